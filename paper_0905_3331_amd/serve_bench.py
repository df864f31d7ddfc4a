"""Serving benchmark: a stream of solve requests over four lattice sizes.

Workload (the serving pattern of many inversions per gauge configuration,
Sec. 3.2, as a request stream): lattices 8^3x16, 16^3x32, 24^3x48 and
32^3x64 drawn with weights 0.4/0.3/0.2/0.1, each with its own resident
random SU(3) gauge field (eps = 0.3, seed 3100 + size index); per request
kappa = 0.1632, mut drawn uniformly from [0.002, 0.02], a Gaussian source
(one of a few per size, drawn per request) and relative tolerance 1e-8 on the
FP64 true residual, FP32 inner CG with FP32 two-row links.  Arrivals are a
Poisson process (seed 3000).

Runs, on one GPU: each size alone (an idle server, one request at a time),
a burst of requests submitted at once (saturation throughput), then Poisson
streams at fractions of that throughput.  Prints one JSON object with p50/p99
latency and solves/s per run, and per size.

    python -m paper_0905_3331_amd.serve_bench [--requests 2000] [--loads 0.5,0.8]
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from collections import deque

import numpy as np

SIZES = [(16, 8, 8, 8), (32, 16, 16, 16), (48, 24, 24, 24), (64, 32, 32, 32)]
NAMES = ["8^3x16", "16^3x32", "24^3x48", "32^3x64"]
WEIGHTS = [0.4, 0.3, 0.2, 0.1]
KAPPA = 0.1632
MU_RANGE = (0.002, 0.02)
TOL = 1e-8
THETA = (1.0, 0.0, 0.0, 0.0)
N_SRC = 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(tmq, torch, srv):
    import synth

    lids, srcs = [], []
    for j, d in enumerate(SIZES):
        t0 = time.time()
        U = synth.random_gauge(d, eps=0.3, seed=3100 + j)
        lids.append(srv.add_lattice(d, torch.from_numpy(U).to("cuda")))
        del U
        srcs.append([torch.from_numpy(synth.gaussian_odd(d, seed=3000 + 100 * j + k)).to("cuda")
                     for k in range(N_SRC)])
        log(f"lattice {NAMES[j]} ready ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return lids, srcs


def draw(n, seed=3000):
    rng = np.random.default_rng(seed)
    size = rng.choice(len(SIZES), size=n, p=WEIGHTS)
    mu = rng.uniform(*MU_RANGE, size=n)
    src = rng.integers(0, N_SRC, size=n)
    gaps = rng.exponential(1.0, size=n)  # unit-rate inter-arrival gaps
    return size, mu, src, gaps


class Pool:
    """Recycled solution buffers per lattice size."""

    def __init__(self, torch, srcs):
        self.torch = torch
        self.free = [[] for _ in SIZES]
        self.proto = [s[0] for s in srcs]

    def get(self, j):
        return self.free[j].pop() if self.free[j] else self.torch.empty_like(self.proto[j])

    def put(self, j, x):
        self.free[j].append(x)


def run(tmq, srv, lids, srcs, pool, size, mu, src, times, opts):
    """Submit request i at times[i] seconds after the start (None: all at once);
    returns per-request records."""
    srv.reset_stats()
    n = len(size)
    out = [None] * n
    live = deque()

    def collect(block=False):
        while live:
            t, i, j, x = live[0]
            r = srv.wait(t) if block else srv.poll(t)
            if r is None:
                # later requests may have finished first: check the rest once
                for k in range(1, len(live)):
                    t2, i2, j2, x2 = live[k]
                    r2 = srv.poll(t2)
                    if r2 is not None:
                        out[i2] = r2[1]
                        pool.put(j2, x2)
                        live[k] = None
                while None in live:
                    live.remove(None)
                return
            out[i] = r[1]
            pool.put(j, x)
            live.popleft()

    t0 = time.perf_counter()
    for i in range(n):
        if times is not None:
            while True:
                wait = times[i] - (time.perf_counter() - t0)
                if wait <= 0:
                    break
                collect()
                time.sleep(min(wait, 2e-4))
        j = int(size[i])
        x = pool.get(j)
        p = tmq.params(KAPPA, float(mu[i]), THETA)
        t = srv.submit(lids[j], p, srcs[j][int(src[i])], opts, x=x, sync=False)
        live.append((t, i, j, x))
    while live:
        collect(block=True)
    wall = time.perf_counter() - t0
    return out, srv.stats(), wall


def summarise(recs, st, wall, size):
    lat = np.array([r.seconds for r in recs])
    ok = all(r.status == 0 and r.true_rel_residual <= TOL for r in recs)
    per = {}
    for j, name in enumerate(NAMES):
        m = size == j
        if m.any():
            lj = lat[m]
            per[name] = {"n": int(m.sum()), "p50_ms": float(np.percentile(lj, 50) * 1e3),
                         "p99_ms": float(np.percentile(lj, 99) * 1e3),
                         "iters_mean": float(np.mean([recs[i].iters for i in np.nonzero(m)[0]]))}
    return {"requests": len(recs), "all_converged": ok,
            "max_true_rel_residual": float(max(r.true_rel_residual for r in recs)),
            "solves_per_s": st["solves_per_s"], "wall_s": wall,
            "p50_ms": st["p50_s"] * 1e3, "p99_ms": st["p99_s"] * 1e3, "mean_ms": st["mean_s"] * 1e3,
            "mean_wait_ms": st["mean_wait_s"] * 1e3, "peak_running": st["peak_running"],
            "peak_gb": st["peak_bytes"] / 1e9, "engines": st["engines"], "steps": st["steps"],
            "per_size": per}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=2000, help="requests per Poisson run")
    ap.add_argument("--burst", type=int, default=400, help="requests of the saturation run")
    ap.add_argument("--loads", default="0.5,0.8,0.95", help="Poisson rates as fractions of saturation throughput")
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=0.0, help="0: 60%% of free device memory")
    ap.add_argument("--sloppy", default="fp32")
    args = ap.parse_args(argv)

    import torch

    from paper_0905_3331_amd import tmq

    if not torch.cuda.is_available():
        raise SystemExit("serve_bench needs a GPU")
    opts = tmq.solver_opts(tol=TOL, sloppy=args.sloppy, sloppy_link="fp32" if args.sloppy == "fp32" else "fp16")
    result = {"workload": "serving stream 8^3x16/16^3x32/24^3x48/32^3x64 (0.4/0.3/0.2/0.1), kappa 0.1632, "
                          "mut U[0.002,0.02], tol 1e-8 (FP64 true residual), inner " + args.sloppy,
              "max_batch": args.max_batch}
    with tmq.Server(budget_bytes=int(args.budget_gb * 1e9), max_batch=args.max_batch) as srv:
        lids, srcs = setup(tmq, torch, srv)
        pool = Pool(torch, srcs)
        # warm-up: every size once (kernel autotuning happens here)
        for j in range(len(SIZES)):
            run(tmq, srv, lids, srcs, pool, np.array([j] * 3), np.full(3, 0.004), np.arange(3), None, opts)
        alone = {}
        for j, name in enumerate(NAMES):
            lat = []
            for k in range(5):
                recs, st, _ = run(tmq, srv, lids, srcs, pool, np.array([j]), np.array([0.002 + 0.004 * k]),
                                  np.array([k % N_SRC]), None, opts)
                lat.append(recs[0].seconds)
            alone[name] = {"p50_ms": float(np.median(lat) * 1e3), "iters": recs[0].iters}
            log(f"alone {name}: {alone[name]}")
        result["alone"] = alone
        size, mu, src, gaps = draw(args.burst, seed=3001)
        recs, st, wall = run(tmq, srv, lids, srcs, pool, size, mu, src, None, opts)
        burst = summarise(recs, st, wall, size)
        result["burst"] = burst
        cap = burst["solves_per_s"]
        log(f"burst: {cap:.1f} solves/s, p50 {burst['p50_ms']:.1f} ms")
        result["poisson"] = []
        for load in [float(v) for v in args.loads.split(",") if v]:
            size, mu, src, gaps = draw(args.requests, seed=3000)
            rate = load * cap
            times = np.cumsum(gaps) / rate
            recs, st, wall = run(tmq, srv, lids, srcs, pool, size, mu, src, times, opts)
            s = summarise(recs, st, wall, size)
            s.update({"load": load, "rate_per_s": rate})
            result["poisson"].append(s)
            log(f"poisson load {load}: {s['solves_per_s']:.1f} solves/s p50 {s['p50_ms']:.1f} ms "
                f"p99 {s['p99_ms']:.1f} ms")
    print(json.dumps(result))
    return result


if __name__ == "__main__":
    main()
