#!/usr/bin/env python3
"""Benchmark: even/odd twisted-mass CG at 32^3 x 64 on one MI355X.

A step is one solve of Qhat^+ Qhat^- x = b to a true relative residual of
1e-10 with the mixed-precision solver (FP16 spinors with per-site FP32 scale,
FP16 two-row links, FP32 arithmetic, FP64 reliable updates), with the gauge
field and the source already resident in HBM.  The hopping half-sweeps inside
the timed steps are timed with HIP events on their launch stream; the
reported value is the algorithmic bandwidth (each input spinor, link and
output counted once) of the plain half-sweeps of the inner operator, K1 and K2
of eqs. (eo3)/(eo4) in 16-bit storage; the half-sweeps that carry the fused
CG update and the FP64 half-sweeps of the reliable updates are reported
beside it.  The same solve in plain FP64 CG is timed beside it for the
mixed-vs-FP64 time-to-solution, and the FP64 oracle is timed on the host
cores on a bounded sample of the same operator and on the whole CG of the
24^3 x 48 workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

WORKLOAD = {
    "dims": (64, 32, 32, 32),  # T, LZ, LY, LX
    "kappa": 0.1632,
    "mu_tilde": 0.004,
    "theta": (1.0, 0.0, 0.0, 0.0),
    "eps": 0.3,
    "gauge_seed": 1002,
    "source_seed": 2200,
    "tol": 1e-10,
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def measured_traffic(family, key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    from paper_0905_3331_amd.profile_hop import kernel_hash

    path = os.path.join(ROOT, "profiles", "hop_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get(family, {}).get(key)


def cpu_baseline(U, b, w, budget_s, full):
    import numpy as np

    import oracle
    import synth

    vh = b.shape[0]
    bytes_qq = 2 * (1536 + 1728) * vh  # same algorithmic model, full 3x3 links (what the oracle reads)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.QhatQhat(U, b, w["kappa"], w["mu_tilde"], w["theta"])
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
        log(f"cpu oracle Qhat^+Qhat^- #{n}: {el:.1f}s")
    # the oracle's whole CG to 1e-10 on the 24^3x48 workload (kappa 0.1632,
    # 2 kappa mu 0.004, links eps 0.3 seed 1001, Gaussian source seed 2100)
    d1 = (48, 24, 24, 24)
    log("cpu oracle: CG to 1e-10 on 24^3x48 (inputs generated first, not timed)")
    U1 = synth.random_gauge(d1, eps=0.3, seed=1001)
    b1 = synth.gaussian_odd(d1, seed=2100)
    t1 = time.perf_counter()
    x1, i1 = oracle.cg(U1, b1, w["kappa"], w["mu_tilde"], w["theta"], tol=1e-10)
    cg1 = time.perf_counter() - t1
    del U1, b1, x1
    log(f"cpu oracle CG 24^3x48: {cg1:.1f} s, {i1['iters']} iterations")
    cgfull = None
    if full:
        log("cpu oracle: CG to 1e-10 on the 32^3x64 workload")
        t2 = time.perf_counter()
        _, i2 = oracle.cg(U, b, w["kappa"], w["mu_tilde"], w["theta"], tol=1e-10)
        cgfull = {"s": round(time.perf_counter() - t2, 2), "iters": i2["iters"]}
        log(f"cpu oracle CG 32^3x64: {cgfull}")
    # the oracle's own CG to 1e-10 on the small full-lattice workload (4^4, kappa 0.16,
    # 2 kappa mu 0.01), timed whole
    d4 = (4, 4, 4, 4)
    U4 = synth.random_gauge(d4, eps=0.3, seed=1000)
    b4 = synth.gaussian_spinor(d4 + (4, 3), seed=2000).reshape(-1, 4, 3)
    t1 = time.perf_counter()
    _, i4 = oracle.cg(U4, b4, 0.16, 0.01, w["theta"], eo=False, tol=1e-10)
    cg4 = time.perf_counter() - t1
    return {
        "value": round(bytes_qq * n / el / 1e9, 3),
        "unit": "GB/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{n} applications of the FP64 oracle's Qhat^+Qhat^- (4 hopping half-sweeps) on the "
                  f"32^3x64 workload, {el:.1f} s; bytes counted with the same algorithmic model",
        "seconds_per_QhatQhat": round(el / n, 3),
        "cg_24c48_s_to_1e-10": round(cg1, 2),
        "cg_24c48_iters": i1["iters"],
        "cg_32c64_s_to_1e-10": cgfull["s"] if cgfull else None,
        "cg_32c64_iters": cgfull["iters"] if cgfull else None,
        "cg_4444_full_ms_to_1e-10": round(cg4 * 1e3, 2),
        "cg_4444_full_iters": i4["iters"],
        **host_cpu(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sloppy", default="fp16", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--link", default="fp16", choices=["fp32", "fp16"])
    ap.add_argument("--cpu-seconds", type=float, default=6.0, help="budget of the CPU oracle's operator sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the CPU oracle's whole CG on the 32^3x64 workload (about 35 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "a lattice would shard by domain decomposition, which is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_0905_3331_amd import tmq

    w = WORKLOAD
    dims = w["dims"]
    log(f"generating the {dims} gauge field (eps {w['eps']}, seed {w['gauge_seed']})")
    U = synth.random_gauge(dims, eps=w["eps"], seed=w["gauge_seed"])
    b = synth.gaussian_odd(dims, seed=w["source_seed"])
    lat = tmq.Lattice(dims, device=0)
    lat.load_gauge(U)
    bd = torch.from_numpy(b).to("cuda:0")
    xd = torch.empty_like(bd)
    p = tmq.params(w["kappa"], w["mu_tilde"], w["theta"])
    mixed = tmq.solver_opts(tol=w["tol"], sloppy=args.sloppy, sloppy_link=args.link)
    fp64 = tmq.solver_opts(tol=w["tol"], sloppy="fp64")
    vh = b.shape[0]

    # calibration: a plain copy kernel, 1 GiB read + 1 GiB written per launch
    copy_gbs = tmq.stream_copy_gbps(1 << 30, reps=5)
    log(f"copy kernel: {copy_gbs:.0f} GB/s")

    log(f"warmup: {args.warmup} mixed solves")
    for _ in range(args.warmup):
        lat.solve(p, bd, mixed, x=xd)
    torch.cuda.synchronize()

    # ---------------------------------------------------------- timed region
    log(f"timed: {args.steps} mixed solves with per-launch hop timing")
    lat.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        _, info = lat.solve(p, bd, mixed, x=xd)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inner = "hop16" if args.sloppy != "fp32" else "hop32"
    fams = ("hop", "hop64", inner, inner + ":pure", inner + ":k1", inner + ":k2", inner + ":fused")
    stats = {f: lat.kernel_stats(f) for f in fams}
    lat.set_kernel_timing(False)
    ms_per_step = (t1 - t0) / args.steps * 1e3

    def gbs(st):
        return st["bytes"] / (st["ms"] * 1e-3) / 1e9 if st["ms"] > 0 else None

    def avg_us(st):
        return round(st["ms"] / st["launches"] * 1e3, 2) if st["launches"] else None

    hop = stats["hop"]
    pure = stats[inner + ":pure"]
    value = gbs(pure)
    log(f"mixed: {ms_per_step:.2f} ms/solve, {infos[-1].iters} iters, {infos[-1].reliable_updates} reliable updates, "
        f"inner half-sweeps {value:.0f} GB/s, all hop launches {gbs(hop):.0f} GB/s")

    # un-instrumented time to solution, mixed and FP64
    def timed_solves(opts, k):
        for _ in range(max(1, args.warmup)):
            lat.solve(p, bd, opts, x=xd)
        torch.cuda.synchronize()
        s = time.perf_counter()
        for _ in range(k):
            _, inf = lat.solve(p, bd, opts, x=xd)
        torch.cuda.synchronize()
        return (time.perf_counter() - s) / k * 1e3, inf

    mixed_ms, mixed_info = timed_solves(mixed, args.steps)
    x_mixed = xd.cpu().numpy()
    log(f"mixed (no events): {mixed_ms:.2f} ms/solve")
    # the paper's own reduced-precision CG (FP64 vectors, the operator switched to its 32-bit form at
    # sqrt(tol)) for comparison; with a 16-bit operator that scheme stalls (its FP64 recursion
    # outruns the operator's accuracy), so it runs with FP32 storage as in the paper
    switch = tmq.solver_opts(tol=w["tol"], sloppy="fp32", sloppy_link="fp32", mode="switch")
    switch_ms, switch_info = timed_solves(switch, max(1, args.steps // 2))
    log(f"switch mode: {switch_ms:.2f} ms/solve, {switch_info.iters} iters")
    lat.set_kernel_timing(True)
    fp64_ms_ev, fp64_info = timed_solves(fp64, 1)
    st64 = lat.kernel_stats("hop64")
    lat.set_kernel_timing(False)
    fp64_ms, fp64_info = timed_solves(fp64, args.steps)
    x_fp64 = xd.cpu().numpy()
    log(f"fp64: {fp64_ms:.2f} ms/solve, {fp64_info.iters} iters")

    dom_name = inner + ":pure"
    dom = pure
    dom_gbs = value
    per_launch_bytes = dom["bytes"] / max(dom["launches"], 1)
    traffic = measured_traffic(dom_name, "hbm_bytes_per_launch")

    verify = None
    if not args.no_verify:
        import oracle

        log("oracle true residuals of the GPU solutions (FP64, host)")
        verify = {
            "mixed_true_rel_residual": oracle.true_residual(U, b, x_mixed, w["kappa"], w["mu_tilde"], w["theta"]),
            "fp64_true_rel_residual": oracle.true_residual(U, b, x_fp64, w["kappa"], w["mu_tilde"], w["theta"]),
        }

    cpu = None
    if not args.no_cpu:
        log(f"cpu baseline: oracle on the host cores for ~{args.cpu_seconds:.0f} s, then its 24^3x48 CG")
        cpu = cpu_baseline(U, b, w, args.cpu_seconds, args.cpu_full)

    # ------------------------------------------ outside the timed region
    # gauge ingest (canonical FP64 links -> the resident copies, with the SU(3)
    # check) and the FP16 spinor codec, each timed on its own
    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    Ud = torch.from_numpy(U).to("cuda:0")
    t_in = timed(lambda: lat.load_gauge(Ud), 3)
    V = int(np.prod(dims))
    in_bytes = V * 4 * 9 * 16
    out_bytes = V * 4 * (144 + 96 + 48 + 24)  # FP64 full, FP64/FP32/FP16 two-row copies
    del Ud
    t_enc = timed(lambda: lat.encode(bd, "fp16"), 5)
    enc_bytes = vh * (192 + 48 + 4)
    ingest = {"gauge_ingest_ms": round(t_in * 1e3, 3), "gauge_ingest_GBps": round((in_bytes + out_bytes) / t_in / 1e9, 1),
              "fp16_encode_ms": round(t_enc * 1e3, 3), "fp16_encode_GBps": round(enc_bytes / t_enc / 1e9, 1)}
    log(f"gauge ingest {ingest['gauge_ingest_ms']} ms, fp16 encode {ingest['fp16_encode_ms']} ms")

    line = {
        "metric": "Hopping-matrix GB/s (% HBM peak); mixed vs FP64 CG time-to-1e-10 at 32^3x64",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"even/odd twisted-mass CG on Qhat^+Qhat^-, 32^3x64, tol 1e-10; inner {args.sloppy} spinors "
                        f"+ {args.link} two-row links with f32 arithmetic, f64 reliable updates",
            "lattice": "32^3x64",
            "kappa": w["kappa"],
            "two_kappa_mu": w["mu_tilde"],
            "theta": list(w["theta"]),
            "links": "random SU(3) exp(i 0.3 H), reunitarised",
            "source": "Gaussian complex, unit variance per component",
            "tol": w["tol"],
        },
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "value_kernels": f"the plain {args.sloppy} half-sweeps K1 and K2 (no fused epilogue) of the timed solves",
        "hop_gflops": round(pure["flops"] / (pure["ms"] * 1e-3) / 1e9, 1),
        "inner_hop": {part: {"GBps": round(gbs(stats[f"{inner}:{part}"]) or 0.0, 1),
                             "avg_us": avg_us(stats[f"{inner}:{part}"]),
                             "launches": stats[f"{inner}:{part}"]["launches"],
                             "algorithmic_bytes_per_launch": round(stats[f"{inner}:{part}"]["bytes"] /
                                                                   max(stats[f"{inner}:{part}"]["launches"], 1))}
                      for part in ("k1", "k2", "fused")},
        "reliable_update_hop64": {"GBps": round(gbs(stats["hop64"]) or 0.0, 1), "avg_us": avg_us(stats["hop64"]),
                                  "launches": stats["hop64"]["launches"]},
        "all_hop_launches_GBps": round(gbs(hop), 1),
        "hop_launches": hop["launches"],
        "mixed_ms_to_1e-10": round(mixed_ms, 3),
        "mixed_iters": mixed_info.iters,
        "mixed_reliable_updates": mixed_info.reliable_updates,
        "fp64_ms_to_1e-10": round(fp64_ms, 3),
        "fp64_iters": fp64_info.iters,
        "speedup_mixed_vs_fp64": round(fp64_ms / mixed_ms, 3),
        "paper_switch_mode_ms_to_1e-10": round(switch_ms, 3),
        "paper_switch_mode_iters": switch_info.iters,
        "paper_switch_mode_true_rel_residual": switch_info.true_rel_residual,
        "fp64_hop_GBps": round(st64["bytes"] / (st64["ms"] * 1e-3) / 1e9, 1) if st64["ms"] > 0 else None,
        "roofline": {
            "kernel": f"hop half-sweeps K1 and K2 ({dom_name}: {args.sloppy} spinors, {args.link} two-row links)",
            "bound": "hbm",
            "achieved": round(dom_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(per_launch_bytes),
            "avg_launch_us": avg_us(dom),
            "launches": dom["launches"],
            "copy_kernel_GBps": round(copy_gbs, 1),
            "frac_of_copy": round(dom_gbs / copy_gbs, 4),
        },
        "cpu_baseline": cpu,
        "ingest_and_codec": ingest,
        "verify": verify,
        "autotune": lat.tuning_report(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
