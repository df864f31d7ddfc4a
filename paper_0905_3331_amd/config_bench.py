"""Timings of the other benchmark workloads (one MI355X).

  4^4 full     plain FP64 CG on the full-lattice Q^+Q^- (no even/odd), 4^4,
               kappa 0.16, 2 kappa mu 0.01, Gaussian source, tol 1e-10
  24^3x48      even/odd Qhat^+Qhat^-: FP64 CG vs FP32-inner / FP64-outer CG,
               kappa 0.1632, 2 kappa mu 0.004, 5 Gaussian sources, tol 1e-10;
               hop half-sweep bandwidth per storage precision
  24^3x48 x48  48 right-hand sides in one batch: 12 spin-colour point sources
               at one odd site x 2 kappa mu in {0.002, 0.004, 0.008, 0.016},
               FP32 inner / FP64 outer, tol 1e-10 each; against the same 48
               solved one after another; the same batch with FP16 inner spinors
               and links

  doublet      the mass non-degenerate doublet of eq. (Dh) at 32^3x64 with the
               paper's doublet run parameters (kappa 0.17, 2 kappa mubar 0.1105,
               2 kappa epsbar 0.0935): doublet hop half-sweep bandwidth per
               storage precision (links read once for both flavours), and CG on
               Qhat_h^+ Qhat_h^- to 1e-10, FP64 vs FP32-inner vs FP16-inner,
               3 Gaussian doublet sources, median

  minv         24^3x48 (kappa 0.1632, 2 kappa mu 0.004, tol 1e-10): the full-lattice
               M^+ psi = phi by the even/odd factorisation with CG on the normal
               equations (FP64 and FP16-inner) against BiCGstab on Qhat^+ itself
               (FP64); the odd-site system Qhat^+ x = b by BiCGstab against CG on
               Qhat^+ Qhat^- followed by Qhat^-; a propagator (the 12
               spin-colour point sources of one site) batched against one
               after another; the one-end-trick pion
               correlator of one complex Z2 time-slice source (FP16-inner)

  hopcache     the Qhat^+ half-sweeps at 32^3x64 and at 8x32^3 (the share of one
               of 8 GPUs when 32^3x64 is split along t; periodic here), each
               precision timed back to back and with a 1 GiB copy before every
               operator application, which evicts L2 and the 256 MB Infinity
               Cache: whether the bandwidth figures are HBM or cache figures

Links are random SU(3) exp(i 0.3 H), reunitarised (seeds 1000 + workload);
theta = (1, 0, 0, 0).  Prints one JSON object.  The solutions' accuracy
against the FP64 oracle is checked by the GPU tests at these shapes.

    python -m paper_0905_3331_amd.config_bench
"""
from __future__ import annotations

import argparse
import os
import json
import sys
import time

import numpy as np

THETA = (1.0, 0.0, 0.0, 0.0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def median_time(fn, reps):
    import torch

    ts = []
    out = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def full_4444(tmq, torch, synth, reps):
    dims = (4, 4, 4, 4)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1000))
    b = torch.from_numpy(synth.gaussian_spinor(dims + (4, 3), seed=2000).reshape(-1, 4, 3)).cuda()
    p = tmq.params(0.16, 0.01, THETA)
    opts = tmq.solver_opts(tol=1e-10)
    lat.solve_full(p, b, opts)
    t, (x, info) = median_time(lambda: lat.solve_full(p, b, opts), reps)
    lat.close()
    return {"lattice": "4^4", "operator": "full Q^+Q^-, FP64 CG", "ms_to_1e-10": t * 1e3, "iters": info.iters,
            "true_rel_residual": info.true_rel_residual}


def hop_rates(tmq, torch, synth, lat, dims, reps=20):
    b = torch.from_numpy(synth.gaussian_odd(dims, seed=3)).cuda()
    out = torch.empty_like(b)
    p = tmq.params(0.1632, 0.004, THETA)
    res = {}
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        lat.apply_Qhat(p, +1, b, out, prec=prec)
        torch.cuda.synchronize()
        lat.set_kernel_timing(True)
        for _ in range(reps):
            lat.apply_Qhat(p, +1, b, out, prec=prec)
        st = lat.kernel_stats("hop")
        lat.set_kernel_timing(False)
        res[prec] = {"avg_us": st["ms"] / st["launches"] * 1e3,
                     "GBps": st["bytes"] / (st["ms"] * 1e-3) / 1e9,
                     "GFLOPs": st["flops"] / (st["ms"] * 1e-3) / 1e9}
    return res


def eo_24c48(tmq, torch, synth, reps):
    dims = (48, 24, 24, 24)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1001))
    p = tmq.params(0.1632, 0.004, THETA)
    out = {"lattice": "24^3x48", "hop": hop_rates(tmq, torch, synth, lat, dims)}
    for name, opts in (("fp64", tmq.solver_opts(tol=1e-10)),
                       ("fp32_inner", tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")),
                       ("fp16_inner", tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")),
                       ("fp32_switch_paper", tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32",
                                                             mode="switch"))):
        times, iters, rus, res = [], [], [], []
        for k in range(5):
            b = torch.from_numpy(synth.gaussian_odd(dims, seed=2100 + k)).cuda()
            lat.solve(p, b, opts)
            t, (x, info) = median_time(lambda: lat.solve(p, b, opts), reps)
            times.append(t)
            iters.append(info.iters)
            rus.append(info.reliable_updates)
            res.append(info.true_rel_residual)
        out[name] = {"ms_to_1e-10_median_of_5_sources": float(np.median(times)) * 1e3,
                     "iters": iters, "reliable_updates": rus, "max_true_rel_residual": max(res)}
    out["speedup_fp32_inner_vs_fp64"] = out["fp64"]["ms_to_1e-10_median_of_5_sources"] / \
        out["fp32_inner"]["ms_to_1e-10_median_of_5_sources"]
    lat.close()
    return out


def batch_24c48(tmq, torch, synth, reps):
    dims = (48, 24, 24, 24)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1003))
    vh = int(np.prod(dims)) // 2
    site = int(np.random.default_rng(2300).integers(0, vh))
    muts = (0.002, 0.004, 0.008, 0.016)
    ps, bs = [], []
    for mut in muts:
        for k in range(12):
            bs.append(torch.from_numpy(synth.point_source_odd(dims, site, k // 3, k % 3)).cuda())
            ps.append(tmq.params(0.1632, mut, THETA))
    opts = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    xs = [torch.empty_like(b) for b in bs]
    lat.solve_batch(ps, bs, opts, xs=xs)  # tunes the batched launches
    t_batch, (_, infos) = median_time(lambda: lat.solve_batch(ps, bs, opts, xs=xs), reps)
    lat.set_kernel_timing(True)
    lat.solve_batch(ps, bs, opts, xs=xs)
    st = lat.kernel_stats("hop")
    lat.set_kernel_timing(False)

    def alone():
        inf = []
        for i in range(len(bs)):
            _, f = lat.solve(ps[i], bs[i], opts, x=xs[i])
            inf.append(f)
        return inf

    t_alone, infos_alone = median_time(alone, 1)
    # the same batch with FP16 spinors and links in the inner iteration
    o16 = tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")
    lat.solve_batch(ps, bs, o16, xs=xs)  # tunes the FP16 batched launches
    t16, (_, inf16) = median_time(lambda: lat.solve_batch(ps, bs, o16, xs=xs), reps)
    x16 = [x.clone() for x in xs]
    lat.solve_batch(ps, bs, opts, xs=xs)
    x32 = [x.clone() for x in xs]
    # both again with the iteration bodies captured as HIP graphs (the first
    # solve runs each body once plainly, then captures one graph per ring entry)
    os.environ["TMQ_ENGINE_GRAPHS"] = "1"
    lat.solve_batch(ps, bs, opts, xs=xs)
    tg32, _ = median_time(lambda: lat.solve_batch(ps, bs, opts, xs=xs), reps)
    same32 = all(torch.equal(a, b) for a, b in zip(xs, x32))
    lat.solve_batch(ps, bs, o16, xs=xs)
    tg16, _ = median_time(lambda: lat.solve_batch(ps, bs, o16, xs=xs), reps)
    same16 = all(torch.equal(a, b) for a, b in zip(xs, x16))
    del os.environ["TMQ_ENGINE_GRAPHS"]
    report = lat.tuning_report()
    lat.close()
    return {"lattice": "24^3x48", "nrhs": len(bs), "point_site": site,
            "batch_ms": t_batch * 1e3, "per_rhs_ms": t_batch * 1e3 / len(bs),
            "one_after_another_ms": t_alone * 1e3, "speedup_batch_vs_alone": t_alone / t_batch,
            "iters": [f.iters for f in infos], "all_converged": all(f.status == 0 for f in infos),
            "max_true_rel_residual": max(f.true_rel_residual for f in infos),
            "batch_hop_GBps_links_once": st["bytes"] / (st["ms"] * 1e-3) / 1e9,
            "batch_hop_launch_us": st["ms"] / st["launches"] * 1e3,
            "fp16_inner_batch_ms": t16 * 1e3, "fp16_inner_iters": [f.iters for f in inf16],
            "fp16_inner_all_converged": all(f.status == 0 for f in inf16),
            "fp16_inner_max_true_rel_residual": max(f.true_rel_residual for f in inf16),
            "hip_graph_bodies": {"fp32_inner_batch_ms": tg32 * 1e3, "fp16_inner_batch_ms": tg16 * 1e3,
                                 "same_solutions_bit_for_bit": same32 and same16},
            "batch_tuning": report.get("batch")}


def batch_sweep(tmq, torch, synth, reps):
    """The batched FP32 half-sweeps of 48 right-hand sides at 24^3x48 for every
    block order (z-slabs, t-slabs, plain) and RHS group size: short solves
    (three iterations) with the variant and group forced (TMQ_HOP_VARIANT,
    TMQ_HOP_GROUP), each preceded by a 1 MiB copy-kernel launch pair that
    marks it in a counter run (profile_hop --summarize-batch-sweep), and its
    half-sweeps timed with events.  Under rocprofv3 --pmc FETCH_SIZE this
    gives each configuration's HBM reads per launch."""
    dims = (48, 24, 24, 24)
    vh = int(np.prod(dims)) // 2
    U = synth.random_gauge(dims, eps=0.3, seed=1003)
    bs = [torch.from_numpy(synth.gaussian_odd(dims, seed=5000 + i)).cuda() for i in range(48)]
    ps = [tmq.params(0.1632, 0.002 * (1 + i % 4), THETA) for i in range(48)]
    opts = tmq.solver_opts(tol=1e-14, sloppy="fp32", sloppy_link="fp32", max_iter=3)
    rows = []
    for var in (1, 3, 0):
        os.environ["TMQ_HOP_VARIANT"] = str(var)
        lat = tmq.Lattice(dims)
        lat.load_gauge(U)
        for g in (1, 2, 4, 8, 16, 32, 48):
            os.environ["TMQ_HOP_GROUP"] = str(g)
            lat.solve_batch(ps, bs, opts, check=False)  # tunes (first time) and warms
            tmq.stream_copy_gbps(1 << 20, reps=1)       # marker
            lat.set_kernel_timing(True)
            lat.solve_batch(ps, bs, opts, check=False)
            st = {k: lat.kernel_stats("hop32:" + k) for k in ("k1", "k2", "fused")}
            lat.set_kernel_timing(False)
            rows.append({"variant": var, "group": g,
                         **{f"{k}_us": v["ms"] / max(v["launches"], 1) * 1e3 for k, v in st.items()},
                         **{f"{k}_algorithmic_bytes": v["bytes"] / max(v["launches"], 1) for k, v in st.items()}})
            # reads of a K1 launch: its bytes less the 48 FP32 outputs it writes
            rows[-1]["k1_algorithmic_read_bytes"] = rows[-1]["k1_algorithmic_bytes"] - 48 * vh * 96.0
            log(f"variant {var} group {g}: K1 {rows[-1]['k1_us']:.0f} us")
        del os.environ["TMQ_HOP_GROUP"]
        lat.close()
    del os.environ["TMQ_HOP_VARIANT"]
    return {"lattice": "24^3x48", "nrhs": 48, "rows": rows}


def batch_profile(tmq, torch, synth, reps):
    """One tuned 48-right-hand-side batch solve of the batch workload (FP32
    inner) for counter runs: rocprofv3 --pmc FETCH_SIZE (or WRITE_SIZE) --
    python3 -m paper_0905_3331_amd.config_bench --only batchprof.  The copy
    kernel runs first for the counters' calibration (1 GiB read and written)."""
    gbs = tmq.stream_copy_gbps(1 << 30, reps=1)
    dims = (48, 24, 24, 24)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1003))
    vh = int(np.prod(dims)) // 2
    site = int(np.random.default_rng(2300).integers(0, vh))
    ps, bs = [], []
    for mut in (0.002, 0.004, 0.008, 0.016):
        for k in range(12):
            bs.append(torch.from_numpy(synth.point_source_odd(dims, site, k // 3, k % 3)).cuda())
            ps.append(tmq.params(0.1632, mut, THETA))
    opts = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    xs = [torch.empty_like(b) for b in bs]
    lat.solve_batch(ps, bs, opts, xs=xs)  # tunes
    lat.set_kernel_timing(True)
    _, infos = lat.solve_batch(ps, bs, opts, xs=xs)
    st = {k: lat.kernel_stats("hop32:" + k) for k in ("k1", "k2", "fused")}
    lat.set_kernel_timing(False)
    report = lat.tuning_report()
    lat.close()
    return {"copy_GBps": gbs, "iters": [f.iters for f in infos],
            "fp32_half_sweeps": {k: {"launches": v["launches"], "avg_us": v["ms"] / max(v["launches"], 1) * 1e3,
                                     "algorithmic_bytes_per_launch": v["bytes"] / max(v["launches"], 1)}
                                 for k, v in st.items()},
            "batch_tuning": report.get("batch")}


def nd_32c64(tmq, torch, synth, reps):
    dims = (64, 32, 32, 32)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1002))
    p = tmq.nd_params(0.17, 0.1105, 0.0935, THETA)

    def src(seed):
        return torch.from_numpy(np.stack([synth.gaussian_odd(dims, seed=seed),
                                          synth.gaussian_odd(dims, seed=seed + 1)])).cuda()

    out = {"lattice": "32^3x64", "kappa": 0.17, "mubar_tilde": 0.1105, "epsbar_tilde": 0.0935, "hop": {}}
    b = src(2400)
    o = torch.empty_like(b)
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        lat.apply_Qhat_nd(p, +1, b, o, prec=prec)
        torch.cuda.synchronize()
        lat.set_kernel_timing(True)
        for _ in range(20):
            lat.apply_Qhat_nd(p, +1, b, o, prec=prec)
        st = lat.kernel_stats("hop")
        lat.set_kernel_timing(False)
        out["hop"][prec] = {"avg_us": st["ms"] / st["launches"] * 1e3,
                            "GBps": st["bytes"] / (st["ms"] * 1e-3) / 1e9,
                            "GFLOPs": st["flops"] / (st["ms"] * 1e-3) / 1e9}
    for name, opts in (("fp64", tmq.solver_opts(tol=1e-10)),
                       ("fp32_inner", tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")),
                       ("fp16_inner", tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16"))):
        times, iters, rus, res = [], [], [], []
        for k in range(3):
            bk = src(2410 + 2 * k)
            lat.solve_nd(p, bk, opts)
            t, (x, info) = median_time(lambda: lat.solve_nd(p, bk, opts), reps)
            times.append(t)
            iters.append(info.iters)
            rus.append(info.reliable_updates)
            res.append(info.true_rel_residual)
        out[name] = {"ms_to_1e-10_median_of_3_sources": float(np.median(times)) * 1e3,
                     "iters": iters, "reliable_updates": rus, "max_true_rel_residual": max(res)}
    out["speedup_fp16_inner_vs_fp64"] = out["fp64"]["ms_to_1e-10_median_of_3_sources"] / \
        out["fp16_inner"]["ms_to_1e-10_median_of_3_sources"]
    lat.close()
    return out


def minv_24c48(tmq, torch, synth, reps):
    dims = (48, 24, 24, 24)
    lat = tmq.Lattice(dims)
    lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1001))
    p = tmq.params(0.1632, 0.004, THETA)
    out = {"lattice": "24^3x48"}
    phi = torch.from_numpy(synth.gaussian_spinor(dims + (4, 3), seed=2600).reshape(-1, 4, 3)).cuda()
    for name, opts in (("cg_fp64", tmq.solver_opts(tol=1e-10)),
                       ("cg_fp16_inner", tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")),
                       ("bicgstab_fp64", tmq.solver_opts(tol=1e-10, mode="bicgstab"))):
        lat.solve_M(p, +1, phi, opts)
        t, (psi, info) = median_time(lambda: lat.solve_M(p, +1, phi, opts), reps)
        out["M_inverse_" + name] = {"ms": t * 1e3, "iters": info.iters, "true_rel_residual": info.true_rel_residual}
    b = torch.from_numpy(synth.gaussian_odd(dims, seed=2601)).cuda()
    o64 = tmq.solver_opts(tol=1e-10)
    lat.solve_Qhat(p, +1, b, o64)
    t, (x, info) = median_time(lambda: lat.solve_Qhat(p, +1, b, o64), reps)
    out["Qhat_plus_bicgstab_fp64"] = {"ms": t * 1e3, "iters": info.iters, "true_rel_residual": info.true_rel_residual}

    def cg_route():
        y, inf = lat.solve(p, b, o64)
        return lat.apply_Qhat(p, -1, y), inf

    cg_route()
    t, (x, info) = median_time(cg_route, reps)
    out["Qhat_plus_cg_normal_fp64"] = {"ms": t * 1e3, "iters": info.iters}
    # a propagator: the 12 spin-colour point sources at one site, batched and one after another
    V = int(np.prod(dims))
    site = int(np.random.default_rng(2603).integers(0, V))
    srcs = []
    for k in range(12):
        e = torch.zeros((V, 4, 3), dtype=torch.complex128, device="cuda")
        e[site, k // 3, k % 3] = 1.0
        srcs.append(e)
    for name, opts in (("fp64", tmq.solver_opts(tol=1e-10)),
                       ("fp16_inner", tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16"))):
        lat.solve_M_batch(p, +1, srcs, opts)
        tb, (_, infos) = median_time(lambda: lat.solve_M_batch(p, +1, srcs, opts), reps)
        ta, _ = median_time(lambda: [lat.solve_M(p, +1, e, opts) for e in srcs], 1)
        out["propagator_12_point_sources_" + name] = {
            "batch_ms": tb * 1e3, "one_after_another_ms": ta * 1e3, "speedup": ta / tb,
            "iters": [i.iters for i in infos], "max_true_rel_residual": max(i.true_rel_residual for i in infos)}
    xi = torch.from_numpy(synth.z2_timeslice_source(dims, 0, seed=2602).reshape(-1, 4, 3)).cuda()
    o16 = tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")
    lat.pion_correlator(p, xi, o16)
    t, (c, ph, info) = median_time(lambda: lat.pion_correlator(p, xi, o16), reps)
    out["pion_correlator_fp16_inner"] = {"ms": t * 1e3, "iters": info.iters,
                                         "C_0_to_4": [float(v) for v in c[:5]]}
    lat.close()
    return out


def hop_cache(tmq, torch, synth, reps):
    big_a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    big_b = torch.empty_like(big_a)
    p = tmq.params(0.1632, 0.004, THETA)
    out = {}
    for dims in ((64, 32, 32, 32), (8, 32, 32, 32)):
        lat = tmq.Lattice(dims)
        lat.load_gauge(synth.random_gauge(dims, eps=0.3, seed=1005))
        b = torch.from_numpy(synth.gaussian_odd(dims, seed=2500)).cuda()
        o = torch.empty_like(b)
        key = "x".join(map(str, dims))
        out[key] = {}
        for prec in ("fp64", "fp32", "fp16"):
            lat.apply_Qhat(p, +1, b, o, prec=prec)  # tunes the launches
            torch.cuda.synchronize()
            row = {}
            for mode in ("back_to_back", "cache_evicted"):
                lat.set_kernel_timing(True)
                for _ in range(10 * reps):
                    if mode == "cache_evicted":
                        big_b.copy_(big_a)
                    lat.apply_Qhat(p, +1, b, o, prec=prec)
                st = lat.kernel_stats("hop")
                lat.set_kernel_timing(False)
                row[mode] = {"avg_us": st["ms"] / st["launches"] * 1e3,
                             "GBps": st["bytes"] / (st["ms"] * 1e-3) / 1e9}
            out[key][prec] = row
        lat.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--only", default="full,eo,batch,nd,minv,hopcache")
    args = ap.parse_args(argv)
    import torch

    import synth
    from paper_0905_3331_amd import tmq

    if not torch.cuda.is_available():
        raise SystemExit("config_bench needs a GPU")
    want = args.only.split(",")
    res = {}
    if "full" in want:
        log("4^4 full-lattice FP64 CG")
        res["full_4444"] = full_4444(tmq, torch, synth, max(args.reps, 5))
    if "eo" in want:
        log("24^3x48 even/odd: FP64 vs mixed")
        res["eo_24c48"] = eo_24c48(tmq, torch, synth, args.reps)
    if "batch" in want:
        log("24^3x48 batch of 48")
        res["batch_24c48_48rhs"] = batch_24c48(tmq, torch, synth, args.reps)
    if "batchsweep" in want:
        log("24^3x48 batch of 48, block orders x RHS groups")
        res["batch_sweep"] = batch_sweep(tmq, torch, synth, args.reps)
    if "batchprof" in want:
        log("24^3x48 batch of 48, one solve for counter runs")
        res["batch_profile"] = batch_profile(tmq, torch, synth, args.reps)
    if "nd" in want:
        log("32^3x64 flavour doublet")
        res["doublet_32c64"] = nd_32c64(tmq, torch, synth, args.reps)
    if "minv" in want:
        log("24^3x48 full-lattice inversion, BiCGstab, correlator")
        res["minv_24c48"] = minv_24c48(tmq, torch, synth, args.reps)
    if "hopcache" in want:
        log("32^3x64 and 8x32^3 half-sweeps, back to back and with the caches evicted")
        res["hop_cache"] = hop_cache(tmq, torch, synth, args.reps)
    print(json.dumps(res))
    return res


if __name__ == "__main__":
    main()
