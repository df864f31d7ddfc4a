"""Drive the hopping kernels for profiling (rocprofv3 kernel traces and counters).

Runs one calibration copy of a known size (kernel ``k_stream_copy``: reads and
writes --copy-mib MiB once each), then --reps applications of Qhat^+ (two hop
half-sweeps, K1 without and K2 with the site term) per requested spinor
precision on a random SU(3) lattice.  The algorithmic bytes of each launch and
the tuned variant are printed, so that counter readings (FETCH_SIZE,
WRITE_SIZE per dispatch) can be scaled by the copy's and compared.

    rocprofv3 --kernel-trace --stats -- python3 -m paper_0905_3331_amd.profile_hop
    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_0905_3331_amd.profile_hop
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="64,32,32,32", help="T,LZ,LY,LX")
    ap.add_argument("--prec", default="fp64,fp16", help="comma list of fp64, fp32, fp16, bf16")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()

    import torch

    import synth
    from paper_0905_3331_amd import tmq

    dims = tuple(int(v) for v in args.dims.split(","))
    copy_bytes = args.copy_mib << 20
    gbs = tmq.stream_copy_gbps(copy_bytes, reps=1)
    print(json.dumps({"calibration": "k_stream_copy", "bytes_read": copy_bytes, "bytes_written": copy_bytes,
                      "launches": 2, "GBps": round(gbs, 1)}), flush=True)
    U = synth.random_gauge(dims, seed=7)
    lat = tmq.Lattice(dims)
    lat.load_gauge(U)
    b = torch.from_numpy(synth.gaussian_odd(dims, seed=3)).cuda()
    out = torch.empty_like(b)
    p = tmq.params(0.1632, 0.004)
    for prec in args.prec.split(","):
        lat.apply_Qhat(p, +1, b, out, prec=prec)  # tunes the variant
        torch.cuda.synchronize()
        lat.set_kernel_timing(True)
        for _ in range(args.reps):
            lat.apply_Qhat(p, +1, b, out, prec=prec)
        st = lat.kernel_stats("hop")
        lat.set_kernel_timing(False)
        print(json.dumps({"prec": prec, "dims": dims, "hop_launches": st["launches"],
                          "avg_us": round(st["ms"] / st["launches"] * 1e3, 2),
                          "algorithmic_bytes_per_launch": st["bytes"] / st["launches"],
                          "GBps": round(st["bytes"] / st["ms"] / 1e6, 1)}), flush=True)
    print(json.dumps(lat.tuning_report()), flush=True)
    lat.close()


if __name__ == "__main__":
    main()
