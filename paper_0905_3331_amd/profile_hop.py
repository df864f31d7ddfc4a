"""Drive the hopping kernels for profiling (rocprofv3 kernel traces and counters),
and summarise what rocprofv3 wrote.

Runs one calibration copy of a known size (kernel ``k_stream_copy``: reads and
writes --copy-mib MiB once each), then --reps applications of Qhat^+ (two hop
half-sweeps, K1 without and K2 with the site term) per requested spinor
precision on a random SU(3) lattice.  The algorithmic bytes of each launch and
the tuned variant are printed, so that counter readings (FETCH_SIZE,
WRITE_SIZE per dispatch) can be scaled by the copy's and compared.

    rocprofv3 --kernel-trace --stats -- python3 -m paper_0905_3331_amd.profile_hop
    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_0905_3331_amd.profile_hop

Summaries (no GPU needed):

    python -m paper_0905_3331_amd.profile_hop --summarize-trace STATS_CSV --cmd "..." --out FILE.md
    python -m paper_0905_3331_amd.profile_hop --summarize-pmc FETCH_CSV WRITE_CSV --copy-bytes N \
        --cmd "..." --out profiles/hop_traffic.json

    python -m paper_0905_3331_amd.profile_hop --summarize-valu COUNTER_CSV --cmd "..." --out FILE.md

The traffic summary scales each counter by what it reads for the plain copy
kernel (k_stream_copy, N bytes read and N written per launch), averages it
over the dispatches of each hop family (hop16: FP16/BF16 spinors, hop32,
hop64) and records the hash of the kernel sources, so that a benchmark can
tell whether the figures belong to the current kernels.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# sources that determine the hop kernels' memory traffic
KERNEL_SOURCES = ("hop_impl.h", "hop.hip", "hop_f64.hip", "hop_f32.hip", "hop_f16.hip", "hop_b16.hip",
                  "hop16_f16.hip", "hop16_b16.hip",
                  "fields.h", "spin.h", "views.h", "kernels.h", "devutil.h", "fastdiv.h")


def code_text(src: str) -> str:
    """The code of a C++ source without its comments and blank lines, so that
    editing a comment leaves the kernel hash unchanged (string literals in
    these sources hold no comment markers)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in src.splitlines())
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_hash() -> str:
    """Hash of the code (comments aside) of the sources that make the hop kernels."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0905_3331_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def is_hop(name: str) -> bool:
    """A hop half-sweep kernel: the general hop_kernel or the 16-bit hop16_kernel."""
    return "hop_kernel<" in name or "hop16_kernel<" in name


def hop_family(name: str):
    if not is_hop(name):
        return None
    if "Sp16" in name:
        return "hop16"
    if "SpF32" in name:
        return "hop32"
    if "SpF64" in name:
        return "hop64"
    return None


def hop_template_args(name: str):
    """Template arguments of a hop kernel instantiation, as text, in order:
    hop_kernel: spinor format, link format, SELF, NORM, NT, ORD, SB, G, EP, ND;
    hop16_kernel: spinor format, SELF, NORM, ORD, SB, EP, ND, PM, K2F, BATCH."""
    key = "hop16_kernel<" if "hop16_kernel<" in name else "hop_kernel<"
    i = name.find(key)
    if i < 0:
        return None
    depth, cur, args = 0, "", []
    for ch in name[i + len(key):]:
        if ch == "<":
            depth += 1
        elif ch == ">":
            if depth == 0:
                args.append(cur.strip())
                return args
            depth -= 1
        if ch == "," and depth == 0:
            args.append(cur.strip())
            cur = ""
        else:
            cur += ch
    return None


def hop_part(name: str):
    """Which half-sweep an instantiation is: "k1" (no site term of its own
    parity: K1 of eq. (eo3)), "k2" (K2 of eq. (eo4) storing its output),
    "fused" (K2 with the CG update or the true residual fused), or None."""
    a = hop_template_args(name)
    if a and "hop16_kernel<" in name and len(a) >= 8:
        self_, ep = a[1] == "true", a[5]
    elif a and len(a) >= 10:
        self_, ep = a[2] == "true", a[8]
    else:
        return None
    if ep != "0":
        return "fused"
    return "k2" if self_ else "k1"


def _counter_rows(path, counter):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def traffic_markdown(res, title, algorithmic=None):
    """Markdown of a traffic summary (summarize_pmc's result): the family and
    half-sweep averages, then every instantiation.  algorithmic: optional
    {family or part: algorithmic bytes per launch} printed beside them."""
    algorithmic = algorithmic or {}
    lines = [f"# {title}", "", "Commands (GPU box, repo root; one pass per counter):", "", "    " + res["command"], "",
             f"Calibration: the plain copy kernel (k_stream_copy) reads and writes {res['copy_bytes']} bytes per launch; "
             f"HBM read bytes = FETCH_SIZE x 1024 x {res['fetch_scale']:.4f}, write bytes = WRITE_SIZE x 1024 x "
             f"{res['write_scale']:.4f}.", "",
             f"Kernel sources hash: {res['kernel_hash']} (bench.py reports these figures as `roofline.traffic` only while "
             "the hash matches the sources).", "",
             "| family or half-sweep | dispatches (fetch, write) | HBM read MB/launch | HBM write MB/launch | "
             "total MB/launch | algorithmic MB/launch |", "|---|---|---|---|---|---|"]
    for k in sorted(x for x in res if x.startswith("hop")):
        d = res[k]
        alg = algorithmic.get(k)
        lines.append(f"| {k} | {d['dispatches'][0]}, {d['dispatches'][1]} | {d['read_bytes_per_launch'] / 1e6:.1f} | "
                     f"{d['write_bytes_per_launch'] / 1e6:.1f} | {d['hbm_bytes_per_launch'] / 1e6:.1f} | "
                     f"{'%.1f' % (alg / 1e6) if alg else '-'} |")
    lines += ["", "Per instantiation (the few-dispatch rows are autotuner candidates):", "",
              "| kernel | dispatches | read MB | write MB |", "|---|---|---|---|"]
    for k in sorted(res["per_kernel"]):
        v = res["per_kernel"][k]
        name = k.replace("tmq::", "").split("(")[0]
        lines.append(f"| `{name}` | {v.get('dispatches', 0)} | {v.get('read_bytes_per_launch', 0) / 1e6:.1f} | "
                     f"{v.get('write_bytes_per_launch', 0) / 1e6:.1f} |")
    lines.append("")
    return "\n".join(lines)


def summarize_pmc(fetch_csv, write_csv, copy_bytes, cmd, out):
    f = _counter_rows(fetch_csv, "FETCH_SIZE")
    w = _counter_rows(write_csv, "WRITE_SIZE")
    copy = [k for k in f if "k_stream_copy" in k]
    if not copy or not [k for k in w if "k_stream_copy" in k]:
        raise SystemExit("no k_stream_copy dispatch in the counter files")
    fcopy = sum(f[copy[0]]) / len(f[copy[0]]) * 1024.0
    wk = [k for k in w if "k_stream_copy" in k][0]
    wcopy = sum(w[wk]) / len(w[wk]) * 1024.0
    fscale, wscale = copy_bytes / fcopy, copy_bytes / wcopy
    # instantiations launched only while the autotuner timed its candidates
    # (a few dispatches each) are left out of the family averages
    def used(rows):
        top = collections.Counter()
        for k, v in rows.items():
            fa = hop_family(k)
            if fa:
                top[fa] = max(top[fa], len(v))
        return {k for k, v in rows.items() if hop_family(k) and len(v) >= 0.1 * top[hop_family(k)]}

    fam = collections.defaultdict(lambda: {"fetch": [], "write": []})
    per_kernel = {}
    fu, wu = used(f), used(w)
    def groups(k):
        # the family, and its parts: ":pure" (K1 and K2), ":k1", ":k2", ":fused"
        fa, part = hop_family(k), hop_part(k)
        out = [fa]
        if part:
            out.append(f"{fa}:{part}")
            if part != "fused":
                out.append(f"{fa}:pure")
        return out

    for k, v in f.items():
        fa = hop_family(k)
        if fa:
            per_kernel.setdefault(k, {})["read_bytes_per_launch"] = sum(v) / len(v) * 1024.0 * fscale
            per_kernel[k]["dispatches"] = len(v)
            if k in fu:
                for gname in groups(k):
                    fam[gname]["fetch"] += [x * 1024.0 * fscale for x in v]
    for k, v in w.items():
        fa = hop_family(k)
        if fa:
            per_kernel.setdefault(k, {})["write_bytes_per_launch"] = sum(v) / len(v) * 1024.0 * wscale
            if k in wu:
                for gname in groups(k):
                    fam[gname]["write"] += [x * 1024.0 * wscale for x in v]
    res = {"kernel_hash": kernel_hash(), "command": cmd, "copy_bytes": copy_bytes,
           "fetch_scale": fscale, "write_scale": wscale, "per_kernel": per_kernel}
    for fa, d in fam.items():
        if d["fetch"] and d["write"]:
            res[fa] = {"hbm_bytes_per_launch": sum(d["fetch"]) / len(d["fetch"]) + sum(d["write"]) / len(d["write"]),
                       "read_bytes_per_launch": sum(d["fetch"]) / len(d["fetch"]),
                       "write_bytes_per_launch": sum(d["write"]) / len(d["write"]),
                       "dispatches": [len(d["fetch"]), len(d["write"])]}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "per_kernel"}))


def summarize_trace(stats_csv, cmd, out):
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# Kernel trace: " + os.path.basename(out).replace(".md", ""), "",
             "Command (repo root, one MI355X, rocprofv3 --kernel-trace --stats):", "", "    " + cmd, "",
             "| kernel | calls | total ms | share | avg us |", "|---|---|---|---|---|"]
    fam = collections.defaultdict(lambda: [0, 0.0])
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        n, t = int(r["Calls"]), float(r["TotalDurationNs"])
        name = r["Name"].replace("tmq::", "")
        if len(name) > 110:
            name = name[:107] + "..."
        if t / tot >= 0.002:
            lines.append(f"| `{name}` | {n} | {t / 1e6:.2f} | {100 * t / tot:.1f} % | {t / n / 1e3:.2f} |")
        fa = hop_family(r["Name"])
        if fa:
            fam[fa][0] += n
            fam[fa][1] += t
    lines += ["", "Hop families (all instantiations together):", "", "| family | launches | avg us |", "|---|---|---|"]
    for fa, (n, t) in sorted(fam.items()):
        lines.append(f"| {fa} | {n} | {t / n / 1e3:.2f} |")
    lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def summarize_valu(counter_csv, cmd, out, xcds=8, simds=1024, min_dispatches=20):
    """VALU instructions per wave and VALU busy fraction of each hop kernel.

    rocprofv3 reports each counter per dispatch summed over shader engines and
    XCDs; a wave of a one-RHS launch holds 64 sites, so VALU instructions per
    wave are those executed per site.  Busy = SQ_ACTIVE_INST_VALU (quad-cycles,
    all waves) x 4 / SIMDs / the per-XCD GRBM_GUI_ACTIVE (the sum over XCDs
    divided by their number).
    """
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in csv.DictReader(open(counter_csv)):
        k = r["Kernel_Name"]
        if not is_hop(k):
            continue
        acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    lines = ["# VALU work of the hop kernels in the 32^3x64 mixed solve (rocprofv3 counters)", "",
             "Command (repo root, one MI355X; kernels run serialised under counter collection, so only counts",
             "and ratios are used, not times):", "", "    " + cmd, "",
             f"Kernel sources hash: {kernel_hash()}.  Busy = SQ_ACTIVE_INST_VALU x 4 / {simds} SIMDs / "
             f"(GRBM_GUI_ACTIVE / {xcds} XCDs); instructions per wave = SQ_INSTS_VALU / SQ_WAVES, which is",
             "per site for launches with one right-hand side per lane (64 sites per wave).", "",
             "| kernel (template args as in the traffic summary) | dispatches | waves | VALU instr per wave | VALU busy |",
             "|---|---|---|---|---|"]
    for k in sorted(acc, key=lambda k: -len(disp[k])):
        n = len(disp[k])
        if n < min_dispatches:
            continue
        v = acc[k]
        waves = v["SQ_WAVES"] / n
        per_wave = v["SQ_INSTS_VALU"] / v["SQ_WAVES"]
        busy = v["SQ_ACTIVE_INST_VALU"] * 4 / simds / (v["GRBM_GUI_ACTIVE"] / xcds)
        name = k.replace("tmq::", "").split("(")[0]
        lines.append(f"| `{name}` | {n} | {waves:.0f} | {per_wave:.0f} | {100 * busy:.0f} % |")
    lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def summarize_batch_sweep(fetch_csv, sweep_json, cmd, out):
    """HBM reads per launch of the batched FP32 half-sweeps of each (block
    order, RHS group) configuration of config_bench's batchsweep section: the
    dispatches after each copy-kernel marker pair belong to the next row of
    the sweep (in order); reads are scaled by the marker copy's own reading."""
    res = json.load(open(sweep_json))
    rows = res["batch_sweep"]["rows"] if "batch_sweep" in res else res["rows"]
    disp = collections.OrderedDict()
    for r in csv.DictReader(open(fetch_csv)):
        if r["Counter_Name"] != "FETCH_SIZE":
            continue
        d = int(r["Dispatch_Id"])
        disp.setdefault(d, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
    seq = [disp[d] for d in sorted(disp)]
    copies = [v for k, v in seq if "k_stream_copy" in k]
    if not copies:
        raise SystemExit("no copy-kernel markers in the counter file")
    scale = (1 << 20) / (sorted(copies)[len(copies) // 2] * 1024.0)  # the 1 MiB marker copies
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    ci, prev = -1, False
    for k, v in seq:
        if "k_stream_copy" in k:
            ci += not prev
            prev = True
            continue
        prev = False
        part = hop_part(k)
        if ci >= 0 and hop_family(k) == "hop32" and part:
            acc[ci][part].append(v * 1024.0 * scale)
    lines = ["# Batched FP32 half-sweeps, 48 right-hand sides at 24^3x48: block order x RHS group", "",
             "Commands (GPU box; the sweep, then one counter pass over the same sweep):", "", "    " + cmd, "",
             f"Kernel sources hash: {kernel_hash()}.  Reads scaled by the 1 MiB marker copies (x {scale:.4f}); "
             "times from events in a run without the profiler.", "",
             "| block order | RHS group | K1 us | K2 us | fused K2 us | K1 HBM read MB | K1 algorithmic read MB | ratio |",
             "|---|---|---|---|---|---|---|---|"]
    names = {1: "z-slabs", 3: "t-slabs", 0: "plain"}
    for i, r in enumerate(rows):
        k1 = acc[i].get("k1", [])
        rd = sum(k1) / len(k1) if k1 else float("nan")
        alg = r.get("k1_algorithmic_read_bytes", float("nan"))
        lines.append(f"| {names.get(r['variant'], r['variant'])} | {r['group']} | {r['k1_us']:.0f} | {r['k2_us']:.0f} | "
                     f"{r['fused_us']:.0f} | {rd / 1e6:.0f} | {alg / 1e6:.0f} | {rd / alg:.2f} |")
    lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="64,32,32,32", help="T,LZ,LY,LX")
    ap.add_argument("--prec", default="fp64,fp16", help="comma list of fp64, fp32, fp16, bf16")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--summarize-trace", metavar="STATS_CSV")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--summarize-valu", metavar="COUNTER_CSV")
    ap.add_argument("--summarize-batch-sweep", nargs=2, metavar=("FETCH_CSV", "SWEEP_JSON"))
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--out")
    args = ap.parse_args()
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace, args.cmd, args.out)
    if args.summarize_valu:
        return summarize_valu(args.summarize_valu, args.cmd, args.out)
    if args.summarize_batch_sweep:
        return summarize_batch_sweep(args.summarize_batch_sweep[0], args.summarize_batch_sweep[1], args.cmd, args.out)
    if args.summarize_pmc:
        return summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.copy_bytes, args.cmd, args.out)

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
