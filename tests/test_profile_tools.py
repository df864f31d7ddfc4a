"""Host logic of the profile summaries (no GPU): the counter scaling behind
`roofline.traffic`, the VALU summary, and the kernel-hash gate in bench.py."""
import csv
import json
import os

import pytest

from paper_0905_3331_amd import profile_hop

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
K1 = "void tmq::hop_kernel<tmq::Sp16<false>, tmq::L16R, false, false, true, 1, false, 1, 0, false>(args)"
CAND = "void tmq::hop_kernel<tmq::Sp16<false>, tmq::L16R, false, false, true, 3, false, 1, 0, false>(args)"
F64 = "void tmq::hop_kernel<tmq::SpF64, tmq::L64R, false, false, true, 1, false, 1, 0, false>(args)"
COPY = "k_stream_copy(float4 const*, float4*, long)"


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_summarize_pmc_scales_by_the_copy_kernel(tmp_path):
    copy_bytes = 1 << 30
    # the copy reads and writes copy_bytes; FETCH_SIZE sees half of its reads (scale 2), WRITE_SIZE all
    fetch = [(COPY, "FETCH_SIZE", copy_bytes / 2 / 1024)] * 2
    write = [(COPY, "WRITE_SIZE", copy_bytes / 1024)] * 2
    fetch += [(K1, "FETCH_SIZE", 100000.0)] * 32 + [(K1, "FETCH_SIZE", 120000.0)] * 8
    write += [(K1, "WRITE_SIZE", 50000.0)] * 40
    # an autotuner candidate (fewer than a tenth of the family's most-launched
    # kernel's dispatches) stays out of the family average
    fetch += [(CAND, "FETCH_SIZE", 9e9)]
    write += [(CAND, "WRITE_SIZE", 9e9)]
    fetch += [(F64, "FETCH_SIZE", 700000.0)] * 4
    write += [(F64, "WRITE_SIZE", 200000.0)] * 4
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = tmp_path / "t.json"
    profile_hop.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), copy_bytes, "cmd", str(out))
    d = json.load(open(out))
    assert d["kernel_hash"] == profile_hop.kernel_hash()
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    h16 = d["hop16"]
    assert h16["dispatches"] == [40, 40]
    assert h16["read_bytes_per_launch"] == pytest.approx((32 * 100000.0 + 8 * 120000.0) / 40 * 1024 * 2)
    assert h16["write_bytes_per_launch"] == pytest.approx(50000.0 * 1024)
    assert h16["hbm_bytes_per_launch"] == pytest.approx(h16["read_bytes_per_launch"] + h16["write_bytes_per_launch"])
    assert d["hop64"]["read_bytes_per_launch"] == pytest.approx(700000.0 * 1024 * 2)
    assert d["per_kernel"][CAND]["dispatches"] == 1  # listed, but not averaged


def test_summarize_pmc_needs_the_copy_kernel(tmp_path):
    _write(tmp_path / "f.csv", [(K1, "FETCH_SIZE", 1.0)])
    _write(tmp_path / "w.csv", [(K1, "WRITE_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        profile_hop.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1 << 30, "cmd",
                                  str(tmp_path / "t.json"))


def test_summarize_valu_per_wave_and_busy(tmp_path):
    waves, per_wave, busy, grbm_xcd = 16384.0, 1632.0, 0.68, 150000.0
    rows = []
    for _ in range(30):
        rows += [(K1, "SQ_WAVES", waves), (K1, "SQ_INSTS_VALU", waves * per_wave),
                 (K1, "SQ_ACTIVE_INST_VALU", busy * 1024 * grbm_xcd / 4), (K1, "GRBM_GUI_ACTIVE", 8 * grbm_xcd),
                 (K1, "SQ_WAVE_CYCLES", 1.0)]
    rows += [(CAND, "SQ_WAVES", 1.0), (CAND, "SQ_INSTS_VALU", 1.0), (CAND, "SQ_ACTIVE_INST_VALU", 1.0),
             (CAND, "GRBM_GUI_ACTIVE", 1.0)]
    # one dispatch per group of counter rows
    with open(tmp_path / "v.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i // 5 if k == K1 else 10000, "Kernel_Name": k, "Counter_Name": c,
                        "Counter_Value": v})
    out = tmp_path / "v.md"
    profile_hop.summarize_valu(str(tmp_path / "v.csv"), "cmd", str(out))
    text = open(out).read()
    line = [l for l in text.splitlines() if "Sp16<false>, L16R, false, false, true, 1" in l][0]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[1:] == ["30", "16384", "1632", "68 %"]
    assert "true, 3," not in text  # the one-dispatch candidate is left out


def test_bench_takes_traffic_only_for_the_current_kernels(tmp_path, monkeypatch):
    import bench

    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    path = tmp_path / "profiles" / "hop_traffic.json"
    path.write_text(json.dumps({"kernel_hash": profile_hop.kernel_hash(), "hop16": {"hbm_bytes_per_launch": 4.2e8}}))
    assert bench.measured_traffic("hop16", "hbm_bytes_per_launch") == 4.2e8
    path.write_text(json.dumps({"kernel_hash": "0" * 16, "hop16": {"hbm_bytes_per_launch": 4.2e8}}))
    assert bench.measured_traffic("hop16", "hbm_bytes_per_launch") is None
    os.remove(path)
    assert bench.measured_traffic("hop16", "hbm_bytes_per_launch") is None


def test_summarize_trace_family_averages(tmp_path):
    rows = [(K1, 100, 6.1e6), (CAND, 4, 0.3e6), (F64, 50, 11.0e6), (COPY, 2, 0.7e6)]
    with open(tmp_path / "s.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs"])
        w.writeheader()
        for n, c, t in rows:
            w.writerow({"Name": n, "Calls": c, "TotalDurationNs": t})
    out = tmp_path / "s.md"
    profile_hop.summarize_trace(str(tmp_path / "s.csv"), "cmd", str(out))
    fam = {l.split("|")[1].strip(): l for l in open(out).read().splitlines() if l.startswith("| hop")}
    # the family average counts every instantiation: (6.1 + 0.3) ms over 104 launches
    assert fam["hop16"].split("|")[2].strip() == "104"
    assert float(fam["hop16"].split("|")[3]) == pytest.approx(6.4e6 / 104 / 1e3, abs=0.01)
    assert float(fam["hop64"].split("|")[3]) == pytest.approx(220.0, abs=0.01)


H16K1 = "void tmq::hop16_kernel<tmq::Sp16<false>, false, false, 1, true, 0, false, 1>(tmq::HopArgs<tmq::Sp16<false>, tmq::L16R>)"
H16K2 = "void tmq::hop16_kernel<tmq::Sp16<false>, true, true, 1, true, 0, false, 1, true>(tmq::HopArgs<tmq::Sp16<false>, tmq::L16R>)"
H16CG = "void tmq::hop16_kernel<tmq::Sp16<false>, true, true, 1, true, 1, false, 1>(tmq::HopArgs<tmq::Sp16<false>, tmq::L16R>)"
H16BK1 = ("void tmq::hop16_kernel<tmq::Sp16<false>, false, false, 2, false, 0, false, 1, false, true>"
          "(tmq::HopArgs<tmq::Sp16<false>, tmq::L16R>)")
H16BCG = ("void tmq::hop16_kernel<tmq::Sp16<false>, true, true, 1, true, 1, false, 1, false, true>"
          "(tmq::HopArgs<tmq::Sp16<false>, tmq::L16R>)")
GK2 = "void tmq::hop_kernel<tmq::SpF64, tmq::L64R, true, true, true, 1, false, 1, 0, false>(args)"
GRES = "void tmq::hop_kernel<tmq::SpF64, tmq::L64R, true, true, true, 1, false, 1, 2, false>(args)"


def test_hop_parts_of_both_kernels():
    """The half-sweep kind is read from the template arguments of either kernel:
    K1 (no own-parity site term), K2 (storing its output), fused (CG or residual)."""
    assert profile_hop.hop_family(H16K1) == "hop16" and profile_hop.hop_family(F64) == "hop64"
    assert [profile_hop.hop_part(k) for k in (H16K1, H16K2, H16CG)] == ["k1", "k2", "fused"]
    assert [profile_hop.hop_part(k) for k in (H16BK1, H16BCG)] == ["k1", "fused"]  # batched launches
    assert [profile_hop.hop_part(k) for k in (F64, GK2, GRES)] == ["k1", "k2", "fused"]
    assert profile_hop.hop_part(COPY) is None and profile_hop.hop_family(COPY) is None


def test_summarize_pmc_parts(tmp_path):
    """Family averages split into ":pure" (K1 and K2), ":k1", ":k2", ":fused"."""
    copy_bytes = 1 << 30
    fetch = [(COPY, "FETCH_SIZE", copy_bytes / 2 / 1024)] * 2
    write = [(COPY, "WRITE_SIZE", copy_bytes / 1024)] * 2
    fetch += [(H16K1, "FETCH_SIZE", 100.0)] * 20 + [(H16K2, "FETCH_SIZE", 200.0)] * 10 + [(H16CG, "FETCH_SIZE", 400.0)] * 10
    write += [(H16K1, "WRITE_SIZE", 10.0)] * 20 + [(H16K2, "WRITE_SIZE", 10.0)] * 10 + [(H16CG, "WRITE_SIZE", 30.0)] * 10
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = tmp_path / "t.json"
    profile_hop.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), copy_bytes, "cmd", str(out))
    d = json.load(open(out))
    k = 1024.0
    assert d["hop16:k1"]["read_bytes_per_launch"] == pytest.approx(200.0 * k)
    assert d["hop16:k2"]["read_bytes_per_launch"] == pytest.approx(400.0 * k)
    assert d["hop16:fused"]["write_bytes_per_launch"] == pytest.approx(30.0 * k)
    # pure: 20 K1 and 10 K2 launches averaged per launch
    assert d["hop16:pure"]["read_bytes_per_launch"] == pytest.approx((20 * 200.0 + 10 * 400.0) / 30 * k)
    assert d["hop16:pure"]["dispatches"] == [30, 30]


def test_summarize_batch_sweep_attributes_dispatches(tmp_path):
    """Each configuration's half-sweeps are the dispatches after its marker copy pair."""
    sweep = {"rows": [{"variant": 1, "group": 8, "k1_us": 1.0, "k2_us": 2.0, "fused_us": 3.0,
                       "k1_algorithmic_read_bytes": 1000.0 * 1024},
                      {"variant": 0, "group": 48, "k1_us": 1.0, "k2_us": 2.0, "fused_us": 3.0,
                       "k1_algorithmic_read_bytes": 1000.0 * 1024}]}
    K1_32 = "void tmq::hop_kernel<tmq::SpF32, tmq::L32R, false, false, false, 1, false, 1, 0, false>(args)"
    marker = (1 << 20) / 1024.0  # KiB the 1 MiB marker copy reads (scale 1)
    rows = [(COPY, "FETCH_SIZE", marker)] * 2 + [(K1_32, "FETCH_SIZE", 2000.0)] * 3
    rows += [(COPY, "FETCH_SIZE", marker)] * 2 + [(K1_32, "FETCH_SIZE", 3000.0)] * 3
    _write(tmp_path / "f.csv", rows)
    (tmp_path / "s.json").write_text(json.dumps(sweep))
    out = tmp_path / "o.md"
    profile_hop.summarize_batch_sweep(str(tmp_path / "f.csv"), str(tmp_path / "s.json"), "cmd", str(out))
    text = out.read_text()
    assert "| z-slabs | 8 | 1 | 2 | 3 | 2 | 1 | 2.00 |" in text
    assert "| plain | 48 | 1 | 2 | 3 | 3 | 1 | 3.00 |" in text


def test_kernel_hash_ignores_comments():
    """The kernel hash covers code, not comments: a comment edit keeps it, a code edit changes it."""
    src = "int a = 1;  // one\n/* block\n comment */\nint b = 2;\n\n"
    assert profile_hop.code_text(src) == "int a = 1;\nint b = 2;"
    assert profile_hop.code_text(src.replace("one", "two")) == profile_hop.code_text(src)
    assert profile_hop.code_text(src.replace("2;", "3;")) != profile_hop.code_text(src)

