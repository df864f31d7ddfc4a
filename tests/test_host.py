"""CPU tests of the GPU library's host side: the C ABI loads and exports every
declared entry point, argument validation, and the spin-projector table and
two-row link reconstruction of the kernels (compiled for the host)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import dense
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmq.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tmq_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    path = os.path.join(ROOT, "paper_0905_3331_amd", "libtmq.so")
    if not os.path.exists(path):
        from paper_0905_3331_amd.build import build

        build()
    return ctypes.CDLL(path)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_0905_3331_amd import tmq

    assert set(declared_functions()) <= set(tmq.EXPORTED)


def test_argument_validation_without_gpu():
    from paper_0905_3331_amd import tmq

    with pytest.raises(tmq.TmqError) as e:
        tmq.Lattice((4, 4, 3, 4))
    assert e.value.code == tmq.TMQ_EINVAL
    with pytest.raises(tmq.TmqError):
        tmq.footprint_bytes((4, 4, 4, 5))
    assert tmq.footprint_bytes((4, 4, 4, 4)) > 0
    # FP16 mixed solve state is smaller than FP64 solve state at 32^3 x 64
    f64 = tmq.footprint_bytes((64, 32, 32, 32), tmq.solver_opts(sloppy="fp64"))
    f16 = tmq.footprint_bytes((64, 32, 32, 32), tmq.solver_opts(sloppy="fp16"))
    assert 0 < f16 < f64 + 2e9


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structs of the binding have the compiler's layout of include/tmq.h."""
    from paper_0905_3331_amd import tmq

    exe = tmp_path / "abi_layout"
    src = os.path.join(ROOT, "tests", "cpu_helpers", "abi_layout.c")
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), src])
    want = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        k, v = line.split()
        want[k] = int(v)
    for cls in (tmq.tmq_params, tmq.tmq_nd_params, tmq.tmq_solver_opts, tmq.tmq_solve_info, tmq.tmq_server_config,
                tmq.tmq_server_stats):
        name = cls.__name__
        assert ctypes.sizeof(cls) == want[name], name
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == want[f"{name}.{f}"], (name, f)


def test_server_needs_a_device():
    from paper_0905_3331_amd import tmq

    with pytest.raises(tmq.TmqError) as e:
        tmq.Server(device=-1)
    assert e.value.code in (tmq.TMQ_EDEVICE, tmq.TMQ_EINVAL)


@pytest.fixture(scope="module")
def spinlib(tmp_path_factory):
    out = tmp_path_factory.mktemp("spin") / "libspin.so"
    src = os.path.join(ROOT, "tests", "cpu_helpers", "spin_table.cpp")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", str(out), src])
    return ctypes.CDLL(str(out))


@pytest.mark.parametrize("mu", range(4))
@pytest.mark.parametrize("sign", [+1, -1])
def test_spin_projector_table(spinlib, mu, sign):
    dp = ctypes.POINTER(ctypes.c_double)
    rng = np.random.default_rng(mu * 2 + (sign > 0))
    for _ in range(3):
        psi = (rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))).astype(np.complex128)
        out = np.zeros((4, 3), np.complex128)
        spinlib.spin_project_reconstruct(mu, sign, psi.ctypes.data_as(dp), out.ctypes.data_as(dp))
        expect = (np.eye(4) + sign * dense.G[mu]) @ psi
        assert np.allclose(out, expect, atol=1e-15)


def test_su3_two_row_reconstruction(spinlib):
    dp = ctypes.POINTER(ctypes.c_double)
    U = synth.random_su3(50, 1.0, np.random.default_rng(3))
    for u in U:
        rows = np.ascontiguousarray(u[:2])
        third = np.zeros(3, np.complex128)
        spinlib.su3_reconstruct(rows.ctypes.data_as(dp), third.ctypes.data_as(dp))
        assert np.max(np.abs(third - u[2])) < 1e-15


def test_fastdiv_multipliers(tmp_path):
    """The 16-bit hop kernel decodes a site index by multiply-high divisions
    (Granlund-Montgomery round-up multipliers).  Against plain integer division:
    every divisor up to 4096 and the lattice-sized ones around powers of two,
    numerators at random below 2^31 and at the quotient boundaries q d - 1, q d."""
    out = tmp_path / "libfastdiv.so"
    src = os.path.join(ROOT, "tests", "cpu_helpers", "fastdiv_check.cpp")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", str(out), src])
    lib = ctypes.CDLL(str(out))
    up = ctypes.POINTER(ctypes.c_uint32)
    rng = np.random.default_rng(11)
    divisors = list(range(1, 4097))
    for p in range(12, 32):
        divisors += [(1 << p) - 1, 1 << p, (1 << p) + 1, 3 << (p - 2), 5 << (p - 3)]
    divisors += [int(v) for v in rng.integers(1, 1 << 26, 200)]
    for d in [d for d in divisors if d <= 1 << 31]:  # the documented range
        qmax = ((1 << 31) - 1) // d
        qs = np.unique(np.concatenate([[0, 1, 2, qmax], rng.integers(0, qmax + 1, 16)]))
        edge = np.concatenate([qs * d, qs * d - 1, qs * d + d - 1])
        n = np.concatenate([rng.integers(0, 1 << 31, 64), edge])
        n = n[(n >= 0) & (n < (1 << 31))].astype(np.uint32)
        q = np.zeros_like(n)
        lib.fastdiv_quotients(d, n.ctypes.data_as(up), q.ctypes.data_as(up), len(n))
        assert np.array_equal(q, n // np.uint32(d)), d


# ------------------------------------------------ hop block orders (host replay)
# A replay of the hop kernel's map from (block, lane) to output site for each
# block order, as written in hop_impl.h / hop.hip: every site of the parity is
# computed exactly once per field (per flavour for doublet lane pairs), and no
# active lane addresses a site outside the field.

HOP_BLOCK = 256


def _hop_grid(n):
    g = (n + HOP_BLOCK - 1) // HOP_BLOCK
    return (g + 7) // 8 * 8


def _grid_variant(dims, order, lps):
    T, LZ, LY, LX = dims
    plane, vh = LY * (LX // 2), T * LZ * LY * (LX // 2)
    if order == "plain":
        return _hop_grid(lps * vh)
    if order == "zslab":
        zc = LZ // 8 + (1 if LZ % 8 else 0)
        return 8 * ((lps * T * zc * plane + HOP_BLOCK - 1) // HOP_BLOCK)
    tc = T // 8 + (1 if T % 8 else 0)
    return 8 * ((lps * LZ * tc * plane + HOP_BLOCK - 1) // HOP_BLOCK)


def _replay(dims, order, lps):
    T, LZ, LY, LX = dims
    XH = LX // 2
    plane, vh = LY * XH, T * LZ * LY * XH
    nblk = _grid_variant(dims, order, lps)
    spb = HOP_BLOCK // lps
    hits = np.zeros((lps, vh), dtype=np.int64)
    tid = np.arange(HOP_BLOCK)
    ls, fl = (tid >> 1, tid & 1) if lps == 2 else (tid, np.zeros_like(tid))
    for b in range(nblk):
        j, sb = b & 7, b >> 3
        if order == "plain":
            h = (j * (nblk >> 3) + sb) * spb + ls
            active = h < vh
        elif order == "zslab":
            zb, zr = LZ >> 3, LZ & 7
            zc, z0 = zb + (1 if j < zr else 0), j * zb + min(j, zr)
            S = zc * plane
            l = sb * spb + ls
            active = l < T * S
            t, rem = l // S, l % S
            z = z0 + rem // plane
            r2 = rem - (z - z0) * plane
            y, xh = r2 // XH, r2 % XH
            h = ((t * LZ + z) * plane) + y * XH + xh
        else:
            tb, tr = T >> 3, T & 7
            tc, t0 = tb + (1 if j < tr else 0), j * tb + min(j, tr)
            P = tc * plane
            l = sb * spb + ls
            active = l < LZ * P
            z, rem = l // P, l % P
            t = t0 + rem // plane
            r2 = rem - (t - t0) * plane
            y, xh = r2 // XH, r2 % XH
            h = ((t * LZ + z) * plane) + y * XH + xh
        assert np.all(h[active] >= 0) and np.all(h[active] < vh), (dims, order, b)
        np.add.at(hits, (fl[active], h[active]), 1)
    return hits


@pytest.mark.parametrize("dims", [(8, 8, 6, 10), (10, 4, 6, 6), (48, 24, 24, 24), (12, 10, 2, 4), (2, 2, 2, 2)],
                         ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("lps", [1, 2])
def test_hop_block_orders_cover_every_site_once(dims, lps):
    T, LZ = dims[0], dims[1]
    orders = ["plain"] + (["zslab"] if LZ >= 8 else []) + (["tslab"] if T >= 8 else [])
    for order in orders:
        hits = _replay(dims, order, lps)
        assert np.all(hits == 1), (dims, order, lps, hits.min(), hits.max())


@pytest.mark.parametrize("dims", [(48, 24, 24, 24), (16, 8, 16, 12)], ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("order", ["plain", "zslab", "tslab"])
def test_batched_grid_covers_every_block_and_tuple_once(dims, order):
    """The batched grid (tuples of RHS in groups of GR, each XCD sweeping its
    share of site blocks once per group) computes every (tuple, block) pair
    exactly once, ragged last group included."""
    nblk = _grid_variant(dims, order, 1)
    nb = nblk // 8
    for ntup, GR in ((7, 3), (12, 12), (5, 1)):
        seen = np.zeros((ntup, nblk), dtype=np.int64)
        for b in range(nblk * ntup):
            j, k = b & 7, b >> 3
            gr = k // (nb * GR)
            gsize = min(GR, ntup - gr * GR)
            within = k - gr * nb * GR
            sb = within // gsize
            tup = gr * GR + (within - sb * gsize)
            assert 0 <= tup < ntup and 0 <= sb < nb
            seen[tup, 8 * sb + j] += 1
        assert np.all(seen == 1), (dims, order, ntup, GR)
