"""FP64 CPU oracle for the twisted-mass operator, its even/odd Schur complement and CG.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark to judge the GPU library.  The library never
imports it and it imports nothing from the library.

The arithmetic lives in ``tmq_oracle.c`` (plain C, FP64, dense gamma matrices);
this module compiles it with gcc on first use and wraps it with ctypes.  The
spinor codec reference (FP16/BF16 with a per-site FP32 scale) is plain numpy.

Every function takes and returns fields in the canonical host layout of
``synth``: gauge (T,LZ,LY,LX,4,3,3), full spinors (T,LZ,LY,LX,4,3), odd-site
fields (V/2,4,3), all complex128.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tmq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.orc_odd_sites.restype = ctypes.c_long
            lib.orc_cg.restype = ctypes.c_int
            lib.orc_true_residual.restype = ctypes.c_double
            lib.orc_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"dims must be 4 even extents (T, LZ, LY, LX), got {dims}")
    return (ctypes.c_int * 4)(*dims), dims


def _c(a: np.ndarray, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.size != int(np.prod(shape)):
        raise ValueError(f"expected {int(np.prod(shape))} complex values, got {a.size}")
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _theta(theta):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.shape != (4,):
        raise ValueError("theta must have 4 entries (t, x, y, z)")
    return th


def volume(dims) -> int:
    T, LZ, LY, LX = dims
    return T * LZ * LY * LX


def gammas() -> np.ndarray:
    """gamma_0..gamma_3 and gamma_5 of Appendix A, shape (5, 4, 4)."""
    out = np.zeros((5, 4, 4), dtype=np.complex128)
    _load().orc_gammas(_p(out))
    return out


def odd_sites(dims) -> np.ndarray:
    """Site indices of the odd sites in increasing order."""
    cd, dims = _dims(dims)
    out = np.zeros(volume(dims) // 2, dtype=np.int64)
    n = _load().orc_odd_sites(cd, out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    assert n == volume(dims) // 2
    return out


def hop(U, psi, theta):
    """H psi on the full lattice (hopping term of eq. (eo0) with the Sec. 4.1.2 phase)."""
    dims = U.shape[:4]
    cd, dims = _dims(dims)
    U = _c(U)
    psi = _c(psi, dims + (4, 3))
    out = np.empty(dims + (4, 3), dtype=np.complex128)
    _load().orc_hop(cd, _p(U), _p(_theta(theta)), _p(psi), _p(out))
    return out


def M(U, psi, kappa, mut, sign, theta):
    """M^{sign} psi = (1 + sign i mut gamma_5) psi - kappa H psi, full lattice."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    psi = _c(psi, dims + (4, 3))
    out = np.empty(dims + (4, 3), dtype=np.complex128)
    _load().orc_M(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut), ctypes.c_int(sign),
                  _p(_theta(theta)), _p(psi), _p(out))
    return out


def Q(U, psi, kappa, mut, sign, theta):
    """Q^{sign} psi = gamma_5 M^{sign} psi, full lattice (eq. (eo1))."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    psi = _c(psi, dims + (4, 3))
    out = np.empty(dims + (4, 3), dtype=np.complex128)
    _load().orc_Q(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut), ctypes.c_int(sign),
                  _p(_theta(theta)), _p(psi), _p(out))
    return out


def Qhat(U, psi_odd, kappa, mut, sign, theta):
    """Qhat^{sign} psi_o on the odd sites (eq. (eo4) with eq. (eo3))."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    psi = _c(psi_odd, (volume(dims) // 2, 4, 3))
    out = np.empty((volume(dims) // 2, 4, 3), dtype=np.complex128)
    _load().orc_Qhat(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut), ctypes.c_int(sign),
                     _p(_theta(theta)), _p(psi), _p(out))
    return out


def QhatQhat(U, psi_odd, kappa, mut, theta):
    """Qhat^+ Qhat^- psi_o (Qhat^- first)."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    psi = _c(psi_odd, (volume(dims) // 2, 4, 3))
    out = np.empty((volume(dims) // 2, 4, 3), dtype=np.complex128)
    _load().orc_QhatQhat(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut),
                         _p(_theta(theta)), _p(psi), _p(out))
    return out


def QQ(U, psi, kappa, mut, theta):
    """Q^+ Q^- psi on the full lattice (Q^- first)."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    psi = _c(psi, dims + (4, 3))
    out = np.empty(dims + (4, 3), dtype=np.complex128)
    _load().orc_QQ(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut),
                   _p(_theta(theta)), _p(psi), _p(out))
    return out


def cg(U, b, kappa, mut, theta, eo=True, tol=1e-10, relative=True, max_iter=10000,
       history=False):
    """Textbook CG on Qhat^+Qhat^- (eo) or Q^+Q^- (full), x_0 = 0 (Sec. 4.4).

    Returns (x, info) with info = {converged, iters, alpha, beta, rr}.
    """
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    n_sites = volume(dims) // 2 if eo else volume(dims)
    b = _c(b, (n_sites, 4, 3))
    x = np.empty_like(b)
    alpha = np.zeros(max_iter)
    beta = np.zeros(max_iter)
    rr = np.zeros(max_iter + 1)
    it = ctypes.c_int(0)
    st = _load().orc_cg(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut), _p(_theta(theta)),
                        ctypes.c_int(1 if eo else 0), _p(b), _p(x), ctypes.c_double(tol),
                        ctypes.c_int(1 if relative else 0), ctypes.c_int(max_iter),
                        _p(alpha), _p(beta), _p(rr), ctypes.byref(it))
    k = it.value
    info = {"converged": st == 0, "iters": k}
    if history:
        info.update(alpha=alpha[:k].copy(), beta=beta[:k].copy(), rr=rr[:k + 1].copy())
    return x.reshape(b.shape), info


def true_residual(U, b, x, kappa, mut, theta, eo=True) -> float:
    """||b - A x|| / ||b|| with A = Qhat^+Qhat^- (eo) or Q^+Q^- (full), in FP64."""
    cd, dims = _dims(U.shape[:4])
    U = _c(U)
    n_sites = volume(dims) // 2 if eo else volume(dims)
    b = _c(b, (n_sites, 4, 3))
    x = _c(x, (n_sites, 4, 3))
    return float(_load().orc_true_residual(cd, _p(U), ctypes.c_double(kappa), ctypes.c_double(mut),
                                           _p(_theta(theta)), ctypes.c_int(1 if eo else 0),
                                           _p(b), _p(x)))


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ------------------------------------------------------------------ codec
# Reduced-precision storage of spinors (the paper stores intermediate
# half-spinors in reduced precision, Sec. 4.1): per site, scale = the largest
# |real or imaginary part| over the 24 reals, rounded to FP32 (RNE); each real
# is stored as  fp16_or_bf16( fp32( value / scale ) ), both roundings RNE, the
# division in FP64.  An all-zero site stores scale 0 and zero codes.  Decoding
# is fp32(code) * scale in FP32.


def _f32_to_bf16_bits(f: np.ndarray) -> np.ndarray:
    u = f.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)


def _bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32)


def encode_site_scaled(psi: np.ndarray, kind: str):
    """Encode an (n,4,3) complex field: returns (codes uint16 (n,24), scale float32 (n,))."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(-1, 12)
    re = psi.view(np.float64).reshape(-1, 24)  # (re, im) interleaved per component
    scale = np.max(np.abs(re), axis=1).astype(np.float32)
    s64 = scale.astype(np.float64)
    safe = np.where(s64 > 0, s64, 1.0)
    y = (re / safe[:, None]).astype(np.float32)
    y[s64 == 0] = 0
    if kind == "fp16":
        codes = y.astype(np.float16).view(np.uint16)
    elif kind == "bf16":
        codes = _f32_to_bf16_bits(y)
    else:
        raise ValueError(kind)
    return codes, scale


def decode_site_scaled(codes: np.ndarray, scale: np.ndarray, kind: str) -> np.ndarray:
    """Inverse of encode_site_scaled, values in FP32 returned as complex128 (n,4,3)."""
    if kind == "fp16":
        y = codes.view(np.float16).astype(np.float32)
    else:
        y = _bf16_bits_to_f32(codes)
    v = (y * scale.astype(np.float32)[:, None]).astype(np.float64)
    return v.view(np.complex128).reshape(-1, 4, 3)


# ------------------------------------------------------ flavour doublet
#
# The mass non-degenerate doublet of eq. (Dh), D_h = D_W 1_f + i mubar g5 tau^3
# + epsbar tau^1, in the hopping normalisation of eq. (eo0): with A the site
# term 1 + i mubar g5 tau^3 + epsbar tau^1 (mubar and epsbar standing for
# 2 kappa mubar and 2 kappa epsbar),
#     M_h psi = A psi - kappa H psi      (H flavour-diagonal),
# and Q_h = g5 M_h.  Its even/odd reduction follows the factorisation of
# App. B for the doublet: Qhat_h = g5 (A_oo - kappa^2 H_oe A_ee^-1 H_eo) on
# the odd sites, A_ee^-1 the inverse of the 8x8 site matrix (flavour x spin).
# sign = -1 flips the sign of mubar (Qhat_h^- is the adjoint of Qhat_h^+).
# Doublet fields are (2, ...) arrays: flavour index first (upper, lower).

_TAU = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)


def doublet_site_matrix(mubar, epsbar):
    """The 8x8 site term A = 1 + i mubar g5 tau^3 + epsbar tau^1 of eq. (Dh),
    indexed (flavour, spin), built from the dense gamma_5 of App. A."""
    g5 = gammas()[4]
    return (np.eye(8) + 1j * mubar * np.kron(_TAU[2], g5) + epsbar * np.kron(_TAU[0], np.eye(4)))


def _site_apply(A8, psi2):
    """(A8 psi)(x) for a doublet field (2, n, 4, 3): A8 acts on (flavour, spin)."""
    n = psi2.shape[1]
    v = np.transpose(psi2, (1, 0, 2, 3)).reshape(n, 8, 3)
    w = np.einsum("ab,nbc->nac", A8, v)
    return np.transpose(w.reshape(n, 2, 4, 3), (1, 0, 2, 3))


def _gamma5(psi):
    return np.einsum("st,...tc->...sc", gammas()[4], psi)


def Mh(U, psi2, kappa, mubar, epsbar, theta):
    """M_h psi on the full lattice for a doublet psi2 (2, T, LZ, LY, LX, 4, 3)."""
    dims = tuple(U.shape[:4])
    V = volume(dims)
    psi2 = np.asarray(psi2, dtype=np.complex128).reshape((2,) + dims + (4, 3))
    loc = _site_apply(doublet_site_matrix(mubar, epsbar), psi2.reshape(2, V, 4, 3))
    out = np.empty_like(psi2)
    for f in range(2):
        out[f] = loc[f].reshape(dims + (4, 3)) - kappa * hop(U, psi2[f], theta)
    return out


def _hop_parity(U, part, theta, src_sites, dst_sites):
    """H restricted to parity blocks: the field `part` on src_sites, H applied, read on dst_sites."""
    dims = tuple(U.shape[:4])
    full = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    full[src_sites] = part
    return hop(U, full.reshape(dims + (4, 3)), theta).reshape(volume(dims), 4, 3)[dst_sites]


def Qhat_nd(U, psi2_odd, kappa, mubar, epsbar, sign, theta):
    """Qhat_h^{sign} psi on the odd sites of a doublet (2, V/2, 4, 3)."""
    dims = tuple(U.shape[:4])
    V = volume(dims)
    odd = odd_sites(dims)
    even = np.setdiff1d(np.arange(V), odd)
    psi2 = np.asarray(psi2_odd, dtype=np.complex128).reshape(2, V // 2, 4, 3)
    A8 = doublet_site_matrix(sign * mubar, epsbar)
    Ainv = np.linalg.inv(A8)
    t_e = np.stack([_hop_parity(U, psi2[f], theta, odd, even) for f in range(2)])
    s_e = _site_apply(Ainv, t_e)
    w_o = np.stack([_hop_parity(U, s_e[f], theta, even, odd) for f in range(2)])
    return _gamma5(_site_apply(A8, psi2) - kappa * kappa * w_o)


def QhatQhat_nd(U, psi2_odd, kappa, mubar, epsbar, theta):
    """Qhat_h^+ Qhat_h^- psi (Qhat_h^- first) on a doublet of odd-site fields."""
    return Qhat_nd(U, Qhat_nd(U, psi2_odd, kappa, mubar, epsbar, -1, theta), kappa, mubar, epsbar, +1, theta)


def cg_nd(U, b2, kappa, mubar, epsbar, theta, tol=1e-10, max_iter=10000):
    """Textbook CG (Sec. 4.4) on Qhat_h^+ Qhat_h^- for a doublet source, x_0 = 0,
    inner products over both flavours; stops when |r|^2 <= tol^2 |b|^2."""
    b = np.asarray(b2, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    target = tol * tol * rr
    k = 0
    while rr > target and k < max_iter:
        ap = QhatQhat_nd(U, p, kappa, mubar, epsbar, theta)
        alpha = rr / float(np.vdot(p, ap).real)
        x += alpha * p
        r -= alpha * ap
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    return x, {"converged": rr <= target, "iters": k}


def true_residual_nd(U, b2, x2, kappa, mubar, epsbar, theta) -> float:
    """||b - Qhat_h^+ Qhat_h^- x|| / ||b|| in FP64 for doublet fields."""
    b = np.asarray(b2, dtype=np.complex128)
    r = b - QhatQhat_nd(U, x2, kappa, mubar, epsbar, theta)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(b.ravel()))


# ------------------------------------------------------------ BiCGstab
#
# The stabilised bi-conjugate gradient method (one of the solvers the paper
# lists for D chi = phi, Sec. 4.4; van der Vorst's algorithm as given in the
# textbooks the paper cites), applied to the odd-site operator Qhat^{sign}
# itself rather than to the normal equations.  Shadow residual = the initial
# residual; x_0 = 0; stops when |r|^2 <= tol^2 |b|^2 on the iterated
# residual; complex inner products <a, b> = sum conj(a) b.

def bicgstab(U, b, kappa, mut, sign, theta, tol=1e-10, max_iter=10000):
    """Solve Qhat^{sign} x = b; returns (x, {converged, iters, breakdown})."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    rhat = r.copy()
    bb = float(np.vdot(b, b).real)
    target = tol * tol * bb
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    k = 0
    rr = bb
    while rr > target and k < max_iter:
        rho_new = np.vdot(rhat, r)
        if rho_new == 0 or omega == 0:
            return x, {"converged": False, "iters": k, "breakdown": True}
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = Qhat(U, p, kappa, mut, sign, theta)
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        t = Qhat(U, s, kappa, mut, sign, theta)
        tt = float(np.vdot(t, t).real)
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rr = float(np.vdot(r, r).real)
        k += 1
    return x, {"converged": rr <= target, "iters": k, "breakdown": False}


# ------------------------------------------------- consumers of the solver
#
# The HMC force solves of eq. (eo6) and the one-end-trick correlator of the
# online measurements (eqs. (source), (oneend)).

def solve_M(U, phi, kappa, mut, sign, theta, tol=1e-12):
    """psi = (M^{sign})^-1 phi on the full lattice by the plain route
    Q^{sign} = g5 M^{sign}: psi = (Q^{sign})^-1 g5 phi = Q^{-sign} (Q^+ Q^-)^-1 g5 phi
    (Q^+ Q^- = Q^- Q^+ on the full lattice), with the oracle's CG."""
    dims = tuple(U.shape[:4])
    phi = np.asarray(phi, dtype=np.complex128).reshape(dims + (4, 3))
    g5phi = _gamma5(phi)
    y, info = cg(U, g5phi.reshape(-1, 4, 3), kappa, mut, theta, eo=False, tol=tol)
    assert info["converged"], info
    return Q(U, y.reshape(dims + (4, 3)), kappa, mut, -sign, theta)


def timeslice_bilinear(psi, gamma, t0=0):
    """C(t) = sum over the sites of time slice (t0 + t) mod T of psi^+ Gamma psi
    (spin matrix Gamma, colour summed); psi a full field (T, LZ, LY, LX, 4, 3)."""
    psi = np.asarray(psi, dtype=np.complex128)
    per_t = np.einsum("tzyxsc,su,tzyxuc->t", psi.conj(), np.asarray(gamma, dtype=np.complex128), psi)
    return np.roll(per_t, -t0)


def pion_correlator(U, xi, kappa, mut, theta, t0=0, tol=1e-12):
    """One-end-trick estimator of the pseudoscalar correlator for one noise
    sample xi (a full field, non-zero on time slice t0): phi = (M^+)^-1 xi and
    C(t) = sum over the spatial sites at time t0 + t of |phi|^2, for M in the
    hopping normalisation of eq. (eo0)."""
    phi = solve_M(U, xi, kappa, mut, +1, theta, tol=tol)
    return timeslice_bilinear(phi, np.eye(4), t0).real, phi
