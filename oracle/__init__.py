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
