"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

This module holds no arithmetic of the method itself (no hopping term, no
gamma matrices, no solver): it only draws random gauge links and spinor
fields in the canonical host layout, so that both the oracle and the GPU path
can be fed the very same FP64 arrays.

Canonical host layout (little-endian complex128, C order):
  dims            = (T, LZ, LY, LX), every extent even
  site index      lex = ((t*LZ + z)*LY + y)*LX + x
  gauge field U   shape (T, LZ, LY, LX, 4, 3, 3); direction mu = 0:t 1:x 2:y 3:z,
                  U[..., mu, a, b] is row a, column b of the link U(x, mu)
  full spinor     shape (T, LZ, LY, LX, 4, 3) = (site, spin, colour)
  odd-site field  shape (V/2, 4, 3): the odd sites ((t+x+y+z) odd) in
                  increasing lexicographic order

The site order t, z, y, x with spin and then colour fastest follows the
paper's propagator/source file index order (Sec. 4.7).

Recipes (workloads of the kind the paper runs on, Sec. 6 and Appendix B):
  * links:   U = reunitarise(exp(i*eps*H)), H = sum_a h_a lambda_a/2 with
             h_a ~ N(0,1) i.i.d. and lambda_a the Gell-Mann matrices.
             Reunitarise = Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1),
             so that det U = 1 up to rounding.
  * spinors: every complex component is (a + i b)/sqrt(2), a, b ~ N(0,1),
             i.e. E|z|^2 = 1 per complex component.
  * point sources: unit vector at one site, one spin, one colour.
Random numbers come from numpy's PCG64 (``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import os

import numpy as np

__all__ = [
    "gell_mann",
    "random_su3",
    "random_gauge",
    "unit_gauge",
    "gaussian_spinor",
    "gaussian_odd",
    "point_source_odd",
    "z2_timeslice_source",
    "volume",
    "check_dims",
]


def check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"dims must be 4 even extents >= 2 (T, LZ, LY, LX), got {dims}")
    return dims


def volume(dims) -> int:
    T, LZ, LY, LX = check_dims(dims)
    return T * LZ * LY * LX


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j
    l[1, 1, 0] = 1j
    l[2, 0, 0] = 1
    l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j
    l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j
    l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def _reunitarise(U: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0, 1; row 2 = conj(row0 x row1). In place on a (n,3,3) array."""
    r0 = U[:, 0, :]
    r0 /= np.sqrt(np.sum(np.abs(r0) ** 2, axis=1))[:, None]
    r1 = U[:, 1, :]
    proj = np.sum(np.conj(r0) * r1, axis=1)
    r1 -= proj[:, None] * r0
    r1 /= np.sqrt(np.sum(np.abs(r1) ** 2, axis=1))[:, None]
    U[:, 2, 0] = np.conj(r0[:, 1] * r1[:, 2] - r0[:, 2] * r1[:, 1])
    U[:, 2, 1] = np.conj(r0[:, 2] * r1[:, 0] - r0[:, 0] * r1[:, 2])
    U[:, 2, 2] = np.conj(r0[:, 0] * r1[:, 1] - r0[:, 1] * r1[:, 0])
    return U


def random_su3(n: int, eps: float, rng: np.random.Generator, chunk: int = 1 << 20) -> np.ndarray:
    """n random SU(3) matrices exp(i eps H), H = sum_a h_a lambda_a / 2, reunitarised."""
    import torch  # CPU only: a batched matrix exponential

    lam = gell_mann() / 2.0
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        h = rng.standard_normal((e - s, 8))
        H = np.tensordot(h, lam, axes=(1, 0))  # (m, 3, 3) Hermitian traceless
        A = torch.from_numpy(1j * eps * H)
        out[s:e] = torch.linalg.matrix_exp(A).numpy()
    return _reunitarise(out)


def _cache_path(kind: str, dims, eps, seed):
    root = os.environ.get("TMQ_SYNTH_CACHE")
    if not root:
        return None
    os.makedirs(root, exist_ok=True)
    return os.path.join(root, f"{kind}_{'x'.join(map(str, dims))}_{eps}_{seed}.npy")


def random_gauge(dims, eps: float = 0.3, seed: int = 0) -> np.ndarray:
    """Random SU(3) gauge field in the canonical layout, shape (T,LZ,LY,LX,4,3,3).

    Set TMQ_SYNTH_CACHE to a directory to memoise large fields on disk.
    """
    dims = check_dims(dims)
    path = _cache_path("gauge", dims, eps, seed)
    if path and os.path.exists(path):
        return np.load(path, mmap_mode=None)
    rng = np.random.default_rng(seed)
    n = volume(dims) * 4
    U = random_su3(n, eps, rng).reshape(dims + (4, 3, 3))
    if path:
        np.save(path, U)
    return U


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link is the identity."""
    dims = check_dims(dims)
    U = np.zeros(dims + (4, 3, 3), dtype=np.complex128)
    for a in range(3):
        U[..., a, a] = 1.0
    return U


def gaussian_spinor(shape, seed: int = 0) -> np.ndarray:
    """Complex Gaussian field, E|z|^2 = 1 per component; shape is (..., 4, 3)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(tuple(shape) + (2,))
    return ((a[..., 0] + 1j * a[..., 1]) / np.sqrt(2.0)).astype(np.complex128)


def gaussian_odd(dims, seed: int = 0) -> np.ndarray:
    """Gaussian source on the odd sites, shape (V/2, 4, 3)."""
    return gaussian_spinor((volume(dims) // 2, 4, 3), seed)


def point_source_odd(dims, site_odd: int, spin: int, colour: int) -> np.ndarray:
    """Unit point source at odd-site index ``site_odd`` (spin, colour)."""
    b = np.zeros((volume(dims) // 2, 4, 3), dtype=np.complex128)
    b[site_odd, spin, colour] = 1.0
    return b


def z2_timeslice_source(dims, t0: int, seed: int = 0) -> np.ndarray:
    """Complex Z2 noise (each component (+-1 +- i)/sqrt(2), so that E[xi_i^* xi_j] =
    delta_ij and E[xi_i xi_j] = 0) on every spin-colour component of time slice t0,
    zero elsewhere; full field (T, LZ, LY, LX, 4, 3)."""
    dims = check_dims(dims)
    rng = np.random.default_rng(seed)
    xi = np.zeros(dims + (4, 3), dtype=np.complex128)
    sgn = rng.integers(0, 2, size=dims[1:] + (4, 3, 2)) * 2 - 1
    xi[t0] = (sgn[..., 0] + 1j * sgn[..., 1]) / np.sqrt(2.0)
    return xi
