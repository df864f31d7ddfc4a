"""Dense brute-force constructions of the paper's operators, for pinning the oracle.

These build the operator as an explicit (12V x 12V) matrix, by assembling sparse
blocks from the definitions, which is a different route from the oracle's
matrix-free loop:

* ``M_hopping``: eq. (eo0) of Appendix B assembled term by term (blocks are
  accumulated with +=, so on an extent of 2 the forward and backward
  neighbours, which coincide, both contribute).
* ``M_covariant``: the Wilson operator of eq. (DW) built literally from the
  covariant differences of eq. (covariant), 2 kappa (D_W + m_0) + i mut gamma_5
  with m_0 = 1/(2 kappa) - 4.  The paper's eq. (DW) has (1 - gamma) on the
  forward hop while eq. (eo0) has (1 + gamma); the two differ by a gamma_5
  conjugation, which the tests apply.
* ``shift``: the gauge-covariant shift T_mu psi(x) = U(x,mu) psi(x+mu), with
  either the phase spread over every hop (Sec. 4.1.2) or, literally, the
  twisted boundary condition psi(x + L) = e^{i theta pi} psi(x) of Sec. 2.4
  applied only to hops that cross the boundary.

Index of a dense vector: site * 12 + spin * 3 + colour, site = canonical
lexicographic index ((t*LZ + z)*LY + y)*LX + x.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.sparse as sp

_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gamma_matrices.txt")


def load_gammas():
    """gamma_0..gamma_3, gamma_5 from the golden fixture (Appendix A), shape (5,4,4)."""
    mats, cur = [], None
    with open(_GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("gamma"):
                cur = []
                mats.append(cur)
                continue
            cur.append([complex(*map(float, e.split(","))) for e in line.split()])
    return np.array(mats, dtype=np.complex128)


G = load_gammas()
G5 = G[4]
I4 = np.eye(4)
I3 = np.eye(3)


def site_coords(dims):
    """Coordinates (t, x, y, z) of every site, in lexicographic order (numpy unravel)."""
    T, LZ, LY, LX = dims
    t, z, y, x = np.unravel_index(np.arange(T * LZ * LY * LX), (T, LZ, LY, LX))
    return np.stack([t, x, y, z], axis=1)


def extents(dims):
    T, LZ, LY, LX = dims
    return np.array([T, LX, LY, LZ])  # along mu = t, x, y, z


def site_index(dims, c):
    T, LZ, LY, LX = dims
    return np.ravel_multi_index((c[..., 0], c[..., 3], c[..., 2], c[..., 1]), (T, LZ, LY, LX))


def parities(dims):
    return site_coords(dims).sum(axis=1) % 2


def shift(U, mu, theta, mode="spread"):
    """Sparse (12V x 12V) matrix of T_mu psi(x) = phase * (1_spin x U(x,mu)) psi(x + mu)."""
    dims = U.shape[:4]
    V = int(np.prod(dims))
    L = extents(dims)
    c = site_coords(dims)
    Uf = U.reshape(V, 4, 3, 3)
    rows, cols, vals = [], [], []
    for s in range(V):
        cn = c[s].copy()
        cross = cn[mu] == L[mu] - 1
        cn[mu] = (cn[mu] + 1) % L[mu]
        f = int(site_index(dims, cn))
        if mode == "spread":
            ph = np.exp(1j * np.pi * theta[mu] / L[mu])
        elif mode == "boundary":
            ph = np.exp(1j * np.pi * theta[mu]) if cross else 1.0
        else:
            raise ValueError(mode)
        blk = ph * np.kron(I4, Uf[s, mu])
        r, q = np.nonzero(np.ones((12, 12)))
        rows.append(12 * s + r)
        cols.append(12 * f + q)
        vals.append(blk[r, q])
    return sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(12 * V, 12 * V)
    )


def spin_op(m, V):
    """Sparse (12V x 12V) matrix of a site-diagonal spin matrix m (4x4)."""
    return sp.kron(sp.eye(V), sp.csr_matrix(np.kron(m, I3)), format="csr")


def M_hopping(U, kappa, mut, sign, theta, mode="spread"):
    """Dense M^{sign} from eq. (eo0): (1 + sign i mut g5) - kappa sum_mu [(1+g)T + (1-g)T^+]."""
    dims = U.shape[:4]
    V = int(np.prod(dims))
    M = spin_op(I4 + 1j * sign * mut * G5, V)
    for mu in range(4):
        T = shift(U, mu, theta, mode)
        M = M - kappa * (spin_op(I4 + G[mu], V) @ T + spin_op(I4 - G[mu], V) @ T.conj().T)
    return M.toarray()


def M_covariant(U, kappa, mut, sign, theta, mode="spread"):
    """Dense 2 kappa (D_W + m0) + sign i mut g5 from eqs. (DW) and (covariant), m0 = 1/(2 kappa) - 4."""
    dims = U.shape[:4]
    V = int(np.prod(dims))
    one = sp.eye(12 * V, format="csr")
    DW = sp.csr_matrix((12 * V, 12 * V), dtype=np.complex128)
    for mu in range(4):
        T = shift(U, mu, theta, mode)
        nab = T - one  # forward covariant difference
        nab_star = one - T.conj().T  # backward covariant difference
        DW = DW + 0.5 * (spin_op(G[mu], V) @ (nab + nab_star) - nab_star @ nab)
    m0 = 1.0 / (2.0 * kappa) - 4.0
    M = 2.0 * kappa * (DW + m0 * one) + spin_op(1j * sign * mut * G5, V)
    return M.toarray()


def boundary_gauge_transform(dims, theta):
    """Diagonal W = e^{i pi sum_mu theta_mu x_mu / L_mu}: maps the spread-phase operator
    to the boundary-phase one, M_spread = W^+ M_boundary W."""
    c = site_coords(dims)
    L = extents(dims)
    ph = np.exp(1j * np.pi * (c * (np.asarray(theta) / L)).sum(axis=1))
    return np.repeat(ph, 12)


def eo_blocks(dims):
    """Dense-vector indices of the even and the odd sites (sites in lexicographic order)."""
    par = parities(dims)
    ev = np.nonzero(par == 0)[0]
    od = np.nonzero(par == 1)[0]
    e_idx = (12 * ev[:, None] + np.arange(12)[None, :]).ravel()
    o_idx = (12 * od[:, None] + np.arange(12)[None, :]).ravel()
    return e_idx, o_idx


def schur_Qhat(M, dims):
    """gamma_5 (M_oo - M_oe inv(M_ee) M_eo) with a dense numerical inverse."""
    e, o = eo_blocks(dims)
    Mee = M[np.ix_(e, e)]
    Meo = M[np.ix_(e, o)]
    Moe = M[np.ix_(o, e)]
    Moo = M[np.ix_(o, o)]
    S = Moo - Moe @ np.linalg.solve(Mee, Meo)
    nodd = len(o) // 12
    g5 = np.kron(np.eye(nodd), np.kron(G5, I3))
    return g5 @ S


def dense_of(apply, n, shape):
    """Matrix of a linear map given as a function on arrays of ``shape`` (n unknowns)."""
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = np.asarray(apply(e.reshape(shape))).ravel()
    return A
