"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the printed
gamma matrices and their algebra, dense brute-force matrices assembled from
the definitions (eq. (eo0); eqs. (DW)/(covariant); the literal twisted
boundary condition), free-field closed forms, plane waves, gamma_5
hermiticity, gauge covariance, the kappa = 0 limit, and a dense linear solve.
"""
import numpy as np
import pytest

import oracle
import synth
import dense

THETA_AP = np.array([1.0, 0.0, 0.0, 0.0])  # antiperiodic in time
THETA_GEN = np.array([1.0, 0.3, -0.7, 0.45])  # generic twisted boundary phases


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ----------------------------------------------------------------- gammas


def test_gammas_match_appendix_A():
    g = oracle.gammas()
    assert np.array_equal(g, dense.G)


def test_gamma_algebra():
    g = dense.G
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)  # Hermitian
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * (m == n) * np.eye(4))
        assert np.allclose(g[4] @ g[m] + g[m] @ g[4], 0)
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], g[4])  # gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3


# --------------------------------------------------------------- geometry


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 2, 4), (8, 4, 4, 6)])
def test_odd_sites(dims):
    odd = oracle.odd_sites(dims)
    V = int(np.prod(dims))
    assert len(odd) == V // 2
    assert np.all(np.diff(odd) > 0)
    assert np.all(dense.parities(dims)[odd] == 1)
    # with LX even, consecutive (x even, x odd) pairs hold one site of each parity,
    # so the k-th odd site is at index 2k or 2k+1
    assert np.array_equal(odd >> 1, np.arange(V // 2))


# ------------------------------------------------------- dense operators

SMALL = [(2, 2, 2, 2), (4, 6, 2, 4)]


@pytest.fixture(scope="module", params=SMALL, ids=lambda d: "x".join(map(str, d)))
def small_case(request):
    dims = request.param
    U = synth.random_gauge(dims, eps=0.6, seed=11)
    return dims, U


def _oracle_M_dense(U, kappa, mut, sign, theta):
    dims = U.shape[:4]
    n = 12 * int(np.prod(dims))
    return dense.dense_of(lambda v: oracle.M(U, v, kappa, mut, sign, theta), n, dims + (4, 3))


@pytest.mark.parametrize("sign", [+1, -1])
def test_M_matches_eo0_assembly(small_case, sign):
    dims, U = small_case
    A = _oracle_M_dense(U, 0.17, 0.05, sign, THETA_GEN)
    B = dense.M_hopping(U, 0.17, 0.05, sign, THETA_GEN)
    assert rel(A, B) < 1e-14


@pytest.mark.parametrize("sign", [+1, -1])
def test_M_matches_covariant_wilson_form(small_case, sign):
    """eq. (eo0) = gamma_5 [2 kappa (D_W + m0) + i mut g5] gamma_5 with D_W from eq. (DW)."""
    dims, U = small_case
    kappa, mut = 0.13, 0.07
    A = _oracle_M_dense(U, kappa, mut, sign, THETA_GEN)
    B = dense.M_covariant(U, kappa, mut, sign, THETA_GEN)
    V = int(np.prod(dims))
    g5 = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))
    assert rel(A, g5 @ B @ g5) < 1e-13


def test_spread_phase_equals_twisted_boundary_condition(small_case):
    """The per-hop phase is the BC psi(x+L) = e^{i theta pi} psi(x) after a site-diagonal unitary."""
    dims, U = small_case
    A = _oracle_M_dense(U, 0.15, 0.02, +1, THETA_GEN)
    B = dense.M_hopping(U, 0.15, 0.02, +1, THETA_GEN, mode="boundary")
    w = dense.boundary_gauge_transform(dims, THETA_GEN)
    assert rel(A, (w.conj()[:, None] * B) * w[None, :]) < 1e-14
    # and the phase is not trivially absent: with theta = 0 the operator differs
    C = _oracle_M_dense(U, 0.15, 0.02, +1, np.zeros(4))
    assert rel(A, C) > 1e-3


@pytest.mark.parametrize("sign", [+1, -1])
def test_Qhat_matches_dense_schur_complement(small_case, sign):
    dims, U = small_case
    kappa, mut = 0.16, 0.03
    V = int(np.prod(dims))
    A = dense.dense_of(lambda v: oracle.Qhat(U, v, kappa, mut, sign, THETA_GEN), 6 * V, (V // 2, 4, 3))
    M = dense.M_hopping(U, kappa, mut, sign, THETA_GEN)
    B = dense.schur_Qhat(M, dims)
    assert rel(A, B) < 1e-13


def test_Q_full_is_gamma5_M(small_case):
    dims, U = small_case
    psi = synth.gaussian_spinor(dims + (4, 3), seed=5)
    a = oracle.Q(U, psi, 0.16, 0.01, -1, THETA_AP)
    b = oracle.M(U, psi, 0.16, 0.01, -1, THETA_AP)
    b[..., 2:, :] *= -1
    assert rel(a, b) == 0.0


# -------------------------------------------------------------- free field


def _momenta(dims, theta):
    L = dense.extents(dims)
    grids = np.meshgrid(*[(2 * np.pi * np.arange(L[m]) + theta[m] * np.pi) / L[m] for m in range(4)],
                        indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)  # (V, 4) over mu = t, x, y, z


@pytest.mark.parametrize("dims", [(4, 6, 2, 4), (6, 4, 4, 2)])
def test_free_plane_waves(dims):
    """U = 1: H e^{iqx} u = sum_mu (2 cos p_mu + 2 i gamma_mu sin p_mu) e^{iqx} u, p = q + theta pi / L."""
    U = synth.unit_gauge(dims)
    L = dense.extents(dims)
    c = dense.site_coords(dims)
    rng = np.random.default_rng(3)
    for _ in range(4):
        n = np.array([rng.integers(0, L[m]) for m in range(4)])
        q = 2 * np.pi * n / L
        p = q + THETA_GEN * np.pi / L
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        wave = np.exp(1j * (c @ q))
        psi = (wave[:, None, None] * u[None]).reshape(dims + (4, 3))
        h = sum(2 * np.cos(p[m]) * np.eye(4) + 2j * np.sin(p[m]) * dense.G[m] for m in range(4))
        expect = (wave[:, None, None] * (h @ u)[None]).reshape(dims + (4, 3))
        assert rel(oracle.hop(U, psi, THETA_GEN), expect) < 1e-14


def test_free_field_M_spectrum():
    """Eigenvalues a(p) +- i sqrt(sum_mu b_mu^2 + mut^2), a = 1 - 2k sum cos p, b = 2k sin p."""
    dims = (4, 2, 2, 4)
    kappa, mut = 0.16, 0.05
    U = synth.unit_gauge(dims)
    A = _oracle_M_dense(U, kappa, mut, +1, THETA_GEN)
    p = _momenta(dims, THETA_GEN)
    a = 1 - 2 * kappa * np.cos(p).sum(axis=1)
    w = np.sqrt((2 * kappa * np.sin(p)) ** 2 @ np.ones(4) + mut ** 2)
    expect = np.concatenate([np.repeat(a + 1j * w, 6), np.repeat(a - 1j * w, 6)])
    got = np.linalg.eigvals(A)

    def canon(z):
        return z[np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))]

    assert np.max(np.abs(canon(got) - canon(expect))) < 1e-12


def qq_free_eigenvalues(dims, kappa, mut, theta):
    """Closed form of the Qhat^+Qhat^- spectrum for U = 1 (each momentum of the full zone 6-fold)."""
    p = _momenta(dims, theta)
    c = 2 * np.cos(p).sum(axis=1)
    s2 = 4 * (np.sin(p) ** 2).sum(axis=1)
    d = 1 + mut ** 2
    alpha = 1 - kappa ** 2 * (c ** 2 - s2) / d
    beta = mut * (1 + kappa ** 2 * (c ** 2 + s2) / d)
    delta = 2 * kappa ** 2 * c / d
    return np.repeat(alpha ** 2 + beta ** 2 + delta ** 2 * s2, 6)


def test_free_field_QhatQhat_spectrum():
    dims = (4, 4, 4, 4)
    kappa, mut = 0.1632, 0.004
    U = synth.unit_gauge(dims)
    n = 6 * int(np.prod(dims))
    A = dense.dense_of(lambda v: oracle.QhatQhat(U, v, kappa, mut, THETA_AP), n, (n // 12, 4, 3))
    assert np.allclose(A, A.conj().T, atol=1e-14)
    got = np.sort(np.linalg.eigvalsh(A))
    expect = np.sort(qq_free_eigenvalues(dims, kappa, mut, THETA_AP))
    assert np.max(np.abs(got - expect)) < 1e-13


# ------------------------------------------------------------- invariants


def test_gamma5_hermiticity_dense(small_case):
    dims, U = small_case
    A = _oracle_M_dense(U, 0.16, 0.04, +1, THETA_GEN)
    B = _oracle_M_dense(U, 0.16, 0.04, -1, THETA_GEN)
    V = int(np.prod(dims))
    g5 = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))
    assert rel(g5 @ A @ g5, B.conj().T) < 1e-15


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 4)])
def test_Qhat_adjoint(dims):
    """(Qhat^+)^dagger = Qhat^-: <y, Qhat^+ x> = <Qhat^- y, x>."""
    U = synth.random_gauge(dims, seed=21)
    x = synth.gaussian_odd(dims, seed=1)
    y = synth.gaussian_odd(dims, seed=2)
    kappa, mut = 0.1632, 0.004
    lhs = np.vdot(y, oracle.Qhat(U, x, kappa, mut, +1, THETA_AP))
    rhs = np.vdot(oracle.Qhat(U, y, kappa, mut, -1, THETA_AP), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # Qhat itself is not Hermitian
    lhs2 = np.vdot(y, oracle.Qhat(U, x, kappa, mut, -1, THETA_AP))
    assert abs(lhs - lhs2) / abs(lhs) > 1e-6


def _colour(Om, psi):
    return np.einsum("sab,sib->sia", Om, psi)


@pytest.mark.parametrize("dims", [(4, 4, 2, 6), (4, 4, 4, 4)])
def test_gauge_covariance(dims):
    """U -> Om(x) U(x,mu) Om(x+mu)^+, psi -> Om psi: M[U^Om] Om psi = Om M[U] psi; same for Qhat."""
    U = synth.random_gauge(dims, seed=31)
    V = int(np.prod(dims))
    rng = np.random.default_rng(32)
    Om = synth.random_su3(V, 1.5, rng)
    c = dense.site_coords(dims)
    L = dense.extents(dims)
    Ug = np.empty_like(U).reshape(V, 4, 3, 3)
    Uf = U.reshape(V, 4, 3, 3)
    for mu in range(4):
        cn = c.copy()
        cn[:, mu] = (cn[:, mu] + 1) % L[mu]
        fwd = dense.site_index(dims, cn)
        Ug[:, mu] = Om @ Uf[:, mu] @ Om[fwd].conj().transpose(0, 2, 1)
    Ug = Ug.reshape(U.shape)
    psi = synth.gaussian_spinor((V, 4, 3), seed=33)
    a = oracle.M(Ug, _colour(Om, psi).reshape(dims + (4, 3)), 0.16, 0.01, +1, THETA_GEN)
    b = _colour(Om, oracle.M(U, psi.reshape(dims + (4, 3)), 0.16, 0.01, +1, THETA_GEN).reshape(V, 4, 3))
    assert rel(a.reshape(V, 4, 3), b) < 1e-14
    odd = oracle.odd_sites(dims)
    po = synth.gaussian_odd(dims, seed=34)
    a = oracle.Qhat(Ug, _colour(Om[odd], po), 0.1632, 0.004, -1, THETA_AP)
    b = _colour(Om[odd], oracle.Qhat(U, po, 0.1632, 0.004, -1, THETA_AP))
    assert rel(a, b) < 1e-14


def test_kappa_zero():
    """kappa = 0: Qhat^+Qhat^- = (1 + mut^2) 1, so CG converges in one step to b/(1+mut^2)."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=41)
    b = synth.gaussian_odd(dims, seed=42)
    mut = 0.3
    assert rel(oracle.QhatQhat(U, b, 0.0, mut, THETA_AP), (1 + mut ** 2) * b) < 1e-15
    x, info = oracle.cg(U, b, 0.0, mut, THETA_AP, tol=1e-12)
    assert info["converged"] and info["iters"] == 1
    assert rel(x, b / (1 + mut ** 2)) < 1e-14  # alpha carries the rounding of two sums over 1536 terms


def test_mee_inverse_closed_form():
    """eq. (eo3): (1 +- i mut g5)^{-1} = (1 -+ i mut g5) / (1 + mut^2)."""
    for mut in (0.004, 0.3, 2.0):
        for s in (+1, -1):
            A = np.eye(4) + 1j * s * mut * dense.G5
            B = (np.eye(4) - 1j * s * mut * dense.G5) / (1 + mut ** 2)
            assert np.allclose(A @ B, np.eye(4), atol=1e-15)


# --------------------------------------------------------------------- CG


def test_cg_matches_dense_solve():
    dims = (2, 2, 2, 2)
    U = synth.random_gauge(dims, seed=51)
    kappa, mut = 0.1632, 0.004
    n = 6 * 16
    A = dense.dense_of(lambda v: oracle.QhatQhat(U, v, kappa, mut, THETA_AP), n, (8, 4, 3))
    b = synth.gaussian_odd(dims, seed=52)
    xs = np.linalg.solve(A, b.ravel())
    ev = np.linalg.eigvalsh(A)
    x, info = oracle.cg(U, b, kappa, mut, THETA_AP, tol=1e-10, history=True)
    assert info["converged"]
    assert rel(x.ravel(), xs) <= (ev[-1] / ev[0]) * 1e-10
    # Ritz values of the Lanczos matrix built from the CG coefficients lie inside
    # the spectrum and the largest one reaches lambda_max
    a, bt = info["alpha"], info["beta"]
    k = len(a)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1 / a[i] + (bt[i - 1] / a[i - 1] if i else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(bt[i]) / a[i]
    ritz = np.linalg.eigvalsh(T)
    assert ritz.min() >= ev[0] * (1 - 1e-8) and ritz.max() <= ev[-1] * (1 + 1e-8)
    # CG stops once the residual is small, so the extreme Ritz values are close but not exact
    assert abs(ritz.max() - ev[-1]) / ev[-1] < 1e-3
    assert abs(ritz.min() - ev[0]) / ev[0] < 1e-2


def test_cg_full_operator_4444():
    """Plain FP64 full-lattice Q^+Q^- solve on 4^4, kappa 0.16, 2 kappa mu 0.01, tol 1e-10."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=1000)
    b = synth.gaussian_spinor(dims + (4, 3), seed=2000).reshape(-1, 4, 3)
    x, info = oracle.cg(U, b, 0.16, 0.01, THETA_AP, eo=False, tol=1e-10)
    assert info["converged"]
    assert oracle.true_residual(U, b, x, 0.16, 0.01, THETA_AP, eo=False) < 2e-10


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 4, 4)])
def test_cg_free_field_terminates(dims):
    """In exact arithmetic CG stops after at most as many steps as A has distinct eigenvalues."""
    kappa, mut = 0.1632, 0.004
    U = synth.unit_gauge(dims)
    b = synth.gaussian_odd(dims, seed=61)
    ndist = len(np.unique(np.round(qq_free_eigenvalues(dims, kappa, mut, THETA_AP), 10)))
    x, info = oracle.cg(U, b, kappa, mut, THETA_AP, tol=1e-10)
    assert info["converged"] and info["iters"] <= ndist + 1
    assert oracle.true_residual(U, b, x, kappa, mut, THETA_AP) < 2e-10


def test_cg_eo_residual_and_max_iter():
    dims = (8, 4, 4, 4)
    U = synth.random_gauge(dims, seed=71)
    b = synth.gaussian_odd(dims, seed=72)
    x, info = oracle.cg(U, b, 0.1632, 0.004, THETA_AP, tol=1e-10)
    assert info["converged"] and 20 < info["iters"] < 80
    assert oracle.true_residual(U, b, x, 0.1632, 0.004, THETA_AP) < 2e-10
    x2, info2 = oracle.cg(U, b, 0.1632, 0.004, THETA_AP, tol=1e-10, max_iter=3)
    assert not info2["converged"] and info2["iters"] == 3


# -------------------------------------------------------------- generators


def test_su3_generator():
    rng = np.random.default_rng(81)
    U = synth.random_su3(20000, 0.3, rng)
    eye = np.eye(3)
    assert np.max(np.abs(U @ U.conj().transpose(0, 2, 1) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14
    # <Re tr U>/3 ~ 1 - eps^2 <tr H^2>/6 = 1 - 0.09 * 4 / 6 = 0.94 (to O(eps^4))
    m = np.mean(np.real(np.trace(U, axis1=1, axis2=2))) / 3
    assert abs(m - 0.941) < 0.003


# ------------------------------------------------------------------- codec


@pytest.mark.parametrize("kind", ["fp16", "bf16"])
def test_codec_reference(kind):
    import torch

    psi = synth.gaussian_odd((4, 4, 4, 4), seed=91) * np.exp(np.random.default_rng(1).normal(size=(128, 1, 1)))
    psi[3] = 0
    codes, scale = oracle.encode_site_scaled(psi, kind)
    # the rounding agrees with torch's FP32 -> FP16 / BF16 conversion (RNE)
    re = psi.reshape(-1, 12).view(np.float64).reshape(-1, 24)
    s = np.where(scale > 0, scale.astype(np.float64), 1.0)
    y = torch.from_numpy((re / s[:, None]).astype(np.float32))
    tdt = torch.float16 if kind == "fp16" else torch.bfloat16
    ref = y.to(tdt).view(torch.int16).numpy().view(np.uint16)
    ref[3] = 0
    assert np.array_equal(codes, ref)
    back = oracle.decode_site_scaled(codes, scale, kind)
    bound = 2.0 ** (-11 if kind == "fp16" else -8)
    err = np.abs(back.reshape(-1, 12).view(np.float64).reshape(-1, 24) - re)
    assert np.all(err <= bound * scale[:, None] * (1 + 1e-6))
    assert scale[3] == 0 and np.all(back[3] == 0)


# ---------------------------------------------------------- flavour doublet
# eq. (Dh) in the hopping normalisation; mubar, epsbar stand for 2 kappa mubar
# and 2 kappa epsbar (the doublet run of the paper's test-run table: kappa
# 0.17, 2 kappa mubar 0.1105, 2 kappa epsbar 0.0935).
ND_KAPPA, ND_MUBAR, ND_EPSBAR = 0.17, 0.1105, 0.0935
TAU = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]


def _dense_Mh(U, kappa, mubar, epsbar, theta):
    """Dense doublet operator [[M(+mubar), epsbar], [epsbar, M(-mubar)]] assembled from
    the one-flavour eq. (eo0) matrices (flavour-major index)."""
    Mu = dense.M_hopping(U, kappa, mubar, +1, theta)
    Md = dense.M_hopping(U, kappa, mubar, -1, theta)
    one = np.eye(Mu.shape[0])
    return np.block([[Mu, epsbar * one], [epsbar * one, Md]])


def test_doublet_site_term_flavour_rotation():
    """eq. (altDh): the site term of eq. (Dh) rotated in flavour space is the
    (mu_sigma, mu_delta) = (mubar, -epsbar) form.  The rotation that does it
    is (1 - i tau^2) . (1 + i tau^2) / 2 (the paper prints the factors in the
    other order, which gives the same form with both masses negated)."""
    g5 = dense.G5
    for mb, eb in ((ND_MUBAR, ND_EPSBAR), (0.3, -0.2)):
        A = oracle.doublet_site_matrix(mb, eb)
        Ap = np.eye(8) + 1j * mb * np.kron(TAU[0], g5) + (-eb) * np.kron(TAU[2], np.eye(4))
        Rm = np.kron(np.eye(2) - 1j * TAU[1], np.eye(4))
        Rp = np.kron(np.eye(2) + 1j * TAU[1], np.eye(4))
        assert np.abs(Rm @ A @ Rp / 2 - Ap).max() < 1e-15
        # and the inverse the even/odd reduction needs: (1 - i mubar g5 tau^3 - epsbar tau^1) / (1 + mubar^2 - epsbar^2)
        inv = (np.eye(8) - 1j * mb * np.kron(TAU[2], g5) - eb * np.kron(TAU[0], np.eye(4))) / (1 + mb * mb - eb * eb)
        assert np.abs(A @ inv - np.eye(8)).max() < 1e-15


def test_doublet_Mh_matches_dense(small_case):
    dims, U = small_case
    V = int(np.prod(dims))
    A = dense.dense_of(lambda v: oracle.Mh(U, v, ND_KAPPA, ND_MUBAR, ND_EPSBAR, THETA_GEN), 24 * V,
                       (2,) + tuple(dims) + (4, 3))
    B = _dense_Mh(U, ND_KAPPA, ND_MUBAR, ND_EPSBAR, THETA_GEN)
    assert rel(A, B) < 1e-14


@pytest.mark.parametrize("sign", [+1, -1])
def test_Qhat_nd_matches_dense_schur_complement(small_case, sign):
    """Qhat_h = g5 (M_oo - M_oe M_ee^-1 M_eo) of the dense doublet operator,
    the even/odd factorisation of App. B applied to eq. (Dh)."""
    dims, U = small_case
    V = int(np.prod(dims))
    A = dense.dense_of(lambda v: oracle.Qhat_nd(U, v, ND_KAPPA, ND_MUBAR, ND_EPSBAR, sign, THETA_GEN), 12 * V,
                       (2, V // 2, 4, 3))
    M = _dense_Mh(U, ND_KAPPA, sign * ND_MUBAR, ND_EPSBAR, THETA_GEN)
    e, o = dense.eo_blocks(dims)
    e2 = np.concatenate([e, 12 * V + e])
    o2 = np.concatenate([o, 12 * V + o])
    S = M[np.ix_(o2, o2)] - M[np.ix_(o2, e2)] @ np.linalg.solve(M[np.ix_(e2, e2)], M[np.ix_(e2, o2)])
    g5 = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))  # 2 flavours x V/2 odd sites
    assert rel(A, g5 @ S) < 1e-13


def test_Qhat_nd_reduces_to_degenerate():
    """epsbar = 0: the doublet decouples into Qhat^{+-} of eq. (eo4) for the two flavours."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=71)
    psi = np.stack([synth.gaussian_odd(dims, seed=72), synth.gaussian_odd(dims, seed=73)])
    for sign in (+1, -1):
        a = oracle.Qhat_nd(U, psi, ND_KAPPA, ND_MUBAR, 0.0, sign, THETA_AP)
        assert rel(a[0], oracle.Qhat(U, psi[0], ND_KAPPA, ND_MUBAR, sign, THETA_AP)) < 1e-14
        assert rel(a[1], oracle.Qhat(U, psi[1], ND_KAPPA, ND_MUBAR, -sign, THETA_AP)) < 1e-14


def test_Qhat_nd_adjoint_and_tau3():
    """(Qhat_h^+)^dagger = Qhat_h^- ; flipping the sign of epsbar (the convention of
    eq. (Dheo) against eq. (Dh)) is the flavour rotation tau^3 on both sides."""
    dims = (4, 4, 2, 6)
    U = synth.random_gauge(dims, seed=74)
    x = np.stack([synth.gaussian_odd(dims, seed=75), synth.gaussian_odd(dims, seed=76)])
    y = np.stack([synth.gaussian_odd(dims, seed=77), synth.gaussian_odd(dims, seed=78)])
    args = (ND_KAPPA, ND_MUBAR, ND_EPSBAR)
    lhs = np.vdot(y, oracle.Qhat_nd(U, x, *args, +1, THETA_GEN))
    rhs = np.vdot(oracle.Qhat_nd(U, y, *args, -1, THETA_GEN), x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    assert abs(lhs - np.vdot(y, oracle.Qhat_nd(U, x, *args, -1, THETA_GEN))) / abs(lhs) > 1e-6
    t3 = np.array([1.0, -1.0])[:, None, None, None]
    a = oracle.Qhat_nd(U, x, ND_KAPPA, ND_MUBAR, -ND_EPSBAR, +1, THETA_GEN)
    b = t3 * oracle.Qhat_nd(U, t3 * x, *args, +1, THETA_GEN)
    assert rel(a, b) < 1e-15


def test_cg_nd_matches_dense_solve():
    dims = (2, 2, 2, 2)
    U = synth.random_gauge(dims, seed=79)
    args = (ND_KAPPA, ND_MUBAR, ND_EPSBAR)
    n = 2 * 6 * 16
    A = dense.dense_of(lambda v: oracle.QhatQhat_nd(U, v, *args, THETA_AP), n, (2, 8, 4, 3))
    assert rel(A, A.conj().T) < 1e-14
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > 0
    b = np.stack([synth.gaussian_odd(dims, seed=80), synth.gaussian_odd(dims, seed=81)])
    xs = np.linalg.solve(A, b.ravel())
    x, info = oracle.cg_nd(U, b, *args, THETA_AP, tol=1e-10)
    assert info["converged"]
    assert rel(x.ravel(), xs) <= (ev[-1] / ev[0]) * 1e-10
    assert oracle.true_residual_nd(U, b, x, *args, THETA_AP) <= 1e-10


# -------------------------------------------------------------- BiCGstab


def test_bicgstab_matches_dense_solve():
    """BiCGstab on Qhat^{+-} itself against a dense solve of the dense Qhat (2^4 and 4x2^3)."""
    for dims in [(2, 2, 2, 2), (4, 2, 2, 2)]:
        U = synth.random_gauge(dims, seed=91)
        V = int(np.prod(dims))
        b = synth.gaussian_odd(dims, seed=92)
        for sign in (+1, -1):
            A = dense.schur_Qhat(dense.M_hopping(U, 0.1632, 0.004, sign, THETA_AP), dims)
            xs = np.linalg.solve(A, b.ravel())
            sv = np.linalg.svd(A, compute_uv=False)
            x, info = oracle.bicgstab(U, b, 0.1632, 0.004, sign, THETA_AP, tol=1e-11)
            assert info["converged"], info
            assert rel(x.ravel(), xs) <= (sv[0] / sv[-1]) * 1e-11
            assert rel(oracle.Qhat(U, x, 0.1632, 0.004, sign, THETA_AP), b) <= 2e-11
            assert x.shape == (V // 2, 4, 3)


def test_bicgstab_kappa_zero_closed_form():
    """kappa = 0: Qhat^{+-} = g5 (1 +- i mut g5) = g5 +- i mut has the two eigenvalues
    +-1 +- i mut, so the BiCG polynomial of degree 2 annihilates any residual and
    BiCGstab ends within two steps, with x = (g5 -+ i mut) b / (1 + mut^2)."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=93)
    b = synth.gaussian_odd(dims, seed=94)
    mut = 0.3
    for sign in (+1, -1):
        x, info = oracle.bicgstab(U, b, 0.0, mut, sign, THETA_AP, tol=1e-12)
        assert info["converged"] and info["iters"] <= 2
        g5b = b.copy()
        g5b[:, 2:, :] *= -1
        want = (g5b - sign * 1j * mut * b) / (1 + mut ** 2)
        assert rel(x, want) < 1e-14


def test_bicgstab_solves_the_cg_system_consistently():
    """Solving Qhat^+ y = b by BiCGstab, then Qhat^- x = y, gives the CG solution of
    Qhat^+ Qhat^- x = b (4^4, random links)."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=95)
    b = synth.gaussian_odd(dims, seed=96)
    y, i1 = oracle.bicgstab(U, b, 0.1632, 0.004, +1, THETA_AP, tol=1e-12)
    x, i2 = oracle.bicgstab(U, y, 0.1632, 0.004, -1, THETA_AP, tol=1e-12)
    xc, ic = oracle.cg(U, b, 0.1632, 0.004, THETA_AP, tol=1e-12)
    assert i1["converged"] and i2["converged"] and ic["converged"]
    assert rel(x, xc) < 1e-9


# ------------------------------------------------ consumers of the solver


@pytest.mark.parametrize("sign", [+1, -1])
def test_oracle_solve_M_matches_dense(sign):
    dims = (4, 2, 2, 2)
    U = synth.random_gauge(dims, seed=97)
    phi = synth.gaussian_spinor(dims + (4, 3), seed=98)
    psi = oracle.solve_M(U, phi, 0.16, 0.03, sign, THETA_GEN, tol=1e-13)
    want = np.linalg.solve(dense.M_hopping(U, 0.16, 0.03, sign, THETA_GEN), phi.ravel())
    assert rel(psi.ravel(), want) < 1e-10


@pytest.mark.parametrize("t0", [0, 1])
def test_pion_correlator_point_sources_match_dense_propagator(t0):
    """The one-end estimator summed over the 12 unit sources at one site is the
    point-to-all correlator sum_x tr[G(x, y) G(x, y)^+] of the dense propagator
    G = (M^+)^-1 (so the solve, the time-slice sums and the shift by t0 are right)."""
    dims = (4, 2, 2, 2)
    U = synth.random_gauge(dims, seed=99)
    kappa, mut = 0.16, 0.05
    V = int(np.prod(dims))
    G = np.linalg.inv(dense.M_hopping(U, kappa, mut, +1, THETA_AP)).reshape(V, 12, V, 12)
    y = t0 * (V // dims[0])  # site (t0, 0, 0, 0)
    want = np.zeros(dims[0])
    for x in range(V):
        want[(x // (V // dims[0]) - t0) % dims[0]] += float(np.sum(np.abs(G[x, :, y, :]) ** 2))
    got = np.zeros(dims[0])
    total = 0.0
    for k in range(12):
        xi = np.zeros((V, 12), dtype=np.complex128)
        xi[y, k] = 1.0
        c, phi = oracle.pion_correlator(U, xi.reshape(dims + (4, 3)), kappa, mut, THETA_AP, t0=t0)
        got += c
        total += float(np.vdot(phi, phi).real)
    assert rel(got, want) < 1e-10
    assert abs(got.sum() - total) <= 1e-12 * total


def test_heatbath_and_force_solves():
    """eqs. (eo10), (eo6): with phi_o = Qhat^+ r_o, X_o = (Qhat^+ Qhat^-)^-1 phi_o and
    Y_o = Qhat^- X_o give back Y_o = r_o, and S_PF = phi_o^+ X_o = |r_o|^2."""
    dims = (4, 4, 4, 4)
    U = synth.random_gauge(dims, seed=100)
    r = synth.gaussian_odd(dims, seed=101)
    phi = oracle.Qhat(U, r, 0.1632, 0.004, +1, THETA_AP)
    X, info = oracle.cg(U, phi, 0.1632, 0.004, THETA_AP, tol=1e-12)
    Y = oracle.Qhat(U, X, 0.1632, 0.004, -1, THETA_AP)
    assert info["converged"]
    assert rel(Y, r) < 1e-9
    assert abs(np.vdot(phi, X).real - np.vdot(r, r).real) < 1e-9 * np.vdot(r, r).real


# ---------------------------------------------- the acceptance checker
# Every solve is accepted on the FP64 true residual |b - A x| / |b| (Sec. 4.4,
# last paragraph).  These pins fix its value against dense matrices assembled
# from eq. (eo0) by brute force, at residuals far from the converged regime
# (so a missing square root, a squared or doubly normalised result, or the
# wrong operator order would show), not only on converged solutions.


def _dense_normal(U, kappa, mut, theta, eo):
    dims = U.shape[:4]
    Mp = dense.M_hopping(U, kappa, mut, +1, theta)
    Mm = dense.M_hopping(U, kappa, mut, -1, theta)
    if eo:
        return dense.schur_Qhat(Mp, dims) @ dense.schur_Qhat(Mm, dims)  # Qhat^- first
    V = int(np.prod(dims))
    g5 = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))
    return (g5 @ Mp) @ (g5 @ Mm)  # Q^+ Q^- = g5 M^+ g5 M^-


@pytest.mark.parametrize("eo", [True, False], ids=["eo", "full"])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)], ids=lambda d: "x".join(map(str, d)))
def test_true_residual_matches_dense(dims, eo):
    U = synth.random_gauge(dims, eps=0.5, seed=131)
    kappa, mut = 0.1632, 0.004
    A = _dense_normal(U, kappa, mut, THETA_GEN, eo)
    n_sites = int(np.prod(dims)) // (2 if eo else 1)
    shape = (n_sites, 4, 3)
    b = synth.gaussian_spinor(shape, seed=132)
    # x = 0: the residual is b itself, exactly 1
    assert oracle.true_residual(U, b, np.zeros_like(b), kappa, mut, THETA_GEN, eo=eo) == 1.0
    xs = np.linalg.solve(A, b.ravel())
    rng = np.random.default_rng(133)
    for scale in (0.0, 1e-9, 1e-3, 0.3):
        # x* plus a perturbation: residuals from rounding level up to O(1)
        d = rng.normal(size=xs.shape) + 1j * rng.normal(size=xs.shape)
        x = xs + scale * np.linalg.norm(xs) / np.linalg.norm(d) * d
        want = np.linalg.norm(b.ravel() - A @ x) / np.linalg.norm(b.ravel())
        got = oracle.true_residual(U, b, x.reshape(shape), kappa, mut, THETA_GEN, eo=eo)
        if scale == 0.0:
            assert got < 1e-13  # the exact solution, up to rounding
        else:
            # rounding of A x in either computation is ~1e-16 |b| in absolute terms
            assert abs(got - want) <= 1e-12 * want + 1e-14, (scale, got, want)
    # with |b| = 1 the value is the plain |b - A x|
    bn = b / np.linalg.norm(b.ravel())
    x = rng.normal(size=xs.shape) * 1e-2
    want = np.linalg.norm(bn.ravel() - A @ x)
    got = oracle.true_residual(U, bn, x.reshape(shape), kappa, mut, THETA_GEN, eo=eo)
    assert abs(got - want) <= 1e-12 * want


def test_true_residual_nd_matches_dense():
    """The doublet's checker against the dense doublet Schur complement (eq. (Dh),
    App. B), Qhat_h^- applied first, at residuals from 1e-9 to O(1)."""
    dims = (2, 2, 2, 2)
    V = int(np.prod(dims))
    U = synth.random_gauge(dims, eps=0.5, seed=134)
    args = (ND_KAPPA, ND_MUBAR, ND_EPSBAR)
    e, o = dense.eo_blocks(dims)
    e2 = np.concatenate([e, 12 * V + e])
    o2 = np.concatenate([o, 12 * V + o])
    g5 = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))

    def schur(sign):
        M = _dense_Mh(U, ND_KAPPA, sign * ND_MUBAR, ND_EPSBAR, THETA_GEN)
        S = M[np.ix_(o2, o2)] - M[np.ix_(o2, e2)] @ np.linalg.solve(M[np.ix_(e2, e2)], M[np.ix_(e2, o2)])
        return g5 @ S

    A = schur(+1) @ schur(-1)
    b = np.stack([synth.gaussian_odd(dims, seed=135), synth.gaussian_odd(dims, seed=136)])
    assert oracle.true_residual_nd(U, b, np.zeros_like(b), *args, THETA_GEN) == 1.0
    xs = np.linalg.solve(A, b.ravel())
    rng = np.random.default_rng(137)
    for scale in (1e-9, 1e-3, 0.3):
        d = rng.normal(size=xs.shape) + 1j * rng.normal(size=xs.shape)
        x = xs + scale * np.linalg.norm(xs) / np.linalg.norm(d) * d
        want = np.linalg.norm(b.ravel() - A @ x) / np.linalg.norm(b.ravel())
        got = oracle.true_residual_nd(U, b, x.reshape(b.shape), *args, THETA_GEN)
        assert abs(got - want) <= 1e-12 * want + 1e-14, (scale, got, want)


# ------------------------------------------------- C_PGamma of the one-end trick


def _cpg_gammas():
    g = dense.G
    g5 = dense.G5
    rng = np.random.default_rng(141)
    rand = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    # <PP>, <PA> and <PV> with mu = t (A = g5 g0, V = g0), and a generic matrix
    return {"P": g5, "A0": g5 @ g[0], "V0": g[0], "V2": g[2], "random": rand}


@pytest.mark.parametrize("name", list(_cpg_gammas()))
def test_bilinear_gives_the_papers_C_PGamma(name):
    """The one-end trick of eqs. (source)/(oneend): for phi = (M^+)^-1 xi with the
    noise on time slice t0, the time-slice bilinear sum_x phi^+ (g5 Gamma) phi,
    summed over the 12 unit sources of a site y (the complete spin-colour
    basis, for which the noise average of eq. (source) is exact), equals
    C_PGamma = sum_x tr[G_u(x, y) g5 G_d(y, x) Gamma] built from the two dense
    propagators G_u = (M^+)^-1 and G_d = (M^-)^-1.  So Gamma sits at the point
    where the bilinear is formed (the paper's "source" 0), the noise at the
    other end, and g5 Gamma is the matrix the bilinear takes; Gamma = g5 gives
    the pion correlator.  The gamma_5-hermiticity step G_u(x,y) = g5 G_d(y,x)^+ g5
    that the paper uses is checked on the way."""
    gam = _cpg_gammas()[name]
    dims = (4, 2, 2, 2)
    T = dims[0]
    U = synth.random_gauge(dims, seed=142)
    kappa, mut = 0.16, 0.05
    V = int(np.prod(dims))
    Gu = np.linalg.inv(dense.M_hopping(U, kappa, mut, +1, THETA_AP))
    Gd = np.linalg.inv(dense.M_hopping(U, kappa, mut, -1, THETA_AP))
    g5f = np.kron(np.eye(V), np.kron(dense.G5, dense.I3))
    assert rel(Gu, g5f @ Gd.conj().T @ g5f) < 1e-13
    Gu4 = Gu.reshape(V, 4, 3, V, 4, 3)
    Gd4 = Gd.reshape(V, 4, 3, V, 4, 3)
    per_slice = V // T
    for t0 in (0, 1):
        y = t0 * per_slice + 3  # a site of time slice t0
        want = np.zeros(T, dtype=np.complex128)
        for x in range(V):
            # tr over spin and colour of G_u(x, y) g5 G_d(y, x) Gamma
            c = np.einsum("aibj,bc,cjdi,da->", Gu4[x, :, :, y], dense.G5, Gd4[y, :, :, x], gam, optimize=True)
            want[(x // per_slice - t0) % T] += c
        got = np.zeros(T, dtype=np.complex128)
        for k in range(12):
            xi = np.zeros((V, 12), dtype=np.complex128)
            xi[y, k] = 1.0
            phi = (Gu @ xi.ravel()).reshape(dims + (4, 3))
            got += oracle.timeslice_bilinear(phi, dense.G5 @ gam, t0)
        assert rel(got, want) < 1e-12, (t0, got, want)
        # the same through the oracle's own solve (pion_correlator's path for Gamma = g5)
        if name == "P":
            tot = np.zeros(T)
            for k in range(12):
                xi = np.zeros((V, 12), dtype=np.complex128)
                xi[y, k] = 1.0
                tot += oracle.pion_correlator(U, xi.reshape(dims + (4, 3)), kappa, mut, THETA_AP, t0=t0)[0]
            assert rel(tot, want.real) < 1e-10 and np.abs(want.imag).max() < 1e-12 * np.abs(want).max()
