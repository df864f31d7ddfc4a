"""GPU parity of the solver's consumers against the oracle: the HMC force
solves of eq. (eo6) with the heatbath of eq. (eo10) (Y_o gives back r_o,
S_PF = |r_o|^2), the time-slice bilinear contraction, and the
one-end-trick pseudoscalar correlator (eqs. (source), (oneend))."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THETA = np.array([1.0, 0.0, 0.0, 0.0])
THETA_GEN = np.array([1.0, 0.3, -0.7, 0.45])


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def tmq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0905_3331_amd import tmq as t

    return t


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("sloppy", ["fp64", "fp16"])
def test_heatbath_and_force_solves(tmq, sloppy):
    dims = (8, 8, 6, 10)
    U = synth.random_gauge(dims, eps=0.3, seed=130)
    lat = tmq.Lattice(dims)
    lat.load_gauge(U)
    p = tmq.params(0.1632, 0.004, THETA)
    r = synth.gaussian_odd(dims, seed=131)
    phi = lat.apply_Qhat(p, +1, dev(r))  # eq. (eo10)
    o = tmq.solver_opts(tol=1e-10, sloppy=sloppy, sloppy_link="fp16")
    X, Y, S, info = lat.solve_force(p, phi, o)
    assert info.status == 0
    res = oracle.true_residual(U, host(phi), host(X), 0.1632, 0.004, THETA)
    assert res <= 1e-10
    assert rel(host(Y), oracle.Qhat(U, host(X), 0.1632, 0.004, -1, THETA)) < 1e-13
    rr = float(np.vdot(r, r).real)
    print(f"force solves {sloppy}: iters {info.iters} |Y - r|/|r| {rel(host(Y), r):.2e} "
          f"S_PF/|r|^2 - 1 = {S / rr - 1:.2e}")
    assert rel(host(Y), r) < 1e-8
    assert abs(S - rr) < 1e-8 * rr
    lat.close()


@pytest.mark.parametrize("t0", [0, 3])
def test_timeslice_bilinear(tmq, t0):
    dims = (6, 4, 2, 10)
    lat = tmq.Lattice(dims)
    psi = synth.gaussian_spinor(dims + (4, 3), seed=132)
    rng = np.random.default_rng(133)
    g = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    got = lat.timeslice_bilinear(g, dev(psi.reshape(-1, 4, 3)), t0)
    want = oracle.timeslice_bilinear(psi, g, t0)
    assert rel(got, want) < 1e-13
    lat.close()


@pytest.mark.parametrize("sloppy", ["fp64", "fp16"])
def test_pion_correlator(tmq, sloppy):
    dims = (8, 4, 4, 6)
    U = synth.random_gauge(dims, eps=0.3, seed=134)
    lat = tmq.Lattice(dims)
    lat.load_gauge(U)
    t0 = 5
    xi = synth.z2_timeslice_source(dims, t0, seed=135)
    p = tmq.params(0.1632, 0.004, THETA)
    c, phi, info = lat.pion_correlator(p, dev(xi.reshape(-1, 4, 3)),
                                       tmq.solver_opts(tol=1e-11, sloppy=sloppy, sloppy_link="fp16"), t0=t0)
    co, phio = oracle.pion_correlator(U, xi, 0.1632, 0.004, THETA, t0=t0, tol=1e-12)
    print(f"pion correlator {sloppy}: iters {info.iters}, C = {np.array2string(c, precision=4)}")
    assert info.status == 0
    assert rel(host(phi).reshape(phio.shape), phio) < 1e-8
    assert rel(c, co) < 1e-9
    # the correlator decays away from the source
    assert c[0] > c[1] > c[2]
    # through the C ABI without a phi buffer (the library stages the solution itself)
    import ctypes

    from paper_0905_3331_amd.tmq import _lib

    corr = np.zeros(dims[0])
    info2 = tmq.tmq_solve_info()
    o = tmq.solver_opts(tol=1e-11, sloppy=sloppy, sloppy_link="fp16")
    xd = dev(xi.reshape(-1, 4, 3))
    code = _lib.tmq_pion_correlator_dev(lat._h, ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(xd.data_ptr()),
                                        t0, corr.ctypes.data, None, None, ctypes.byref(info2))
    assert code == 0 and np.array_equal(corr, c)
    lat.close()
