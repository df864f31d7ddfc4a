"""GPU parity of the mass non-degenerate flavour doublet (eq. (Dh)): the
even/odd operator Qhat_h^{+-} against the oracle element by element (FP64:
1e-13 relative; FP32/FP16/BF16 storage: bounded by the storage precision),
and CG solves of Qhat_h^+ Qhat_h^- x = b judged by the oracle's FP64 true
residual (<= 1e-10) in every precision mode, batched doublets against their
solves alone bit for bit.  Parameters: the paper's doublet run, kappa 0.17,
2 kappa mubar 0.1105, 2 kappa epsbar 0.0935."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THETA = np.array([1.0, 0.0, 0.0, 0.0])
THETA_GEN = np.array([1.0, 0.3, -0.7, 0.45])
KAPPA, MUBAR, EPSBAR = 0.17, 0.1105, 0.0935


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


def doublet(dims, seed):
    return np.stack([synth.gaussian_odd(dims, seed=seed), synth.gaussian_odd(dims, seed=seed + 1)])


_LAT = {}


def lattice(tmq, dims, seed):
    if (dims, seed) not in _LAT:
        U = synth.random_gauge(dims, eps=0.3, seed=seed)
        lat = tmq.Lattice(dims)
        lat.load_gauge(U)
        _LAT[(dims, seed)] = (lat, U)
    return _LAT[(dims, seed)]


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 10), (8, 8, 6, 10)], ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("sign", [+1, -1])
def test_qhat_nd_fp64(tmq, dims, sign):
    lat, U = lattice(tmq, dims, 301)
    psi = doublet(dims, 302)
    p = tmq.nd_params(KAPPA, MUBAR, EPSBAR, THETA_GEN)
    got = host(lat.apply_Qhat_nd(p, sign, dev(psi)))
    want = oracle.Qhat_nd(U, psi, KAPPA, MUBAR, EPSBAR, sign, THETA_GEN)
    assert rel(got, want) < 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_qhat_nd_random_parameters(tmq, seed):
    """Property test of the doublet operator: random kappa, mubar, epsbar (with
    1 + mubar^2 - epsbar^2 > 0, so that A_ee is invertible), boundary angles,
    operator sign and lattice shape, against the oracle in FP64 and FP16."""
    rng = np.random.default_rng(7400 + seed)
    dims = [(4, 4, 4, 4), (6, 4, 2, 10), (8, 8, 6, 10), (2, 6, 4, 8)][seed]
    kappa = float(rng.uniform(0.05, 0.2))
    mubar = float(rng.uniform(-0.4, 0.4))
    epsbar = float(rng.uniform(-0.4, 0.4))
    assert 1.0 + mubar * mubar - epsbar * epsbar > 0.5
    theta = rng.uniform(-1.0, 1.0, 4)
    sign = int(rng.choice([-1, 1]))
    lat, U = lattice(tmq, dims, 310 + seed)
    psi = doublet(dims, 7500 + seed)
    p = tmq.nd_params(kappa, mubar, epsbar, theta)
    want = oracle.Qhat_nd(U, psi, kappa, mubar, epsbar, sign, theta)
    e64 = rel(host(lat.apply_Qhat_nd(p, sign, dev(psi))), want)
    e16 = rel(host(lat.apply_Qhat_nd(p, sign, dev(psi), prec="fp16")), want)
    print(f"{dims} kappa {kappa:.3f} mubar {mubar:+.3f} epsbar {epsbar:+.3f} sign {sign:+d}: fp64 {e64:.1e} fp16 {e16:.1e}")
    assert e64 < 1e-13 and e16 < 3e-3


@pytest.mark.parametrize("prec,bound", [("fp32", 2e-6), ("fp16", 3e-3), ("bf16", 2.5e-2)])
def test_qhat_nd_reduced_precision_error(tmq, prec, bound):
    dims = (8, 8, 6, 10)
    lat, U = lattice(tmq, dims, 301)
    psi = doublet(dims, 303)
    p = tmq.nd_params(KAPPA, MUBAR, EPSBAR, THETA)
    got = host(lat.apply_Qhat_nd(p, +1, dev(psi), prec=prec))
    err = rel(got, oracle.Qhat_nd(U, psi, KAPPA, MUBAR, EPSBAR, +1, THETA))
    print(f"doublet {prec}: relative error {err:.2e}")
    assert err < bound


def test_qhat_nd_host_api_and_degenerate_limit(tmq):
    """Host pointers give the device result; with epsbar = 0 the flavours are
    Qhat^{+-} of the one-flavour operator (to rounding: the site terms are
    summed in another order)."""
    dims = (6, 4, 2, 10)
    lat, U = lattice(tmq, dims, 301)
    psi = doublet(dims, 304)
    p = tmq.nd_params(KAPPA, MUBAR, EPSBAR, THETA_GEN)
    assert np.array_equal(lat.apply_Qhat_nd(p, -1, psi), host(lat.apply_Qhat_nd(p, -1, dev(psi))))
    p0 = tmq.nd_params(KAPPA, MUBAR, 0.0, THETA_GEN)
    q = tmq.params(KAPPA, MUBAR, THETA_GEN)
    for sign in (+1, -1):
        a = host(lat.apply_Qhat_nd(p0, sign, dev(psi)))
        assert rel(a[0], host(lat.apply_Qhat(q, sign, dev(psi[0])))) < 1e-15
        assert rel(a[1], host(lat.apply_Qhat(q, -sign, dev(psi[1])))) < 1e-15


def test_nd_parameter_validation(tmq):
    lat, _ = lattice(tmq, (4, 4, 4, 4), 301)
    psi = dev(doublet((4, 4, 4, 4), 305))
    with pytest.raises(tmq.TmqError) as e:
        lat.apply_Qhat_nd(tmq.nd_params(KAPPA, 0.1, 1.2), +1, psi)  # 1 + mubar^2 - epsbar^2 < 0
    assert e.value.code == tmq.TMQ_EINVAL
    with pytest.raises(ValueError):
        lat.solve_nd_batch([tmq.nd_params(KAPPA, MUBAR, EPSBAR)] * 33, [psi] * 33, tmq.solver_opts())


@pytest.mark.parametrize("sloppy,link,mode", [("fp64", "fp64", "reliable"), ("fp32", "fp32", "reliable"),
                                              ("fp16", "fp16", "reliable"), ("bf16", "fp16", "reliable"),
                                              ("fp32", "fp32", "switch")])
def test_cg_nd(tmq, sloppy, link, mode):
    dims = (8, 8, 6, 10)
    lat, U = lattice(tmq, dims, 301)
    b = doublet(dims, 306)
    p = tmq.nd_params(KAPPA, MUBAR, EPSBAR, THETA)
    o = tmq.solver_opts(tol=1e-10, sloppy=sloppy, sloppy_link="fp32" if link == "fp64" else link, mode=mode)
    x, info = lat.solve_nd(p, dev(b), o)
    res = oracle.true_residual_nd(U, b, host(x), KAPPA, MUBAR, EPSBAR, THETA)
    print(f"doublet CG {sloppy}/{link}/{mode}: iters {info.iters} reliable {info.reliable_updates} "
          f"true res {res:.2e} (gpu {info.true_rel_residual:.2e})")
    assert info.status == tmq.TMQ_OK and res <= 1e-10
    assert abs(res - info.true_rel_residual) <= 1e-3 * res


def test_cg_nd_matches_oracle_solution(tmq):
    """FP64 CG against the oracle's CG on the same doublet source (4^4): both
    solutions within the bound the tolerance sets."""
    dims = (4, 4, 4, 4)
    lat, U = lattice(tmq, dims, 301)
    b = doublet(dims, 307)
    p = tmq.nd_params(KAPPA, MUBAR, EPSBAR, THETA)
    x, info = lat.solve_nd(p, b, tmq.solver_opts(tol=1e-12))  # host-pointer call
    xo, io = oracle.cg_nd(U, b, KAPPA, MUBAR, EPSBAR, THETA, tol=1e-12)
    assert info.status == 0 and io["converged"]
    assert rel(x, xo) < 1e-8
    assert abs(info.iters - io["iters"]) <= 2


def test_nd_batch_maximum_size(tmq):
    """The largest doublet batch (32 doublets, i.e. 64 flavour fields): every
    doublet meets 1e-10 by the oracle, samples equal their solves alone bit for
    bit, and one more doublet is refused."""
    dims = (4, 4, 4, 4)
    lat, U = lattice(tmq, dims, 301)
    n = tmq.MAX_RHS // 2
    o = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    ps = [tmq.nd_params(KAPPA, 0.05 + 0.01 * (k % 8), 0.02 + 0.005 * (k % 4), THETA) for k in range(n)]
    bs = [dev(doublet(dims, 8300 + 2 * k)) for k in range(n)]
    xs, infos = lat.solve_nd_batch(ps, bs, o)
    for k in range(n):
        pk = ps[k]
        res = oracle.true_residual_nd(U, host(bs[k]), host(xs[k]), KAPPA, pk.mubar_tilde, pk.epsbar_tilde, THETA)
        assert infos[k].status == 0 and res <= 1e-10, (k, res)
    for k in (0, n - 1):
        x1, _ = lat.solve_nd(ps[k], bs[k], o)
        assert torch.equal(x1, xs[k]), k
    with pytest.raises(ValueError):
        lat.solve_nd_batch(ps + ps[:1], bs + bs[:1], o)


@pytest.mark.parametrize("variant", range(5))
def test_nd_batch16_block_orders(tmq, variant, monkeypatch):
    """Batched 16-bit doublet launches (both flavours in a lane) decode blocks
    and sites by multiply-high division and take the site terms of eq. (Dh)
    from a host-side table; on a lattice with XCD slabs of two sizes, a forced
    block order and a smaller last group, each doublet equals its solve alone
    bit for bit."""
    monkeypatch.setenv("TMQ_HOP_VARIANT", str(variant))
    monkeypatch.setenv("TMQ_HOP_GROUP", "4")
    dims = (10, 10, 4, 6)
    U = synth.random_gauge(dims, eps=0.3, seed=302)
    lat = tmq.Lattice(dims)  # a lattice of its own: the forced variant is read at creation
    lat.load_gauge(U)
    o = tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")
    ps = [tmq.nd_params(KAPPA, mb, eb, THETA) for mb, eb in ((0.1105, 0.0935), (0.05, 0.02), (0.2, 0.15))]
    bs = [dev(doublet(dims, 320 + 2 * k)) for k in range(3)]
    xs, infos = lat.solve_nd_batch(ps, bs, o)
    for k in range(3):
        x1, i1 = lat.solve_nd(ps[k], bs[k], o)
        assert torch.equal(x1, xs[k]), k
        assert (i1.iters, i1.reliable_updates) == (infos[k].iters, infos[k].reliable_updates)
        pk = ps[k]
        res = oracle.true_residual_nd(U, host(bs[k]), host(xs[k]), KAPPA, pk.mubar_tilde, pk.epsbar_tilde, THETA)
        assert infos[k].status == 0 and res <= 1e-10, (k, res)
    lat.close()


@pytest.mark.parametrize("sloppy", ["fp64", "fp32", "fp16"])
def test_nd_batch_equals_alone(tmq, sloppy):
    dims = (8, 8, 6, 10)
    lat, U = lattice(tmq, dims, 301)
    o = tmq.solver_opts(tol=1e-10, sloppy=sloppy, sloppy_link="fp16" if sloppy == "fp16" else "fp32")
    ps = [tmq.nd_params(KAPPA, mb, eb, THETA) for mb, eb in ((0.1105, 0.0935), (0.05, 0.02), (0.2, 0.15))]
    bs = [dev(doublet(dims, 310 + 2 * k)) for k in range(3)]
    xs, infos = lat.solve_nd_batch(ps, bs, o)
    for k in range(3):
        x1, i1 = lat.solve_nd(ps[k], bs[k], o)
        assert torch.equal(x1, xs[k]), k
        assert (i1.iters, i1.reliable_updates) == (infos[k].iters, infos[k].reliable_updates)
        pk = ps[k]
        res = oracle.true_residual_nd(U, host(bs[k]), host(xs[k]), KAPPA, pk.mubar_tilde, pk.epsbar_tilde, THETA)
        assert infos[k].status == 0 and res <= 1e-10, (k, res)
