"""GPU checks at the full sizes of the benchmark workloads, in the launch
configuration the benchmarks time: the 32^3x64 headline (FP64 and FP16 Qhat^+
over the whole lattice, the mixed FP16 solve), 24^3x48 FP64 and FP32-inner
even/odd CG (kappa 0.1632, 2 kappa mu 0.004), BiCGstab and the doublet at
24^3x48, and the 48-RHS batch on 24^3x48 (12 point sources x 4 twisted masses).  Solutions are judged by the oracle's FP64 true
residual (the oracle applies Qhat^+Qhat^- once per check), and batched
solutions against their solves alone, bit for bit."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THETA = (1.0, 0.0, 0.0, 0.0)
DIMS = (48, 24, 24, 24)


@pytest.fixture(scope="module")
def tmq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0905_3331_amd import tmq as t

    return t


def test_eo_24c48_fp64_and_mixed(tmq):
    U = synth.random_gauge(DIMS, eps=0.3, seed=1001)
    lat = tmq.Lattice(DIMS)
    lat.load_gauge(U)
    b = synth.gaussian_odd(DIMS, seed=2100)
    p = tmq.params(0.1632, 0.004, THETA)
    for opts in (tmq.solver_opts(tol=1e-10), tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32"),
                 tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16")):
        x, info = lat.solve(p, torch.from_numpy(b).cuda(), opts)
        res = oracle.true_residual(U, b, x.cpu().numpy(), 0.1632, 0.004, THETA)
        print(f"24^3x48 sloppy={opts.sloppy}: iters {info.iters} reliable {info.reliable_updates} "
              f"true res {res:.2e} (gpu {info.true_rel_residual:.2e})")
        assert info.status == 0 and res <= 1e-10
        assert abs(res - info.true_rel_residual) <= 1e-3 * res
    lat.close()


def test_batch_24c48_48rhs(tmq):
    U = synth.random_gauge(DIMS, eps=0.3, seed=1003)
    lat = tmq.Lattice(DIMS)
    lat.load_gauge(U)
    vh = int(np.prod(DIMS)) // 2
    site = int(np.random.default_rng(2300).integers(0, vh))
    ps, bs = [], []
    for mut in (0.002, 0.004, 0.008, 0.016):
        for k in range(12):
            bs.append(synth.point_source_odd(DIMS, site, k // 3, k % 3))
            ps.append(tmq.params(0.1632, mut, THETA))
    opts = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    bd = [torch.from_numpy(b).cuda() for b in bs]
    xs, infos = lat.solve_batch(ps, bd, opts)
    assert all(f.status == 0 for f in infos)
    for i in (0, 17, 47):
        x1, i1 = lat.solve(ps[i], bd[i], opts)
        assert torch.equal(x1, xs[i]), i
        assert (i1.iters, i1.reliable_updates) == (infos[i].iters, infos[i].reliable_updates)
    for i in (0, 13, 26, 39, 47):
        res = oracle.true_residual(U, bs[i], xs[i].cpu().numpy(), 0.1632, ps[i].mu_tilde, THETA)
        assert res <= 1e-10, (i, res)
    lat.close()


def test_doublet_24c48_mixed(tmq):
    """The flavour doublet (eq. (Dh), the paper's doublet run parameters) at
    24^3x48, FP16-inner CG, judged by the oracle's FP64 true residual."""
    U = synth.random_gauge(DIMS, eps=0.3, seed=1001)
    lat = tmq.Lattice(DIMS)
    lat.load_gauge(U)
    b = np.stack([synth.gaussian_odd(DIMS, seed=2500), synth.gaussian_odd(DIMS, seed=2501)])
    p = tmq.nd_params(0.17, 0.1105, 0.0935, THETA)
    x, info = lat.solve_nd(p, torch.from_numpy(b).cuda(), tmq.solver_opts(tol=1e-10, sloppy="fp16",
                                                                           sloppy_link="fp16"))
    res = oracle.true_residual_nd(U, b, x.cpu().numpy(), 0.17, 0.1105, 0.0935, THETA)
    print(f"doublet 24^3x48 fp16 inner: iters {info.iters} reliable {info.reliable_updates} true res {res:.2e}")
    assert info.status == 0 and res <= 1e-10
    assert abs(res - info.true_rel_residual) <= 1e-3 * res
    lat.close()


def test_headline_32c64_operator_and_mixed_solve(tmq):
    """The 32^3x64 workload of the benchmark, in its launch configuration
    (autotuned FP16 half-sweeps): the FP16 Qhat^+ against the oracle on the
    whole lattice (bounded by the FP16 storage), the FP64 Qhat^+ to 1e-13, and
    the mixed FP16 solve to 1e-10 by the oracle's FP64 true residual."""
    dims = (64, 32, 32, 32)
    U = synth.random_gauge(dims, eps=0.3, seed=1002)
    lat = tmq.Lattice(dims)
    lat.load_gauge(U)
    b = synth.gaussian_odd(dims, seed=2200)
    p = tmq.params(0.1632, 0.004, THETA)
    want = oracle.Qhat(U, b, 0.1632, 0.004, +1, THETA)
    bd = torch.from_numpy(b).cuda()
    for prec, bound in (("fp64", 1e-13), ("fp16", 3e-3)):
        got = lat.apply_Qhat(p, +1, bd, prec=prec).cpu().numpy()
        err = float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(want.ravel()))
        print(f"32^3x64 Qhat^+ {prec}: relative error {err:.2e}")
        assert err < bound
    x, info = lat.solve(p, bd, tmq.solver_opts(tol=1e-10, sloppy="fp16", sloppy_link="fp16"))
    res = oracle.true_residual(U, b, x.cpu().numpy(), 0.1632, 0.004, THETA)
    print(f"32^3x64 mixed fp16: iters {info.iters} reliable {info.reliable_updates} true res {res:.2e}")
    assert info.status == 0 and res <= 1e-10
    assert abs(res - info.true_rel_residual) <= 1e-3 * res
    lat.close()


def test_bicgstab_24c48(tmq):
    """BiCGstab on Qhat^+ at 24^3x48: the oracle's Qhat of the solution gives b back to 1e-10."""
    U = synth.random_gauge(DIMS, eps=0.3, seed=1001)
    lat = tmq.Lattice(DIMS)
    lat.load_gauge(U)
    b = synth.gaussian_odd(DIMS, seed=2601)
    p = tmq.params(0.1632, 0.004, THETA)
    x, info = lat.solve_Qhat(p, +1, torch.from_numpy(b).cuda(), tmq.solver_opts(tol=1e-10))
    r = b - oracle.Qhat(U, x.cpu().numpy(), 0.1632, 0.004, +1, THETA)
    res = float(np.linalg.norm(r.ravel()) / np.linalg.norm(b.ravel()))
    print(f"24^3x48 BiCGstab: iters {info.iters} true res {res:.2e}")
    assert info.status == 0 and res <= 1e-10
    lat.close()
