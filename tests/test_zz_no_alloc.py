"""GPU test of the allocation-free operator entry point (tmq_apply_Qhat_noalloc_dev)
against the allocating one (tmq_apply_Qhat_dev), through the C ABI: the same
result bit for bit (same kernels), on two calls in a row that share the fixed
device work space, the second with a smaller lattice; sizes above the fixed
work space are refused with TMQ_EINVAL."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THETA = np.array([1.0, 0.3, -0.7, 0.45])


@pytest.fixture(scope="module")
def tmq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0905_3331_amd import tmq as t

    return t


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_noalloc_equals_allocating_entry_point(tmq, prec):
    # the larger lattice first, then a smaller one in the same work space
    cases = [((16, 8, 8, 10), 801), ((6, 4, 2, 10), 802)]
    p = tmq.params(0.1632, 0.004, THETA)
    for dims, seed in cases:
        U = synth.random_gauge(dims, seed=seed)
        with tmq.Lattice(dims) as lat:
            lat.load_gauge(U)
            psi = dev(synth.gaussian_odd(dims, seed=seed + 10))
            for sign in (+1, -1):
                print(f"noalloc {prec} {dims} sign {sign:+d}", flush=True)
                out_na = torch.full_like(psi, float("nan"))
                lat.apply_Qhat_noalloc(p, sign, psi, out_na, prec=prec)
                ref = lat.apply_Qhat(p, sign, psi, prec=prec)
                assert torch.equal(out_na, ref), (prec, dims, sign)
                if prec == "fp64":
                    want = oracle.Qhat(U, psi.cpu().numpy(), 0.1632, 0.004, sign, THETA)
                    got = out_na.cpu().numpy()
                    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_noalloc_before_any_tuning_and_refusal(tmq):
    """A fresh lattice (nothing tuned yet) gives the allocating entry point's result,
    and a lattice whose work fields exceed the fixed array is refused."""
    dims = (8, 8, 6, 10)
    U = synth.random_gauge(dims, seed=803)
    p = tmq.params(0.15, -0.02, THETA)
    psi = dev(synth.gaussian_odd(dims, seed=804))
    with tmq.Lattice(dims) as lat:
        lat.load_gauge(U)
        out_na = torch.empty_like(psi)
        lat.apply_Qhat_noalloc(p, +1, psi, out_na, prec="fp16")
        assert lat.tuning_report()["hop"] == []  # it did not tune
        assert torch.equal(out_na, lat.apply_Qhat(p, +1, psi, prec="fp16"))
    big = (64, 16, 16, 16)  # FP64: 3 x 131072 x 192 B = 75.5 MB > 64 MiB; FP16 fits
    Ub = synth.random_gauge(big, seed=805)
    with tmq.Lattice(big) as lat:
        lat.load_gauge(Ub)
        psi = dev(synth.gaussian_odd(big, seed=806))
        out_na = torch.empty_like(psi)
        with pytest.raises(tmq.TmqError) as e:
            lat.apply_Qhat_noalloc(p, +1, psi, out_na, prec="fp64")
        assert e.value.code == tmq.TMQ_EINVAL and "work space" in str(e.value)
        lat.apply_Qhat_noalloc(p, +1, psi, out_na, prec="fp16")
        assert torch.equal(out_na, lat.apply_Qhat(p, +1, psi, prec="fp16"))
