"""GPU tests of the solve server (tmq_server_*): served solutions meet their
tolerance by the oracle's FP64 true residual, a request's result is the same
bit for bit whether it runs alone or joins a mix of other requests at any
iteration, and admission keeps the engines' device memory within the budget
(back-pressure with a small artificial budget, rejection of a request that can
never fit)."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THETA = np.array([1.0, 0.0, 0.0, 0.0])
KAPPA = 0.1632


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


_GAUGE = {}


def gauge(dims, seed):
    if (dims, seed) not in _GAUGE:
        _GAUGE[(dims, seed)] = synth.random_gauge(dims, eps=0.3, seed=seed)
    return _GAUGE[(dims, seed)]


def slot_bytes(tmq, dims, opts):
    return tmq.footprint_bytes(dims, opts, 2) - tmq.footprint_bytes(dims, opts, 1)


def test_serve_mixed_sizes_against_oracle(tmq):
    """Requests over three lattice sizes and three inner precisions, submitted
    together: each meets its tolerance by the oracle's FP64 true residual."""
    sizes = [(4, 4, 4, 4), (8, 4, 4, 6), (8, 8, 6, 10)]
    rng = np.random.default_rng(3000)
    with tmq.Server(max_batch=8) as srv:
        ids = [srv.add_lattice(d, dev(gauge(d, 3100 + j))) for j, d in enumerate(sizes)]
        reqs = []
        for i in range(18):
            j = int(rng.integers(0, len(sizes)))
            d = sizes[j]
            mut = float(rng.uniform(0.002, 0.02))
            sloppy = ("fp32", "fp16", "fp64")[i % 3]
            tol = 1e-8 if i % 2 else 1e-10
            b = synth.gaussian_odd(d, seed=4000 + i)
            o = tmq.solver_opts(tol=tol, sloppy=sloppy, sloppy_link="fp16" if sloppy == "fp16" else "fp32")
            t = srv.submit(ids[j], tmq.params(KAPPA, mut, THETA), dev(b), o)
            reqs.append((t, j, b, mut, tol))
        for t, j, b, mut, tol in reqs:
            x, info = srv.wait(t, timeout=60)
            res = oracle.true_residual(gauge(sizes[j], 3100 + j), b, host(x), KAPPA, mut, THETA)
            print(f"request {t} size {sizes[j]} iters {info.iters} ru {info.reliable_updates} "
                  f"res {res:.2e} (gpu {info.true_rel_residual:.2e}) latency {info.seconds * 1e3:.1f} ms")
            assert info.status == tmq.TMQ_OK, info
            assert res <= tol
            assert abs(res - info.true_rel_residual) <= 1e-3 * res + 1e-15
        st = srv.stats()
        assert st["completed"] == 18 and st["failed"] == 0 and st["running"] == 0 and st["queued"] == 0
        assert 0 < st["p50_s"] <= st["p99_s"]
        with pytest.raises(tmq.TmqError):  # retired ticket
            srv.poll(reqs[0][0])


@pytest.mark.parametrize("sloppy", ["fp32", "fp16", "fp64"])
def test_serve_alone_equals_in_mix(tmq, sloppy):
    """A request's solution and iteration counts are identical whether it runs
    alone or joins, at some later iteration, a batch of other requests that
    join and leave around it."""
    dims = (8, 8, 6, 10)
    U = gauge(dims, 3101)
    o = tmq.solver_opts(tol=1e-10, sloppy=sloppy, sloppy_link="fp16" if sloppy == "fp16" else "fp32")
    b = synth.gaussian_odd(dims, seed=5000)
    p = tmq.params(KAPPA, 0.0071, THETA)
    with tmq.Server(max_batch=8) as srv:
        lid = srv.add_lattice(dims, dev(U))
        x_alone, i_alone = srv.wait(srv.submit(lid, p, dev(b), o), timeout=60)
        assert i_alone.status == 0
        others = []
        for k in range(3):
            bo = synth.gaussian_odd(dims, seed=5001 + k)
            others.append(srv.submit(lid, tmq.params(KAPPA, 0.002 + 0.006 * k, THETA), dev(bo), o))
        # let the others iterate for a while before the request joins
        s0 = srv.stats()["steps"]
        t_end = time.time() + 10
        while srv.stats()["steps"] < s0 + 5 and time.time() < t_end:
            time.sleep(1e-4)
        t = srv.submit(lid, p, dev(b), o)
        for k in range(3):
            bo = synth.gaussian_odd(dims, seed=5011 + k)
            others.append(srv.submit(lid, tmq.params(KAPPA, 0.02 - 0.005 * k, THETA), dev(bo), o))
        x_mix, i_mix = srv.wait(t, timeout=60)
        for q in others:
            _, io = srv.wait(q, timeout=60)
            assert io.status == 0
        assert srv.stats()["peak_running"] >= 2
    assert torch.equal(x_alone, x_mix)
    assert (i_alone.iters, i_alone.reliable_updates) == (i_mix.iters, i_mix.reliable_updates)
    assert i_alone.true_rel_residual == i_mix.true_rel_residual
    assert oracle.true_residual(U, b, host(x_mix), KAPPA, 0.0071, THETA) <= 1e-10


def test_serve_admission_back_pressure(tmq):
    """With a budget of 2.5 slots of the small lattice, at most two of its
    requests are admitted at once; a larger lattice's request waits until the
    small engine has drained and been released; a request whose one slot
    exceeds the budget is rejected at submission."""
    small, large, huge = (8, 8, 8, 8), (16, 8, 8, 8), (16, 16, 8, 8)
    o = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    budget = int(2.5 * slot_bytes(tmq, small, o))
    assert slot_bytes(tmq, large, o) < budget < slot_bytes(tmq, huge, o)
    assert 2 * slot_bytes(tmq, small, o) + slot_bytes(tmq, large, o) > budget
    with tmq.Server(budget_bytes=budget, max_batch=16) as srv:
        ls = srv.add_lattice(small, dev(gauge(small, 3102)))
        ll = srv.add_lattice(large, dev(gauge(large, 3103)))
        lh = srv.add_lattice(huge, dev(gauge(huge, 3104)))
        with pytest.raises(tmq.TmqError) as e:
            srv.submit(lh, tmq.params(KAPPA, 0.01, THETA), dev(synth.gaussian_odd(huge, seed=1)), o)
        assert e.value.code == tmq.TMQ_ENOMEM
        reqs = []
        for i in range(7):
            d, lid = (large, ll) if i == 3 else (small, ls)
            b = synth.gaussian_odd(d, seed=6000 + i)
            mut = 0.003 + 0.002 * i
            reqs.append((srv.submit(lid, tmq.params(KAPPA, mut, THETA), dev(b), o), d, b, mut, lid))
        for t, d, b, mut, lid in reqs:
            x, info = srv.wait(t, timeout=60)
            assert info.status == 0
            U = gauge(d, 3102 if lid == ls else 3103)
            assert oracle.true_residual(U, b, host(x), KAPPA, mut, THETA) <= 1e-10
        st = srv.stats()
        print(st)
        assert st["rejected"] == 1 and st["completed"] == 7
        assert st["peak_running"] <= 2
        assert st["peak_bytes"] <= budget


def test_serve_edge_requests(tmq):
    """A zero source finishes at once with x = 0, a NaN source reports
    TMQ_ENAN, max_iter = 3 reports TMQ_ENOCONV with the true residual, and a
    good request in the same batch is unaffected."""
    dims = (4, 4, 4, 4)
    U = gauge(dims, 3105)
    o = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    o3 = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32", max_iter=3)
    good = synth.gaussian_odd(dims, seed=7000)
    bnan = synth.gaussian_odd(dims, seed=7001)
    bnan[3, 1, 2] = np.nan
    p = tmq.params(KAPPA, 0.01, THETA)
    with tmq.Server(max_batch=8) as srv:
        lid = srv.add_lattice(dims, dev(U))
        tz = srv.submit(lid, p, dev(np.zeros_like(good)), o)
        tn = srv.submit(lid, p, dev(bnan), o)
        t3 = srv.submit(lid, p, dev(good), o3)
        tg = srv.submit(lid, p, dev(good), o)
        xz, iz = srv.wait(tz, timeout=60)
        _, i_n = srv.wait(tn, timeout=60)
        x3, i3 = srv.wait(t3, timeout=60)
        xg, ig = srv.wait(tg, timeout=60)
        st = srv.stats()
    assert iz.status == 0 and iz.iters == 0 and not torch.any(xz != 0)
    assert i_n.status == tmq.TMQ_ENAN
    assert i3.status == tmq.TMQ_ENOCONV and i3.iters == 3
    res3 = oracle.true_residual(U, good, host(x3), KAPPA, 0.01, THETA)
    assert abs(res3 - i3.true_rel_residual) <= 1e-6 * res3
    assert ig.status == 0
    assert oracle.true_residual(U, good, host(xg), KAPPA, 0.01, THETA) <= 1e-10
    assert st["failed"] == 2


def test_serve_threads_poll_and_destroy(tmq):
    """Requests submitted from several host threads at once all finish and
    converge; poll reports a pending request as pending; destroying the server
    with requests in flight waits for them and returns."""
    import threading

    dims = (8, 4, 4, 6)
    U = gauge(dims, 3106)
    o = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link="fp32")
    srv = tmq.Server(max_batch=4)
    lid = srv.add_lattice(dims, dev(U))
    bs = [synth.gaussian_odd(dims, seed=8000 + i) for i in range(12)]
    bd = [dev(b) for b in bs]
    torch.cuda.synchronize()
    tickets = [None] * 12

    def worker(k):
        for i in range(k, 12, 3):
            tickets[i] = srv.submit(lid, tmq.params(KAPPA, 0.002 + 0.001 * i, THETA), bd[i], o, sync=False)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    first = srv.poll(tickets[11])  # most likely still queued or running
    assert first is None or first[1].status == 0
    for i, t in enumerate(tickets):
        if i == 11 and first is not None:
            x, info = first
        else:
            x, info = srv.wait(t, timeout=60)
        assert info.status == 0
        res = oracle.true_residual(U, bs[i], host(x), KAPPA, 0.002 + 0.001 * i, THETA)
        assert res <= 1e-10, (i, res)
    st = srv.stats()
    assert st["completed"] == 12 and st["peak_running"] <= 4
    # in flight at destruction: destroy waits for them
    for i in range(4):
        srv.submit(lid, tmq.params(KAPPA, 0.01, THETA), bd[i], o)
    srv.close()



def test_serve_same_spinor_precision_different_link_formats(tmq):
    """Requests with the same inner spinor precision but different inner link
    formats (FP32 spinors with FP16 links, and with FP32 links) need engines of
    their own: both kinds complete, each meets its tolerance, and the server
    holds one engine per link format."""
    d = (8, 4, 4, 6)
    U = gauge(d, 3150)
    with tmq.Server(max_batch=4) as srv:
        lid = srv.add_lattice(d, dev(U))
        reqs = []
        for i in range(6):
            link = "fp16" if i % 2 == 0 else "fp32"
            o = tmq.solver_opts(tol=1e-10, sloppy="fp32", sloppy_link=link)
            b = synth.gaussian_odd(d, seed=4150 + i)
            mut = 0.004 + 0.002 * i
            t = srv.submit(lid, tmq.params(KAPPA, mut, THETA), dev(b), o)
            reqs.append((t, b, mut, link))
        for t, b, mut, link in reqs:
            x, info = srv.wait(t, timeout=60)
            assert info.status == tmq.TMQ_OK, (link, info)
            assert oracle.true_residual(U, b, host(x), KAPPA, mut, THETA) <= 1e-10
        st = srv.stats()
        assert st["completed"] == 6 and st["failed"] == 0
        assert st["engines"] == 2
