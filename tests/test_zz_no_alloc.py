"""The allocation-free run (sa_run_chains_noalloc) against the allocating one
(sa_run_chains) on the same inputs, through the C ABI: best vector, cost,
winner and every stage's statistics bit for bit.  Two calls in a row, the
second one smaller, so the second reads none of the first's leftovers."""
import numpy as np
import pytest

from paper_2506_19866_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_19866_amd import sa
    sa.lib()


def _sa():
    from paper_2506_19866_amd import sa
    return sa


def _reference(P, x0, **kw):
    sa = _sa()
    run = sa.Run(P, x0, **kw)
    x, cost, winner = run.best()
    st = run.stats()
    run.close()
    return x, cost, winner, st


def _noalloc(P, x0, **kw):
    sa = _sa()
    xb = torch.full((P.n_params,), 99, dtype=torch.int8, device="cuda")
    best = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    stats = torch.zeros((kw["n_stages"] * 48,), dtype=torch.uint8, device="cuda")
    sa.run_chains_noalloc(P, x0, xb, best, stats, **kw)
    torch.cuda.synchronize()
    b = best.cpu().numpy()
    return xb.cpu().numpy(), int(b[0]), int(b[1]), sa.decode_stage_stats(stats.cpu().numpy())


def _same(got, ref):
    x, cost, winner, st = got
    rx, rcost, rwinner, rst = ref
    assert cost == rcost and winner == rwinner, (cost, winner, rcost, rwinner)
    assert np.array_equal(x, rx)
    for k in rst:
        assert np.array_equal(st[k], rst[k]), k


def test_noalloc_matches_the_allocating_run_twice():
    sa = _sa()
    cases = [("c3", 16384, dict(n_stages=2, steps_per_stage=120, first_stage=3)),
             ("c1", 40, dict(n_stages=6, steps_per_stage=90))]
    for name, n, extra in cases:
        w = synth.load_workload(name)
        s = synth.bench_schedule(name)
        P = sa.Problem(w)
        x0 = torch.from_numpy(synth.start_vectors(name, w, n)).cuda()
        kw = dict(seed=s["seed"], T0=s["T0"], rho=s["rho"], **extra)
        ref = _reference(P, x0, **kw)
        got = _noalloc(P, x0, **kw)
        print(f"{name}: {n} chains, cost {got[1]} (chain {got[2]})")
        _same(got, ref)


def test_noalloc_priority_model_and_limits():
    sa = _sa()
    w = synth.load_workload("q1")
    s = synth.bench_schedule("q1")
    P = sa.Problem(w)
    x0 = torch.from_numpy(synth.start_vectors("q1", w, 29)).cuda()
    kw = dict(seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=4, steps_per_stage=50)
    _same(_noalloc(P, x0, **kw), _reference(P, x0, **kw))
    # a run beyond the fixed array is refused before any device work
    w3 = synth.load_workload("c3")
    P3 = sa.Problem(w3)
    big = torch.zeros((24000, P3.n_params), dtype=torch.int8, device="cuda")
    xb = torch.zeros((P3.n_params,), dtype=torch.int8, device="cuda")
    best = torch.zeros((2,), dtype=torch.int32, device="cuda")
    with pytest.raises(sa.SAError) as e:
        sa.run_chains_noalloc(P3, big, xb, best, None, seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=10)
    assert e.value.code == sa.SA_ERR_UNSUPPORTED
    # unsupported options are refused too (island restart)
    import ctypes as C
    d = sa._RunDesc(29, 1, 1.0, 0.9, 0, 2, 10, 0, 0, 0, 0, 0, 16, None, 0.1, None, 0, 1, 4, None)
    rc = sa.lib().sa_run_chains_noalloc(P.handle, C.byref(d), C.c_void_p(x0.data_ptr()), C.c_void_p(xb.data_ptr()),
                                        C.c_void_p(best.data_ptr()), None, sa._stream_handle())
    assert rc == sa.SA_ERR_UNSUPPORTED
