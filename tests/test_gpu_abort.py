"""Stopping a queued run at a stage boundary and resuming it (the run
descriptor's abort_flag_host), through the C ABI.

A stage boundary of Table 1's stage loop (§2.4.1) is where the chains reduce,
restart from the winner and cool, so a checkpoint there is the winner's vector
and the stage index.  With the host flag set, every later stage's kernels
return at entry without writing; the run keeps its last completed stage, and
a new run started from the winner at the next stage index continues bit for
bit as the uninterrupted run -- both checked against the CPU oracle's
uninterrupted run.  The flag is only ever set from the host (a host store, or
a stream-ordered copy into the pinned flag); every kernel exits normally."""
import ctypes as C
import time

import numpy as np
import pytest

from oracle.oracle import OracleProblem
from paper_2506_19866_amd import synth
from tests.problems import random_problem

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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).cuda()


def _flag():
    return torch.zeros(1, dtype=torch.int32).pin_memory()


def _check_prefix(st, ref, done):
    assert np.array_equal(st["best_cost"][:done], ref["stage_best"][:done])
    assert np.array_equal(st["winner"][:done], ref["stage_winner"][:done])
    for k in ("accepted", "uphill", "neutral", "infeasible"):
        assert np.array_equal(st[k][:done], ref["stage_" + k][:done]), k
    # stages skipped by the abort report nothing
    assert np.all(st["best_cost"][done:] == -1) and np.all(st["winner"][done:] == -1)
    assert np.all(st["accepted"][done:] == 0)


def _resume_and_compare(P, prob, x_win, done, ref, *, n, S, L, seed, T0, rho, net=0, **kw):
    """A new run from the winner at stage `done` matches the oracle's
    uninterrupted run over the remaining stages."""
    sa = _sa()
    x0 = np.repeat(x_win[None, :], n, axis=0)
    run = sa.Run(P, _dev(x0), seed=seed, T0=T0, rho=rho, first_stage=done, n_stages=S - done,
                 steps_per_stage=L, **kw)
    st = run.stats(net)
    assert np.array_equal(st["best_cost"], ref["stage_best"][done:])
    assert np.array_equal(st["winner"], ref["stage_winner"][done:])
    for k in ("accepted", "uphill", "neutral", "infeasible"):
        assert np.array_equal(st[k], ref["stage_" + k][done:]), k
    x, cost, winner = run.best(net)
    assert cost == ref["cost"] and winner == ref["winner"] and np.array_equal(x, ref["x"])
    run.close()


def test_abort_between_graph_launches_then_resume():
    """Stages 0..2 in one captured graph, then a stream-ordered copy sets the
    flag, then the remaining stages in a second graph: every one of them
    returns at entry (or sa_run_launch already sees the flag and queues
    nothing).  The winner of stage 2 and a run resumed from it at stage 3 match
    the oracle's uninterrupted run bit for bit."""
    sa = _sa()
    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    n, S, L, k = 24, 8, 60, 3
    x0 = synth.start_vectors("c1", w, n)
    kw = dict(seed=s["seed"], T0=s["T0"], rho=s["rho"])
    o = OracleProblem(w)
    ref = o.run(x0, n_stages=S, steps_per_stage=L, n_threads=8, **kw)
    ref_k = o.run(x0, n_stages=k, steps_per_stage=L, n_threads=8, **kw)
    P = sa.Problem(w)
    flag = _flag()
    run = sa.Run(P, _dev(x0), n_stages=S, steps_per_stage=L, use_graph=True, abort_flag=flag, launch=False, **kw)
    run.launch(k)
    flag.copy_(torch.ones(1, dtype=torch.int32, device="cuda"), non_blocking=True)
    try:
        run.launch(S - k)
    except sa.SAError as e:          # the copy had already landed: nothing queued
        assert e.code == sa.SA_ERR_ABORTED
    torch.cuda.synchronize()
    assert run.stages_done() == k
    _check_prefix(run.stats(), ref, k)
    x, cost, winner = run.best()
    assert cost == ref["stage_best"][k - 1] and winner == ref["stage_winner"][k - 1]
    assert cost == ref_k["cost"] and np.array_equal(x, ref_k["x"])
    # while the flag is set nothing more is queued
    if run.launched < S:
        with pytest.raises(sa.SAError) as e:
            run.launch(1)
        assert e.value.code == sa.SA_ERR_ABORTED
    run.close()
    _resume_and_compare(P, w, x, k, ref, n=n, S=S, L=L, use_graph=True, **kw)


def test_abort_from_the_host_during_a_captured_run():
    """The flag is stored from the host while a 100-stage graph runs; whatever
    stage boundary it lands on, the completed stages are the oracle's, the run
    stops cleanly, and resuming from the winner reproduces the uninterrupted
    run."""
    sa = _sa()
    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    n, S, L = 32, 100, 1000
    x0 = synth.start_vectors("c1", w, n)
    kw = dict(seed=s["seed"] + 7, T0=s["T0"], rho=s["rho"])
    ref = OracleProblem(w).run(x0, n_stages=S, steps_per_stage=L, n_threads=8, **kw)
    P = sa.Problem(w)
    flag = _flag()
    run = sa.Run(P, _dev(x0), n_stages=S, steps_per_stage=L, use_graph=True, abort_flag=flag, **kw)
    time.sleep(0.02)
    flag[0] = 1
    done = run.stages_done()
    print(f"abort landed after {done} of {S} stages")
    assert 0 <= done <= S
    _check_prefix(run.stats(), ref, done)
    if done > 0:
        x, cost, winner = run.best()
        assert cost == ref["stage_best"][done - 1] and winner == ref["stage_winner"][done - 1]
    else:
        with pytest.raises(sa.SAError):
            run.best()
        x = None
    run.close()
    if 0 < done < S:
        _resume_and_compare(P, w, x, done, ref, n=n, S=S, L=L, use_graph=True, **kw)


def test_flag_set_before_the_first_stage():
    sa = _sa()
    w = synth.load_workload("c1")
    flag = _flag()
    flag[0] = 5
    run = sa.Run(sa.Problem(w), _dev(synth.start_vectors("c1", w, 8)), seed=1, T0=1.0, rho=0.9, n_stages=3,
                 steps_per_stage=20, abort_flag=flag, launch=False)
    with pytest.raises(sa.SAError) as e:
        run.launch(3)
    assert e.value.code == sa.SA_ERR_ABORTED
    assert run.stages_done() == 0
    with pytest.raises(sa.SAError) as e:
        run.best()
    assert e.value.code == sa.SA_ERR_ARG
    # cleared again, the run proceeds
    flag[0] = 0
    run.launch(3)
    assert run.stages_done() == 3
    run.close()


def test_unpinned_flag_is_rejected():
    """The library itself refuses a flag that is not pinned host memory (the
    binding refuses it earlier, so this goes through ctypes directly)."""
    sa = _sa()
    w = synth.load_workload("c1")
    P = sa.Problem(w)
    x0 = _dev(synth.start_vectors("c1", w, 4))
    plain = np.zeros(1, dtype=np.int32)
    d = sa._RunDesc(4, 1, 1.0, 0.9, 0, 2, 10, 0, 0, 0, 0, 0, 16, None, 0.1, None, 0, 1, 0,
                    plain.ctypes.data)
    probs = (C.c_void_p * 1)(P.handle)
    h = C.c_void_p()
    rc = sa.lib().sa_run_create(probs, 1, C.byref(d), C.c_void_p(x0.data_ptr()), C.byref(h),
                                sa._stream_handle())
    assert rc == sa.SA_ERR_ARG and not h.value
    with pytest.raises(TypeError):
        sa.Run(P, x0, seed=1, T0=1.0, rho=0.9, n_stages=2, steps_per_stage=10,
               abort_flag=torch.zeros(1, dtype=torch.int32))


def test_abort_of_the_many_network_kernel():
    """Two networks in the persistent kernel: abort after 2 of 5 stages (eager
    launches), then resume each network from its own winner."""
    sa = _sa()
    probs = [random_problem(200 + i, n_nodes=N, n_edges=E, n_cond=C, n_steps=8, n_times=3, n_obs=5,
                            noise=0.1, clamps=(1, 1))[0] for i, (N, E, C) in enumerate([(14, 30, 3), (40, 120, 6)])]
    n, S, L, k = 12, 5, 50, 2
    xs = [synth.feasible_params(np.random.default_rng(300 + i), n, p["row_ptr"], p["src"])
          for i, p in enumerate(probs)]
    kw = dict(seed=41, T0=1.5, rho=0.8)
    refs = [OracleProblem(p).run(x, n_stages=S, steps_per_stage=L, net=i, n_threads=8, **kw)
            for i, (p, x) in enumerate(zip(probs, xs))]
    Ps = [sa.Problem(p) for p in probs]
    flag = _flag()
    run = sa.Run(Ps, [_dev(x) for x in xs], n_stages=S, steps_per_stage=L, kernel=sa.SA_KERNEL_PERSISTENT,
                 chains_per_block=2, abort_flag=flag, launch=False, **kw)
    run.launch(k)
    flag.copy_(torch.ones(1, dtype=torch.int32, device="cuda"), non_blocking=True)
    try:
        run.launch(S - k)
    except sa.SAError as e:
        assert e.code == sa.SA_ERR_ABORTED
    assert run.stages_done() == k
    wins = []
    for i, ref in enumerate(refs):
        _check_prefix(run.stats(i), ref, k)
        x, cost, winner = run.best(i)
        assert cost == ref["stage_best"][k - 1] and winner == ref["stage_winner"][k - 1]
        wins.append(x)
    run.close()
    x0 = [_dev(np.repeat(x[None, :], n, axis=0)) for x in wins]
    run = sa.Run(Ps, x0, first_stage=k, n_stages=S - k, steps_per_stage=L, kernel=sa.SA_KERNEL_PERSISTENT,
                 chains_per_block=2, **kw)
    for i, ref in enumerate(refs):
        st = run.stats(i)
        assert np.array_equal(st["best_cost"], ref["stage_best"][k:])
        assert np.array_equal(st["accepted"], ref["stage_accepted"][k:])
        x, cost, winner = run.best(i)
        assert cost == ref["cost"] and winner == ref["winner"] and np.array_equal(x, ref["x"])
    run.close()


def test_abort_of_the_priority_and_traced_kernels():
    """The priority model's stage kernel and the traced (learned-stage) kernel
    stop the same way."""
    sa = _sa()
    wq = synth.load_workload("q1")
    sq = synth.bench_schedule("q1")
    n, S, L, k = 13, 4, 40, 1
    xq = synth.start_vectors("q1", wq, n)
    kw = dict(seed=sq["seed"], T0=sq["T0"], rho=sq["rho"])
    ref = OracleProblem(wq).run(xq, n_stages=S, steps_per_stage=L, n_threads=8, **kw)
    P = sa.Problem(wq)
    flag = _flag()
    run = sa.Run(P, _dev(xq), n_stages=S, steps_per_stage=L, abort_flag=flag, launch=False, **kw)
    run.launch(k)
    flag.copy_(torch.ones(1, dtype=torch.int32, device="cuda"), non_blocking=True)
    try:
        run.launch(S - k)
    except sa.SAError as e:
        assert e.code == sa.SA_ERR_ABORTED
    assert run.stages_done() == k
    _check_prefix(run.stats(), ref, k)
    x, _, _ = run.best()
    run.close()
    _resume_and_compare(P, wq, x, k, ref, n=n, S=S, L=L, **kw)

    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    n, S, L, k = 16, 5, 50, 3
    x0 = synth.start_vectors("c1", w, n)
    kw = dict(seed=s["seed"] + 1, T0=s["T0"], rho=s["rho"])
    ref = OracleProblem(w).run(x0, n_stages=S, steps_per_stage=L, n_threads=8, **kw)
    P = sa.Problem(w)
    trace = torch.zeros((n, S * L * sa.TRACE_RECORD_BYTES), dtype=torch.uint8, device="cuda")
    flag = _flag()
    run = sa.Run(P, _dev(x0), n_stages=S, steps_per_stage=L, trace=trace, trace_every=1, refresh_every=8,
                 abort_flag=flag, launch=False, **kw)
    run.launch(k)
    flag.copy_(torch.ones(1, dtype=torch.int32, device="cuda"), non_blocking=True)
    try:
        run.launch(S - k)
    except sa.SAError as e:
        assert e.code == sa.SA_ERR_ABORTED
    assert run.stages_done() == k
    _check_prefix(run.stats(), ref, k)
    # the skipped stages wrote no trace records
    rec = trace.cpu().numpy().reshape(n, S * L, sa.TRACE_RECORD_BYTES)
    assert np.any(rec[:, :k * L] != 0) and not np.any(rec[:, k * L:] != 0)
    x, _, _ = run.best()
    run.close()
    _resume_and_compare(P, w, x, k, ref, n=n, S=S, L=L, **kw)
