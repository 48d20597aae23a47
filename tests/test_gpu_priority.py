"""GPU parity of the priority-update model (paper §2.1 image with weight,
polarity and threshold; §2.2 priority update; §2.5.3; Table 1) against the
CPU oracle, bit for bit: costs, trajectories, per-stage statistics, winners
and best vectors.  Covers the three lane-segment widths (16, 32 and 64 lanes
per chain), ragged chain counts, several conditions, clamps, penalty mode,
island restart and resume."""
import numpy as np
import pytest

from oracle.oracle import OracleProblem
from paper_2506_19866_amd import synth
from tests.problems import priority_problem

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


# (N, E, C, T, O, clamps): segment widths 16 (N <= 16) and 32, which gather
# regulator states by ballots, and 64, with 8 regulator slots, 16 slots
# (largest in-degree 9-16) or the ballot masks (largest in-degree above 16)
SHAPES = [
    (5, 9, 1, 6, 3, (0, 0)),
    (16, 40, 3, 12, 8, (1, 1)),
    (12, 100, 2, 8, 6, (1, 1)),
    (17, 50, 2, 9, 6, (1, 2)),
    (32, 90, 5, 15, 20, (1, 1)),
    (28, 300, 2, 10, 10, (1, 1)),
    (30, 560, 1, 7, 12, (0, 0)),
    (33, 100, 1, 19, 20, (0, 0)),
    (64, 200, 4, 11, 30, (1, 3)),
    (45, 420, 2, 9, 20, (1, 2)),
    (48, 600, 1, 8, 20, (1, 1)),
]


def _variant(prob):
    """(lanes per chain, regulator slots) the library picks for a network."""
    N, max_in = prob["n_nodes"], int(np.diff(prob["row_ptr"]).max())
    lc = 16 if N <= 16 else 32 if N <= 32 else 64
    return (lc, 0 if lc <= 32 else 8 if max_in <= 8 else 16 if max_in <= 16 else 0)


def test_shapes_cover_every_kernel_variant():
    got = {_variant(priority_problem(300 + N, n_nodes=N, n_edges=E, n_cond=1, n_steps=2, n_obs=2)[0])
           for N, E, *_ in SHAPES}
    assert got == {(16, 0), (32, 0), (64, 8), (64, 16), (64, 0)}


def _vectors(prob, n, seed):
    rng = synth.rng_for(seed)
    xs = synth.priority_random_params(rng, n, prob["n_edges"], prob["n_nodes"])
    feas = synth.priority_feasible_params(rng, n, prob["row_ptr"], prob["src"])
    return np.concatenate([xs, feas])


@pytest.mark.parametrize("N,E,C,T,O,clamps", SHAPES)
@pytest.mark.parametrize("hard", [1, 0])
def test_costs_match_oracle(N, E, C, T, O, clamps, hard):
    prob, hidden = priority_problem(300 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=T, n_obs=O,
                                    noise=0.1, clamps=clamps, hard=hard)
    xs = np.concatenate([_vectors(prob, 37, N), hidden[None, :]])  # 75 vectors: ragged in every width
    o = OracleProblem(prob)
    want = o.cost_batch(xs)
    P = _sa().Problem(prob)
    assert P.n_params == 3 * (N + E)
    got = P.eval_cost(_dev(xs)).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N,E,C,T,O,clamps", SHAPES)
def test_trajectories_match_oracle(N, E, C, T, O, clamps):
    prob, _ = priority_problem(300 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=T, n_obs=O, clamps=clamps)
    xs = _vectors(prob, 11, 7 + N)
    o = OracleProblem(prob)
    got = _sa().Problem(prob).simulate(_dev(xs)).cpu().numpy()
    for i, x in enumerate(xs):
        assert np.array_equal(got[i], o.simulate(x)), i


def test_sparse_observations_and_time_zero():
    prob, _ = priority_problem(501, n_nodes=20, n_edges=60, n_cond=2, n_steps=14, n_obs=7, obs_t=[0, 5, 9, 14],
                               noise=0.2, clamps=(1, 1))
    xs = _vectors(prob, 20, 3)
    assert np.array_equal(_sa().Problem(prob).eval_cost(_dev(xs)).cpu().numpy().astype(np.int64),
                          OracleProblem(prob).cost_batch(xs))


@pytest.mark.parametrize("name", ["q1", "q2", "q3"])
def test_workload_costs(name):
    w = synth.load_workload(name)
    xs = np.concatenate([synth.start_vectors(name, w, 50), w["hidden"][None, :],
                         synth.priority_random_params(synth.rng_for(9), 30, w["n_edges"], w["n_nodes"])])
    got = _sa().Problem(w).eval_cost(_dev(xs)).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, OracleProblem(w).cost_batch(xs))


def _compare_runs(prob, x0, seed, *, T0, rho, n_stages, L, first_stage=0, group_size=0, **kw):
    o = OracleProblem(prob)
    ref = o.run(x0, seed=seed, T0=T0, rho=rho, n_stages=n_stages, steps_per_stage=L, first_stage=first_stage,
                n_threads=8, group_size=group_size)
    sa = _sa()
    run = sa.Run(sa.Problem(prob), _dev(x0), seed=seed, T0=T0, rho=rho, n_stages=n_stages, steps_per_stage=L,
                 first_stage=first_stage, group_size=group_size, **kw)
    st = run.stats()
    x, cost, winner = run.best()
    cb, cx = run.chain_best()
    assert np.array_equal(st["best_cost"], ref["stage_best"])
    assert np.array_equal(st["winner"], ref["stage_winner"])
    for k in ("accepted", "uphill", "neutral", "infeasible"):
        assert np.array_equal(st[k], ref["stage_" + k]), k
    # candidates that keep the trajectory are scored without a simulation
    n = len(x0)
    assert (st["simulated"] <= n * L - st["infeasible"] + n).all() and (st["simulated"] >= n).all()
    assert cost == ref["cost"] and winner == ref["winner"]
    assert np.array_equal(x, ref["x"])
    assert np.array_equal(cb.astype(np.int64), ref["chain_best"])
    assert np.array_equal(cx, ref["chain_xbest"])
    return ref


def test_run_q1():
    w = synth.load_workload("q1")
    s = synth.bench_schedule("q1")
    x0 = synth.start_vectors("q1", w, 21)      # 16-lane segments: 4 chains per wave, ragged
    ref = _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=8, L=70)
    assert ref["cost"] <= ref["stage_best"][0]


def test_run_q2_truncated():
    w = synth.load_workload("q2")
    s = synth.bench_schedule("q2")
    x0 = synth.start_vectors("q2", w, 70)
    _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=3, L=100)


def test_run_q3_truncated():
    w = synth.load_workload("q3")
    s = synth.bench_schedule("q3")
    x0 = synth.start_vectors("q3", w, 9)
    _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=2, L=40)


@pytest.mark.parametrize("N,E,C,T,O,clamps", [SHAPES[3], SHAPES[4], SHAPES[6], SHAPES[9], SHAPES[10]])
def test_run_other_widths_penalty_resume_islands(N, E, C, T, O, clamps):
    prob, _ = priority_problem(300 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=T, n_obs=O, noise=0.1,
                               clamps=clamps, hard=0)
    x0 = synth.priority_random_params(synth.rng_for(N), 13, E, N)    # penalty mode: infeasible starts allowed
    _compare_runs(prob, x0, 55, T0=1.5, rho=0.8, n_stages=4, L=45, first_stage=2, group_size=4)


def test_run_hard_mode_counts_infeasible_and_graph():
    prob, _ = priority_problem(701, n_nodes=12, n_edges=20, n_cond=2, n_steps=8, n_obs=6, noise=0.1)
    x0 = synth.priority_feasible_params(synth.rng_for(5), 10, prob["row_ptr"], prob["src"])
    ref = _compare_runs(prob, x0, 8, T0=2.0, rho=0.7, n_stages=3, L=50, use_graph=True)
    assert ref["stage_infeasible"].sum() > 0


def test_rejections():
    sa = _sa()
    w = synth.load_workload("q1")
    x0 = synth.start_vectors("q1", w, 4)
    P = sa.Problem(w)
    kw = dict(seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=4)
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, _dev(x0), kernel=sa.SA_KERNEL_PERSISTENT, **kw)
    assert e.value.code == sa.SA_ERR_UNSUPPORTED
    c1 = synth.load_workload("c1")
    with pytest.raises(sa.SAError) as e:           # the two models in one run
        sa.Run([P, sa.Problem(c1)], [_dev(x0), _dev(synth.start_vectors("c1", c1, 4))], **kw)
    assert e.value.code == sa.SA_ERR_UNSUPPORTED
    bad = x0.copy()
    bad[0, 3 * w["n_edges"]] = 7                     # a speed outside {1..6, 10..12}
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, _dev(bad), **kw)
    assert e.value.code == sa.SA_ERR_DOMAIN
    infeasible = x0.copy()
    infeasible[0, :w["n_edges"]] = 0                 # every weight 0
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, _dev(infeasible), **kw)
    assert e.value.code == sa.SA_ERR_INFEASIBLE
    big, _ = priority_problem(801, n_nodes=65, n_edges=130, n_cond=1, n_steps=3, n_obs=5)
    with pytest.raises(sa.SAError) as e:
        sa.Problem(big)
    assert e.value.code == sa.SA_ERR_UNSUPPORTED


@pytest.mark.parametrize("name", ["q2", "q3"])
def test_full_size_stages_sampled_chains(name):
    """Two stages of the workload in the launch configuration bench.py times
    (every chain, 500 steps per stage).  Chains are independent within a
    stage, so sampled chains are recomputed by the oracle one by one with
    their own Philox ids: stage 0 from their own start vectors, stage 1 from
    the stage-0 winner the library restarted every chain from."""
    w = synth.load_workload(name)
    s = synth.bench_schedule(name)
    n, L = s["n_chains"], s["steps_per_stage"]
    x0 = synth.start_vectors(name, w, n)
    sa = _sa()
    P = sa.Problem(w)
    o = OracleProblem(w)
    kw = dict(seed=s["seed"], T0=s["T0"], rho=s["rho"], steps_per_stage=L)
    run = sa.Run(P, _dev(x0), n_stages=2, launch=False, **kw)
    run.launch(1)
    cb0, cx0 = run.chain_best()
    st0 = run.stats()
    sample = (0, 1, 5, n // 2 + 3, n - 2, n - 1)
    for chain in sample:
        ref = o.run(x0[chain:chain + 1], n_stages=1, first_chain=chain, **kw)
        assert cb0[chain] == ref["chain_best"][0], chain
        assert np.array_equal(cx0[chain], ref["chain_xbest"][0]), chain
    assert st0["best_cost"][0] == cb0.min() and st0["winner"][0] == int(np.argmin(cb0))
    winner = cx0[int(np.argmin(cb0))]
    run.launch(1)
    cb1, cx1 = run.chain_best()
    for chain in sample:
        ref = o.run(winner[None, :], n_stages=1, first_stage=1, first_chain=chain, **kw)
        assert cb1[chain] == ref["chain_best"][0], chain
        assert np.array_equal(cx1[chain], ref["chain_xbest"][0]), chain
    assert np.array_equal(o.cost_batch(cx1[:6]), cb1[:6].astype(np.int64))


@pytest.mark.parametrize("N,E,C,T,n,L,hard", [
    (2, 2, 1, 1, 1, 1, 1),          # the smallest network, one step, one chain, one annealing step
    (64, 1300, 20, 3, 5, 70, 1),    # the largest segment, in-degree above 16 (ballot masks), many conditions
    (40, 0, 3, 6, 7, 40, 0),        # no edges at all (penalty mode): only node parameters change
    (16, 30, 2, 40, 9, 17, 1),      # a horizon longer than a step block; L not a multiple of the segment
])
def test_run_extreme_shapes(N, E, C, T, n, L, hard):
    if E == 0:
        row_ptr, src = np.zeros(N + 1, np.int32), np.zeros(0, np.int32)
        rng = synth.rng_for(N)
        init, clamp = synth.conditions(rng, N, C, (0, 1))
        prob = dict(n_nodes=N, n_edges=0, row_ptr=row_ptr, src=src, n_cond=C, init=init, clamp=clamp, n_steps=T,
                    obs_t=np.arange(T + 1, dtype=np.int32), obs_n=np.arange(0, N, 3, dtype=np.int32),
                    step_size=1, hard=0, penalty=0, model=synth.MODEL_PRIORITY)
        prob["observed"] = rng.integers(0, 3, size=(C, T + 1, len(prob["obs_n"]))).astype(np.int8)
        x0 = synth.priority_random_params(rng, n, 0, N)
    else:
        prob, _ = priority_problem(900 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=T, n_obs=max(1, N // 3),
                                   noise=0.1, clamps=(0, 2) if C > 1 else (0, 0), hard=hard)
        x0 = synth.priority_feasible_params(synth.rng_for(N + 1), n, prob["row_ptr"], prob["src"])
    _compare_runs(prob, x0, 21, T0=1.3, rho=0.75, n_stages=2, L=L)
    xs = np.concatenate([x0, synth.priority_random_params(synth.rng_for(E + 3), 9, E, N)])
    got = _sa().Problem(prob).eval_cost(_dev(xs)).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, OracleProblem(prob).cost_batch(xs))


def test_several_networks_in_one_run():
    """Three priority-model networks of different segment widths in one run:
    one stage-kernel launch per network and stage, one reduction for all;
    network p draws with Philox network id p, so each must equal the oracle's
    run of that network alone with net = p (island restarts, a graph)."""
    sa = _sa()
    probs = [synth.load_workload("q1"), priority_problem(1201, n_nodes=27, n_edges=80, n_cond=3, n_steps=9,
                                                         n_obs=9, noise=0.1, clamps=(1, 1))[0],
             synth.load_workload("q3")]
    n, S, L, G = 11, 3, 40, 4
    x0 = [synth.priority_feasible_params(synth.rng_for(40 + i), n, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]
    run = sa.Run([sa.Problem(p) for p in probs], [_dev(x) for x in x0], seed=99, T0=1.5, rho=0.8, n_stages=S,
                 steps_per_stage=L, group_size=G, use_graph=True)
    for i, (prob, x) in enumerate(zip(probs, x0)):
        ref = OracleProblem(prob).run(x, seed=99, T0=1.5, rho=0.8, n_stages=S, steps_per_stage=L, net=i,
                                      n_threads=8, group_size=G)
        st = run.stats(i)
        xb, cost, winner = run.best(i)
        cb, cx = run.chain_best(i)
        assert np.array_equal(st["best_cost"], ref["stage_best"]) and np.array_equal(st["winner"], ref["stage_winner"])
        for k in ("accepted", "uphill", "neutral", "infeasible"):
            assert np.array_equal(st[k], ref["stage_" + k]), (i, k)
        assert cost == ref["cost"] and winner == ref["winner"] and np.array_equal(xb, ref["x"]), i
        assert np.array_equal(cb.astype(np.int64), ref["chain_best"]) and np.array_equal(cx, ref["chain_xbest"]), i
