"""GPU parity: the HIP library against the CPU oracle, element by element and
bit for bit (integer work: costs, trajectories, per-stage statistics, winners
and best vectors must be identical).

Sizes: small enough for the oracle to finish in seconds while spanning several
m-tiles/k-tiles, ragged wave counts and every register layout, plus sampled
checks at the full workload sizes in the launch configuration the benchmark
times."""
import numpy as np
import pytest

from oracle.oracle import OracleProblem, candidate_matrix
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


def _gpu_costs(prob, xs, **kw):
    P = _sa().Problem(prob, **kw)
    out = P.eval_cost(_dev(xs)).cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    return out


# ---------------------------------------------------------------------------
# cost of every candidate of tiny networks (exhaustive)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,N,E,C,noise,clamps,d,hard", [
    (31, 3, 5, 2, 0.3, (0, 1), 1, 1),
    (32, 4, 6, 3, 0.2, (1, 1), 1, 1),
    (33, 4, 6, 2, 0.2, (0, 1), 2, 1),
    (34, 3, 6, 1, 0.4, (0, 0), 1, 0),
])
def test_every_candidate_cost_matches(seed, N, E, C, noise, clamps, d, hard):
    prob, _ = random_problem(seed, n_nodes=N, n_edges=E, n_cond=C, n_steps=6, n_times=3,
                             n_obs=min(N, 3), noise=noise, clamps=clamps, step_size=d, hard=hard)
    o = OracleProblem(prob)
    X = candidate_matrix(o.n_params, o.n_edges)
    best, argmin, nmin, oracle_costs = o.brute_force(with_costs=True)
    gpu = _gpu_costs(prob, X)
    assert np.array_equal(gpu, oracle_costs)
    assert gpu.min() == best and int((gpu == best).sum()) == nmin


# ---------------------------------------------------------------------------
# costs and trajectories of random vectors on every workload and layout
# ---------------------------------------------------------------------------
LAYOUTS = [  # (N, E, C, T, K, O): every m-tile count 1..12 and several condition groups
    (5, 12, 1, 4, 2, 2), (16, 40, 4, 6, 3, 5), (20, 60, 8, 15, 4, 10), (33, 90, 16, 8, 3, 11),
    (63, 200, 5, 10, 4, 20), (64, 190, 3, 7, 7, 64), (70, 240, 17, 6, 2, 30), (100, 400, 16, 12, 6, 40),
    (127, 500, 2, 5, 5, 50), (128, 380, 20, 4, 2, 40), (150, 520, 33, 5, 3, 50), (191, 600, 4, 3, 3, 70),
]


@pytest.mark.parametrize("N,E,C,T,K,O", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2])
def test_random_costs_and_trajectories(N, E, C, T, K, O, d):
    prob, hidden = random_problem(1000 + N + C, n_nodes=N, n_edges=E, n_cond=C, n_steps=T,
                                  n_times=K, n_obs=O, noise=0.1, clamps=(0, 3), step_size=d,
                                  topology="preferential")
    rng = np.random.default_rng(N * 7 + d)
    xs = np.concatenate([synth.random_params(rng, 37, E, N),
                         synth.feasible_params(rng, 6, prob["row_ptr"], prob["src"]), hidden[None]])
    o = OracleProblem(prob)
    assert np.array_equal(_gpu_costs(prob, xs), o.cost_batch(xs))
    P = _sa().Problem(prob)
    traj = P.simulate(_dev(xs[:9])).cpu().numpy()
    for i in range(9):
        assert np.array_equal(traj[i], o.simulate(xs[i])), i


def test_observation_at_time_zero_and_penalty():
    prob, _ = random_problem(41, n_nodes=12, n_edges=30, n_cond=3, n_steps=6, n_times=3, n_obs=5,
                             noise=0.3)
    prob = dict(prob, obs_t=np.array([0, 2, 6], np.int32), penalty=7)
    rng = np.random.default_rng(5)
    xs = synth.random_params(rng, 50, prob["n_edges"], prob["n_nodes"])
    assert np.array_equal(_gpu_costs(prob, xs), OracleProblem(prob).cost_batch(xs))


@pytest.mark.parametrize("d", [1, 2])
def test_horizon_beyond_last_observation(d):
    """States after the last observed time enter no cost (the kernels stop
    simulating there); trajectories still cover the whole horizon."""
    prob, _ = random_problem(5100 + d, n_nodes=40, n_edges=140, n_cond=10, n_steps=12, n_times=3, n_obs=12,
                             noise=0.1, clamps=(1, 2), step_size=d)
    prob = dict(prob, n_steps=19)
    rng = np.random.default_rng(51 + d)
    xs = np.concatenate([synth.random_params(rng, 40, prob["n_edges"], prob["n_nodes"]),
                         synth.feasible_params(rng, 8, prob["row_ptr"], prob["src"])])
    o = OracleProblem(prob)
    assert np.array_equal(_gpu_costs(prob, xs), o.cost_batch(xs))
    traj = _sa().Problem(prob).simulate(_dev(xs[:4])).cpu().numpy()
    assert traj.shape[2] == 20
    for i in range(4):
        assert np.array_equal(traj[i], o.simulate(xs[i])), i
    _compare_runs(prob, xs[40:], 13, T0=1.3, rho=0.8, n_stages=2, L=40)


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_workload_costs(name):
    w = synth.load_workload(name)
    rng = np.random.default_rng(9)
    xs = np.concatenate([synth.random_params(rng, 45, w["n_edges"], w["n_nodes"]),
                         synth.start_vectors(name, w, 18), w["hidden"][None]])
    o = OracleProblem(w)
    assert np.array_equal(_gpu_costs(w, xs), o.cost_batch(xs))
    clean = dict(w, observed=w["clean"])
    assert _gpu_costs(clean, w["hidden"][None])[0] == 0


def test_empty_batch_is_a_noop():
    w = synth.load_workload("c1")
    P = _sa().Problem(w)
    out = torch.full((1,), -5, dtype=torch.int32, device="cuda")
    P.eval_cost(torch.empty((0, P.n_params), dtype=torch.int8, device="cuda"), out=out)
    torch.cuda.synchronize()
    assert int(out[0]) == -5


# ---------------------------------------------------------------------------
# annealing runs (Table 1): bit-identical to the oracle
# ---------------------------------------------------------------------------
def _compare_runs(prob, x0, name_seed, *, T0, rho, n_stages, L, first_stage=0, hard=1, group_size=0, **kw):
    o = OracleProblem(prob)
    ref = o.run(x0, seed=name_seed, T0=T0, rho=rho, n_stages=n_stages, steps_per_stage=L,
                first_stage=first_stage, n_threads=8, group_size=group_size)
    sa = _sa()
    P = sa.Problem(prob)
    run = sa.Run(P, _dev(x0), seed=name_seed, T0=T0, rho=rho, n_stages=n_stages, steps_per_stage=L,
                 first_stage=first_stage, group_size=group_size, **kw)
    st = run.stats()
    x, cost, winner = run.best()
    cb, cx = run.chain_best()
    assert np.array_equal(st["best_cost"], ref["stage_best"])
    assert np.array_equal(st["winner"], ref["stage_winner"])
    for k in ("accepted", "uphill", "neutral", "infeasible"):
        assert np.array_equal(st[k], ref["stage_" + k]), k
    # every chain simulates its start vector and every feasible candidate
    n = len(x0)
    assert np.array_equal(st["simulated"], n * L - st["infeasible"] + n)
    assert cost == ref["cost"] and winner == ref["winner"]
    assert np.array_equal(x, ref["x"])
    assert np.array_equal(cb.astype(np.int64), ref["chain_best"])
    assert np.array_equal(cx, ref["chain_xbest"])
    return ref


def test_run_c1_full_schedule():
    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    x0 = synth.start_vectors("c1", w, s["n_chains"])
    ref = _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=s["n_stages"],
                        L=s["steps_per_stage"])
    assert ref["cost"] <= ref["stage_best"][0]


def test_run_c2_truncated():
    w = synth.load_workload("c2")
    s = synth.bench_schedule("c2")
    x0 = synth.start_vectors("c2", w, 70)   # ragged: not a multiple of the block's 4 waves
    _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=3, L=150)


@pytest.mark.parametrize("N,E,C,d,values,clamps,O,by_offset", [
    # clamp value 1 cannot be forced through the accumulator: select
    (40, 130, 12, 1, (1,), (1, 3), 10, 0),
    (120, 600, 16, 1, (0, 1, 2), (1, 3), 30, 0),
    (90, 300, 20, 2, (1, 2), (1, 3), 22, 0),
    # more than 32 clamped nodes: select
    (120, 600, 24, 1, (0, 2), (2, 3), 30, 0),
    # 32 observed nodes fill the first dword: clamped nodes first would add an
    # observed dword, so select
    (70, 250, 16, 1, (0, 2), (1, 2), 32, 0),
    # accumulator offsets: the bias slot in the unused half of the only dword
    # (16 nodes), an odd m-tile count (48), two k-fragments (150; 130 with an
    # odd m-tile count and two condition groups), no clamps at all
    (16, 50, 4, 1, (0, 2), (1, 2), 6, 1),
    (48, 150, 10, 2, (0, 2), (1, 2), 12, 1),
    (150, 500, 8, 1, (0, 2), (1, 2), 40, 1),
    (130, 420, 17, 2, (0, 2), (1, 2), 12, 1),
    (30, 90, 6, 1, (0, 2), (0, 0), 8, 1),
])
def test_run_clamp_hold_paths(N, E, C, d, values, clamps, O, by_offset):
    """The stage kernel holds clamped nodes either by accumulator offsets of
    the first two m-tiles (clamped nodes placed first) or by a select on every
    state dword; both paths, at the layout corner cases, against the oracle."""
    prob, _ = random_problem(400 + N + C, n_nodes=N, n_edges=E, n_cond=C, n_steps=9, n_times=3, n_obs=O,
                             noise=0.1, clamps=clamps, step_size=d, clamp_values=values)
    if 1 in values:
        assert (prob["clamp"] == 1).any()
    assert _sa().Problem(prob).info["clamps_by_offset"] == by_offset
    x0 = synth.feasible_params(np.random.default_rng(N + C), 24, prob["row_ptr"], prob["src"])
    _compare_runs(prob, x0, 13, T0=1.2, rho=0.7, n_stages=3, L=60)


def test_stored_workloads_hold_clamps_by_offset():
    for name in ("c1", "c2", "c3"):
        assert _sa().Problem(synth.load_workload(name)).info["clamps_by_offset"] == 1, name


def test_run_c3_truncated():
    w = synth.load_workload("c3")
    s = synth.bench_schedule("c3")
    x0 = synth.start_vectors("c3", w, 64)
    _compare_runs(w, x0, s["seed"], T0=s["T0"], rho=s["rho"], n_stages=2, L=40)


@pytest.mark.parametrize("G", [1, 5, 8, 21])
def test_run_island_restart_groups(G):
    """Island restart (groups of G chains, the last one ragged for G = 5 and 8;
    G = 21 is every chain) on the specialised kernel, against the oracle."""
    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    x0 = synth.start_vectors("c1", w, 21)
    _compare_runs(w, x0, 123, T0=s["T0"], rho=s["rho"], n_stages=6, L=60, group_size=G)


def test_run_island_restart_c2_graph():
    """Groups of 32 chains of the c2 workload, stages captured in a hipGraph."""
    w = synth.load_workload("c2")
    s = synth.bench_schedule("c2")
    x0 = synth.start_vectors("c2", w, 100)
    _compare_runs(w, x0, 77, T0=s["T0"], rho=s["rho"], n_stages=4, L=50, group_size=32, use_graph=True)


@pytest.mark.parametrize("N,E,C,d,G,first", [(40, 130, 18, 2, 6, 3), (191, 700, 3, 1, 2, 0), (9, 25, 3, 1, 3, 1)])
def test_run_island_restart_other_layouts(N, E, C, d, G, first):
    """Island restart with step size 2, the largest layout, and a run resumed
    mid-schedule (first stage > 0), against the oracle."""
    prob, _ = random_problem(6000 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=7, n_times=3,
                             n_obs=max(2, N // 3), noise=0.1, clamps=(1, 2), step_size=d)
    x0 = synth.feasible_params(np.random.default_rng(N + 1), 11, prob["row_ptr"], prob["src"])
    _compare_runs(prob, x0, 29, T0=1.5, rho=0.8, n_stages=3, L=40, first_stage=first, group_size=G)


def test_island_restart_rejections():
    sa = _sa()
    w = synth.load_workload("c1")
    P = sa.Problem(w)
    x0 = _dev(synth.start_vectors("c1", w, 8))
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, x0, seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=10, group_size=-1, launch=False)
    assert e.value.code == sa.SA_ERR_ARG
    trace = torch.zeros((8, 4 * sa.TRACE_RECORD_BYTES), dtype=torch.uint8, device="cuda")
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, x0, seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=10, group_size=4, trace=trace,
               launch=False)
    assert e.value.code == sa.SA_ERR_UNSUPPORTED


def test_run_resume_mid_schedule_and_penalty_mode():
    w = dict(synth.load_workload("c1"), hard=0)
    s = synth.bench_schedule("c1")
    x0 = synth.random_params(np.random.default_rng(3), 12, w["n_edges"], w["n_nodes"])
    _compare_runs(w, x0, 77, T0=s["T0"], rho=s["rho"], n_stages=5, L=70, first_stage=40, hard=0)


@pytest.mark.parametrize("N,E,C,d", [(9, 25, 3, 1), (40, 130, 18, 2), (150, 600, 5, 1)])
def test_run_other_layouts(N, E, C, d):
    prob, _ = random_problem(2000 + N, n_nodes=N, n_edges=E, n_cond=C, n_steps=7, n_times=3,
                             n_obs=max(2, N // 3), noise=0.1, clamps=(1, 2), step_size=d)
    x0 = synth.feasible_params(np.random.default_rng(N), 9, prob["row_ptr"], prob["src"])
    _compare_runs(prob, x0, 5, T0=1.5, rho=0.8, n_stages=3, L=45)


@pytest.mark.parametrize("N,E,C,T,K,n,L", [
    (30, 100, 64, 6, 7, 5, 33),     # 64 conditions = 4 condition groups; every time observed incl. t = 0
    (191, 700, 3, 4, 2, 3, 20),     # the largest layout (12 m-tiles x 3 k-tiles)
    (25, 70, 6, 9, 4, 1, 130),      # a single chain; L not a multiple of the 64-step Philox batch
])
def test_run_extreme_shapes(N, E, C, T, K, n, L):
    prob, _ = random_problem(3000 + N + C, n_nodes=N, n_edges=E, n_cond=C, n_steps=T, n_times=K,
                             n_obs=max(2, N // 4), noise=0.15, clamps=(0, 2), step_size=1)
    if K == T + 1:
        prob["obs_t"] = np.arange(T + 1, dtype=np.int32)
    x0 = synth.feasible_params(np.random.default_rng(N + C), n, prob["row_ptr"], prob["src"])
    _compare_runs(prob, x0, 11, T0=1.2, rho=0.7, n_stages=2, L=L)


def test_no_stage_launched_has_no_best():
    sa = _sa()
    w = synth.load_workload("c1")
    run = sa.Run(sa.Problem(w), _dev(synth.start_vectors("c1", w, 4)), seed=1, T0=1.0, rho=0.9, n_stages=2,
                 steps_per_stage=10, launch=False)
    with pytest.raises(sa.SAError) as e:
        run.best()
    assert e.value.code == sa.SA_ERR_ARG
    assert run.stats()["best_cost"].size == 0
    with pytest.raises(sa.SAError):
        run.launch(3)   # beyond the schedule
    run.launch(2)
    assert run.stats()["best_cost"].size == 2
    run.close()


@pytest.mark.parametrize("N,tiles", [(12, (1, 1)), (63, (4, 1)), (64, (4, 1)), (120, (8, 1)), (127, (8, 1)),
                                     (128, (9, 2)), (150, (10, 2)), (191, (12, 2))])
def test_register_layout_by_size(N, tiles):
    """Register layout of the simulation: ceil(N/16) m-tiles of 16 rows and
    N//128 + 1 k-fragments of 128 columns (nodes + bias), with at least 9
    m-tiles once there are two fragments."""
    sa = _sa()
    prob, _ = random_problem(4000 + N, n_nodes=N, n_edges=3 * N, n_cond=4, n_steps=4, n_times=2,
                             n_obs=max(2, N // 4), noise=0.0, clamps=(0, 1), step_size=1)
    x0 = synth.feasible_params(np.random.default_rng(N), 2, prob["row_ptr"], prob["src"])
    run = sa.Run(sa.Problem(prob), _dev(x0), seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=4, launch=False)
    info = run.info()
    assert (info["tiles_m"], info["frags_k"]) == tiles
    run.close()


def test_infeasible_start_is_rejected():
    sa = _sa()
    w = synth.load_workload("c1")
    P = sa.Problem(w)
    x0 = synth.start_vectors("c1", w, 4)
    x0[2, :w["n_edges"]] = 0
    with pytest.raises(sa.SAError) as e:
        sa.Run(P, _dev(x0), seed=1, T0=1.0, rho=0.9, n_stages=1, steps_per_stage=10)
    assert e.value.code == sa.SA_ERR_INFEASIBLE


# ---------------------------------------------------------------------------
# full-size workload, benchmark launch configuration, sampled chains
# ---------------------------------------------------------------------------
def test_c3_full_size_stage_sampled_chains():
    """Two stages of the c3 workload in the launch configuration bench.py
    times (16384 chains x 500 steps); every chain is independent within a
    stage, so sampled chains are recomputed by the oracle one by one with
    their own Philox chain ids: stage 0 from their start vectors, stage 1 from
    the stage-0 winner every chain restarted from."""
    w = synth.load_workload("c3")
    s = synth.bench_schedule("c3")
    n, L = s["n_chains"], s["steps_per_stage"]
    x0 = synth.start_vectors("c3", w, n)
    sa = _sa()
    P = sa.Problem(w)
    kw = dict(seed=s["seed"], T0=s["T0"], rho=s["rho"], steps_per_stage=L)
    run = sa.Run(P, _dev(x0), n_stages=2, launch=False, **kw)
    run.launch(1)
    cb, cx = run.chain_best()
    st = run.stats()
    o = OracleProblem(w)
    sample = (0, 1, 4095, 12345, n - 1)
    for chain in sample:
        ref = o.run(x0[chain:chain + 1], n_stages=1, first_chain=chain, **kw)
        assert cb[chain] == ref["chain_best"][0], chain
        assert np.array_equal(cx[chain], ref["chain_xbest"][0]), chain
    assert st["best_cost"][0] == cb.min() and st["winner"][0] == int(np.argmin(cb))
    assert np.array_equal(o.cost_batch(cx[:8]), cb[:8].astype(np.int64))
    winner = cx[int(np.argmin(cb))]
    run.launch(1)
    cb1, cx1 = run.chain_best()
    for chain in sample[:3]:
        ref = o.run(winner[None, :], n_stages=1, first_stage=1, first_chain=chain, **kw)
        assert cb1[chain] == ref["chain_best"][0], chain
        assert np.array_equal(cx1[chain], ref["chain_xbest"][0]), chain
