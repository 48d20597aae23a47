"""GPU parity of the many-network persistent kernel (one launch per stage for
networks of uneven size), its autotuner and the hipGraph-captured launch,
against the oracle and against the single-network kernel."""
import numpy as np
import pytest

from oracle.oracle import OracleProblem
from paper_2506_19866_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sa():
    from paper_2506_19866_amd import sa
    return sa


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).cuda()


def _check_against_oracle(run, probs, x0s, seed, T0, rho, S, L, first_stage=0, nets=None, group_size=0):
    for p, (prob, x0) in enumerate(zip(probs, x0s)):
        net = p if nets is None else nets[p]
        ref = OracleProblem(prob).run(x0, seed=seed, T0=T0, rho=rho, n_stages=S, steps_per_stage=L,
                                      first_stage=first_stage, net=net, n_threads=8, group_size=group_size)
        st = run.stats(p)
        x, cost, winner = run.best(p)
        cb, cx = run.chain_best(p)
        assert np.array_equal(st["best_cost"], ref["stage_best"]), p
        assert np.array_equal(st["winner"], ref["stage_winner"]), p
        for k in ("accepted", "uphill", "neutral", "infeasible"):
            assert np.array_equal(st[k], ref["stage_" + k]), (p, k)
        assert np.array_equal(st["simulated"], len(x0) * L - st["infeasible"] + len(x0)), p
        assert cost == ref["cost"] and winner == ref["winner"], p
        assert np.array_equal(x, ref["x"]), p
        assert np.array_equal(cb.astype(np.int64), ref["chain_best"]), p
        assert np.array_equal(cx, ref["chain_xbest"]), p


@pytest.mark.parametrize("chains_per_block", [1, 2, 4, 8, 0])
def test_persistent_kernel_on_one_network(chains_per_block):
    sa = _sa()
    w = synth.load_workload("c1")
    s = synth.bench_schedule("c1")
    x0 = synth.start_vectors("c1", w, 21)
    run = sa.Run(sa.Problem(w), _dev(x0), seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=6,
                 steps_per_stage=50, kernel=sa.SA_KERNEL_PERSISTENT, chains_per_block=chains_per_block)
    info = run.info()
    assert info["kernel"] == sa.SA_KERNEL_PERSISTENT
    assert info["chains_per_block"] in (1, 2, 4, 8)
    assert (info["tiles_m"], info["frags_k"]) == (1, 1)   # 12 nodes
    if chains_per_block:
        assert info["chains_per_block"] == chains_per_block
    _check_against_oracle(run, [w], [x0], s["seed"], s["T0"], s["rho"], 6, 50)


def _uneven_subset():
    batch = synth.load_batch("c4")
    N = np.array([p["n_nodes"] for p in batch])
    # smallest, largest, and sizes in between (every k-tile count), in workload order
    picks = sorted({int(np.argmin(N)), int(np.argmax(N)), *[int(np.argmin(np.abs(N - v))) for v in (30, 63, 64, 90, 128)]})
    return [batch[i] for i in picks]


@pytest.mark.parametrize("use_graph", [False, True])
def test_uneven_batch_matches_oracle_per_network(use_graph):
    sa = _sa()
    probs = _uneven_subset()
    # one network with step size 2: its own persistent launch in the same stage
    probs = probs + [dict(probs[1], step_size=2)]
    n = 10
    x0s = [synth.feasible_params(np.random.default_rng(i), n, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]
    P = [sa.Problem(p) for p in probs]
    S, L, seed = 3, 40, 99
    run = sa.Run(P, [_dev(x) for x in x0s], seed=seed, T0=2.0, rho=0.8, n_stages=S, steps_per_stage=L,
                 use_graph=use_graph, chains_per_block=0)
    _check_against_oracle(run, probs, x0s, seed, 2.0, 0.8, S, L)


def test_uneven_batch_island_restart():
    """Island restart in the persistent kernel: groups of 3 of 10 chains per
    network (the last group is one chain), every network against the oracle."""
    sa = _sa()
    probs = _uneven_subset()[:5]
    n = 10
    x0s = [synth.feasible_params(np.random.default_rng(30 + i), n, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]
    P = [sa.Problem(p) for p in probs]
    S, L, seed = 3, 40, 17
    run = sa.Run(P, [_dev(x) for x in x0s], seed=seed, T0=2.0, rho=0.8, n_stages=S, steps_per_stage=L,
                 use_graph=True, chains_per_block=2, group_size=3)
    _check_against_oracle(run, probs, x0s, seed, 2.0, 0.8, S, L, group_size=3)


# (nodes, edges, conditions, clamp values, observed nodes): every m-tile count
# of the three size classes, the bias slot in each position it can take
# (inside a computed m-tile, in the unused half of the last dword, past the
# rows), and both ways of holding clamped nodes (a clamp value of 1, or
# clamped and observed nodes that do not fit the first dword, take the select)
_LAYOUT_CASES = [(16, 50, 5, (0, 2), 3), (26, 80, 6, (0, 2), 4), (33, 90, 7, (1, 2), 5), (48, 140, 9, (0, 2), 8),
                 (64, 200, 12, (0, 2), 10), (80, 240, 6, (0, 1, 2), 13), (96, 290, 8, (0, 2), 16),
                 (112, 330, 16, (0, 2), 18), (120, 360, 5, (0, 2), 20), (128, 380, 4, (0, 2), 21),
                 (144, 420, 8, (1,), 24), (144, 420, 6, (0, 2), 24), (150, 450, 10, (0, 2), 18)]


def test_batch_every_tile_count_and_clamp_form():
    """One persistent run over networks of every m-tile count the size classes
    serve, mixing the accumulator-offset and select forms of clamping, each
    network bit-exact against the oracle."""
    from tests.problems import random_problem
    sa = _sa()
    probs = [random_problem(700 + N + C, n_nodes=N, n_edges=E, n_cond=C, n_steps=8, n_times=3, n_obs=O,
                            noise=0.1, clamps=(1, 2), clamp_values=v)[0] for N, E, C, v, O in _LAYOUT_CASES]
    P = [sa.Problem(p) for p in probs]
    forms = [q.info["clamps_by_offset"] for q in P]
    assert forms == [1, 1, 0, 1, 1, 0, 1, 0, 1, 1, 0, 1, 1]
    n = 9
    x0s = [synth.feasible_params(np.random.default_rng(50 + i), n, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]
    S, L, seed = 3, 40, 23
    run = sa.Run(P, [_dev(x) for x in x0s], seed=seed, T0=2.0, rho=0.8, n_stages=S, steps_per_stage=L,
                 use_graph=True, chains_per_block=0)
    _check_against_oracle(run, probs, x0s, seed, 2.0, 0.8, S, L)


def test_batch_independent_of_tiling_and_launch_split():
    """Results do not depend on the chains per workgroup or on how the stages
    are split into launch calls, and equal the oracle's per network."""
    sa = _sa()
    probs = _uneven_subset()[:4]
    n = 8
    x0s = [synth.feasible_params(np.random.default_rng(10 + i), n, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]
    P = [sa.Problem(p) for p in probs]
    a = sa.Run(P, [_dev(x) for x in x0s], seed=5, T0=1.5, rho=0.7, n_stages=4, steps_per_stage=30,
               chains_per_block=2)
    b = sa.Run(P, [_dev(x) for x in x0s], seed=5, T0=1.5, rho=0.7, n_stages=4, steps_per_stage=30,
               chains_per_block=8, launch=False)
    b.launch(1)
    b.launch(3)
    for p in range(len(probs)):
        sa_, sb = a.stats(p), b.stats(p)
        for k in sa_:
            assert np.array_equal(sa_[k], sb[k]), (p, k)
        assert np.array_equal(a.best(p)[0], b.best(p)[0])
    _check_against_oracle(a, probs, x0s, 5, 1.5, 0.7, 4, 30)


def test_full_batched_workload_sampled_chains():
    """The batched workload at its full size (256 networks x 256 chains) for
    one stage in the launch configuration the benchmark uses; sampled chains
    of sampled networks recomputed one by one by the oracle."""
    sa = _sa()
    probs = synth.load_batch("c4")
    s = synth.batch_schedule()
    n = s["n_chains"]
    x0s = synth.batch_start_vectors(probs, n)
    P = [sa.Problem(p) for p in probs]
    L = 40
    run = sa.Run(P, [_dev(x) for x in x0s], seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=1,
                 steps_per_stage=L, chains_per_block=0, use_graph=True)
    N = np.array([p["n_nodes"] for p in probs])
    for p in sorted({0, int(np.argmax(N)), int(np.argmin(N)), 128, 255}):
        cb, cx = run.chain_best(p)
        st = run.stats(p)
        assert st["best_cost"][0] == cb.min() and st["winner"][0] == int(np.argmin(cb))
        o = OracleProblem(probs[p])
        for chain in (0, 101, n - 1):
            ref = o.run(x0s[p][chain:chain + 1], seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=1,
                        steps_per_stage=L, net=p, first_chain=chain)
            assert cb[chain] == ref["chain_best"][0], (p, chain)
            assert np.array_equal(cx[chain], ref["chain_xbest"][0]), (p, chain)
