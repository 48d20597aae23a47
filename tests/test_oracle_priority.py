"""Pins of the oracle's priority-update model (paper §2.1 image with weight,
polarity and threshold; §2.2 speed, memory and step size; §2.5.3
constraints), against hand-worked trajectories, closed forms, the paper's
printed parameter counts, invariants and the independent Python statement.
"""
import math

import numpy as np
import pytest

from oracle import reference
from oracle.oracle import OracleProblem, draw
from paper_2506_19866_amd import synth
from tests.problems import from_edges, golden

PRIORITY = synth.MODEL_PRIORITY


def _params(perm, E, w, p, t, u, m, d):
    """Vector in parameter order from per-given-edge w, p, t and per-node u, m, d."""
    x = np.zeros(3 * E + 3 * len(u), dtype=np.int8)
    for k in range(E):
        x[perm[k]], x[E + perm[k]], x[2 * E + perm[k]] = w[k], p[k], t[k]
    N = len(u)
    x[3 * E:3 * E + N], x[3 * E + N:3 * E + 2 * N], x[3 * E + 2 * N:] = u, m, d
    return x


def _sim(impl, prob, x):
    if impl == "c":
        return OracleProblem(prob).simulate(x)[0].tolist()
    return reference.simulate(prob, x)[0]


@pytest.mark.parametrize("impl", ["c", "python"])
def test_hand_worked_three_node_trajectory(impl):
    g = golden("p1_priority_three_nodes.json")
    edges = [tuple(e) for e in g["edges_src_dst"]]
    prob, perm = from_edges(3, edges, init=g["init"], n_steps=len(g["trajectory"]) - 1, model=PRIORITY)
    x = _params(perm, len(edges), g["w"], g["p"], g["t"], g["u"], g["m"], g["d"])
    assert _sim(impl, prob, x) == g["trajectory"]


@pytest.mark.parametrize("impl", ["c", "python"])
@pytest.mark.parametrize("case", range(3))
def test_highest_priority_class_moves_ties_included(impl, case):
    g = golden("p1_priority_three_nodes.json")
    tc = g["tie_cases"][case]
    # nodes A=0, B=1, Z=2 (clamped at 2)
    prob, perm = from_edges(3, [(2, 0), (2, 1)], init=[0, 0, 2], clamp=[-1, -1, 2],
                            n_steps=len(tc["trajectory_ab"]) - 1, model=PRIORITY)
    x = _params(perm, 2, [1, 1], [1, 1], [1, 1], tc["u"] + [1], [0, 0, 0], [1, 1, 1])
    traj = _sim(impl, prob, x)
    assert [row[:2] for row in traj] == tc["trajectory_ab"]
    assert all(row[2] == 2 for row in traj)


def test_parameter_counts_match_the_paper():
    """§1 and §2.5 print P = 102 (HPG: 9 nodes, 25 edges) and P = 723 (Mtb: 63
    nodes, 178 edges); the priority workloads have exactly those sizes."""
    g = golden("paper_parameter_counts.json")["paper"]
    for name, key in (("q2", "hpg"), ("q3", "mtb")):
        w = synth.load_workload(name)
        assert (w["n_nodes"], w["n_edges"]) == (g[key]["nodes"], g[key]["edges"])
        assert OracleProblem(w).n_params == g[key]["params"]
        assert len(w["hidden"]) == g[key]["params"]
        assert w["observed"].shape[1] == 20          # 20 time points, the initial state included
    assert synth.load_workload("q2")["observed"].shape[2] == 5
    assert synth.load_workload("q3")["observed"].shape[2] == 35


def test_single_free_node_closed_form():
    """One free node driven by a clamped regulator at level a has the constant
    goal g = clamp((a div t) * w * p, 0, 2); it is told at every step until it
    arrives, so it moves d levels at steps m+1, 2(m+1), ...:
    s(k) = s0 + sign(g - s0) * min(|g - s0|, d * floor(k / (m + 1)))."""
    for a in range(3):
        for w in range(3):
            for p in (-1, 0, 1):
                for t in (1, 2):
                    goal = min(max((a // t) * w * p, 0), 2)
                    for m in range(3):
                        for d in (1, 2):
                            for s0 in range(3):
                                for u in (1, 12):
                                    prob, perm = from_edges(2, [(1, 0)], init=[s0, a], clamp=[-1, a],
                                                            n_steps=9, model=PRIORITY)
                                    x = _params(perm, 1, [w], [p], [t], [u, 1], [m, 0], [d, 1])
                                    traj = OracleProblem(prob).simulate(x)[0]
                                    gap = goal - s0
                                    sign = (gap > 0) - (gap < 0)
                                    want = [s0 + sign * min(abs(gap), d * (k // (m + 1))) for k in range(10)]
                                    assert traj[:, 0].tolist() == want, (a, w, p, t, m, d, s0)
                                    assert (traj[:, 1] == a).all()


@pytest.mark.parametrize("m", [0, 1, 2])
def test_uniform_decay_without_regulation(m):
    """With every weight 0 each image is 0.  With equal speeds and equal
    memory every node still above 0 has the same idle and telling counts, so
    the whole class moves together at steps m+1, 2(m+1), ...:
    s_i(k) = max(s_i(0) - d_i * floor(k / (m + 1)), 0)."""
    rng = synth.rng_for(31 + m)
    row_ptr, src = synth.topology_cycle_plus_uniform(rng, 15, 50)
    init, _ = synth.conditions(rng, 15, 3, (0, 0))
    prob = dict(n_nodes=15, n_edges=50, row_ptr=row_ptr, src=src, n_cond=3, init=init,
                clamp=np.full_like(init, -1), n_steps=8, obs_t=np.array([1], np.int32),
                obs_n=np.array([0], np.int32), observed=np.zeros((3, 1, 1), np.int8),
                step_size=1, hard=1, penalty=0, model=PRIORITY)
    x = synth.priority_random_params(rng, 1, 50, 15)[0]
    x[:50] = 0
    x[150:165] = 5
    x[165:180] = m
    d = x[180:195].astype(int)
    traj = OracleProblem(prob).simulate(x)
    for c in range(3):
        for k in range(9):
            want = np.maximum(init[c].astype(int) - d * (k // (m + 1)), 0)
            assert traj[c, k].tolist() == want.tolist()


def test_moves_bounded_by_step_size_and_clamps_hold():
    w = synth.load_workload("q3")
    prob = dict(w, clamp=np.where(np.arange(63) % 9 == 0, 1, -1).astype(np.int8)[None, :])
    o = OracleProblem(prob)
    E, N = w["n_edges"], w["n_nodes"]
    xs = synth.priority_random_params(synth.rng_for(41), 20, E, N)
    for x in xs:
        traj = o.simulate(x)[0].astype(int)
        d = x[3 * E + 2 * N:].astype(int)
        assert (np.abs(np.diff(traj, axis=0)) <= d[None, :]).all()
        assert (traj[:, ::9] == 1).all()
        assert traj.min() >= 0 and traj.max() <= 2


def test_relabeling_invariance():
    """Renaming nodes permutes trajectories and leaves costs unchanged."""
    w = synth.load_workload("q2")
    N, E = w["n_nodes"], w["n_edges"]
    rng = np.random.default_rng(3)
    pi = rng.permutation(N)
    edges = [(int(w["src"][e]), i) for i in range(N) for e in range(w["row_ptr"][i], w["row_ptr"][i + 1])]
    new_edges = [(int(pi[j]), int(pi[i])) for j, i in edges]
    init = np.empty_like(w["init"]); init[:, pi] = w["init"]
    obs_n_new = pi[w["obs_n"]]
    order = np.argsort(obs_n_new)
    prob2, perm = from_edges(N, new_edges, init=init, n_steps=w["n_steps"], obs_t=w["obs_t"],
                             obs_n=obs_n_new[order], observed=w["observed"][:, :, order], model=PRIORITY)
    o1, o2 = OracleProblem(w), OracleProblem(prob2)
    for x in synth.priority_random_params(rng, 20, E, N):
        x2 = np.empty_like(x)
        for blk in range(3):
            x2[blk * E + perm] = x[blk * E:(blk + 1) * E]
            x2[3 * E + blk * N + pi] = x[3 * E + blk * N:3 * E + (blk + 1) * N]
        assert np.array_equal(o2.simulate(x2)[:, :, pi], o1.simulate(x))
        assert o1.cost(x) == o2.cost(x2)


@pytest.mark.parametrize("name", ["q1", "q2", "q3"])
def test_c_oracle_equals_python_statement(name):
    w = synth.load_workload(name)
    o = OracleProblem(w)
    xs = synth.priority_random_params(synth.rng_for(51), 12, w["n_edges"], w["n_nodes"])
    xs = np.concatenate([xs, synth.start_vectors(name, w, 4)])
    for x in xs:
        assert o.simulate(x)[0].tolist() == reference.simulate(w, x)[0]
        assert (o.violations(x), o.cost(x)) == (reference.violations(w, x), reference.cost(w, x))


@pytest.mark.parametrize("name", ["q1", "q3"])
def test_hidden_parameters_fit_clean_data_exactly(name):
    w = synth.load_workload(name)
    clean = dict(w, observed=w["clean"])
    assert OracleProblem(clean).cost(w["hidden"]) == 0
    assert OracleProblem(w).violations(w["hidden"]) == 0


def test_violation_counts():
    """§2.5.3: (a) an out-edge with w != 0, (b) an in-edge with p = +1 and w != 0."""
    # loop 0 -> 1 -> 2 -> 0
    prob, perm = from_edges(3, [(0, 1), (1, 2), (2, 0)], init=[0, 0, 0], model=PRIORITY)
    o = OracleProblem(prob)
    ones = [1, 1, 1]
    assert o.violations(_params(perm, 3, [1, 1, 1], [1, 1, 1], ones, ones, [0] * 3, ones)) == 0
    # w = 0 on 0 -> 1: node 0 loses its out-edge, node 1 its activating in-edge
    assert o.violations(_params(perm, 3, [0, 1, 1], [1, 1, 1], ones, ones, [0] * 3, ones)) == 2
    # p = -1 on 1 -> 2: node 2 has no activating in-edge; out-edges all present
    assert o.violations(_params(perm, 3, [1, 2, 1], [1, -1, 1], ones, ones, [0] * 3, ones)) == 1
    # p = 0 with w != 0 still counts as an out-edge
    assert o.violations(_params(perm, 3, [1, 1, 2], [1, 1, 0], ones, ones, [0] * 3, ones)) == 1


def test_feasible_generator_is_feasible():
    for name in ("q2", "q3"):
        w = synth.load_workload(name)
        o = OracleProblem(w)
        xs = synth.start_vectors(name, w, 64)
        assert all(o.violations(x) == 0 for x in xs)


_DOMAINS = ((0, 1, 2), (-1, 0, 1), (1, 2), synth.SPEEDS_SLOW + synth.SPEEDS_FAST, (0, 1, 2), (1, 2))


def test_proposal_stays_in_domain_never_noop_and_uniform():
    """Table 1 proposal on the priority parameters: a uniformly chosen element
    takes one of the other values of its own domain, uniformly."""
    w = synth.load_workload("q1")
    o = OracleProblem(w)
    E, N, P = w["n_edges"], w["n_nodes"], o.n_params
    bounds = [0, E, 2 * E, 3 * E, 3 * E + N, 3 * E + 2 * N, P]
    x = synth.start_vectors("q1", w, 1)[0]
    counts = np.zeros(P)
    moves = {}
    n = 60000
    for g in range(n):
        i, v = o.propose(x, draw(9, g, 0, 0))
        blk = int(np.searchsorted(bounds, i, side="right")) - 1
        assert v in _DOMAINS[blk] and v != x[i]
        counts[i] += 1
        moves[(i, v)] = moves.get((i, v), 0) + 1
    chi2 = float(((counts - n / P) ** 2 / (n / P)).sum())
    assert chi2 < P + 6 * math.sqrt(2 * P)
    for i in range(P):
        blk = int(np.searchsorted(bounds, i, side="right")) - 1
        others = [v for v in _DOMAINS[blk] if v != x[i]]
        got = np.array([moves.get((i, v), 0) for v in others], dtype=float)
        expect = counts[i] / len(others)
        assert (np.abs(got - expect) < 6 * math.sqrt(expect) + 1).all(), (i, got)


def test_annealing_on_priority_model_improves_and_is_thread_independent():
    w = synth.load_workload("q1")
    o = OracleProblem(w)
    x0 = synth.start_vectors("q1", w, 8)
    kw = dict(seed=7, T0=2.0, rho=0.9, n_stages=20, steps_per_stage=40)
    r1 = o.run(x0, n_threads=1, **kw)
    r2 = o.run(x0, n_threads=4, **kw)
    assert r1["cost"] == r2["cost"] and np.array_equal(r1["x"], r2["x"])
    assert r1["cost"] == o.cost(r1["x"]) and o.violations(r1["x"]) == 0
    assert r1["cost"] <= min(o.cost(x) for x in x0)
