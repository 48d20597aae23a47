"""Pins of the oracle's learned-proposal definitions (oracle/learned.py):
hand-worked features, table invariants, and agreement of its serial run with
the C oracle's plain run wherever the two must coincide."""
import math

import numpy as np
import pytest

from oracle import learned
from oracle.oracle import OracleProblem
from tests.problems import from_edges, golden, random_problem


def _w1_problem():
    g = golden("w1_three_node_loop.json")
    edges = [(j, i) for j, i, _ in g["edges_src_dst_a"]]
    prob, perm = from_edges(3, edges, init=g["init"], n_steps=3, obs_t=g["obs_t"], obs_n=g["obs_n"],
                            observed=[g["observed"]])
    x = np.zeros(6, dtype=np.int8)
    for k, (_, _, a) in enumerate(g["edges_src_dst_a"]):
        x[perm[k]] = a
    return prob, x


def _expect(spec, T):
    f = np.zeros(32, dtype=np.float64)
    for k, v in spec.items():
        f[int(k)] = math.log(T) / 5 if v == "ln(T)/5" else v
    return f


def test_w1_refresh_aggregates_and_features_by_hand():
    gf = golden("w1_move_features.json")
    prob, x = _w1_problem()
    agg = learned.refresh_state(prob, x, gf["T"])
    assert agg["mismatch"] == gf["mismatch"]
    assert agg["msh"].tolist() == gf["msh"]
    assert agg["eh"].tolist() == gf["eh"] and agg["ah"].tolist() == gf["ah"]
    assert agg["mn"] == np.float32(gf["mn"])
    for mv in (gf["move"], gf["theta_move"]):
        spec = mv["features_nonzero"] if "features_nonzero" in mv else gf["features_nonzero"]
        f = learned.move_features(prob, mv["p"], mv["old"], mv["v"], agg, agg["ip"], agg["on"], agg["lt"])
        assert np.allclose(f, _expect(spec, gf["T"]).astype(np.float32), rtol=0, atol=1e-7), (mv, f)
    f = learned.move_features(prob, 1, 1, 0, agg, agg["ip"], agg["on"], agg["lt"])
    assert np.array_equal(f, _expect(gf["features_nonzero"], gf["T"]).astype(np.float32))


def _model(rng, scale=0.3):
    return {"W1": rng.normal(size=(32, 256)) * scale, "w2": rng.normal(size=256) * scale, "b2": 0.1}


def test_table_invariants():
    prob, hidden = random_problem(31, n_nodes=10, n_edges=30, n_cond=3, n_steps=6, n_times=3, n_obs=4)
    rng = np.random.default_rng(3)
    t = learned.proposal_table(prob, hidden, 0.7, _model(rng))
    P = len(hidden)
    assert len(t["moves"]) == 2 * P and t["features"].shape == (2 * P, 32)
    w = t["weights"]
    masked = t["features"][:, 21] != 0
    assert (w[masked] == 0).all()
    assert w.max() == learned.TABLE_SCALE and (w <= learned.TABLE_SCALE).all()
    # weights follow exp of the score differences
    lg = t["logits"]
    top = lg[~masked].max()
    assert np.array_equal(w[~masked], np.floor(np.exp(lg[~masked] - top) * 65536).astype(np.uint64))
    # moves never repeat the current value and cover both other values of every parameter
    for m, (p, old, v) in enumerate(t["moves"]):
        assert p == m // 2 and old == hidden[p] and v != old
    # a network that ignores its input scores every move alike
    flat = {"W1": np.zeros((32, 256)), "w2": np.zeros(256), "b2": -3.0}
    tf = learned.proposal_table(prob, hidden, 0.7, flat)
    assert set(tf["weights"][~masked].tolist()) == {65536}


def test_features_are_bf16_ready_and_mask_matches_constraints():
    prob, hidden = random_problem(32, n_nodes=12, n_edges=36, n_cond=4, n_steps=7, n_times=3, n_obs=5)
    o = OracleProblem(prob)
    t = learned.proposal_table(prob, hidden, 1.3, {"W1": np.zeros((32, 256)), "w2": np.zeros(256), "b2": 0.0})
    for m, (p, old, v) in enumerate(t["moves"]):
        xc = hidden.copy()
        xc[p] = v
        assert (t["features"][m, 21] != 0) == (o.violations(xc) > o.violations(hidden))
    assert (t["features"][:, 24:31] == 0).all() and (t["features"][:, 31] == 1).all()


@pytest.mark.parametrize("hard", [1, 0])
def test_run_without_model_is_the_plain_method(hard):
    prob, _ = random_problem(33, n_nodes=9, n_edges=26, n_cond=3, n_steps=6, n_times=3, n_obs=4,
                             noise=0.1, hard=hard)
    from paper_2506_19866_amd import synth
    rng = synth.rng_for(5)
    x0 = synth.feasible_params(rng, 5, prob["row_ptr"], prob["src"])
    kw = dict(seed=77, T0=1.5, rho=0.8, n_stages=3, steps_per_stage=40)
    ref = OracleProblem(prob).run(x0, **kw)
    got = learned.run(prob, x0, model=None, refresh=8, eps=0.1, **kw)
    assert got["stage_best"] == ref["stage_best"].tolist()
    assert got["stage_winner"] == ref["stage_winner"].tolist()
    assert np.array_equal(got["x"], ref["x"]) and got["cost"] == ref["cost"]
    # every plain step is also what the always-plain learned run takes
    rng2 = np.random.default_rng(1)
    always_plain = learned.run(prob, x0, model=_model(rng2), refresh=8, eps=1.0, **kw)
    assert always_plain["stage_best"] == got["stage_best"] and always_plain["steps"] == got["steps"]


def test_learned_steps_follow_the_table():
    prob, _ = random_problem(34, n_nodes=10, n_edges=30, n_cond=3, n_steps=6, n_times=3, n_obs=4, noise=0.1)
    from paper_2506_19866_amd import synth
    x0 = synth.feasible_params(synth.rng_for(6), 3, prob["row_ptr"], prob["src"])
    model = _model(np.random.default_rng(2), scale=0.5)
    res = learned.run(prob, x0, seed=9, T0=1.0, rho=0.9, n_stages=2, steps_per_stage=48, model=model,
                      refresh=16, eps=0.25, trace_every=1)
    srcs = np.array([s[2] for s in res["steps"]])
    assert (srcs == learned.SOURCE_LEARNED).sum() > 0.5 * len(srcs)
    assert (srcs == learned.SOURCE_PLAIN).sum() > 0.1 * len(srcs)
    # traced records carry the same steps
    assert [(c, g, p, v, d, fl) for c, g, _, p, v, d, fl in res["trace"]] == \
        [(c, g, p, v, dl, a | (fe << 1) | (s << 2)) for c, g, s, p, v, fe, dl, a in res["steps"]]
    # the stage bests decrease and are real costs
    o = OracleProblem(prob)
    assert res["cost"] == o.cost(res["x"])
    assert res["stage_best"][1] <= res["stage_best"][0]
