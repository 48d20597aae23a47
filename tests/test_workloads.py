"""The stored workloads are exactly what their committed recipe produces
(seeded generators + oracle trajectories), and have the documented shapes."""
import numpy as np
import pytest

from oracle import make_workloads
from paper_2506_19866_amd import synth


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "q1", "q2", "q3"])
def test_stored_workload_regenerates(name):
    stored = synth.load_workload(name)
    fresh = make_workloads.make(name)
    for k, v in fresh.items():
        assert np.array_equal(np.asarray(stored[k]), np.asarray(v)), k


def test_stored_batch_regenerates_and_has_the_documented_spread():
    stored = synth.load_batch("c4")
    assert len(stored) == synth.BATCH["n_networks"]
    for i in (0, 5, 77, 255):
        fresh = make_workloads.make(f"c4[{i}]", synth.batch_network_config(i), 4000 + i)
        for k, v in fresh.items():
            assert np.array_equal(np.asarray(stored[i][k]), np.asarray(v)), (i, k)
    N = np.array([p["n_nodes"] for p in stored])
    P = np.array([p["n_nodes"] + p["n_edges"] for p in stored])
    C = np.array([p["n_cond"] for p in stored])
    assert N.min() >= 10 and N.max() <= 150 and P.min() >= 30 and P.max() <= 900
    assert C.min() >= 4 and C.max() <= 16


@pytest.mark.parametrize("name,N,E,P,C", [("c1", 12, 28, 40, 4), ("c2", 20, 82, 102, 8), ("c3", 120, 603, 723, 16)])
def test_workload_shapes(name, N, E, P, C):
    w = synth.load_workload(name)
    assert (w["n_nodes"], w["n_edges"], w["n_nodes"] + w["n_edges"], w["n_cond"]) == (N, E, P, C)
    cfg = synth.CONFIGS[name]
    assert w["observed"].shape == (C, cfg["n_times"], cfg["n_obs"])
    flips = int((w["observed"] != w["clean"]).sum())
    assert flips == synth.n_flips(cfg)


@pytest.mark.parametrize("name,N,E,P,C,K,O", [("q1", 6, 12, 54, 2, 11, 4), ("q2", 9, 25, 102, 1, 20, 5),
                                            ("q3", 63, 178, 723, 1, 20, 35)])
def test_priority_workload_shapes(name, N, E, P, C, K, O):
    w = synth.load_workload(name)
    assert w["model"] == synth.MODEL_PRIORITY
    assert (w["n_nodes"], w["n_edges"], 3 * (w["n_nodes"] + w["n_edges"]), w["n_cond"]) == (N, E, P, C)
    assert w["observed"].shape == (C, K, O) and len(w["hidden"]) == P
    assert w["obs_t"].tolist() == list(range(K))
    cfg = synth.PRIORITY_CONFIGS[name]
    assert int((w["observed"] != w["clean"]).sum()) == synth.n_flips(cfg)
    u = w["hidden"][3 * E:3 * E + N]
    assert set(u.tolist()) <= set(synth.SPEEDS_SLOW + synth.SPEEDS_FAST)
