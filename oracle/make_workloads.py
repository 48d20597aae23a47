"""Writes the stored synthetic workloads ``paper_2506_19866_amd/data/c*.npz``.

TEST INFRASTRUCTURE.  The reference data of a workload are the trajectories of
hidden, randomly drawn feasible parameters at the observed times (the paper's
pseudo-experimental data, §2.5.2), so producing them needs the model; this
script takes that step with the oracle only, once, offline.  Everything else
comes from the seeded generators in ``paper_2506_19866_amd.synth``.

Recipe per workload (seed = 1000 + config number; priority-model workloads
q1-q3: 1100 + number):
  1. topology, hidden feasible parameters, conditions, observed times;
  2. oracle trajectories of the hidden parameters under every condition;
  3. observed nodes drawn with weight 1 + (number of state changes over all
     conditions and steps), favouring dynamic nodes (§2.5.2);
  4. reference data = hidden trajectories at (observed times, observed nodes);
     redrawn (next attempt seed) if fewer than 30% (batched workload: 15%) of
     its entries are non-zero, keeping the best of 100 draws otherwise;
  5. noise: a fixed fraction of entries flipped to another level.

Usage:  python oracle/make_workloads.py [c1 c2 c3 c4 q1 q2 q3]
"""
from __future__ import annotations

import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_HERE))

from oracle.oracle import OracleProblem  # noqa: E402
from paper_2506_19866_amd import synth  # noqa: E402


def make(name: str, cfg: dict | None = None, seed: int | None = None) -> dict:
    cfg = cfg if cfg is not None else synth.config(name)
    base = seed if seed is not None else synth.problem_seed(name)
    min_nonzero = cfg.get("min_nonzero", 0.30)
    best = None
    for attempt in range(100):
        rng = synth.rng_for(base + 7919 * attempt)
        prob = synth.make_structure(cfg, rng)
        N, C, K = prob["n_nodes"], prob["n_cond"], len(prob["obs_t"])
        # observe every node first, to measure activity under the hidden vector
        tmp = dict(prob, obs_n=np.arange(N, dtype=np.int32),
                   observed=np.zeros((C, K, N), dtype=np.int8))
        traj = OracleProblem(tmp).simulate(prob["hidden"])          # [C][T+1][N]
        activity = (np.diff(traj.astype(np.int64), axis=1) != 0).sum(axis=(0, 1))
        obs_n = synth.choose_observed(rng, activity, cfg["n_obs"])
        clean = traj[:, prob["obs_t"], :][:, :, obs_n].astype(np.int8)  # [C][K][O]
        observed = synth.add_noise(rng, clean, cfg["noise"]) if cfg["noise"] > 0 else clean.copy()
        prob.update(obs_n=obs_n, observed=observed, clean=clean, attempt=np.int64(attempt))
        frac = np.count_nonzero(clean) / clean.size
        if frac >= min_nonzero:
            return prob
        if best is None or frac > best[0]:
            best = (frac, prob)
    print(f"{name}: no draw reached {min_nonzero:.0%} non-zero entries; keeping the best ({best[0]:.0%})")
    return best[1]


def make_batch() -> list:
    """The batched workload: every network drawn like the single workloads,
    from its own sizes and seed (network i: seed 4000 + i)."""
    probs = []
    for i in range(synth.BATCH["n_networks"]):
        cfg = synth.batch_network_config(i)
        probs.append(make(f"c4[{i}]", cfg, cfg["seed"]))
    return probs


def main(names):
    os.makedirs(synth.DATA_DIR, exist_ok=True)
    for name in names:
        if name == "c4":
            probs = make_batch()
            path = os.path.join(synth.DATA_DIR, "c4.npz")
            synth.save_batch(path, probs)
            P = [p["n_nodes"] + p["n_edges"] for p in probs]
            print(f"c4: {len(probs)} networks, N {min(p['n_nodes'] for p in probs)}-{max(p['n_nodes'] for p in probs)}, "
                  f"P {min(P)}-{max(P)}, C {min(p['n_cond'] for p in probs)}-{max(p['n_cond'] for p in probs)} -> {path}")
            continue
        prob = make(name)
        path = os.path.join(synth.DATA_DIR, f"{name}.npz")
        synth.save_problem(path, prob)
        n_params = OracleProblem(prob).n_params
        print(f"{name}: model={prob['model']} N={prob['n_nodes']} E={prob['n_edges']} P={n_params} "
              f"C={prob['n_cond']} K={len(prob['obs_t'])} O={len(prob['obs_n'])} "
              f"max_indeg={int(np.diff(prob['row_ptr']).max())} -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c3", "c4"])
