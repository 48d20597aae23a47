"""Small problem builders shared by the tests (no model arithmetic: the
reference data of a generated problem come from the oracle)."""
from __future__ import annotations

import json
import os

import numpy as np

from paper_2506_19866_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def from_edges(n_nodes, edges_src_dst, *, init, clamp=None, n_steps=5, obs_t=(1,), obs_n=(0,),
               observed=None, step_size=1, hard=1, penalty=0, model=0):
    """Problem dict from an explicit edge list (one condition per row of init).
    Returns (prob, perm) where perm[k] is the index of the k-th given edge in
    the canonical (target-grouped) parameter order."""
    row_ptr, src = synth._to_csr(n_nodes, [(j, i) for j, i in edges_src_dst])
    order = sorted(range(len(edges_src_dst)), key=lambda k: (edges_src_dst[k][1], edges_src_dst[k][0]))
    perm = np.empty(len(edges_src_dst), dtype=np.int64)
    for pos, k in enumerate(order):
        perm[k] = pos
    init = np.atleast_2d(np.asarray(init, dtype=np.int8))
    C = init.shape[0]
    clamp = np.full_like(init, -1) if clamp is None else np.atleast_2d(np.asarray(clamp, dtype=np.int8))
    obs_t = np.asarray(obs_t, dtype=np.int32)
    obs_n = np.asarray(obs_n, dtype=np.int32)
    if observed is None:
        observed = np.zeros((C, len(obs_t), len(obs_n)), dtype=np.int8)
    prob = dict(n_nodes=n_nodes, n_edges=len(src), row_ptr=row_ptr, src=src, n_cond=C,
                init=init, clamp=clamp, n_steps=n_steps, obs_t=obs_t, obs_n=obs_n,
                observed=np.asarray(observed, dtype=np.int8).reshape(C, len(obs_t), len(obs_n)),
                step_size=step_size, hard=hard, penalty=penalty, model=model)
    return prob, perm


def random_problem(seed, *, n_nodes, n_edges, n_cond, n_steps, n_times, n_obs, noise=0.0,
                   clamps=(1, 1), step_size=1, hard=1, topology="cycle_plus_uniform", clamp_values=(0, 2)):
    """A seeded random problem whose reference data are the oracle trajectories
    of a hidden feasible vector (plus optional noise).  Returns (prob, hidden)."""
    from oracle.oracle import OracleProblem
    rng = synth.rng_for(seed)
    if topology == "cycle_plus_uniform":
        row_ptr, src = synth.topology_cycle_plus_uniform(rng, n_nodes, n_edges)
    elif topology == "preferential":
        row_ptr, src = synth.topology_preferential(rng, n_nodes, n_edges)
    else:
        row_ptr, src = synth.topology_bounded_indegree(rng, n_nodes, n_edges)
    hidden = synth.feasible_params(rng, 1, row_ptr, src)[0]
    init, clamp = synth.conditions(rng, n_nodes, n_cond, clamps, clamp_values)
    obs_t = synth.observation_times(n_steps, n_times)
    obs_n = np.sort(rng.choice(n_nodes, size=n_obs, replace=False)).astype(np.int32)
    prob = dict(n_nodes=n_nodes, n_edges=n_edges, row_ptr=row_ptr, src=src, n_cond=n_cond,
                init=init, clamp=clamp, n_steps=n_steps, obs_t=obs_t, obs_n=obs_n,
                observed=np.zeros((n_cond, n_times, n_obs), dtype=np.int8),
                step_size=step_size, hard=hard, penalty=0)
    traj = OracleProblem(prob).simulate(hidden)
    clean = traj[:, obs_t, :][:, :, obs_n].astype(np.int8)
    prob["observed"] = synth.add_noise(rng, clean, noise) if noise > 0 else clean
    return prob, hidden


def priority_problem(seed, *, n_nodes, n_edges, n_cond, n_steps, n_obs, obs_t=None, noise=0.0, clamps=(0, 0),
                     hard=1, topology="cycle_plus_uniform"):
    """A seeded random problem of the priority-update model whose reference
    data are the oracle trajectories of a hidden feasible vector (every time
    point observed unless obs_t is given).  Returns (prob, hidden)."""
    from oracle.oracle import OracleProblem
    rng = synth.rng_for(seed)
    if topology == "cycle_plus_uniform":
        row_ptr, src = synth.topology_cycle_plus_uniform(rng, n_nodes, n_edges)
    else:
        row_ptr, src = synth.topology_bounded_indegree(rng, n_nodes, n_edges)
    hidden = synth.priority_feasible_params(rng, 1, row_ptr, src)[0]
    init, clamp = synth.conditions(rng, n_nodes, n_cond, clamps)
    obs_t = np.arange(n_steps + 1, dtype=np.int32) if obs_t is None else np.asarray(obs_t, dtype=np.int32)
    obs_n = np.sort(rng.choice(n_nodes, size=n_obs, replace=False)).astype(np.int32)
    prob = dict(n_nodes=n_nodes, n_edges=n_edges, row_ptr=row_ptr, src=src, n_cond=n_cond,
                init=init, clamp=clamp, n_steps=n_steps, obs_t=obs_t, obs_n=obs_n,
                observed=np.zeros((n_cond, len(obs_t), n_obs), dtype=np.int8),
                step_size=1, hard=hard, penalty=0, model=synth.MODEL_PRIORITY)
    traj = OracleProblem(prob).simulate(hidden)
    clean = traj[:, obs_t, :][:, :, obs_n].astype(np.int8)
    prob["observed"] = synth.add_noise(rng, clean, noise) if noise > 0 else clean
    return prob, hidden
