"""Seeded synthetic inputs: network topologies, parameter vectors, experimental
conditions, observation designs and observation noise.

This module holds none of the method's arithmetic: it never simulates a
trajectory, scores a vector or tests a constraint.  Vectors that must satisfy
the structural constraints of §2.5.3 are feasible by construction (one
designated activating in-edge and one designated non-zero out-edge per node).
The reference data of a workload come from simulating hidden parameters; that
step is not here (it is done once, offline, by the oracle, and the results are
stored under ``data/``).

Shapes follow the paper's workloads (§2.5): sparse directed networks where
every node is both regulated and regulating, ternary states, a few observed
time points on a subset of nodes that favours dynamic ones, and an observation
matrix that includes noise where the paper's data were experimental.

Problem dict layout (all integer numpy arrays, C-contiguous):
    n_nodes N, n_edges E, row_ptr int32[N+1], src int32[E]  (in-edges grouped
    by target ascending, sources ascending within a target: the canonical
    parameter order), n_cond C, init int8[C,N], clamp int8[C,N] (-1 free),
    n_steps T_s, obs_t int32[K], obs_n int32[O], observed int8[C,K,O],
    step_size d, hard (1/0), penalty (0 = default lambda).
"""
from __future__ import annotations

import os

import numpy as np

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------------------
# topologies
# ---------------------------------------------------------------------------
def _to_csr(n_nodes: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """(src, dst) pairs -> (row_ptr, src) grouped by target, sorted by source."""
    edges = sorted({(int(j), int(i)) for j, i in edges}, key=lambda e: (e[1], e[0]))
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int32)
    for _, i in edges:
        row_ptr[i + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    src = np.array([j for j, _ in edges], dtype=np.int32)
    return row_ptr, src


def _covered(n_nodes: int, edges) -> bool:
    outs = {j for j, _ in edges}
    ins = {i for _, i in edges}
    return len(outs) == n_nodes and len(ins) == n_nodes


def topology_bounded_indegree(rng, n_nodes: int, n_edges: int, degrees=(1, 2, 3)):
    """Each node draws an in-degree uniformly from ``degrees``, conditioned on
    the total being ``n_edges``; sources are distinct and never the target.
    Redrawn until every node also has an out-edge."""
    while True:
        deg = rng.choice(np.asarray(degrees), size=n_nodes)
        if int(deg.sum()) != n_edges:
            continue
        edges = []
        for i in range(n_nodes):
            others = np.array([j for j in range(n_nodes) if j != i])
            for j in rng.choice(others, size=int(deg[i]), replace=False):
                edges.append((int(j), i))
        if _covered(n_nodes, edges):
            return _to_csr(n_nodes, edges)


def topology_cycle_plus_uniform(rng, n_nodes: int, n_edges: int):
    """A random directed cycle through all nodes (so every node regulates and
    is regulated), then uniformly random distinct non-self edges."""
    assert n_nodes <= n_edges <= n_nodes * (n_nodes - 1)
    perm = rng.permutation(n_nodes)
    edges = {(int(perm[k]), int(perm[(k + 1) % n_nodes])) for k in range(n_nodes)}
    while len(edges) < n_edges:
        j, i = (int(v) for v in rng.integers(0, n_nodes, size=2))
        if j != i:
            edges.add((j, i))
    return _to_csr(n_nodes, edges)


def topology_preferential(rng, n_nodes: int, n_edges: int):
    """Scale-free regulators: a random cycle for coverage, then each further
    edge picks a uniform target and a source with probability proportional to
    (out-degree + 1), i.e. directed preferential attachment on regulators."""
    assert n_nodes <= n_edges <= n_nodes * (n_nodes - 1)
    perm = rng.permutation(n_nodes)
    edges = {(int(perm[k]), int(perm[(k + 1) % n_nodes])) for k in range(n_nodes)}
    outdeg = np.ones(n_nodes, dtype=np.float64)
    for j, _ in edges:
        outdeg[j] += 1
    while len(edges) < n_edges:
        i = int(rng.integers(0, n_nodes))
        j = int(rng.choice(n_nodes, p=outdeg / outdeg.sum()))
        if j != i and (j, i) not in edges:
            edges.add((j, i))
            outdeg[j] += 1
    return _to_csr(n_nodes, edges)


# ---------------------------------------------------------------------------
# parameter vectors
# ---------------------------------------------------------------------------
def random_params(rng, n: int, n_edges: int, n_nodes: int) -> np.ndarray:
    """Arbitrary vectors (constraints not enforced): a in {-1,0,1}, theta in {0,1,2}."""
    x = rng.integers(0, 3, size=(n, n_edges + n_nodes), dtype=np.int8)
    x[:, :n_edges] -= 1
    return x


def feasible_params(rng, n: int, row_ptr: np.ndarray, src: np.ndarray) -> np.ndarray:
    """Vectors that satisfy both structural constraints of §2.5.3 by
    construction: uniform a and theta, then for every node one uniformly chosen
    out-edge gets a random non-zero sign and one uniformly chosen in-edge gets
    +1 (in-edge choices are applied last; +1 is non-zero, so an edge chosen
    both ways keeps both properties)."""
    row_ptr = np.asarray(row_ptr)
    src = np.asarray(src)
    N = len(row_ptr) - 1
    E = len(src)
    x = random_params(rng, n, E, N)
    rows = np.arange(n)
    out_lists = [np.flatnonzero(src == v) for v in range(N)]
    for v in range(N):
        outs = out_lists[v]
        if len(outs) == 0:
            raise ValueError(f"node {v} has no out-edge: no feasible vector exists")
        pick = outs[rng.integers(0, len(outs), size=n)]
        x[rows, pick] = rng.choice(np.array([-1, 1], dtype=np.int8), size=n)
    for v in range(N):
        lo, hi = int(row_ptr[v]), int(row_ptr[v + 1])
        if hi == lo:
            raise ValueError(f"node {v} has no in-edge: no feasible vector exists")
        x[rows, rng.integers(lo, hi, size=n)] = 1
    return x


# Parameters of the paper's own model with the priority update (§2.1, §2.2):
# x = [w_e] ++ [p_e] ++ [t_e] ++ [u_i] ++ [m_i] ++ [d_i], P = 3E + 3N.
MODEL_SYNCHRONOUS, MODEL_PRIORITY = 0, 1
SPEEDS_SLOW = (1, 2, 3, 4, 5, 6)
SPEEDS_FAST = (10, 11, 12)


def priority_random_params(rng, n: int, n_edges: int, n_nodes: int, fast_fraction: float = 1.0 / 3.0) -> np.ndarray:
    """Arbitrary priority-model vectors (constraints not enforced): w in
    {0,1,2}, p in {-1,0,1}, t in {1,2}; per node a slow or (with probability
    fast_fraction, one third as in §2.5.2) fast speed u, memory m in {0,1,2}
    and step size d in {1,2}."""
    E, N = n_edges, n_nodes
    x = np.empty((n, 3 * E + 3 * N), dtype=np.int8)
    x[:, :E] = rng.integers(0, 3, size=(n, E))
    x[:, E:2 * E] = rng.integers(-1, 2, size=(n, E))
    x[:, 2 * E:3 * E] = rng.integers(1, 3, size=(n, E))
    fast = rng.random((n, N)) < fast_fraction
    x[:, 3 * E:3 * E + N] = np.where(fast, rng.choice(np.array(SPEEDS_FAST, dtype=np.int8), size=(n, N)),
                                     rng.choice(np.array(SPEEDS_SLOW, dtype=np.int8), size=(n, N)))
    x[:, 3 * E + N:3 * E + 2 * N] = rng.integers(0, 3, size=(n, N))
    x[:, 3 * E + 2 * N:] = rng.integers(1, 3, size=(n, N))
    return x


def priority_feasible_params(rng, n: int, row_ptr: np.ndarray, src: np.ndarray) -> np.ndarray:
    """Priority-model vectors that satisfy §2.5.3 by construction: for every
    node one uniformly chosen out-edge gets w in {1,2} and one uniformly chosen
    in-edge gets w in {1,2} and p = +1 (a non-zero w keeps the out-edge
    property of an edge chosen both ways)."""
    row_ptr = np.asarray(row_ptr)
    src = np.asarray(src)
    N = len(row_ptr) - 1
    E = len(src)
    x = priority_random_params(rng, n, E, N)
    rows = np.arange(n)
    for v in range(N):
        outs = np.flatnonzero(src == v)
        if len(outs) == 0:
            raise ValueError(f"node {v} has no out-edge: no feasible vector exists")
        x[rows, outs[rng.integers(0, len(outs), size=n)]] = rng.integers(1, 3, size=n)
    for v in range(N):
        lo, hi = int(row_ptr[v]), int(row_ptr[v + 1])
        if hi == lo:
            raise ValueError(f"node {v} has no in-edge: no feasible vector exists")
        pick = rng.integers(lo, hi, size=n)
        x[rows, pick] = rng.integers(1, 3, size=n)
        x[rows, E + pick] = 1
    return x


# ---------------------------------------------------------------------------
# experimental design
# ---------------------------------------------------------------------------
def conditions(rng, n_nodes: int, n_cond: int, clamps_per_cond=(1, 1), clamp_values=(0, 2)):
    """Initial states uniform in {0,1,2}; each condition clamps a uniformly
    drawn number (in the inclusive range ``clamps_per_cond``) of distinct nodes
    to a value drawn from ``clamp_values`` (a perturbation: knock-down or
    over-expression)."""
    init = rng.integers(0, 3, size=(n_cond, n_nodes), dtype=np.int8)
    clamp = np.full((n_cond, n_nodes), -1, dtype=np.int8)
    lo, hi = clamps_per_cond
    for c in range(n_cond):
        k = int(rng.integers(lo, hi + 1))
        nodes = rng.choice(n_nodes, size=k, replace=False)
        clamp[c, nodes] = rng.choice(np.asarray(clamp_values, dtype=np.int8), size=k)
    return init, clamp


def observation_times(n_steps: int, n_times: int) -> np.ndarray:
    """Evenly spread observed steps floor(k*T_s/K), k = 1..K."""
    return np.array([(k * n_steps) // n_times for k in range(1, n_times + 1)], dtype=np.int32)


def choose_observed(rng, activity: np.ndarray, n_obs: int) -> np.ndarray:
    """Observed nodes without replacement, with probability proportional to
    1 + activity (the paper prefers nodes with a more dynamic time course,
    §2.5.2); returned sorted."""
    w = 1.0 + np.asarray(activity, dtype=np.float64)
    picked = rng.choice(len(w), size=n_obs, replace=False, p=w / w.sum())
    return np.sort(picked).astype(np.int32)


def add_noise(rng, observed: np.ndarray, fraction: float) -> np.ndarray:
    """Flips exactly round(fraction * size) entries, chosen by a seeded
    permutation, each to one of the two other levels uniformly."""
    flat = observed.reshape(-1).copy()
    n_flip = int(round(fraction * flat.size))
    where = rng.permutation(flat.size)[:n_flip]
    shift = rng.integers(1, 3, size=n_flip)
    flat[where] = ((flat[where].astype(np.int64) + shift) % 3).astype(np.int8)
    return flat.reshape(observed.shape)


# ---------------------------------------------------------------------------
# workload recipes (sizes of the paper's two networks, §2.5, scaled as the
# configurations below state)
# ---------------------------------------------------------------------------
CONFIGS = {
    # 12 nodes, 28 edges, 40 parameters; tiny enough for full oracle runs
    "c1": dict(n_nodes=12, n_edges=28, topology="bounded_indegree", n_cond=4, clamps=(1, 1),
               n_steps=10, n_times=3, n_obs=6, noise=0.0,
               chains=64, stages=100, steps_per_stage=100, T0=2.0, T_end=0.01),
    # HPG scale: 102 parameters (paper §2.5.1)
    "c2": dict(n_nodes=20, n_edges=82, topology="cycle_plus_uniform", n_cond=8, clamps=(1, 1),
               n_steps=15, n_times=4, n_obs=10, noise=0.10,
               chains=4096, stages=100, steps_per_stage=500, T0=2.0, T_end=0.01),
    # Mtb scale: 723 parameters (paper §2.5.2)
    "c3": dict(n_nodes=120, n_edges=603, topology="preferential", n_cond=16, clamps=(1, 3),
               n_steps=20, n_times=5, n_obs=40, noise=0.05,
               chains=16384, stages=200, steps_per_stage=500, T0=2.0, T_end=0.01),
}


# The paper's own model (priority update, P = 3E + 3N) at the sizes of its two
# networks (§2.5): one condition, 20 time points including the initial state,
# every one observed.
PRIORITY_CONFIGS = {
    # tiny: 6 nodes, 12 edges, 54 parameters
    "q1": dict(model=MODEL_PRIORITY, n_nodes=6, n_edges=12, topology="bounded_indegree", n_cond=2, clamps=(0, 0),
               n_steps=10, n_obs=4, noise=0.0,
               chains=64, stages=60, steps_per_stage=100, T0=2.0, T_end=0.01),
    # HPG axis: 9 nodes, 25 edges, 102 parameters, 5 observed nodes (§2.5.1)
    "q2": dict(model=MODEL_PRIORITY, n_nodes=9, n_edges=25, topology="cycle_plus_uniform", n_cond=1, clamps=(0, 0),
               n_steps=19, n_obs=5, noise=0.10,
               chains=4096, stages=100, steps_per_stage=500, T0=2.0, T_end=0.01),
    # Mtb host-pathogen: 63 nodes, 178 edges, 723 parameters, 35 observed nodes (§2.5.2)
    "q3": dict(model=MODEL_PRIORITY, n_nodes=63, n_edges=178, topology="cycle_plus_uniform", n_cond=1, clamps=(0, 0),
               n_steps=19, n_obs=35, noise=0.0,
               chains=16384, stages=200, steps_per_stage=500, T0=2.0, T_end=0.01),
}


# Batched uneven workload: 256 independent networks of 10-150 nodes, each with
# its own conditions and data, 256 chains per network in one persistent launch.
BATCH = dict(name="c4", n_networks=256, nodes=(10, 150), mean_indegree=(2.0, 5.0), conditions=(4, 16),
             steps=(10, 20), times=(3, 5), clamps=(1, 2), noise=0.05,
             chains=256, stages=100, steps_per_stage=200, T0=2.0, T_end=0.01)


def batch_network_config(i: int) -> dict:
    """Sizes of network i of the batched workload (seed 4000 + i)."""
    rng = rng_for(4000 + i)
    N = int(rng.integers(BATCH["nodes"][0], BATCH["nodes"][1] + 1))
    k = float(rng.uniform(*BATCH["mean_indegree"]))
    C = int(rng.integers(BATCH["conditions"][0], BATCH["conditions"][1] + 1))
    T = int(rng.integers(BATCH["steps"][0], BATCH["steps"][1] + 1))
    K = int(rng.integers(BATCH["times"][0], BATCH["times"][1] + 1))
    return dict(n_nodes=N, n_edges=int(round(k * N)), topology="cycle_plus_uniform", n_cond=C,
                clamps=BATCH["clamps"], n_steps=T, n_times=K, n_obs=-(-N // 3), noise=BATCH["noise"],
                seed=4000 + i, min_nonzero=0.15)


def load_batch(name: str = "c4") -> list:
    """The stored batched workload as a list of problem dicts."""
    path = os.path.join(DATA_DIR, f"{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        files = {k: z[k] for k in z.files}
    n = int(files["n_networks"])
    out = []
    for i in range(n):
        pre = f"n{i}_"
        prob = {k[len(pre):]: v for k, v in files.items() if k.startswith(pre)}
        for k in _INT_KEYS:
            prob[k] = int(prob[k]) if k in prob else 0
        out.append(prob)
    return out


def save_batch(path: str, probs: list) -> None:
    arrays = {"n_networks": np.int64(len(probs))}
    for i, prob in enumerate(probs):
        for k, v in prob.items():
            arrays[f"n{i}_{k}"] = np.int64(v) if k in _INT_KEYS else np.asarray(v)
    np.savez_compressed(path, **arrays)


def batch_start_vectors(probs: list, n_chains: int) -> list:
    """Per-network starting vectors of the batched workload (feasible)."""
    return [feasible_params(rng_for(6000 + i), n_chains, p["row_ptr"], p["src"]) for i, p in enumerate(probs)]


def batch_schedule() -> dict:
    return dict(n_chains=BATCH["chains"], n_stages=BATCH["stages"], steps_per_stage=BATCH["steps_per_stage"],
                T0=BATCH["T0"], rho=cooling_factor(BATCH["T0"], BATCH["T_end"], BATCH["stages"]), seed=2004)


def problem_seed(name: str) -> int:
    return (1100 if name.startswith("q") else 1000) + int(name[1:])


def run_seed(name: str) -> int:
    return (2100 if name.startswith("q") else 2000) + int(name[1:])


def config(name: str) -> dict:
    return PRIORITY_CONFIGS[name] if name in PRIORITY_CONFIGS else CONFIGS[name]


def cooling_factor(T0: float, T_end: float, n_stages: int) -> float:
    """rho such that stage n_stages-1 is at T_end (configs give T0 -> T_end)."""
    if n_stages <= 1:
        return 1.0
    return float((T_end / T0) ** (1.0 / (n_stages - 1)))


def make_structure(cfg: dict, rng) -> dict:
    """Everything of a workload except the reference data: topology, hidden
    parameters, conditions and observed times."""
    N, E = cfg["n_nodes"], cfg["n_edges"]
    topo = cfg["topology"]
    if topo == "bounded_indegree":
        row_ptr, src = topology_bounded_indegree(rng, N, E)
    elif topo == "cycle_plus_uniform":
        row_ptr, src = topology_cycle_plus_uniform(rng, N, E)
    elif topo == "preferential":
        row_ptr, src = topology_preferential(rng, N, E)
    else:
        raise ValueError(topo)
    priority = cfg.get("model", MODEL_SYNCHRONOUS) == MODEL_PRIORITY
    hidden = (priority_feasible_params if priority else feasible_params)(rng, 1, row_ptr, src)[0]
    init, clamp = conditions(rng, N, cfg["n_cond"], cfg["clamps"])
    if priority:  # every time point observed, the initial state included (§2.5)
        obs_t = np.arange(cfg["n_steps"] + 1, dtype=np.int32)
    else:
        obs_t = observation_times(cfg["n_steps"], cfg["n_times"])
    return dict(n_nodes=N, n_edges=E, row_ptr=row_ptr, src=src, n_cond=cfg["n_cond"],
                init=init, clamp=clamp, n_steps=cfg["n_steps"], obs_t=obs_t,
                step_size=1, hard=1, penalty=0, model=MODEL_PRIORITY if priority else MODEL_SYNCHRONOUS,
                hidden=hidden)


# ---------------------------------------------------------------------------
# stored workloads
# ---------------------------------------------------------------------------
_INT_KEYS = ("n_nodes", "n_edges", "n_cond", "n_steps", "step_size", "hard", "penalty", "model")


def save_problem(path: str, prob: dict) -> None:
    arrays = {k: np.asarray(v) for k, v in prob.items() if k not in _INT_KEYS}
    scalars = {k: np.int64(prob[k]) for k in _INT_KEYS}
    np.savez_compressed(path, **arrays, **scalars)


def load_problem(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    for k in _INT_KEYS:
        out[k] = int(out[k]) if k in out else 0  # files written before "model" existed: model 0
    return out


def load_workload(name: str) -> dict:
    """A stored workload ('c1', 'c2', 'c3'): problem dict plus 'hidden' (the
    generating parameters) and 'clean' (noise-free reference data)."""
    return load_problem(os.path.join(DATA_DIR, f"{name}.npz"))


def start_vectors(name: str, prob: dict, n_chains: int) -> np.ndarray:
    """Per-chain starting vectors of a workload's runs (feasible)."""
    gen = priority_feasible_params if prob.get("model", 0) == MODEL_PRIORITY else feasible_params
    return gen(rng_for(run_seed(name) + 7), n_chains, prob["row_ptr"], prob["src"])


def bench_schedule(name: str) -> dict:
    cfg = config(name)
    return dict(n_chains=cfg["chains"], n_stages=cfg["stages"],
                steps_per_stage=cfg["steps_per_stage"], T0=cfg["T0"],
                rho=cooling_factor(cfg["T0"], cfg["T_end"], cfg["stages"]), seed=run_seed(name))


def n_flips(cfg: dict) -> int:
    n_times = cfg["n_steps"] + 1 if cfg.get("model", MODEL_SYNCHRONOUS) == MODEL_PRIORITY else cfg["n_times"]
    n = cfg["n_cond"] * n_times * cfg["n_obs"]
    return int(round(cfg["noise"] * n))


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)

