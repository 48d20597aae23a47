"""The learned proposal, stated plainly: move features, the network's scores,
the integer sampling table, and a serial annealing run that draws its
candidates from that table.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH: the GPU's refresh (feature
simulation, features, network, table) and its learned annealing steps are
checked against these definitions.  Everything here is plain Python / numpy
plus the C oracle's Simulate, Cost and Philox; nothing is shared with the GPU
library.

This is an extension beyond the paper.  Table 1's GetCandidate changes one
uniformly drawn parameter to one of its two other values; the learned
proposal draws the (parameter, new value) pair from a distribution scored by
a small network, refreshed every R steps from the chain's current vector.
Everything after the candidate is drawn -- the structural constraints of
§2.5.3, the full Simulate of §2.2, the score of §2.3, Metropolis and the stage
restart of Table 1 -- is the plain method, unchanged, so the exact integer
cost decides every step (no Hastings correction: SA is used as an optimizer).

Definitions (all values are float32 computed in the order written; the
network's inputs are then rounded to bfloat16, nearest-even):

Refresh of a chain at vector x, stage temperature T:
  S = Simulate(x) at the observed times, all conditions, all nodes.
  per node i:  SS_i = sum_{c,k} S_c(t_k)[i];  msh_i = f32(SS_i) / f32(2 C K)
  per observed node i (observation index o):
      SW_i = sum_{c,k} W,  WR_i = sum W R,  WS_i = sum W S,  WA_i = sum W |S - R|
      eh_i = f32(WR_i - WS_i) / f32(2 SW_i),  ah_i = f32(WA_i) / f32(2 SW_i)
  unobserved nodes: eh = ah = 0
  mn = f32(M(x)) / f32(sum of all W);   lt = f32(ln(T) / 5)   (ln in double)

Features of the move (p -> v), old = x[p], for an edge p = (j -> i) or the
threshold of node i (p = E + i):
  f0..f2  one-hot code(old)         f3..f5  one-hot code(v)
  f6      1 for a threshold          f7  e = (v - old)/2 (edge), (old - v)/2 (threshold)
  f8      node i observed            f9  eh_i            f10  ah_i
  f11     msh_j (edge)               f12 msh_i
  f13     e * eh_i                   f14 (e * msh_j) * eh_i (edge), f13 (threshold)
  f15     node j observed (edge)     f16 eh_j (edge)
  f17     in-degree(i) / 8           f18 out-degree(j) / 8 (edge)
  f19     lt                         f20 mn
  f21     1 if the move raises V (a node loses its last non-zero out-edge or
          its last +1 in-edge)
  f22     (+1 in-edges of i) / 8     f23 (non-zero out-edges of j) / 8 (edge)
  f24..f30  0                        f31 1 (carries the hidden bias)
  Edge-only features are 0 for a threshold.

Network (bf16 weights, float32 accumulation on the GPU):
  z_h = sum_k bf16(W1[k][h]) * bf16(f_k);  a_h = bf16(max(z_h, 0))
  logit = sum_h bf16(w2[h]) * a_h + b2
Table: rows m = 0..2P-1 are the moves (p = m // 2, new code =
  (code(x[p]) + 1 + m % 2) mod 3); a move is masked in HARD mode when f21 = 1.
  weight_m = floor(exp(logit_m - max over unmasked logits) * 65536), 0 if
  masked; cum = inclusive prefix sums (uint32).

Step of the learned run (Philox block (u0..u3) of the plain method):
  if the table is used, (u3 >> 32) >= eps_u32 and total = cum[-1] > 0:
      r = ((u0 >> 32) * total) >> 32; m = first index with cum[m] > r;
      the move (p, v) is row m of the table as built at the refresh; if x[p]
      already equals v (the chain moved since the refresh) the plain
      candidate is used instead (source 2), else the move is used (source 1)
  otherwise the plain candidate (source 0; source 3 when the table was
  empty).  The plain candidate is GetCandidate of Table 1 from u0, u1.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import mlp_reference
from oracle.oracle import OracleProblem, draw, stage_temperature, threshold
from oracle.reference import weights

N_FEATURES = 32
TABLE_SCALE = 65536
SOURCE_PLAIN, SOURCE_LEARNED, SOURCE_STALE, SOURCE_EMPTY = 0, 1, 2, 3
f32 = np.float32


def eps_threshold(eps: float) -> int:
    """u3's top 32 bits below this value select the plain candidate."""
    return min(int(math.floor(eps * 4294967296.0)), 4294967295) if eps < 1.0 else 4294967296


def edge_list(prob):
    row_ptr = np.asarray(prob["row_ptr"], dtype=np.int64)
    src = np.asarray(prob["src"], dtype=np.int64)
    dst = np.repeat(np.arange(int(prob["n_nodes"])), np.diff(row_ptr))
    return src, dst


def code(p: int, E: int, val: int) -> int:
    return val + 1 if p < E else val


def value(p: int, E: int, c: int) -> int:
    return c - 1 if p < E else c


def refresh_state(prob, x, T: float) -> dict:
    """Per-node aggregates of the vector x (refresh definitions above)."""
    N, E = int(prob["n_nodes"]), int(prob["n_edges"])
    C = int(prob["n_cond"])
    obs_t = np.asarray(prob["obs_t"], dtype=np.int64)
    obs_n = np.asarray(prob["obs_n"], dtype=np.int64)
    K, O = len(obs_t), len(obs_n)
    traj = OracleProblem(prob).simulate(x).astype(np.int64)          # [C][T+1][N]
    S = traj[:, obs_t, :]                                            # [C][K][N]
    R = np.asarray(prob["observed"], dtype=np.int64).reshape(C, K, O)
    W = np.asarray(weights(prob), dtype=np.int64)                    # [C][K][O]
    SS = S.sum(axis=(0, 1))
    msh = np.array([f32(SS[i]) / f32(2 * C * K) for i in range(N)], dtype=np.float32)
    eh = np.zeros(N, dtype=np.float32)
    ah = np.zeros(N, dtype=np.float32)
    observed = np.zeros(N, dtype=bool)
    So = S[:, :, obs_n]
    M = 0
    for o in range(O):
        i = int(obs_n[o])
        sw = int(W[:, :, o].sum())
        wr = int((W[:, :, o] * R[:, :, o]).sum())
        ws = int((W[:, :, o] * So[:, :, o]).sum())
        wa = int((W[:, :, o] * np.abs(So[:, :, o] - R[:, :, o])).sum())
        M += wa
        observed[i] = True
        eh[i] = f32(wr - ws) / f32(2 * sw)
        ah[i] = f32(wa) / f32(2 * sw)
    src, dst = edge_list(prob)
    a = np.asarray(x[:E], dtype=np.int64)
    ip = np.bincount(dst[a == 1], minlength=N)
    on = np.bincount(src[a != 0], minlength=N)
    return {"msh": msh, "eh": eh, "ah": ah, "observed": observed,
            "mn": f32(M) / f32(int(W.sum())), "lt": f32(math.log(T) / 5.0),
            "mismatch": M, "x": np.array(x, dtype=np.int8, copy=True), "ip": ip, "on": on}


def counts(prob, x):
    N, E = int(prob["n_nodes"]), int(prob["n_edges"])
    src, dst = edge_list(prob)
    a = np.asarray(x[:E], dtype=np.int64)
    return np.bincount(dst[a == 1], minlength=N).tolist(), np.bincount(src[a != 0], minlength=N).tolist()


def statics(prob) -> dict:
    """Per-problem constants the features read: edge endpoints and degrees."""
    N = int(prob["n_nodes"])
    src, dst = edge_list(prob)
    return {"src": src.tolist(), "dst": dst.tolist(), "E": int(prob["n_edges"]),
            "indeg": np.diff(np.asarray(prob["row_ptr"], dtype=np.int64)).tolist(),
            "outdeg": np.bincount(src, minlength=N).tolist()}


def raises_violations(prob, p: int, old: int, v: int, ip, on, st=None) -> bool:
    st = st or statics(prob)
    if p >= st["E"]:
        return False
    j, i = st["src"][p], st["dst"][p]
    on_new = on[j] + (v != 0) - (old != 0)
    ip_new = ip[i] + (v == 1) - (old == 1)
    return (on_new == 0 and on[j] > 0) or (ip_new == 0 and ip[i] > 0)


def move_features(prob, p: int, old: int, v: int, agg: dict, ip, on, lt, st=None) -> np.ndarray:
    """The 32 float32 features of the move p: old -> v (definitions above)."""
    st = st or statics(prob)
    E, src, dst, indeg, outdeg = st["E"], st["src"], st["dst"], st["indeg"], st["outdeg"]
    f = np.zeros(N_FEATURES, dtype=np.float32)
    edge = p < E
    i = dst[p] if edge else p - E
    j = src[p] if edge else -1
    f[code(p, E, old)] = 1
    f[3 + code(p, E, v)] = 1
    f[6] = 0 if edge else 1
    e = f32(v - old) / f32(2) if edge else f32(old - v) / f32(2)
    f[7] = e
    f[8] = 1 if agg["observed"][i] else 0
    f[9] = agg["eh"][i]
    f[10] = agg["ah"][i]
    f[12] = agg["msh"][i]
    f[13] = e * agg["eh"][i]
    f[14] = f[13]
    if edge:
        f[11] = agg["msh"][j]
        f[14] = (e * agg["msh"][j]) * agg["eh"][i]
        f[15] = 1 if agg["observed"][j] else 0
        f[16] = agg["eh"][j]
        f[18] = f32(outdeg[j]) / f32(8)
        f[23] = f32(on[j]) / f32(8)
    f[17] = f32(indeg[i]) / f32(8)
    f[19] = lt
    f[20] = agg["mn"]
    f[21] = 1 if raises_violations(prob, p, old, v, ip, on, st) else 0
    f[22] = f32(ip[i]) / f32(8)
    f[31] = 1
    return f


def table_moves(prob, x):
    """(p, old, v) of the 2P table rows for the vector x."""
    E = int(prob["n_edges"])
    P = len(x)
    out = []
    for m in range(2 * P):
        p = m // 2
        old = int(x[p])
        out.append((p, old, value(p, E, (code(p, E, old) + 1 + m % 2) % 3)))
    return out


def logits(model: dict, X) -> np.ndarray:
    """The network's scores of feature rows X [n][32] (float64 arithmetic on
    the bf16-rounded inputs, hidden activations rounded to bf16)."""
    Xb = mlp_reference.bf16(X)
    W1 = mlp_reference.bf16(model["W1"])
    w2 = mlp_reference.bf16(model["w2"])
    a = mlp_reference.bf16(np.maximum(Xb @ W1, 0.0))
    return a @ w2 + float(np.float32(model["b2"]))


def proposal_table(prob, x, T: float, model: dict) -> dict:
    """Features, scores and integer table of the refresh at x."""
    agg = refresh_state(prob, x, T)
    hard = int(prob.get("hard", 1)) != 0
    moves = table_moves(prob, x)
    st = statics(prob)
    X = np.stack([move_features(prob, p, old, v, agg, agg["ip"], agg["on"], agg["lt"], st) for p, old, v in moves])
    lg = logits(model, X)
    masked = (X[:, 21] != 0) & hard
    w = np.zeros(len(moves), dtype=np.uint64)
    if (~masked).any():
        lmax = lg[~masked].max()
        w[~masked] = np.floor(np.exp(lg[~masked] - lmax) * TABLE_SCALE).astype(np.uint64)
    return {"features": X, "logits": lg, "weights": w, "cum": np.cumsum(w), "moves": moves, "agg": agg}


def run(prob, x0, *, seed: int, T0: float, rho: float, n_stages: int, steps_per_stage: int,
        model: dict | None, refresh: int, eps: float, first_stage: int = 0, net: int = 0,
        trace_every: int = 0, first_chain: int = 0) -> dict:
    """Serial annealing with learned candidates (model None: plain candidates,
    with the refreshes still taken so that traced steps carry features).
    Follows Table 1 for everything after the candidate is drawn.  Chain c of
    x0 draws as chain first_chain + c (a sample of a larger run)."""
    o = OracleProblem(prob)
    E, P = int(prob["n_edges"]), o.n_params
    hard = int(prob.get("hard", 1)) != 0
    x0 = np.asarray(x0, dtype=np.int8).reshape(-1, P)
    n = x0.shape[0]
    L = int(steps_per_stage)
    eps_u = eps_threshold(eps)
    st = statics(prob)
    src, dst = st["src"], st["dst"]
    start = [x0[c].copy() for c in range(n)]
    start_cost = [o.cost(x0[c]) for c in range(n)]
    out = {"stage_best": [], "stage_winner": [], "steps": [], "trace": []}
    for ks in range(n_stages):
        k = first_stage + ks
        T = stage_temperature(T0, rho, k)
        bests, xbests = [], []
        for c in range(n):
            x = start[c].copy()
            cur = start_cost[c]
            best, xbest = cur, x.copy()
            ip, on = counts(prob, x)
            vcur = o.violations(x)
            table = None
            for it in range(L):
                g = k * L + it
                if it % refresh == 0:
                    table = proposal_table(prob, x, T, model) if model is not None else None
                    agg = table["agg"] if table is not None else refresh_state(prob, x, T)
                u = [int(w) for w in draw(seed, g, first_chain + c, net)]
                top = [w >> 32 for w in u]
                source = SOURCE_PLAIN
                p = v = None
                if table is not None and top[3] >= eps_u:
                    total = int(table["cum"][-1])
                    if total > 0:
                        r = (top[0] * total) >> 32
                        m = int(np.searchsorted(table["cum"], r, side="right"))
                        p, _, v = table["moves"][m]
                        source = SOURCE_LEARNED
                        if int(x[p]) == v:
                            source = SOURCE_STALE
                            p = v = None
                    else:
                        source = SOURCE_EMPTY
                if p is None:
                    p = (top[0] * P) >> 32
                    v = value(p, E, (code(p, E, int(x[p])) + 1 + (u[1] >> 63)) % 3)
                old = int(x[p])
                vc = vcur
                if p < E:
                    j, i = src[p], dst[p]
                    on_new = on[j] + int(v != 0) - int(old != 0)
                    ip_new = ip[i] + int(v == 1) - int(old == 1)
                    vc += int(on_new == 0) - int(on[j] == 0) + int(ip_new == 0) - int(ip[i] == 0)
                feasible = not (hard and vc > 0)
                delta, accept = 0, False
                if feasible:
                    xc = x.copy()
                    xc[p] = v
                    cand = o.cost(xc)
                    delta = cand - cur
                    accept = delta <= 0 or top[2] < threshold(T, delta)
                if trace_every and g % trace_every == 0:
                    f = move_features(prob, p, old, v, agg, ip, on, agg["lt"], st)
                    out["trace"].append((c, g, f, p, v, delta, int(accept) | (int(feasible) << 1) | (source << 2)))
                out["steps"].append((c, g, source, p, v, int(feasible), delta, int(accept)))
                if accept:
                    x[p] = v
                    if p < E:
                        on[j], ip[i] = on_new, ip_new
                    vcur, cur = vc, cand
                    if cand < best:
                        best, xbest = cand, x.copy()
            bests.append(best)
            xbests.append(xbest)
        w = int(np.argmin(bests))          # lowest chain id among equal costs
        out["stage_best"].append(bests[w])
        out["stage_winner"].append(w)
        start = [xbests[w].copy() for _ in range(n)]
        start_cost = [bests[w]] * n
    out["x"], out["cost"] = start[0], start_cost[0]
    return out
