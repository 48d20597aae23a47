"""Pure-Python statement of the model and objective, for tiny networks only.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  A second, independent
statement of the same definitions as the C oracle (plain loops over Python
ints), used to cross-check it on every candidate of tiny networks.

Definitions (paper §2.1 image equation, §2.2 update, §2.3 objective, §2.5.3
constraints; synchronous reading, a_e = p*w with t = 1, theta subtracted):

    h_i(t)   = sum over in-edges e = (j -> i) of a_e * s_j(t-1)
    target   = min(max(h_i(t) - theta_i, 0), 2)
    s_i(t)   = s_i(t-1) moved towards target by at most d levels
    W        = |G| + 1 where G is 0 at the first observed time and the
               difference between consecutive observed times after it
    M(x)     = sum over (condition, observed time, observed node) of W * |S - R|
    V(x)     = #(nodes with no non-zero out-edge) + #(nodes with no +1 in-edge)
    cost(x)  = M(x) + lambda * V(x),  lambda = 1 + 2 * sum(W) unless given

The priority-update model (prob["model"] == 1) is stated in _simulate_priority.
"""
from __future__ import annotations


def _edges(prob):
    """List of (src, dst) in parameter order (grouped by target)."""
    row_ptr = [int(v) for v in prob["row_ptr"]]
    src = [int(v) for v in prob["src"]]
    out = []
    for i in range(int(prob["n_nodes"])):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            out.append((src[e], i))
    return out


def _simulate_priority(prob, x):
    """The priority update (§2.1 image with weight, polarity and threshold;
    §2.2 speed, memory and step size), stated per node as a small record:

        K_i       = sum over in-edges e = (j -> i) of (s_j // t_e) * w_e * p_e
        wants     = clamp(K_i, 0, 2) != s_i          (from the states of t-1)
        streak    = consecutive steps with 'wants' (reset when it fails)
        ready     = wants and streak >= m_i + 1
        priority  = u_i * (steps since the node last moved, or since t = 0)
        the ready nodes whose priority equals the largest one move towards
        clamp(K_i, 0, 2) by at most d_i levels and restart both counts.
    """
    N = int(prob["n_nodes"])
    E = int(prob["n_edges"])
    T = int(prob["n_steps"])
    C = int(prob["n_cond"])
    x = [int(v) for v in x]
    w, pol, thr = x[:E], x[E:2 * E], x[2 * E:3 * E]
    speed, mem, dmax = x[3 * E:3 * E + N], x[3 * E + N:3 * E + 2 * N], x[3 * E + 2 * N:3 * E + 3 * N]
    edges = _edges(prob)
    init = [int(v) for v in list(prob["init"].reshape(-1))]
    clamp = [int(v) for v in list(prob["clamp"].reshape(-1))]
    result = []
    for c in range(C):
        held = {i: clamp[c * N + i] for i in range(N) if clamp[c * N + i] >= 0}
        s = [held.get(i, init[c * N + i]) for i in range(N)]
        nodes = [{"idle": 0, "streak": 0} for _ in range(N)]
        traj = [list(s)]
        for _ in range(T):
            img = [0] * N
            for e, (j, i) in enumerate(edges):
                img[i] += (s[j] // thr[e]) * w[e] * pol[e]
            goal = [min(max(v, 0), 2) for v in img]
            ranked = {}
            for i in range(N):
                if i in held:
                    continue
                rec = nodes[i]
                rec["idle"] += 1
                rec["streak"] = rec["streak"] + 1 if goal[i] != s[i] else 0
                if rec["streak"] >= mem[i] + 1:
                    ranked.setdefault(speed[i] * rec["idle"], []).append(i)
            new = list(s)
            if ranked:
                for i in ranked[max(ranked)]:
                    gap = goal[i] - s[i]
                    step = min(abs(gap), dmax[i])
                    new[i] = s[i] + (step if gap > 0 else -step)
                    nodes[i] = {"idle": 0, "streak": 0}
            s = new
            traj.append(list(s))
        result.append(traj)
    return result


def simulate(prob, x):
    """Returns traj[c][t][i] as nested lists."""
    if int(prob.get("model", 0)) == 1:
        return _simulate_priority(prob, x)
    N = int(prob["n_nodes"])
    E = int(prob["n_edges"])
    T = int(prob["n_steps"])
    C = int(prob["n_cond"])
    d = int(prob.get("step_size", 1))
    x = [int(v) for v in x]
    a, theta = x[:E], x[E:]
    edges = _edges(prob)
    init = [int(v) for v in list(prob["init"].reshape(-1))]
    clamp = [int(v) for v in list(prob["clamp"].reshape(-1))]
    result = []
    for c in range(C):
        held = {i: clamp[c * N + i] for i in range(N) if clamp[c * N + i] >= 0}
        s = [held.get(i, init[c * N + i]) for i in range(N)]
        traj = [list(s)]
        for _ in range(T):
            h = [0] * N
            for e, (j, i) in enumerate(edges):
                h[i] += a[e] * s[j]
            new = []
            for i in range(N):
                if i in held:
                    new.append(held[i])
                    continue
                target = min(max(h[i] - theta[i], 0), 2)
                if d == 1:
                    if target > s[i]:
                        new.append(s[i] + 1)
                    elif target < s[i]:
                        new.append(s[i] - 1)
                    else:
                        new.append(s[i])
                else:
                    new.append(target)
            s = new
            traj.append(list(s))
        result.append(traj)
    return result


def weights(prob):
    C = int(prob["n_cond"])
    K = len(prob["obs_t"])
    O = len(prob["obs_n"])
    R = prob["observed"].reshape(C, K, O)
    W = [[[1] * O for _ in range(K)] for _ in range(C)]
    for c in range(C):
        for k in range(1, K):
            for o in range(O):
                W[c][k][o] = 1 + abs(int(R[c, k, o]) - int(R[c, k - 1, o]))
    return W


def mismatch(prob, x):
    C = int(prob["n_cond"])
    K = len(prob["obs_t"])
    O = len(prob["obs_n"])
    R = prob["observed"].reshape(C, K, O)
    W = weights(prob)
    traj = simulate(prob, x)
    m = 0
    for c in range(C):
        for k, t in enumerate(prob["obs_t"]):
            for o, node in enumerate(prob["obs_n"]):
                m += W[c][k][o] * abs(traj[c][int(t)][int(node)] - int(R[c, k, o]))
    return m


def violations(prob, x):
    N = int(prob["n_nodes"])
    E = int(prob["n_edges"])
    edges = _edges(prob)
    if int(prob.get("model", 0)) == 1:   # w_e != 0 counts as an edge; activating: p_e = +1 and w_e != 0
        present = [int(x[e]) != 0 for e in range(E)]
        activating = [present[e] and int(x[E + e]) == 1 for e in range(E)]
    else:
        present = [int(x[e]) != 0 for e in range(E)]
        activating = [int(x[e]) == 1 for e in range(E)]
    v = 0
    for node in range(N):
        if not any(j == node and present[e] for e, (j, _) in enumerate(edges)):
            v += 1
        if not any(i == node and activating[e] for e, (_, i) in enumerate(edges)):
            v += 1
    return v


def penalty_weight(prob):
    lam = int(prob.get("penalty", 0))
    if lam > 0:
        return lam
    return 1 + 2 * sum(sum(sum(row) for row in wk) for wk in weights(prob))


def cost(prob, x):
    return mismatch(prob, x) + penalty_weight(prob) * violations(prob, x)
