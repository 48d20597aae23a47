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


def simulate(prob, x):
    """Returns traj[c][t][i] as nested lists."""
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
    edges = _edges(prob)
    v = 0
    for node in range(N):
        if not any(j == node and int(x[e]) != 0 for e, (j, _) in enumerate(edges)):
            v += 1
        if not any(i == node and int(x[e]) == 1 for e, (_, i) in enumerate(edges)):
            v += 1
    return v


def penalty_weight(prob):
    lam = int(prob.get("penalty", 0))
    if lam > 0:
        return lam
    return 1 + 2 * sum(sum(sum(row) for row in wk) for wk in weights(prob))


def cost(prob, x):
    return mismatch(prob, x) + penalty_weight(prob) * violations(prob, x)
