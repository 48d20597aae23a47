"""What incremental re-simulation (re-simulating only what a one-parameter
change affects, instead of Table 1's full Simulate(x_candidate)) could save,
measured with the oracle on the Mtb-scale workloads of both models.  These
are the estimates behind the decision not to build it for the synchronous
kernels and to build only the exact skip for the priority kernel; run with
-s to see the figures.

For random feasible single-parameter candidates of a current vector (the
start vector and an annealed one):
  * the fraction whose trajectory up to the last observed time is identical
    to the current one (the most any exact skip can save);
  * the first time step at which the candidate's trajectory differs (a
    re-simulation restarted there saves the steps before it);
and, for the synchronous model, the fraction a per-node test finds exact: the
changed node's target clamp(h, 0, 2) (§2.1) unchanged at every step and
condition along the current trajectory, which by induction over the steps
keeps the trajectory."""
import numpy as np
import pytest

from oracle.oracle import OracleProblem
from paper_2506_19866_amd import synth


def _current_vectors(name, w, o):
    s = synth.bench_schedule(name)
    x0 = synth.start_vectors(name, w, 8)
    r = o.run(x0, seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=40, steps_per_stage=150, n_threads=8)
    return {"start": x0[0].copy(), "annealed": r["x"].copy()}


def _candidates(rng, x, lo_hi, n_trials):
    """(index, new value) pairs, uniform index, one of the other values."""
    out = []
    for _ in range(n_trials):
        i = int(rng.integers(0, len(x)))
        lo, hi = lo_hi(i)
        vals = [v for v in range(lo, hi + 1) if v != int(x[i])]
        out.append((i, int(rng.choice(vals))))
    return out


def test_synchronous_model_gains_little_from_resimulation():
    w = synth.load_workload("c3")
    o = OracleProblem(w)
    E, N = w["n_edges"], w["n_nodes"]
    src = w["src"]
    dst = np.repeat(np.arange(N), np.diff(w["row_ptr"]))
    tlast = int(np.max(w["obs_t"]))
    held = w["clamp"] >= 0                                      # [C][N]
    rng = np.random.default_rng(17)
    for label, x in _current_vectors("c3", w, o).items():
        traj = o.simulate(x)[:, :tlast + 1, :].astype(np.int64)
        a, th = x[:E].astype(np.int64), x[E:].astype(np.int64)
        # h_i(t) for t = 1..tlast from the states at t - 1 (image minus threshold)
        H = np.zeros((traj.shape[0], tlast, N), dtype=np.int64)
        for t in range(tlast):
            np.add.at(H[:, t, :], (slice(None), dst), traj[:, t, src] * a[None, :])
        H -= th[None, None, :]
        v0 = o.violations(x)
        same = exact_test = feasible = 0
        first = []
        for i, new in _candidates(rng, x, lambda i: (-1, 1) if i < E else (0, 2), 300):
            xc = x.copy()
            xc[i] = new
            if o.violations(xc) > v0:      # hard mode: rejected without a simulation
                continue
            feasible += 1
            tc = o.simulate(xc)[:, :tlast + 1, :]
            eq = np.array_equal(tc, traj)
            same += eq
            if not eq:
                first.append(int(np.argmax(np.any(tc != traj, axis=(0, 2)))))
            if i < E:
                n, d = dst[i], (new - int(x[i])) * traj[:, :tlast, src[i]]
            else:
                n, d = i - E, -(new - int(x[i])) * np.ones((traj.shape[0], tlast), dtype=np.int64)
            keeps = (np.clip(H[:, :, n] + d, 0, 2) == np.clip(H[:, :, n], 0, 2)) | held[:, n][:, None]
            if np.all(keeps):
                exact_test += 1
                assert eq, "the per-node test claimed an unchanged trajectory that changed"
        f_same, f_test, mean_first = same / feasible, exact_test / feasible, float(np.mean(first))
        print(f"c3 {label}: {feasible} feasible candidates, identical trajectory {f_same:.3f}, "
              f"found by the per-node test {f_test:.3f}, first differing step {mean_first:.2f} of {tlast}")
        # the premise of not building it: almost every candidate changes the trajectory from the first step
        assert f_same < 0.15 and mean_first < 2.0


def test_priority_model_restart_from_first_affected_step():
    """The priority model (§2.2): candidates that keep the trajectory are what
    the exact skip of its stage kernel takes; for the others, the first step
    at which the trajectory actually differs bounds what a restart could save,
    and a rule computable from the current trajectory alone -- for an edge
    j -> i, the first step whose source state s_j(k - 1) is one whose
    contribution (s div t) * w * p changes; for a node's u, m or d, step 1 --
    gives what an implementation would save."""
    w = synth.load_workload("q3")
    o = OracleProblem(w)
    E, N = w["n_edges"], w["n_nodes"]
    src = w["src"]
    T = int(np.max(w["obs_t"]))
    # domains of x = [w] [p] [t] (edges) [u] [m] [d] (nodes)
    doms = [(0, 2)] * E + [(-1, 1)] * E + [(1, 2)] * E + [(1, 12)] * N + [(0, 2)] * N + [(1, 2)] * N
    speeds = [1, 2, 3, 4, 5, 6, 10, 11, 12]
    rng = np.random.default_rng(23)

    def contribution(xv, e):
        wt, pol, thr = int(xv[e]), int(xv[E + e]), int(xv[2 * E + e])
        return np.array([(sv // thr) * wt * pol for sv in range(3)])
    for label, x in _current_vectors("q3", w, o).items():
        traj = o.simulate(x)[:, :T + 1, :]
        v0 = o.violations(x)
        same = feasible = 0
        first, rule = [], []
        for i, new in _candidates(rng, x, lambda i: doms[i], 300):
            if 3 * E <= i < 3 * E + N and new not in speeds:
                new = int(rng.choice([u for u in speeds if u != int(x[i])]))
            xc = x.copy()
            xc[i] = new
            if o.violations(xc) > v0:
                continue
            feasible += 1
            tc = o.simulate(xc)[:, :T + 1, :]
            if np.array_equal(tc, traj):
                same += 1
                continue
            first.append(int(np.argmax(np.any(tc != traj, axis=(0, 2)))))
            k_rule = 1
            if i < 3 * E:
                e = i % E
                changed = np.flatnonzero(contribution(x, e) != contribution(xc, e))
                hit = np.isin(traj[:, :T, src[e]], changed).any(axis=0)     # by step k - 1
                k_rule = int(np.argmax(hit)) + 1 if hit.any() else T
            assert k_rule <= first[-1], "the rule placed the first affected step after the first difference"
            rule.append(k_rule)
        ideal = (float(np.mean(first)) - 1) / T
        practical = (float(np.mean(rule)) - 1) / T
        print(f"q3 {label}: {feasible} feasible candidates, identical trajectory {same / feasible:.3f} (the exact "
              f"skip's share); the others first differ at step {np.mean(first):.2f} of {T}: a restart there would "
              f"skip {ideal:.3f} of their steps, one at the rule's first affected step {practical:.3f}")
        assert 0.0 <= practical <= ideal


def test_priority_model_image_margin_skip_is_exact():
    """The priority kernel's second exact skip: an edge j -> i whose change
    alters node i's image K_i only at steps where K_i stays saturated
    (min K_i + lo >= 2 or max K_i + hi <= 0 over the steps where i is free,
    lo/hi the changes at the source states it takes) leaves every goal
    clamp(K_i, 0, 2) (§2.1) and so the trajectory unchanged.  Checked here
    against full simulations; prints the share of candidates it adds to the
    contribution-table rule."""
    w = synth.load_workload("q3")
    o = OracleProblem(w)
    E, N = w["n_edges"], w["n_nodes"]
    src = w["src"]
    dst = np.repeat(np.arange(N), np.diff(w["row_ptr"]))
    T = int(np.max(w["obs_t"]))
    free = w["clamp"] < 0                                   # [C][N]
    doms = [(0, 2)] * E + [(-1, 1)] * E + [(1, 2)] * E
    rng = np.random.default_rng(29)

    def table(xv, e):
        return np.array([(sv // int(xv[2 * E + e])) * int(xv[e]) * int(xv[E + e]) for sv in range(3)])
    for label, x in _current_vectors("q3", w, o).items():
        traj = o.simulate(x)[:, :T + 1, :].astype(np.int64)
        K = np.zeros((traj.shape[0], T, N), dtype=np.int64)       # images at steps 1..T from states at 0..T-1
        for e in range(E):
            K[:, :, dst[e]] += (traj[:, :T, src[e]] // int(x[2 * E + e])) * int(x[e]) * int(x[E + e])
        big = 1 << 20
        kmin = np.where(free[:, None, :], K, big).min(axis=(0, 1))
        kmax = np.where(free[:, None, :], K, -big).max(axis=(0, 1))
        v0 = o.violations(x)
        feasible = table_rule = margin_rule = 0
        for _ in range(400):
            i = int(rng.integers(0, 3 * E))
            new = int(rng.choice([v for v in range(doms[i][0], doms[i][1] + 1) if v != int(x[i])]))
            xc = x.copy()
            xc[i] = new
            if o.violations(xc) > v0:
                continue
            feasible += 1
            e = i % E
            d = table(xc, e) - table(x, e)
            seen = np.unique(traj[:, :T, src[e]])
            dv = [int(d[sv]) for sv in seen if d[sv] != 0]
            if not dv:
                table_rule += 1
                continue
            lo, hi = min(0, min(dv)), max(0, max(dv))
            if kmin[dst[e]] + lo >= 2 or kmax[dst[e]] + hi <= 0:
                margin_rule += 1
                assert np.array_equal(o.simulate(xc)[:, :T + 1, :], traj), "margin rule skipped a changed trajectory"
        print(f"q3 {label}: of {feasible} feasible edge candidates the table rule skips {table_rule / feasible:.3f}, "
              f"the image-margin rule {margin_rule / feasible:.3f} more")
        assert margin_rule > 0
