"""The CPU oracle under the address, undefined-behaviour and thread
sanitizers of the host compiler: a C driver (oracle_sanitize_driver.c) calls
the oracle's entry points on small problems of both models -- costs,
mismatches, violations and trajectories of several vectors, a multi-threaded
annealing run with and without island restarts, and the exhaustive search --
and its printed results must equal those of the same calls through the
oracle's Python binding, with no sanitizer report (any report aborts the
driver with a non-zero status)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.oracle import OracleProblem
from paper_2506_19866_amd import synth
from tests.problems import priority_problem, random_problem

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "sa_oracle.c")]
FLAVOURS = {
    "address+undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "thread": ["-fsanitize=thread"],
}


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    out = {}
    d = tmp_path_factory.mktemp("sanitize")
    for name, flags in FLAVOURS.items():
        exe = str(d / ("driver_" + name.replace("+", "_")))
        r = subprocess.run(["gcc", "-std=c11", "-O1", "-g", *flags, *SOURCES, "-o", exe, "-lm", "-lpthread"],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out[name] = exe
    return out


def _ints(a):
    return " ".join(str(int(v)) for v in np.asarray(a).ravel())


def _write_input(path, prob, vecs, run, x0, brute):
    lines = [_ints([prob["n_nodes"], prob["n_edges"], prob["n_cond"], prob["n_steps"], len(prob["obs_t"]),
                    len(prob["obs_n"]), prob.get("step_size", 1), prob.get("hard", 1), prob.get("penalty", 0),
                    prob.get("model", 0)]),
             _ints(prob["row_ptr"]), _ints(prob["src"]), _ints(prob["init"]), _ints(prob["clamp"]),
             _ints(prob["obs_t"]), _ints(prob["obs_n"]), _ints(prob["observed"]),
             str(len(vecs)), _ints(vecs),
             f"{run['n_chains']} {run['seed']} {run['T0']!r} {run['rho']!r} {run['n_stages']} {run['L']} "
             f"{run['n_threads']} {run['group']}",
             _ints(x0), "1" if brute else "0"]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _expected(prob, vecs, run, x0, brute):
    o = OracleProblem(prob)
    out = []
    for x in vecs:
        traj = o.simulate(x).astype(np.int64).ravel()
        w = np.arange(traj.size, dtype=np.int64) % 9973 + 1
        out.append(f"vec {o.cost(x)} {o.mismatch(x)} {o.violations(x)} {int(np.dot(w, traj))}")
    ref = o.run(x0, seed=run["seed"], T0=run["T0"], rho=run["rho"], n_stages=run["n_stages"],
                steps_per_stage=run["L"], n_threads=run["n_threads"], group_size=run["group"])
    status = 0 if (not prob.get("hard", 1) or all(o.violations(x) == 0 for x in x0)) else -1
    out.append(f"run {status} {ref['cost']} {ref['winner']}")
    for s in range(run["n_stages"]):
        out.append(f"stage {ref['stage_best'][s]} {ref['stage_winner'][s]} {ref['stage_accepted'][s]} "
                   f"{ref['stage_uphill'][s]} {ref['stage_neutral'][s]} {ref['stage_infeasible'][s]}")
    out += [f"chain {c}" for c in ref["chain_best"]]
    out.append("xbest " + _ints(ref["x"]))
    if brute:
        best, _, nmin, _ = o.brute_force()
        out.append(f"brute {best} {nmin}")
    return out


def _cases():
    rng = np.random.default_rng(11)
    sync, _ = random_problem(3, n_nodes=12, n_edges=30, n_cond=4, n_steps=8, n_times=3, n_obs=5, noise=0.1,
                             clamps=(1, 2))
    soft, _ = random_problem(4, n_nodes=10, n_edges=24, n_cond=3, n_steps=7, n_times=2, n_obs=4, noise=0.2,
                             clamps=(0, 1), step_size=2, hard=0)
    tiny, _ = random_problem(5, n_nodes=3, n_edges=5, n_cond=2, n_steps=5, n_times=2, n_obs=2, noise=0.3,
                             clamps=(0, 1))
    prio, _ = priority_problem(6, n_nodes=9, n_edges=25, n_cond=2, n_steps=10, n_obs=5, noise=0.1, clamps=(0, 1))
    out = []
    for name, prob, group, brute in (("synchronous", sync, 0, False), ("penalty, d = 2", soft, 2, False),
                                     ("tiny, exhaustive", tiny, 0, True), ("priority model", prio, 3, False)):
        if prob.get("model", 0) == synth.MODEL_PRIORITY:
            x0 = synth.priority_feasible_params(rng, 7, prob["row_ptr"], prob["src"])
            vecs = np.concatenate([x0[:2], synth.priority_feasible_params(rng, 1, prob["row_ptr"], prob["src"])])
        else:
            x0 = synth.feasible_params(rng, 7, prob["row_ptr"], prob["src"])
            P = prob["n_edges"] + prob["n_nodes"]
            rand = np.concatenate([rng.integers(-1, 2, size=(2, prob["n_edges"])),
                                   rng.integers(0, 3, size=(2, prob["n_nodes"]))], axis=1).astype(np.int8)
            vecs = np.concatenate([x0[:2], rand]).reshape(-1, P)
        run = dict(n_chains=len(x0), seed=77, T0=1.5, rho=0.8, n_stages=3, L=40, n_threads=3, group=group)
        out.append((name, prob, vecs, run, x0, brute))
    return out


@pytest.mark.parametrize("flavour", list(FLAVOURS))
def test_oracle_clean_under_sanitizers(drivers, tmp_path, flavour):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    for k, (name, prob, vecs, run, x0, brute) in enumerate(_cases()):
        path = str(tmp_path / f"case{k}.txt")
        _write_input(path, prob, vecs, run, x0, brute)
        r = subprocess.run([drivers[flavour], path], capture_output=True, text=True, env=env, timeout=300)
        if flavour == "thread" and r.returncode != 0 and "unexpected memory mapping" in r.stderr:
            pytest.skip("this kernel's address-space layout is not supported by the thread sanitizer runtime")
        assert r.returncode == 0, f"{name}: {r.stderr[-3000:]}"
        assert r.stdout.strip().split("\n") == _expected(prob, vecs, run, x0, brute), name
