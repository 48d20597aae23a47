"""ctypes front end of the serial C oracle (``sa_oracle.c``).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH: only the test suite, the
smoke check and the CPU-baseline leg of the benchmark import this module.  It
shares nothing with the GPU library except the seeded input generators, which
hold none of the method's arithmetic.

A problem is passed as a plain dict of numpy arrays (the layout of
``paper_2506_19866_amd.synth``): ``row_ptr``, ``src``, ``init``, ``clamp``,
``obs_t``, ``obs_n``, ``observed`` plus the scalars ``n_nodes``, ``n_edges``,
``n_cond``, ``n_steps``, ``step_size``, ``hard``, ``penalty``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (plain -O2, no fast-math: exp and the
    double cooling product must follow IEEE semantics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_edges", C.c_int32),
        ("row_ptr", C.c_void_p), ("src", C.c_void_p),
        ("n_cond", C.c_int32), ("init", C.c_void_p), ("clamp", C.c_void_p),
        ("n_steps", C.c_int32),
        ("n_obs_t", C.c_int32), ("obs_t", C.c_void_p),
        ("n_obs_n", C.c_int32), ("obs_n", C.c_void_p),
        ("observed", C.c_void_p),
        ("step_size", C.c_int32), ("hard", C.c_int32), ("penalty", C.c_int64),
        ("model", C.c_int32),
    ]


class _RunArgs(C.Structure):
    _fields_ = [
        ("n_chains", C.c_int64), ("seed", C.c_uint64), ("net", C.c_int32),
        ("T0", C.c_double), ("rho", C.c_double),
        ("first_stage", C.c_int32), ("n_stages", C.c_int32),
        ("steps_per_stage", C.c_int32), ("n_threads", C.c_int32), ("first_chain", C.c_int64),
        ("group_size", C.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        vp = C.c_void_p
        L.ora_philox4x64_10.argtypes = [vp, vp, vp]
        L.ora_simulate.argtypes = [P, vp, vp]
        L.ora_mismatch.argtypes = [P, vp]; L.ora_mismatch.restype = C.c_int64
        L.ora_violations.argtypes = [P, vp]; L.ora_violations.restype = C.c_int32
        L.ora_cost.argtypes = [P, vp]; L.ora_cost.restype = C.c_int64
        L.ora_cost_batch.argtypes = [P, vp, C.c_int64, vp]
        L.ora_weight_sum.argtypes = [P]; L.ora_weight_sum.restype = C.c_int64
        L.ora_lambda.argtypes = [P]; L.ora_lambda.restype = C.c_int64
        L.ora_stage_temperature.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.ora_stage_temperature.restype = C.c_double
        L.ora_count_stages.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_count_stages.restype = C.c_int64
        L.ora_threshold.argtypes = [C.c_double, C.c_int64]; L.ora_threshold.restype = C.c_uint32
        L.ora_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, vp]
        L.ora_propose.argtypes = [P, vp, vp, vp]; L.ora_propose.restype = C.c_int64
        L.ora_run.argtypes = [P, C.POINTER(_RunArgs), vp] + [vp] * 11
        L.ora_run.restype = C.c_int
        L.ora_brute_force.argtypes = [P, vp, vp, vp]; L.ora_brute_force.restype = C.c_int64
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleProblem:
    """Holds contiguous copies of the problem arrays and the C struct that
    points at them (the arrays must outlive every call)."""

    def __init__(self, prob: dict):
        self.n_nodes = int(prob["n_nodes"])
        self.n_edges = int(prob["n_edges"])
        # model 0: the synchronous ternary model (P = E + N); model 1: the
        # paper's priority update with (w, p, t) per edge, (u, m, d) per node
        self.model = int(prob.get("model", 0))
        self.n_params = (3 if self.model == 1 else 1) * (self.n_nodes + self.n_edges)
        self.n_cond = int(prob["n_cond"])
        self.n_steps = int(prob["n_steps"])
        self._keep = {
            "row_ptr": np.ascontiguousarray(prob["row_ptr"], dtype=np.int32),
            "src": np.ascontiguousarray(prob["src"], dtype=np.int32),
            "init": np.ascontiguousarray(prob["init"], dtype=np.int8).reshape(-1),
            "clamp": np.ascontiguousarray(prob["clamp"], dtype=np.int8).reshape(-1),
            "obs_t": np.ascontiguousarray(prob["obs_t"], dtype=np.int32),
            "obs_n": np.ascontiguousarray(prob["obs_n"], dtype=np.int32),
            "observed": np.ascontiguousarray(prob["observed"], dtype=np.int8).reshape(-1),
        }
        k = self._keep
        self.struct = _Problem(
            self.n_nodes, self.n_edges, _ptr(k["row_ptr"]), _ptr(k["src"]),
            self.n_cond, _ptr(k["init"]), _ptr(k["clamp"]), self.n_steps,
            len(k["obs_t"]), _ptr(k["obs_t"]), len(k["obs_n"]), _ptr(k["obs_n"]),
            _ptr(k["observed"]), int(prob.get("step_size", 1)), int(prob.get("hard", 1)),
            int(prob.get("penalty", 0)), self.model)
        self.ref = C.byref(self.struct)

    # -- model -------------------------------------------------------------
    def simulate(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.int8)
        out = np.empty((self.n_cond, self.n_steps + 1, self.n_nodes), dtype=np.int8)
        lib().ora_simulate(self.ref, _ptr(x), _ptr(out))
        return out

    def mismatch(self, x) -> int:
        x = np.ascontiguousarray(x, dtype=np.int8)
        return int(lib().ora_mismatch(self.ref, _ptr(x)))

    def violations(self, x) -> int:
        x = np.ascontiguousarray(x, dtype=np.int8)
        return int(lib().ora_violations(self.ref, _ptr(x)))

    def cost(self, x) -> int:
        x = np.ascontiguousarray(x, dtype=np.int8)
        return int(lib().ora_cost(self.ref, _ptr(x)))

    def cost_batch(self, xs) -> np.ndarray:
        xs = np.ascontiguousarray(xs, dtype=np.int8).reshape(-1, self.n_params)
        out = np.empty(xs.shape[0], dtype=np.int64)
        lib().ora_cost_batch(self.ref, _ptr(xs), xs.shape[0], _ptr(out))
        return out

    def weight_sum(self) -> int:
        return int(lib().ora_weight_sum(self.ref))

    def penalty_weight(self) -> int:
        return int(lib().ora_lambda(self.ref))

    def propose(self, x, u) -> tuple[int, int]:
        x = np.ascontiguousarray(x, dtype=np.int8)
        u = np.ascontiguousarray(u, dtype=np.uint64)
        nv = np.zeros(1, dtype=np.int8)
        i = lib().ora_propose(self.ref, _ptr(x), _ptr(u), _ptr(nv))
        return int(i), int(nv[0])

    # -- annealing ---------------------------------------------------------
    def run(self, x0, *, seed: int, T0: float, rho: float, n_stages: int,
            steps_per_stage: int, first_stage: int = 0, net: int = 0,
            n_threads: int = 1, first_chain: int = 0, group_size: int = 0) -> dict:
        """Table 1 over the chains of x0; group_size G > 0 restarts each group
        of G consecutive chains from its own best at every stage boundary
        (the grouped reduction suggested in §4) instead of from the global best."""
        x0 = np.ascontiguousarray(x0, dtype=np.int8).reshape(-1, self.n_params)
        n = x0.shape[0]
        S = int(n_stages)
        args = _RunArgs(n, int(seed), int(net), float(T0), float(rho), int(first_stage), S,
                        int(steps_per_stage), int(n_threads), int(first_chain), int(group_size))
        out = {
            "x": np.zeros(self.n_params, dtype=np.int8),
            "cost": np.zeros(1, dtype=np.int64), "winner": np.zeros(1, dtype=np.int64),
            "stage_best": np.zeros(S, dtype=np.int64), "stage_winner": np.zeros(S, dtype=np.int64),
            "stage_accepted": np.zeros(S, dtype=np.uint64), "stage_uphill": np.zeros(S, dtype=np.uint64),
            "stage_neutral": np.zeros(S, dtype=np.uint64), "stage_infeasible": np.zeros(S, dtype=np.uint64),
            "chain_best": np.zeros(n, dtype=np.int64),
            "chain_xbest": np.zeros((n, self.n_params), dtype=np.int8),
        }
        rc = lib().ora_run(self.ref, C.byref(args), _ptr(x0), *[_ptr(out[k]) for k in (
            "x", "cost", "winner", "stage_best", "stage_winner", "stage_accepted", "stage_uphill",
            "stage_neutral", "stage_infeasible", "chain_best", "chain_xbest")])
        if rc != 0:
            raise ValueError("a starting vector breaks a structural constraint (hard mode)")
        out["cost"] = int(out["cost"][0])
        out["winner"] = int(out["winner"][0])
        return out

    def brute_force(self, with_costs: bool = False):
        """Every candidate of the ternary (synchronous) model's 3^P vectors."""
        if self.model != 0:
            raise ValueError("exhaustive search covers the ternary synchronous model only")
        total = 3 ** self.n_params
        argmin = np.zeros(self.n_params, dtype=np.int8)
        nmin = np.zeros(1, dtype=np.int64)
        costs = np.zeros(total, dtype=np.int64) if with_costs else None
        best = lib().ora_brute_force(self.ref, _ptr(argmin), _ptr(nmin),
                                     _ptr(costs) if with_costs else None)
        return int(best), argmin, int(nmin[0]), costs


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed: int, g: int, chain: int, net: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_draw(seed, g, chain, net, _ptr(out))
    return out


def stage_temperature(T0: float, rho: float, k: int) -> float:
    return float(lib().ora_stage_temperature(T0, rho, k))


def count_stages(T0: float, T_min: float, rho: float) -> int:
    return int(lib().ora_count_stages(T0, T_min, rho))


def threshold(T: float, delta: int) -> int:
    return int(lib().ora_threshold(T, delta))


def candidate_matrix(n_params: int, n_edges: int) -> np.ndarray:
    """All 3^P vectors in the enumeration order of ``brute_force`` (digit i of
    m in base 3, least significant first, read as a code)."""
    total = 3 ** n_params
    m = np.arange(total, dtype=np.int64)
    X = np.empty((total, n_params), dtype=np.int8)
    for i in range(n_params):
        code = (m // (3 ** i)) % 3
        X[:, i] = code - 1 if i < n_edges else code
    return X
