"""Python binding of libsa_anneal.so (include/sa_anneal.h).

Argument marshalling only: every step of the annealing, the simulation and
the scoring runs in the library's HIP kernels.  torch supplies device memory
and the current stream.  The binding refuses to run when the library is not
built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsa_anneal.so")

SA_OK = 0
SA_ERR_ARG, SA_ERR_DOMAIN, SA_ERR_TOPOLOGY, SA_ERR_INFEASIBLE = -1, -2, -3, -4
SA_ERR_DEVICE, SA_ERR_OOM, SA_ERR_UNSUPPORTED, SA_ERR_OVERFLOW, SA_ERR_ABORTED = -5, -6, -7, -8, -9
SA_HARD, SA_PENALTY = 0, 1
SA_MODEL_SYNCHRONOUS, SA_MODEL_PRIORITY = 0, 1
SA_KERNEL_AUTO, SA_KERNEL_PERSISTENT = 0, 1
SA_PROPOSAL_PLAIN, SA_PROPOSAL_LEARNED = 0, 1
SA_SOURCE_PLAIN, SA_SOURCE_LEARNED, SA_SOURCE_STALE, SA_SOURCE_EMPTY = 0, 1, 2, 3
TRACE_RECORD_BYTES = 80
# sa_trace_record: 32 bf16 feature bit patterns, candidate, cost change, flags
TRACE_DTYPE = np.dtype([("features", "<u2", (32,)), ("param", "<i4"), ("value", "<i4"), ("delta", "<i4"),
                        ("flags", "<u4")])

EXPORTS = ("sa_create_problem", "sa_destroy_problem", "sa_problem_get_info", "sa_eval_cost",
           "sa_simulate", "sa_run_create", "sa_run_launch", "sa_run_chains", "sa_best", "sa_stats",
           "sa_chain_best", "sa_stage_times", "sa_run_get_info", "sa_run_stages_done", "sa_destroy_run", "sa_run_chains_noalloc", "sa_mlp_create",
           "sa_mlp_destroy", "sa_mlp_get_params", "sa_mlp_set_params", "sa_mlp_forward", "sa_mlp_gradients",
           "sa_mlp_train_step", "sa_measure_peak", "sa_last_error")
SA_PEAK_VALU_XOR, SA_PEAK_VALU_ADD, SA_PEAK_VALU_BITOP3, SA_PEAK_CVT_FP4, SA_PEAK_MFMA_FP4 = 0, 1, 2, 3, 4
SA_PEAK_CVT_FP6, SA_PEAK_MFMA_FP4_FP6, SA_PEAK_LDS_READ = 5, 6, 7
MLP_INPUTS, MLP_HIDDEN = 32, 256
MLP_N_PARAMS = MLP_INPUTS * MLP_HIDDEN + MLP_HIDDEN + 1


class SAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sa error {code}: {msg}")
        self.code = code


class _ProblemDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_edges", C.c_int32),
        ("in_row_ptr", C.c_void_p), ("in_src", C.c_void_p),
        ("n_conditions", C.c_int32), ("init_state", C.c_void_p), ("clamp", C.c_void_p),
        ("n_steps", C.c_int32),
        ("n_obs_times", C.c_int32), ("obs_times", C.c_void_p),
        ("n_obs_nodes", C.c_int32), ("obs_nodes", C.c_void_p),
        ("observed", C.c_void_p),
        ("step_size", C.c_int32), ("constraint_mode", C.c_int32), ("penalty", C.c_int32),
        ("model", C.c_int32),
    ]


class _ProblemInfo(C.Structure):
    _fields_ = [(k, C.c_int32) for k in (
        "n_params", "n_nodes", "n_edges", "n_conditions", "n_steps", "n_obs_times", "n_obs_nodes",
        "weight_sum", "penalty", "max_cost", "clamps_by_offset", "obs_dwords")]


class _RunDesc(C.Structure):
    _fields_ = [
        ("n_chains", C.c_int64), ("seed", C.c_uint64), ("T0", C.c_double), ("rho", C.c_double),
        ("first_stage", C.c_int32), ("n_stages", C.c_int32), ("steps_per_stage", C.c_int32),
        ("record_times", C.c_int32), ("kernel", C.c_int32), ("chains_per_block", C.c_int32),
        ("use_graph", C.c_int32),
        ("proposal", C.c_int32), ("refresh_every", C.c_int32), ("model", C.c_void_p), ("eps_plain", C.c_double),
        ("trace_dev", C.c_void_p), ("trace_capacity", C.c_int64), ("trace_every", C.c_int32),
        ("group_size", C.c_int64), ("abort_flag_host", C.c_void_p),
    ]


class _RunInfo(C.Structure):
    _fields_ = [("n_probs", C.c_int32), ("kernel", C.c_int32), ("chains_per_block", C.c_int32),
                ("stages_launched", C.c_int32), ("tiles_m", C.c_int32), ("frags_k", C.c_int32)]


class _StageStats(C.Structure):
    _fields_ = [
        ("best_cost", C.c_int32), ("winner", C.c_int32),
        ("accepted", C.c_uint64), ("uphill", C.c_uint64), ("neutral", C.c_uint64),
        ("infeasible", C.c_uint64), ("simulated", C.c_uint64),
    ]


_lib = None


def lib():
    """Loads the built library (never builds it: run build() first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built; run paper_2506_19866_amd.build.build()")
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.sa_create_problem.argtypes = [C.POINTER(_ProblemDesc), C.POINTER(vp)]
        L.sa_destroy_problem.argtypes = [vp]
        L.sa_problem_get_info.argtypes = [vp, C.POINTER(_ProblemInfo)]
        L.sa_eval_cost.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.sa_simulate.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.sa_run_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_RunDesc), vp, C.POINTER(vp), vp]
        L.sa_run_launch.argtypes = [vp, C.c_int32, vp]
        L.sa_run_chains.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(_RunDesc), vp, C.POINTER(vp), vp]
        L.sa_best.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.sa_stats.argtypes = [vp, C.c_int32, vp]
        L.sa_chain_best.argtypes = [vp, C.c_int32, vp, vp]
        L.sa_stage_times.argtypes = [vp, C.c_int32, vp]
        L.sa_run_get_info.argtypes = [vp, C.POINTER(_RunInfo)]
        L.sa_run_stages_done.argtypes = [vp, C.POINTER(C.c_int32)]
        L.sa_run_chains_noalloc.argtypes = [vp, C.POINTER(_RunDesc), vp, vp, vp, vp, vp]
        L.sa_destroy_run.argtypes = [vp]
        L.sa_mlp_create.argtypes = [vp, C.POINTER(vp)]
        L.sa_mlp_destroy.argtypes = [vp]
        L.sa_mlp_get_params.argtypes = [vp, vp]
        L.sa_mlp_set_params.argtypes = [vp, vp]
        L.sa_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.sa_mlp_gradients.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.sa_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, vp, vp]
        L.sa_measure_peak.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
        L.sa_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "sa_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != SA_OK:
        raise SAError(rc, lib().sa_last_error().decode())


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _device_tensor(t, dtype, shape_last=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"expected shape [n, {shape_last}], got {tuple(t.shape)}")
    return t


class Problem:
    """A network with its conditions and reference data (problem dict layout of
    paper_2506_19866_amd.synth), staged on the current HIP device."""

    def __init__(self, prob: dict, *, constraint_mode: int | None = None, penalty: int | None = None):
        self._arrays = {
            "row_ptr": np.ascontiguousarray(prob["row_ptr"], dtype=np.int32),
            "src": np.ascontiguousarray(prob["src"], dtype=np.int32),
            "init": np.ascontiguousarray(prob["init"], dtype=np.int8).reshape(-1),
            "clamp": np.ascontiguousarray(prob["clamp"], dtype=np.int8).reshape(-1),
            "obs_t": np.ascontiguousarray(prob["obs_t"], dtype=np.int32),
            "obs_n": np.ascontiguousarray(prob["obs_n"], dtype=np.int32),
            "observed": np.ascontiguousarray(prob["observed"], dtype=np.int8).reshape(-1),
        }
        a = self._arrays
        mode = constraint_mode if constraint_mode is not None else (SA_HARD if int(prob.get("hard", 1)) else SA_PENALTY)
        lam = int(penalty if penalty is not None else prob.get("penalty", 0))
        d = _ProblemDesc(
            int(prob["n_nodes"]), int(prob["n_edges"]), a["row_ptr"].ctypes.data,
            a["src"].ctypes.data if len(a["src"]) else None,
            int(prob["n_cond"]), a["init"].ctypes.data, a["clamp"].ctypes.data, int(prob["n_steps"]),
            len(a["obs_t"]), a["obs_t"].ctypes.data, len(a["obs_n"]), a["obs_n"].ctypes.data,
            a["observed"].ctypes.data, int(prob.get("step_size", 1)), mode, lam, int(prob.get("model", 0)))
        h = C.c_void_p()
        _check(lib().sa_create_problem(C.byref(d), C.byref(h)))
        self._h = h
        info = _ProblemInfo()
        _check(lib().sa_problem_get_info(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in _ProblemInfo._fields_}
        self.n_params = info.n_params
        self.n_nodes = info.n_nodes
        self.n_cond = info.n_conditions
        self.n_steps = info.n_steps

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().sa_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval_cost(self, x, out=None, stream=None):
        """x: int8 CUDA tensor [n, P] -> int32 CUDA tensor [n] (asynchronous)."""
        import torch
        x = _device_tensor(x, torch.int8, self.n_params)
        n = x.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=x.device)
        _device_tensor(out, torch.int32)
        _check(lib().sa_eval_cost(self._h, C.c_void_p(x.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                  _stream_handle(stream)))
        return out

    def simulate(self, x, out=None, stream=None):
        """x: int8 CUDA tensor [n, P] -> int8 CUDA tensor [n, C, T_s+1, N]."""
        import torch
        x = _device_tensor(x, torch.int8, self.n_params)
        n = x.shape[0]
        if out is None:
            out = torch.empty((n, self.n_cond, self.n_steps + 1, self.n_nodes), dtype=torch.int8, device=x.device)
        _device_tensor(out, torch.int8)
        _check(lib().sa_simulate(self._h, C.c_void_p(x.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                 _stream_handle(stream)))
        return out


class Run:
    """Parallel annealing (Table 1) of one problem or of several independent
    problems in one persistent launch per stage.  launch=False only sets the
    run up; launch(k) queues the next k stages."""

    def __init__(self, problems, x0, *, seed: int, T0: float, rho: float, n_stages: int,
                 steps_per_stage: int, first_stage: int = 0, stream=None, launch: bool = True,
                 record_times: bool = False, kernel: int = SA_KERNEL_AUTO, chains_per_block: int = 0,
                 use_graph: bool = False, model: "Mlp | None" = None, refresh_every: int = 16,
                 eps_plain: float = 0.1, trace=None, trace_every: int = 1, group_size: int = 0,
                 abort_flag=None):
        """problems: a Problem or a list of them; x0: int8 CUDA tensor [n_chains, P]
        for one problem, or a list (one [n_chains, P_p] tensor per problem).
        model: learned proposal with this network; trace: uint8 CUDA tensor
        [n_chains, capacity * 80] receiving sa_trace_record rows (decode with
        decode_trace).  group_size G > 0: island restart, each group of G
        consecutive chains restarts from its own best (0: the global best).
        abort_flag: a pinned int32 CPU tensor (torch pin_memory); setting its
        first element non-zero stops the run at the next stage boundary
        (stages_done() then counts the stages that completed)."""
        import torch
        if isinstance(problems, Problem):
            problems, x0 = [problems], [x0]
        self.problems = list(problems)
        xs = [_device_tensor(x, torch.int8, p.n_params) for p, x in zip(self.problems, x0)]
        n = xs[0].shape[0]
        if any(x.shape[0] != n for x in xs):
            raise ValueError("every problem needs the same number of chains")
        self._x0 = torch.cat([x.reshape(-1) for x in xs]) if len(xs) > 1 else xs[0]
        self.problem = self.problems[0]
        self.n_chains = n
        self.n_stages = n_stages
        self.launched = 0
        trace_ptr, cap = None, 0
        if trace is not None:
            trace = _device_tensor(trace, torch.uint8)
            if trace.dim() != 2 or trace.shape[0] != n or trace.shape[1] % TRACE_RECORD_BYTES:
                raise ValueError("trace must be uint8 [n_chains, capacity * 80]")
            trace_ptr, cap = trace.data_ptr(), trace.shape[1] // TRACE_RECORD_BYTES
        self._trace, self.model = trace, model
        abort_ptr = None
        if abort_flag is not None:
            if (not isinstance(abort_flag, torch.Tensor) or abort_flag.is_cuda or abort_flag.dtype != torch.int32
                    or not abort_flag.is_pinned() or abort_flag.numel() < 1):
                raise TypeError("abort_flag must be a pinned int32 CPU tensor")
            abort_ptr = abort_flag.data_ptr()
        self._abort = abort_flag
        d = _RunDesc(n, int(seed) & (2**64 - 1), float(T0), float(rho), int(first_stage), int(n_stages),
                     int(steps_per_stage), 1 if record_times else 0, int(kernel), int(chains_per_block),
                     1 if use_graph else 0, SA_PROPOSAL_LEARNED if model is not None else SA_PROPOSAL_PLAIN,
                     int(refresh_every), model.handle if model is not None else None, float(eps_plain),
                     trace_ptr, int(cap), int(trace_every), int(group_size), abort_ptr)
        probs = (C.c_void_p * len(self.problems))(*[p.handle for p in self.problems])
        h = C.c_void_p()
        _check(lib().sa_run_create(probs, len(self.problems), C.byref(d), C.c_void_p(self._x0.data_ptr()),
                                   C.byref(h), _stream_handle(stream)))
        self._h = h
        if launch:
            self.launch(n_stages, stream=stream)

    def launch(self, n_stages: int, stream=None):
        _check(lib().sa_run_launch(self._h, int(n_stages), _stream_handle(stream)))
        self.launched += n_stages

    def stages_done(self) -> int:
        """Stages that completed (all launched ones unless the abort flag
        stopped the run).  Synchronises."""
        d = C.c_int32()
        _check(lib().sa_run_stages_done(self._h, C.byref(d)))
        return d.value

    def info(self) -> dict:
        i = _RunInfo()
        _check(lib().sa_run_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _RunInfo._fields_}

    def best(self, prob: int = 0):
        x = np.zeros(self.problems[prob].n_params, dtype=np.int8)
        cost, winner = C.c_int32(), C.c_int32()
        _check(lib().sa_best(self._h, prob, x.ctypes.data, C.byref(cost), C.byref(winner)))
        return x, cost.value, winner.value

    def stats(self, prob: int = 0) -> dict:
        arr = (_StageStats * max(self.launched, 1))()
        _check(lib().sa_stats(self._h, prob, C.cast(arr, C.c_void_p)))
        return {k: np.array([getattr(arr[i], k) for i in range(self.launched)],
                            dtype=np.int64 if k in ("best_cost", "winner") else np.uint64)
                for k, _ in _StageStats._fields_}

    def chain_best(self, prob: int = 0):
        cost = np.zeros(self.n_chains, dtype=np.int32)
        x = np.zeros((self.n_chains, self.problems[prob].n_params), dtype=np.int8)
        _check(lib().sa_chain_best(self._h, prob, cost.ctypes.data, x.ctypes.data))
        return cost, x

    def stage_times_ms(self) -> np.ndarray:
        """Stage-kernel durations (HIP events on the launch stream)."""
        ms = np.zeros(max(self.launched, 1), dtype=np.float32)
        _check(lib().sa_stage_times(self._h, 0, ms.ctypes.data))
        return ms[:self.launched]

    def close(self):
        if getattr(self, "_h", None):
            lib().sa_destroy_run(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 16 << 20


def run_chains_noalloc(problem: Problem, x0, x_best, best, stats=None, *, seed: int, T0: float, rho: float,
                       n_stages: int, steps_per_stage: int, first_stage: int = 0, stream=None) -> None:
    """sa_run_chains_noalloc: the whole schedule with the run state in the
    library's fixed device array (no device allocation in the call).  x0: int8
    CUDA tensor [n_chains, P]; outputs (CUDA tensors, written on the stream):
    x_best int8 [P], best int32 [2] (cost, winner chain), stats uint8
    [n_stages * 48] (sa_stage_stats records) or None."""
    import torch
    x0 = _device_tensor(x0, torch.int8, problem.n_params)
    x_best = _device_tensor(x_best, torch.int8)
    best = _device_tensor(best, torch.int32)
    if x_best.numel() < problem.n_params or best.numel() < 2:
        raise ValueError("x_best needs P entries and best 2")
    sp = None
    if stats is not None:
        stats = _device_tensor(stats, torch.uint8)
        if stats.numel() < n_stages * C.sizeof(_StageStats):
            raise ValueError("stats needs n_stages * 48 bytes")
        sp = stats.data_ptr()
    d = _RunDesc(x0.shape[0], int(seed) & (2**64 - 1), float(T0), float(rho), int(first_stage), int(n_stages),
                 int(steps_per_stage), 0, SA_KERNEL_AUTO, 0, 0, SA_PROPOSAL_PLAIN, 16, None, 0.1, None, 0, 1, 0,
                 None)
    _check(lib().sa_run_chains_noalloc(problem.handle, C.byref(d), C.c_void_p(x0.data_ptr()),
                                       C.c_void_p(x_best.data_ptr()), C.c_void_p(best.data_ptr()),
                                       C.c_void_p(sp) if sp else None, _stream_handle(stream)))


def decode_stage_stats(raw: np.ndarray) -> dict:
    """sa_stage_stats records (bytes) as arrays, like Run.stats()."""
    arr = (_StageStats * (len(raw) // C.sizeof(_StageStats))).from_buffer_copy(np.ascontiguousarray(raw).tobytes())
    return {k: np.array([getattr(a, k) for a in arr], dtype=np.int64 if k in ("best_cost", "winner") else np.uint64)
            for k, _ in _StageStats._fields_}


def pack_mlp_params(W1, w2, b2) -> np.ndarray:
    """Flat float32 parameter array: W1 [32][256] row-major (row 31 is the
    hidden bias, fed by the constant input 31), w2 [256], b2."""
    W1 = np.asarray(W1, dtype=np.float32).reshape(MLP_INPUTS, MLP_HIDDEN)
    w2 = np.asarray(w2, dtype=np.float32).reshape(MLP_HIDDEN)
    return np.concatenate([W1.reshape(-1), w2, np.asarray([b2], dtype=np.float32)])


def unpack_mlp_params(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float32)
    nw = MLP_INPUTS * MLP_HIDDEN
    return {"W1": flat[:nw].reshape(MLP_INPUTS, MLP_HIDDEN).copy(), "w2": flat[nw:nw + MLP_HIDDEN].copy(),
            "b2": float(flat[-1])}


class Mlp:
    """The proposal network (32 -> 256 ReLU -> 1) on the current HIP device.
    Feature rows are torch.bfloat16 tensors [n, 32]; labels float32 [n]."""

    def __init__(self, params):
        flat = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if flat.size != MLP_N_PARAMS:
            raise ValueError(f"expected {MLP_N_PARAMS} parameters, got {flat.size}")
        h = C.c_void_p()
        _check(lib().sa_mlp_create(flat.ctypes.data, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def params(self) -> np.ndarray:
        out = np.empty(MLP_N_PARAMS, dtype=np.float32)
        _check(lib().sa_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, params) -> None:
        flat = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if flat.size != MLP_N_PARAMS:
            raise ValueError(f"expected {MLP_N_PARAMS} parameters, got {flat.size}")
        _check(lib().sa_mlp_set_params(self._h, flat.ctypes.data))

    def forward(self, x, stream=None):
        import torch
        x = _device_tensor(x, torch.bfloat16, MLP_INPUTS)
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(lib().sa_mlp_forward(self._h, x.data_ptr(), x.shape[0], out.data_ptr(), _stream_handle(stream)))
        return out

    def gradients(self, x, y, stream=None):
        import torch
        x = _device_tensor(x, torch.bfloat16, MLP_INPUTS)
        y = _device_tensor(y, torch.float32)
        if y.dim() != 1 or y.shape[0] != x.shape[0]:
            raise ValueError("labels must be [n]")
        grad = torch.empty(MLP_N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().sa_mlp_gradients(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], grad.data_ptr(),
                                      loss.data_ptr(), _stream_handle(stream)))
        return grad, loss

    def train_step(self, x, y, lr: float, stream=None, loss=None):
        """One Adam step; returns the device scalar holding the batch's loss."""
        import torch
        x = _device_tensor(x, torch.bfloat16, MLP_INPUTS)
        y = _device_tensor(y, torch.float32)
        if y.dim() != 1 or y.shape[0] != x.shape[0]:
            raise ValueError("labels must be [n]")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().sa_mlp_train_step(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], float(lr),
                                       loss.data_ptr(), _stream_handle(stream)))
        return loss

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sa_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_trace(trace) -> np.ndarray:
    """sa_trace_record rows of a trace tensor [n_chains, capacity * 80] as a
    numpy structured array [n_chains, capacity] (features as float32)."""
    raw = trace.cpu().numpy() if hasattr(trace, "cpu") else np.asarray(trace)
    rec = np.ascontiguousarray(raw).view(TRACE_DTYPE).reshape(raw.shape[0], -1)
    return rec


def bf16_bits_to_float(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def measure_peak(kind: int, stream=None) -> tuple[float, float]:
    """Measured device-wide rate of one instruction kind (SA_PEAK_*): 32-bit
    lane-ops per second for the VALU kinds, values converted per second for
    the packing conversions, flops per second for the matrix products; and
    the timed launch's ms."""
    rate, ms = C.c_double(), C.c_double()
    _check(lib().sa_measure_peak(int(kind), C.byref(rate), C.byref(ms), _stream_handle(stream)))
    return rate.value, ms.value
