"""The C ABI boundary on the CPU: the library loads, exports every entry point
that include/sa_anneal.h declares, and rejects malformed problems with the
documented codes before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2506_19866_amd import sa, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sa_anneal.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sa_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("sa_create_problem", "sa_run_chains", "sa_eval_cost", "sa_best"):
        assert required in names
    assert set(names) == set(sa.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = sa.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(prob, **over):
    a = dict(
        row_ptr=np.ascontiguousarray(prob["row_ptr"], dtype=np.int32),
        src=np.ascontiguousarray(prob["src"], dtype=np.int32),
        init=np.ascontiguousarray(prob["init"], dtype=np.int8).reshape(-1),
        clamp=np.ascontiguousarray(prob["clamp"], dtype=np.int8).reshape(-1),
        obs_t=np.ascontiguousarray(prob["obs_t"], dtype=np.int32),
        obs_n=np.ascontiguousarray(prob["obs_n"], dtype=np.int32),
        observed=np.ascontiguousarray(prob["observed"], dtype=np.int8).reshape(-1))
    scal = dict(n_nodes=prob["n_nodes"], n_edges=prob["n_edges"], n_cond=prob["n_cond"],
                n_steps=prob["n_steps"], step_size=1, mode=sa.SA_HARD, penalty=0, model=0)
    for k, v in over.items():
        if k in a:
            a[k] = v
        else:
            scal[k] = v
    d = sa._ProblemDesc(
        scal["n_nodes"], scal["n_edges"], a["row_ptr"].ctypes.data, a["src"].ctypes.data,
        scal["n_cond"], a["init"].ctypes.data, a["clamp"].ctypes.data, scal["n_steps"],
        len(a["obs_t"]), a["obs_t"].ctypes.data, len(a["obs_n"]), a["obs_n"].ctypes.data,
        a["observed"].ctypes.data, scal["step_size"], scal["mode"], scal["penalty"], scal["model"])
    return d, a


def _create(prob, **over):
    d, keep = _desc(prob, **over)
    h = C.c_void_p()
    rc = sa.lib().sa_create_problem(C.byref(d), C.byref(h))
    if rc == sa.SA_OK:
        sa.lib().sa_destroy_problem(h)
    return rc, sa.lib().sa_last_error().decode()


@pytest.fixture(scope="module")
def c1():
    return synth.load_workload("c1")


def test_null_arguments(c1):
    lib = sa.lib()
    assert lib.sa_create_problem(None, None) == sa.SA_ERR_ARG
    h = C.c_void_p()
    assert lib.sa_create_problem(None, C.byref(h)) == sa.SA_ERR_ARG
    assert lib.sa_eval_cost(None, None, 0, None, None) == sa.SA_ERR_ARG
    assert lib.sa_best(None, 0, None, None, None) == sa.SA_ERR_ARG
    assert lib.sa_destroy_problem(None) == sa.SA_OK
    assert lib.sa_destroy_run(None) == sa.SA_OK


@pytest.mark.parametrize("over,code", [
    (dict(n_nodes=0), sa.SA_ERR_ARG),
    (dict(n_steps=0), sa.SA_ERR_ARG),
    (dict(step_size=3), sa.SA_ERR_DOMAIN),
    (dict(mode=7), sa.SA_ERR_ARG),
    (dict(penalty=-1), sa.SA_ERR_DOMAIN),
    (dict(model=2), sa.SA_ERR_ARG),
    (dict(model=-1), sa.SA_ERR_ARG),
])
def test_scalar_validation(c1, over, code):
    rc, msg = _create(c1, **over)
    assert rc == code and msg


def test_domain_and_topology_validation(c1):
    init = np.array(c1["init"], dtype=np.int8).reshape(-1)
    init[5] = 3
    assert _create(c1, init=init)[0] == sa.SA_ERR_DOMAIN
    clamp = np.array(c1["clamp"], dtype=np.int8).reshape(-1)
    clamp[0] = -2
    assert _create(c1, clamp=clamp)[0] == sa.SA_ERR_DOMAIN
    obs = np.array(c1["observed"], dtype=np.int8).reshape(-1)
    obs[3] = -1
    assert _create(c1, observed=obs)[0] == sa.SA_ERR_DOMAIN
    t = np.array(c1["obs_t"], dtype=np.int32)
    assert _create(c1, obs_t=t[::-1].copy())[0] == sa.SA_ERR_DOMAIN      # not increasing
    t2 = t.copy(); t2[-1] = c1["n_steps"] + 1
    assert _create(c1, obs_t=t2)[0] == sa.SA_ERR_DOMAIN                  # beyond T_s
    on = np.array(c1["obs_n"], dtype=np.int32); on[1] = on[0]
    assert _create(c1, obs_n=on)[0] == sa.SA_ERR_DOMAIN                  # repeated node
    src = np.array(c1["src"], dtype=np.int32)
    row = np.array(c1["row_ptr"])
    bad = src.copy(); bad[row[2]] = 2                                     # self-loop on node 2
    assert _create(c1, src=bad)[0] == sa.SA_ERR_TOPOLOGY
    bad = src.copy(); bad[0] = 99
    assert _create(c1, src=bad)[0] == sa.SA_ERR_TOPOLOGY
    rp = row.astype(np.int32).copy(); rp[-1] -= 1
    assert _create(c1, row_ptr=rp)[0] == sa.SA_ERR_TOPOLOGY


def test_hard_mode_needs_in_and_out_edges():
    # node 2 has no out-edge: constraints (a)/(b) could never hold (§2.5.3)
    row_ptr = np.array([0, 1, 2, 3], dtype=np.int32)
    src = np.array([1, 0, 1], dtype=np.int32)
    prob = dict(n_nodes=3, n_edges=3, row_ptr=row_ptr, src=src, n_cond=1,
                init=np.zeros((1, 3), np.int8), clamp=np.full((1, 3), -1, np.int8), n_steps=3,
                obs_t=np.array([1], np.int32), obs_n=np.array([0], np.int32),
                observed=np.zeros((1, 1, 1), np.int8))
    assert _create(prob)[0] == sa.SA_ERR_TOPOLOGY


def test_overflow_is_reported():
    # lambda * 2N must fit in int32
    w = synth.load_workload("c3")
    assert _create(w, penalty=2**30)[0] == sa.SA_ERR_OVERFLOW


def test_unsupported_sizes():
    N = 200
    row_ptr = np.arange(N + 1, dtype=np.int32)
    src = np.array([(i + 1) % N for i in range(N)], dtype=np.int32)
    prob = dict(n_nodes=N, n_edges=N, row_ptr=row_ptr, src=src, n_cond=1,
                init=np.zeros((1, N), np.int8), clamp=np.full((1, N), -1, np.int8), n_steps=2,
                obs_t=np.array([1], np.int32), obs_n=np.array([0], np.int32),
                observed=np.zeros((1, 1, 1), np.int8))
    assert _create(prob)[0] == sa.SA_ERR_UNSUPPORTED
    # the priority-update model keeps a chain's nodes on the lanes of one wave
    for N in (65, 200):
        row_ptr = np.arange(N + 1, dtype=np.int32)
        src = np.array([(i + 1) % N for i in range(N)], dtype=np.int32)
        prob = dict(n_nodes=N, n_edges=N, row_ptr=row_ptr, src=src, n_cond=1,
                    init=np.zeros((1, N), np.int8), clamp=np.full((1, N), -1, np.int8), n_steps=2,
                    obs_t=np.array([1], np.int32), obs_n=np.array([0], np.int32),
                    observed=np.zeros((1, 1, 1), np.int8))
        rc, msg = _create(prob, model=sa.SA_MODEL_PRIORITY)
        assert rc == sa.SA_ERR_UNSUPPORTED and "priority" in msg


def test_mlp_rejects_bad_params_before_touching_a_device():
    lib = sa.lib()
    h = C.c_void_p()
    assert lib.sa_mlp_create(None, C.byref(h)) == sa.SA_ERR_ARG
    bad = np.zeros(sa.MLP_N_PARAMS, dtype=np.float32)
    bad[17] = np.nan
    assert lib.sa_mlp_create(bad.ctypes.data, C.byref(h)) == sa.SA_ERR_DOMAIN
    assert "not finite" in lib.sa_last_error().decode()
    assert lib.sa_mlp_forward(None, None, 0, None, None) == sa.SA_ERR_ARG
    assert lib.sa_mlp_destroy(None) == sa.SA_OK


def test_mlp_param_packing_round_trip():
    rng = np.random.default_rng(0)
    W1, w2 = rng.normal(size=(32, 256)).astype(np.float32), rng.normal(size=256).astype(np.float32)
    flat = sa.pack_mlp_params(W1, w2, 0.5)
    assert flat.size == sa.MLP_N_PARAMS == 8449
    p = sa.unpack_mlp_params(flat)
    assert np.array_equal(p["W1"], W1) and np.array_equal(p["w2"], w2) and p["b2"] == 0.5
