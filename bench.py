#!/usr/bin/env python3
"""Benchmark: simulated-annealing chain-steps per second on the 723-parameter
(Mtb-scale) workload, one MI355X.

A step is one temperature stage of Table 1 over the whole workload: every one
of the 16384 chains runs 500 proposal/simulation/score/Metropolis steps, then
the global restart from the best chain.  --steps K times K consecutive stages
of the workload's schedule from its first stage (K = 200 is the complete
schedule); --warmup W stages run first on a separate, discarded run.

Prints ONE JSON line on stdout (progress goes to stderr).  The roofline figure
is for the stage kernel, timed with HIP events recorded by the library on the
launch stream; the CPU baseline is the oracle timed on a bounded sample of the
same workload on the host cores.

Other workloads and modes: --workload c1/c2 (smaller synchronous networks),
c4 (256 uneven networks in one persistent launch per stage), q1/q2/q3 (the
paper's own priority-update model; q2 and q3 have the HPG and Mtb networks'
parameter counts); --mode learned / learned-cost (the learned proposal against
the plain one), --mode sweep (the chain counts of the paper's Table 2).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# chip figures (MI355X): 256 CUs of 4 SIMDs at 2.4 GHz; a SIMD issues one
# wave64 VALU instruction every 4 cycles (16 lanes per cycle), so the 32-bit
# integer ALU peak is 256 x 64 lane-ops per clock = 39.3e12 lane-ops/s (the
# published 157.3 TFLOP/s fp32 vector rate is this times 2 flops per FMA times
# 2 for packed-fp32 instructions, which integer work does not have).  The dense
# fp4 matrix peak is the published 10.1 PFLOP/s.  Both are checked against
# the measured rates of sa_measure_peak (--mode peaks).
CU, CLOCK_HZ = 256, 2.4e9
ALU_PEAK_OPS = CU * 64 * CLOCK_HZ
FP4_DENSE_PEAK_FLOPS = 10.1e15
HBM_PEAK_BYTES = 8.0e12
# LDS: 256 CUs x 256 bytes per clock x 2.4 GHz; the measured 16-byte read
# rate of sa_measure_peak (reported beside it) is 96% of that, more than 128
# bytes per clock could deliver
LDS_PEAK_BYTES = CU * 256 * CLOCK_HZ
PROFILES = os.path.join(ROOT, "profiles")
STAGE_KERNEL_SOURCES = ("paper_2506_19866_amd/csrc/sa_k_stage.hip", "paper_2506_19866_amd/csrc/sa_chain.h",
                        "paper_2506_19866_amd/csrc/sa_device.h", "paper_2506_19866_amd/csrc/sa_internal.h")
PRIORITY_KERNEL_SOURCES = ("paper_2506_19866_amd/csrc/sa_k_priority.hip", "paper_2506_19866_amd/csrc/sa_priority.h",
                           "paper_2506_19866_amd/csrc/sa_device.h", "paper_2506_19866_amd/csrc/sa_internal.h")
# committed HBM byte counts per kernel: (summary file, the sources it was taken with)
PMC_SUMMARIES = {"stage": ("stage_kernel_c3_pmc.json", STAGE_KERNEL_SOURCES),
                 "priority": ("pr_stage_kernel_q3_pmc.json", PRIORITY_KERNEL_SOURCES)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_hash(sources) -> str:
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stage_kernel_hash(kind: str = "stage") -> str:
    return sources_hash(PMC_SUMMARIES[kind][1])


def algorithmic_alu_ops(prob: dict) -> int:
    """Integer operations per full simulation of one candidate that must go
    through the vector ALU whatever unit does the regulator contraction:
    per (condition, step, node) update 2 ops (bound the image to {0,1,2},
    move towards it), per observation term 2 ops (|S - R|, weighted add)."""
    C, T, N = prob["n_cond"], prob["n_steps"], prob["n_nodes"]
    K, O = len(prob["obs_t"]), len(prob["obs_n"])
    return 2 * C * T * N + 2 * C * K * O


def algorithmic_alu_ops_priority(prob: dict) -> int:
    """The same count for the priority-update model: per (condition, step,
    edge) 2 ops (the regulator term's multiply-add, its threshold division
    taken as an operand choice), per (condition, step, node) 6 ops (bound the
    image, the told test, the memory count, the priority product, the
    comparison with the step's highest priority, the bounded move), per
    observation term 2 ops."""
    C, T, N, E = prob["n_cond"], prob["n_steps"], prob["n_nodes"], prob["n_edges"]
    K, O = len(prob["obs_t"]), len(prob["obs_n"])
    return 2 * C * T * E + 6 * C * T * N + 2 * C * K * O


def regulator_macs(prob: dict) -> int:
    """Regulator terms per full simulation (one multiply-add per condition,
    step and edge), the part of the work the synchronous kernels run on the
    fp4 matrix cores."""
    return prob["n_cond"] * prob["n_steps"] * prob["n_edges"]


def measured_peaks() -> dict:
    """Device-wide rates of the instructions the kernels are bound by
    (sa_measure_peak): 32-bit lane-ops/s of v_xor / v_add / v_bitop3, values
    per second of the fp4 (2 per instruction) and fp6 (32 per instruction)
    packing conversions, flops/s of the fp4 x fp4 and fp4 x fp6 products,
    bytes/s of 16-byte LDS reads."""
    from paper_2506_19866_amd import sa
    kinds = {"valu_xor": sa.SA_PEAK_VALU_XOR, "valu_add": sa.SA_PEAK_VALU_ADD, "valu_bitop3": sa.SA_PEAK_VALU_BITOP3,
             "cvt_fp4": sa.SA_PEAK_CVT_FP4, "mfma_fp4": sa.SA_PEAK_MFMA_FP4, "cvt_fp6": sa.SA_PEAK_CVT_FP6,
             "mfma_fp4_fp6": sa.SA_PEAK_MFMA_FP4_FP6, "lds_read": sa.SA_PEAK_LDS_READ}
    out = {k: sa.measure_peak(v)[0] for k, v in kinds.items()}
    out["valu"] = max(out["valu_xor"], out["valu_add"], out["valu_bitop3"])
    return out


def counters_from_profiles(launch_key: str, kind: str = "stage"):
    """Issued instructions per stage-kernel launch from the committed SQ
    counter summary, or None when it is missing or the kernel sources changed
    since it was taken."""
    name = {"stage": "stage_kernel_c3_sq_pmc.json", "priority": "pr_stage_kernel_q3_sq_pmc.json"}[kind]
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256_16") != stage_kernel_hash(kind) or rec.get("launch") != launch_key:
        return None
    return rec


def alu_roofline(ops_per_launch: float, avg_launch_s: float, peaks: dict | None, kernel: str, traffic,
                 counters=None, macs_per_launch: float | None = None, dense_macs_per_launch: float | None = None,
                 lds_bytes_per_launch: float | None = None, lds_what: str = "") -> dict:
    """The roofline object: algorithmic integer ALU work against the derived
    ALU peak (and the measured one), plus the matrix-core part of the work
    against the dense fp4 peak, the HBM and LDS bandwidth the launch used,
    and, from committed counters, the VALU instructions the kernel actually
    issued."""
    achieved = ops_per_launch / avg_launch_s
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12, "unit": "TOP/s",
         "frac": achieved / ALU_PEAK_OPS, "traffic": traffic, "kernel": kernel,
         "avg_launch_ms": avg_launch_s * 1e3, "ops_per_launch": ops_per_launch,
         "peak_note": "derived from unit counts: 256 CUs x 64 lanes per clock x 2.4 GHz (32-bit integer lane-ops)"}
    if peaks:
        r["peak_measured"] = peaks["valu"] / 1e12
        r["frac_measured"] = achieved / peaks["valu"]
    if macs_per_launch is not None:
        m = {"achieved": 2 * macs_per_launch / avg_launch_s / 1e12, "peak": FP4_DENSE_PEAK_FLOPS / 1e12,
             "unit": "TFLOP/s", "what": "2 x regulator multiply-adds of the simulations run (algorithmic)"}
        m["frac"] = m["achieved"] / m["peak"]
        if dense_macs_per_launch is not None:
            m["executed"] = 2 * dense_macs_per_launch / avg_launch_s / 1e12
            m["executed_frac"] = m["executed"] / m["peak"]
        if peaks:
            m["peak_measured"] = peaks["mfma_fp4"] / 1e12
        r["mfma"] = m
    if traffic:
        r["hbm"] = {"achieved": traffic / avg_launch_s / 1e9, "peak": HBM_PEAK_BYTES / 1e9, "unit": "GB/s",
                    "frac": traffic / avg_launch_s / HBM_PEAK_BYTES,
                    "what": "copy-calibrated FETCH_SIZE + WRITE_SIZE bytes per launch (traffic) / its duration"}
    if lds_bytes_per_launch is not None:
        lds = {"achieved": lds_bytes_per_launch / avg_launch_s / 1e9, "peak": LDS_PEAK_BYTES / 1e9, "unit": "GB/s",
               "frac": lds_bytes_per_launch / avg_launch_s / LDS_PEAK_BYTES, "what": lds_what,
               "peak_note": "256 CUs x 256 bytes per clock x 2.4 GHz"}
        if peaks and peaks.get("lds_read"):
            lds["peak_measured"] = peaks["lds_read"] / 1e9
            lds["frac_measured"] = lds_bytes_per_launch / avg_launch_s / peaks["lds_read"]
        r["lds"] = lds
    if counters:
        issued = counters["sq_insts_valu_per_launch"] * 64 / (counters["avg_launch_ms"] * 1e-3)
        r["valu_issued"] = {"lane_ops_per_s": issued / 1e12, "unit": "TOP/s",
                            "frac": issued / ALU_PEAK_OPS,
                            "frac_measured": issued / peaks["valu"] if peaks else None,
                            "source": counters.get("file", "profiles"),
                            "note": "SQ_INSTS_VALU x 64 lanes per launch / its duration: every issued VALU "
                                    "instruction (incl. the packing conversions and the matrix instructions' "
                                    "VALU-side count), not only the algorithmic ops"}
    return r


def traffic_from_profiles(launch_key: str, kind: str = "stage"):
    """HBM bytes per stage-kernel launch from the committed PMC summary, or
    None when it is missing or the kernel sources changed since."""
    path = os.path.join(PROFILES, PMC_SUMMARIES[kind][0])
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256_16") != stage_kernel_hash(kind) or rec.get("launch") != launch_key:
        return None
    return rec.get("hbm_bytes_per_launch")


# one-core oracle samples per workload: (chains, steps), a second or less each
SERIAL_SAMPLE = {"c1": (64, 100), "c2": (16, 500), "c3": (4, 500), "q1": (64, 100), "q2": (16, 500),
                 "q3": (4, 500)}


def cpu_baseline(name: str, prob: dict, sched: dict, target_s: float) -> dict:
    from oracle.oracle import OracleProblem
    from paper_2506_19866_amd import synth
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o = OracleProblem(prob)
    L = sched["steps_per_stage"]
    probe_chains, probe_steps = threads, 20
    x = synth.start_vectors(name, prob, probe_chains)
    t0 = time.perf_counter()
    o.run(x, seed=sched["seed"], T0=sched["T0"], rho=sched["rho"], n_stages=1,
          steps_per_stage=probe_steps, n_threads=threads)
    rate = probe_chains * probe_steps / (time.perf_counter() - t0)
    for _ in range(2):  # a short probe underestimates fast oracles: rescale once if the sample ran short
        chains = max(threads, int(rate * target_s / L) // threads * threads)
        x = synth.start_vectors(name, prob, chains)
        t0 = time.perf_counter()
        o.run(x, seed=sched["seed"], T0=sched["T0"], rho=sched["rho"], n_stages=1,
              steps_per_stage=L, n_threads=threads)
        dt = time.perf_counter() - t0
        rate = chains * L / dt
        if dt >= 0.5 * target_s:
            break
    out = {"value": chains * L / dt, "unit": "chain-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{name} stage 0 of its schedule: {chains} chains x {L} steps "
                     f"({chains * L} chain-steps, {dt:.1f} s, {threads} threads, serial C oracle per chain)"}
    # one core: a few chains of the same stage on one thread
    serial_chains = SERIAL_SAMPLE.get(name, (4, L))
    x = synth.start_vectors(name, prob, serial_chains[0])
    t0 = time.perf_counter()
    o.run(x, seed=sched["seed"], T0=sched["T0"], rho=sched["rho"], n_stages=1, steps_per_stage=serial_chains[1],
          n_threads=1)
    dt1 = time.perf_counter() - t0
    out["serial_1core"] = {"value": serial_chains[0] * serial_chains[1] / dt1, "unit": "chain-steps/s", "cores": 1,
                           "sample": f"{name}: {serial_chains[0]} chains x {serial_chains[1]} steps of stage 0, "
                                     f"one thread ({dt1:.2f} s)"}
    return out


def bench_batch(args) -> int:
    """The batched workload: every network's chains in one persistent launch
    per stage, the stages of the timed region captured in one hipGraph."""
    import torch
    from paper_2506_19866_amd import sa, synth
    probs = synth.load_batch("c4")
    s = synth.batch_schedule()
    n, L = s["n_chains"], s["steps_per_stage"]
    x0 = [torch.from_numpy(x).cuda() for x in synth.batch_start_vectors(probs, n)]
    P = [sa.Problem(p) for p in probs]
    torch.cuda.synchronize()
    if args.warmup > 0:
        warm = sa.Run(P, x0, seed=s["seed"] + 1, T0=s["T0"], rho=s["rho"], n_stages=args.warmup,
                      steps_per_stage=L, chains_per_block=4)
        warm.best()
        warm.close()
    t0 = time.perf_counter()
    run = sa.Run(P, x0, seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=args.steps, steps_per_stage=L,
                 launch=False, chains_per_block=0, use_graph=True)
    torch.cuda.synchronize()
    log(f"[bench] c4 setup incl. autotune: {time.perf_counter() - t0:.2f} s, chosen {run.info()}")
    t0 = time.perf_counter()
    run.launch(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    chain_steps = len(probs) * n * L * args.steps
    value = chain_steps / elapsed
    ops = 0.0
    for i, prob in enumerate(probs):
        st = run.stats(i)
        sims_i = float(np.mean(st["simulated"].astype(np.float64)))
        ops += sims_i * algorithmic_alu_ops(prob)
    avg_stage_s = elapsed / args.steps
    peaks = measured_peaks()
    roofline = alu_roofline(ops, avg_stage_s, peaks, "persistent_kernel<MX,KX,D>", None)
    roofline["note"] = "stage time incl. the reduction (graph launch)"
    log(f"[bench] c4: {args.steps} stages in {elapsed:.3f} s: {value:.4g} chain-steps/s")
    out = {
        "metric": "SA chain-steps/s, batched uneven networks", "value": value, "unit": "chain-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp4",
        "data": "synthetic (seeded generator + oracle-simulated reference data, stored workload)",
        "config": {"workload": f"c4: {len(probs)} networks of 10-150 nodes, {n} chains each x {L} steps per stage, "
                               f"one persistent launch per stage, stages in one hipGraph",
                   "chains_per_block": run.info()["chains_per_block"]},
        "roofline": roofline,
    }
    print(json.dumps(out), flush=True)
    run.close()
    return 0


def _curve(run, sched_L, n):
    """(cumulative stage-kernel seconds, global best after each stage,
    fraction of steps that were accepted improving moves)."""
    st = run.stats()
    ms = run.stage_times_ms().astype(np.float64)
    improving = (st["accepted"] - st["uphill"] - st["neutral"]).astype(np.float64).sum()
    return (np.cumsum(ms) * 1e-3, np.minimum.accumulate(st["best_cost"].astype(np.int64)),
            float(improving / (n * sched_L * len(ms))))


def _auc(score, label) -> float:
    """Probability that a random positive row outranks a random negative one
    (ties count half): the Mann-Whitney statistic."""
    order = np.argsort(score, kind="mergesort")
    ranks = np.empty(len(score), dtype=np.float64)
    s_sorted = score[order]
    i = 0
    while i < len(score):
        j = i
        while j + 1 < len(score) and s_sorted[j + 1] == s_sorted[i]:
            j += 1
        ranks[order[i:j + 1]] = 0.5 * (i + j) + 1
        i = j + 1
    pos = label > 0.5
    n1, n0 = int(pos.sum()), int((~pos).sum())
    if n1 == 0 or n0 == 0:
        return float("nan")
    return float((ranks[pos].sum() - n1 * (n1 + 1) / 2) / (n1 * n0))


def _time_to(curve, target):
    t, best, _ = curve
    hit = np.flatnonzero(best <= target)
    return float(t[hit[0]]) if hit.size else None


def bench_learned(args) -> int:
    """The learned proposal against the plain one on the Mtb-scale workload:
    traces of plain runs on the HPG-scale workload (about args.trace_rows
    rows), the network trained on them, then plain and learned runs of the
    full c3 schedule for args.eval_seeds run seeds, compared by the
    stage-kernel time they need to reach (a) a target cost fixed before the
    evaluation (args.target; the default 1277 is the cost 80% of the plain
    runs reached on the seeds the refresh interval and plain fraction were
    chosen on, k = 0..9) and (b) the cost of the generating parameters on the
    noisy data.  The default seeds, k = 10..19 (run seed = 2003 + 100 k), are
    held out from that choice.  Trace collection and training are timed on
    their own and are not in the time to target."""
    import torch
    from paper_2506_19866_amd import proposal, sa, synth
    p2, s2 = synth.load_workload(args.trace_workload), synth.bench_schedule(args.trace_workload)
    P2 = sa.Problem(p2)
    n2, L2 = s2["n_chains"], s2["steps_per_stage"]
    x2 = torch.from_numpy(synth.start_vectors(args.trace_workload, p2, n2)).cuda()
    te = max(1, (n2 * s2["n_stages"] * L2) // args.trace_rows)
    t0 = time.perf_counter()
    X, y, _ = proposal.collect(P2, x2, seed=s2["seed"], T0=s2["T0"], rho=s2["rho"], n_stages=s2["n_stages"],
                               steps_per_stage=L2, trace_every=te, refresh_every=args.refresh)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    pos = float(y.mean().item())
    log(f"[learned] traces: {X.shape[0]} rows from {args.trace_workload} (every {te}th step), {pos:.4f} improving, "
        f"{t_collect:.2f} s")
    # hold out every tenth row (by position) to measure how well the network ranks moves
    held = torch.arange(X.shape[0], device=X.device) % 10 == 9
    Xt, yt, Xh, yh = X[~held].contiguous(), y[~held].contiguous(), X[held].contiguous(), y[held].contiguous()
    net = sa.Mlp(proposal.init_params(args.model_seed))
    t0 = time.perf_counter()
    losses = proposal.train(net, Xt, yt, epochs=args.epochs, batch=8192, lr=args.lr, seed=args.model_seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    auc = _auc(net.forward(Xh).float().cpu().numpy(), yh.cpu().numpy())
    log(f"[learned] held-out rows: {Xh.shape[0]}, ranking AUC of improving moves {auc:.3f}")
    del X, y, Xt, yt, Xh, yh

    p3, s3 = synth.load_workload("c3"), synth.bench_schedule("c3")
    P3 = sa.Problem(p3)
    n3, L3, S3 = s3["n_chains"], s3["steps_per_stage"], s3["n_stages"]
    x3 = torch.from_numpy(synth.start_vectors("c3", p3, n3)).cuda()
    hidden_cost = int(P3.eval_cost(torch.from_numpy(p3["hidden"][None, :]).cuda()).item())
    curves = {"plain": [], "learned": []}
    for k in range(args.seed_offset, args.seed_offset + args.eval_seeds):
        seed = s3["seed"] + 100 * k
        for kind in ("plain", "learned"):
            extra = dict(model=net, refresh_every=args.refresh, eps_plain=args.eps) if kind == "learned" else {}
            run = sa.Run(P3, x3, seed=seed, T0=s3["T0"], rho=s3["rho"], n_stages=S3, steps_per_stage=L3,
                         record_times=True, **extra)
            curves[kind].append(_curve(run, L3, n3))
            run.close()
            log(f"[learned] seed {seed} {kind}: final best {int(curves[kind][-1][1][-1])} "
                f"in {curves[kind][-1][0][-1]:.2f} s of stage kernels, "
                f"{curves[kind][-1][2]:.5f} of steps accepted improving moves")
    finals = {k: [int(c[1][-1]) for c in v] for k, v in curves.items()}
    target = args.target
    tt = {k: [_time_to(c, target) for c in v] for k, v in curves.items()}
    th = {k: [_time_to(c, hidden_cost) for c in v] for k, v in curves.items()}
    total = {k: [float(c[0][-1]) for c in v] for k, v in curves.items()}

    def med(vals):
        """Median with runs that never reach the target counted as infinitely
        slow (None when that median is infinite)."""
        m = float(np.median([np.inf if v is None else v for v in vals]))
        return m if np.isfinite(m) else None

    def boot_median_ci(vals, reps=4000, seed=0):
        """95% bootstrap interval of the median (unreached = infinitely slow;
        an infinite end is reported as None)."""
        x = np.array([np.inf if v is None else v for v in vals], dtype=np.float64)
        rng = np.random.default_rng(seed)
        meds = np.median(x[rng.integers(0, len(x), size=(reps, len(x)))], axis=1)
        lo = np.percentile(meds, 2.5, method="lower")
        hi = np.percentile(meds, 97.5, method="higher")
        return [float(lo) if np.isfinite(lo) else None, float(hi) if np.isfinite(hi) else None]

    # paired by seed: the learned run reaches the target first (ties and
    # double misses are neither), with a two-sided sign test
    wins = losses_ = 0
    for a, b in zip(tt["learned"], tt["plain"]):
        la, pb = np.inf if a is None else a, np.inf if b is None else b
        wins += la < pb
        losses_ += pb < la
    from math import comb
    n_sign = wins + losses_
    p_sign = min(1.0, 2 * sum(comb(n_sign, i) for i in range(0, min(wins, losses_) + 1)) / 2 ** n_sign) \
        if n_sign else 1.0
    value = med(tt["learned"])
    out = {
        "metric": "c3 stage-kernel time to the target cost (fixed before the evaluation), learned proposal",
        "value": value, "unit": "s",
        "n_gpus": 1, "steps": S3, "warmup": 0, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4 simulation, bf16 network",
        "data": f"synthetic (traces from {args.trace_workload} plain runs; evaluation on the stored c3 workload)",
        "config": {"workload": f"c3 ({n3} chains x {L3} steps x {S3} stages), network trained on {te}-strided "
                               f"traces of {args.trace_workload} plain runs", "refresh_every": args.refresh,
                   "eps_plain": args.eps,
                   "eval_seeds": args.eval_seeds, "epochs": args.epochs},
        "plain_time_to_target_s": tt["plain"], "learned_time_to_target_s": tt["learned"],
        "plain_median_s": med(tt["plain"]), "target_cost": target,
        "seeds": [s3["seed"] + 100 * k for k in range(args.seed_offset, args.seed_offset + args.eval_seeds)],
        "median_ci95_s": {k: boot_median_ci(v) for k, v in tt.items()},
        "paired_learned_first": wins, "paired_plain_first": losses_, "sign_test_p": p_sign,
        "final_best_median_ci95": {k: boot_median_ci(v) for k, v in finals.items()},
        "learned_over_plain": (value / med(tt["plain"])) if value is not None and med(tt["plain"]) else None,
        "learned_median_incl_trace_and_training_s": (value + t_collect + t_train) if value is not None else None,
        "reached": {k: sum(v is not None for v in vals) for k, vals in tt.items()},
        "final_best_median": {k: float(np.median(v)) for k, v in finals.items()},
        "hidden_params_cost": hidden_cost, "plain_time_to_hidden_s": th["plain"],
        "learned_time_to_hidden_s": th["learned"],
        "reached_hidden": {k: sum(v is not None for v in vals) for k, vals in th.items()}, "final_best": finals,
        "schedule_stage_kernel_s": total, "trace_collect_s": t_collect, "train_s": t_train,
        "train_epoch_losses": losses, "improving_fraction": pos, "held_out_auc": auc,
        "improving_steps_fraction": {k: [c[2] for c in v] for k, v in curves.items()},
    }
    print(json.dumps(out), flush=True)
    net.close()
    return 0


def bench_learned_cost(args) -> int:
    """Per-stage cost of the learned kernel on c3 against the plain stage
    kernel: the learned kernel without a network (refreshing the per-node
    aggregates only) and with a network at several refresh intervals.  The
    network's weights do not change the work; a freshly initialised one is
    used.  One JSON line per configuration, mean stage-kernel ms over the
    stages after the first."""
    import torch
    from paper_2506_19866_amd import proposal, sa, synth
    prob, s = synth.load_workload("c3"), synth.bench_schedule("c3")
    n, L = s["n_chains"], s["steps_per_stage"]
    x0 = torch.from_numpy(synth.start_vectors("c3", prob, n)).cuda()
    P = sa.Problem(prob)
    net = sa.Mlp(proposal.init_params(args.model_seed))
    trace = torch.zeros((n, sa.TRACE_RECORD_BYTES), dtype=torch.uint8, device="cuda")
    configs = [("plain", {})]
    for R in args.refresh_list:
        configs.append((f"aggregates only, refresh {R}", dict(trace=trace, trace_every=1 << 30, refresh_every=R)))
        configs.append((f"learned, refresh {R}", dict(model=net, refresh_every=R, eps_plain=args.eps)))
    for label, kw in configs:
        run = sa.Run(P, x0, seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=args.steps, steps_per_stage=L,
                     record_times=True, **kw)
        ms = run.stage_times_ms()
        run.close()
        print(json.dumps({"config": label, "stage_ms": float(np.mean(ms[1:] if len(ms) > 1 else ms)),
                          "stages": args.steps}), flush=True)
    net.close()
    return 0


# default target costs of the sweep per workload
SWEEP_TARGETS = {"c1": [10, 5, 0], "c2": [400, 350, 300], "c3": [1400, 1350, 1300], "q1": [5, 0],
                 "q2": [60, 50, 44], "q3": [20, 10, 5, 0]}


def bench_sweep(args) -> int:
    """Chain-count sweep over the thread counts of the paper's Table 2 (32,
    256, 1024, 10240, 102400) on the full schedule of --workload (c3 by
    default; q3 is the paper's own model at the Mtb network's size), with
    Table 1's global restart and with the island restart in groups of --group
    chains (the reduction suggested in §4).  One JSON line per configuration:
    throughput, stage-kernel time of the schedule, final best cost and the
    stage-kernel time until the global best first reaches each target cost."""
    import torch
    from paper_2506_19866_amd import sa, synth
    name = args.workload if args.workload != "c4" else "c3"
    if args.targets is None:
        args.targets = SWEEP_TARGETS[name]
    prob, s = synth.load_workload(name), synth.bench_schedule(name)
    L, S = s["steps_per_stage"], s["n_stages"]
    P = sa.Problem(prob)
    for n in args.chain_list:
        x0 = torch.from_numpy(synth.start_vectors(name, prob, n)).cuda()
        for group in (0, args.group):
            if group and group >= n:
                continue
            run = sa.Run(P, x0, seed=s["seed"], T0=s["T0"], rho=s["rho"], n_stages=S, steps_per_stage=L,
                         record_times=True, group_size=group)
            ms = run.stage_times_ms()
            best = run.stats()["best_cost"]
            run.close()
            t = np.cumsum(ms) * 1e-3
            reach = {}
            for target in args.targets:
                hit = np.nonzero(best <= target)[0]
                reach[str(target)] = float(t[hit[0]]) if hit.size else None
            out = {"workload": name, "chains": n, "restart": f"island {group}" if group else "global", "stages": S,
                   "chain_steps_per_s": n * L * S / float(t[-1]), "schedule_stage_kernel_s": float(t[-1]),
                   "final_best": int(best[-1]), "time_to_target_s": reach}
            log(f"[sweep] {out}")
            print(json.dumps(out), flush=True)
        del x0
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed temperature stages")
    ap.add_argument("--warmup", type=int, default=2, help="untimed stages on a discarded run")
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "q1", "q2", "q3"],
                    help="c4 = the batched workload (256 uneven networks, one persistent launch per stage); "
                         "q1-q3 = the paper's priority-update model (q2 HPG-sized, q3 Mtb-sized)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mode", default="throughput",
                    choices=["throughput", "learned", "learned-cost", "sweep", "peaks"],
                    help="learned: train the proposal network on c2 traces and compare time-to-target on c3; "
                         "learned-cost: per-stage cost of the learned kernel against the plain one on c3; "
                         "sweep: chain counts of the paper's Table 2 with global and island restarts on c3")
    ap.add_argument("--chain-list", type=int, nargs="+", default=[32, 256, 1024, 10240, 102400])
    ap.add_argument("--group", type=int, default=32, help="sweep: chains per island restart group")
    ap.add_argument("--targets", type=int, nargs="+", default=None,
                    help="sweep: target costs (default per workload)")
    ap.add_argument("--refresh-list", type=int, nargs="+", default=[16, 64, 256])
    ap.add_argument("--trace-rows", type=int, default=1 << 20)
    ap.add_argument("--trace-workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--refresh", type=int, default=256, help="learned: steps between proposal-table refreshes")
    ap.add_argument("--eps", type=float, default=0.9,
                    help="learned: fraction of candidates drawn by Table 1's plain rule")
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--seed-offset", type=int, default=10,
                    help="learned: first evaluation seed index k (run seed 2003 + 100 k); 0-9 chose R and eps")
    ap.add_argument("--target", type=int, default=1277,
                    help="learned: target cost, fixed before the evaluation")
    ap.add_argument("--model-seed", type=int, default=2005)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer five times: the reference kernel of known "
                         "traffic that scales the HBM byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU (asked for {max(args.gpus, world)}): the multi-GPU path is "
              "a design (one all-reduce of the 64-bit best key per stage), not a build", file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)
        return 0
    from paper_2506_19866_amd import sa, synth
    if args.mode == "peaks":
        peaks = measured_peaks()
        print(json.dumps({"mode": "peaks",
                          "unit": "lane-ops/s (valu_*), values/s (cvt_*), flop/s (mfma_*), bytes/s (lds_read)",
                          "derived_alu_peak": ALU_PEAK_OPS, "published_fp4_dense_peak": FP4_DENSE_PEAK_FLOPS,
                          **peaks}), flush=True)
        return 0
    if args.mode == "learned":
        return bench_learned(args)
    if args.mode == "learned-cost":
        return bench_learned_cost(args)
    if args.mode == "sweep":
        return bench_sweep(args)

    name = args.workload
    if name == "c4":
        return bench_batch(args)
    prob = synth.load_workload(name)
    sched = synth.bench_schedule(name)
    n, L = sched["n_chains"], sched["steps_per_stage"]
    priority = prob.get("model", 0) == synth.MODEL_PRIORITY
    x0 = torch.from_numpy(synth.start_vectors(name, prob, n)).cuda()
    P = sa.Problem(prob)
    log(f"[bench] workload {name}: N={prob['n_nodes']} E={prob['n_edges']} "
        f"P={P.n_params} C={prob['n_cond']} chains={n} L={L}")
    torch.cuda.synchronize()

    if args.warmup > 0:
        warm = sa.Run(P, x0, seed=sched["seed"] + 1, T0=sched["T0"], rho=sched["rho"],
                      n_stages=args.warmup, steps_per_stage=L)
        warm.best()
        warm.close()
        log(f"[bench] warmup: {args.warmup} stages done")

    run = sa.Run(P, x0, seed=sched["seed"], T0=sched["T0"], rho=sched["rho"], n_stages=args.steps,
                 steps_per_stage=L, launch=False, record_times=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.launch(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = run.stats()
    stage_ms = run.stage_times_ms()
    info = run.info()
    _, best_cost, _ = run.best()
    chain_steps = n * L * args.steps
    value = chain_steps / elapsed
    log(f"[bench] {args.steps} stages in {elapsed:.3f} s: {value:.4g} chain-steps/s, "
        f"best cost {best_cost} (stage 0 best {int(stats['best_cost'][0])})")

    # roofline of the stage kernel: algorithmic ALU work of the simulations it
    # ran (one per chain at stage start and one per feasible proposal, less the
    # priority model's candidates that keep the current trajectory)
    per_sim = algorithmic_alu_ops_priority(prob) if priority else algorithmic_alu_ops(prob)
    sims = stats["simulated"].astype(np.float64)
    ops_per_launch = float(np.mean(sims)) * per_sim
    avg_launch_s = float(np.mean(stage_ms)) * 1e-3
    launch_key = f"{name}:{n}x{L}"
    if priority:
        lc = 16 if prob["n_nodes"] <= 16 else 32 if prob["n_nodes"] <= 32 else 64
        max_in = int(np.diff(prob["row_ptr"]).max())
        kernel = f"pr_stage_kernel<{lc},{0 if lc <= 32 else 8 if max_in <= 8 else 16 if max_in <= 16 else 0}>"
        traffic = traffic_from_profiles(launch_key, "priority")
        model = (f"the paper's priority-update model, {prob['n_nodes']} nodes, {prob['n_edges']} edges, "
                 f"{P.n_params} params (w, p, t per edge; u, m, d per node)")
    else:
        hold = "false" if P.info["clamps_by_offset"] else "true"
        kernel = f"stage_kernel<{info['tiles_m']},{info['frags_k']},{int(prob.get('step_size', 1))},{hold}>"
        traffic = traffic_from_profiles(launch_key)
        model = (f"Mtb-scale, {prob['n_nodes']} nodes, {prob['n_edges']} edges, {P.n_params} ternary params "
                 f"(synchronous update)")
    peaks = measured_peaks()
    log(f"[bench] measured peaks: VALU {peaks['valu'] / 1e12:.1f} T lane-ops/s, fp4 conversion "
        f"{peaks['cvt_fp4'] / 1e12:.1f} T values/s, fp4 matrix {peaks['mfma_fp4'] / 1e12:.0f} TFLOP/s")
    counters = counters_from_profiles(launch_key, "priority" if priority else "stage")
    macs = dense = None
    if not priority:
        sims_mean = float(np.mean(sims))
        macs = sims_mean * regulator_macs(prob)
        t_last = int(np.max(prob["obs_t"]))
        cols = -(-prob["n_cond"] // 16) * 16
        dense = sims_mean * cols * t_last * 16 * info["tiles_m"] * 128 * info["frags_k"]
    sims_mean = float(np.mean(sims))
    if priority:
        # every simulated step reads one observation dword per lane, and each
        # node-lane fetches its regulators' states by one lane permute per
        # regulator slot (LDS-pipe traffic, 4 bytes per lane)
        steps = prob["n_cond"] * (prob["n_steps"] + 1)
        lc = 16 if prob["n_nodes"] <= 16 else 32 if prob["n_nodes"] <= 32 else 64
        max_in = int(np.diff(prob["row_ptr"]).max())
        slots = 0 if lc <= 32 else 8 if max_in <= 8 else 16 if max_in <= 16 else 0
        per_sim = steps * lc * 4 + prob["n_cond"] * prob["n_steps"] * lc * slots * 4
        lds_what = ("per simulation C*(T+1)*LC observation dwords + C*T*LC*slots lane-permute dwords, 4 bytes each "
                    "(the permutes are the kernel's own gathers, not algorithmic reads)")
    else:
        # the scoring reads, at every observed time, the reference and weight
        # dwords of the lane's observed slots from LDS
        cg = -(-prob["n_cond"] // 16)
        per_sim = len(prob["obs_t"]) * P.info["obs_dwords"] * 2 * 4 * 64 * cg
        lds_what = "per simulation K x (scored dwords) x 2 tables x 4 bytes x 64 lanes x condition groups"
    roofline = alu_roofline(ops_per_launch, avg_launch_s, peaks, kernel, traffic, counters, macs, dense,
                            sims_mean * per_sim, lds_what)
    roofline["simulations_per_launch"] = float(np.mean(sims))
    roofline["candidates_per_launch"] = float(n * L)
    out = {
        "metric": "SA chain-steps/s at 723-param scale" if P.n_params == 723 else "SA chain-steps/s",
        "value": value, "unit": "chain-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32" if priority else "fp4",
        "data": "synthetic (seeded generator + oracle-simulated reference data, stored workload)",
        "config": {"workload": f"{name}: {model}, {prob['n_cond']} conditions, "
                               f"{prob['n_steps']} steps; {n} chains x {L} steps per stage, "
                               f"{args.steps} stages of a {sched['n_stages']}-stage schedule T0={sched['T0']}",
                   "chains": n, "steps_per_stage": L, "stages_timed": args.steps,
                   "best_cost": int(best_cost)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(name, prob, sched, args.cpu_seconds)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.4g} chain-steps/s "
            f"on {out['cpu_baseline']['cores']} threads")
    print(json.dumps(out), flush=True)
    run.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
