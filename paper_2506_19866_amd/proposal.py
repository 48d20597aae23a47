"""Training the learned proposal: traced plain runs give (move features,
outcome) rows, the network is fitted to them with the library's training
kernels, and the trained network drives learned runs.

Plumbing only: the traces are written by the annealing kernel, the forward,
backward and Adam steps run in the library's kernels; torch slices the trace
records and shuffles row indices on the device.

The learned proposal is an extension of Table 1's GetCandidate (not in the
paper).  A row's label is 1 when its move was accepted and lowered the cost
(an improving move), else 0: neutral moves are accepted with certainty and
say nothing about descent.
"""
from __future__ import annotations

import numpy as np

from . import sa


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation of the 32 -> 256 -> 1 network (W1 scaled for
    the 24 used inputs, zero bias row, small output layer)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(sa.MLP_INPUTS, sa.MLP_HIDDEN)) * np.sqrt(2.0 / 24)
    W1[24:] = 0.0
    w2 = rng.normal(size=sa.MLP_HIDDEN) * np.sqrt(1.0 / sa.MLP_HIDDEN)
    return sa.pack_mlp_params(W1, w2, -2.0)


def trace_rows(trace):
    """Feature rows (bfloat16 [M, 32]), cost changes and flags (int32 [M]) of
    a trace tensor [n_chains, capacity * 80], on its device.  Slots a run did
    not reach (flags 0 and param 0 with all-zero features) are kept out."""
    import torch
    n = trace.shape[0]
    rec = trace.view(n, -1, sa.TRACE_RECORD_BYTES)
    feats = rec[:, :, :64].contiguous().view(torch.bfloat16).reshape(-1, sa.MLP_INPUTS)
    ints = rec[:, :, 64:].contiguous().view(torch.int32).reshape(-1, 4)
    delta, flags = ints[:, 2].contiguous(), ints[:, 3].contiguous()
    present = feats[:, 31] != 0          # input 31 is the constant 1 in every written record
    return feats[present].contiguous(), delta[present].contiguous(), flags[present].contiguous()


def improving_labels(delta, flags):
    import torch
    return (((flags & 1) != 0) & (delta < 0)).to(torch.float32)


def collect(problem: "sa.Problem", x0, *, seed: int, T0: float, rho: float, n_stages: int, steps_per_stage: int,
            trace_every: int, refresh_every: int = 16):
    """Runs a plain schedule with a step trace and returns (features, labels,
    run statistics)."""
    import torch
    n = x0.shape[0]
    total = n_stages * steps_per_stage
    cap = (total + trace_every - 1) // trace_every
    trace = torch.zeros((n, cap * sa.TRACE_RECORD_BYTES), dtype=torch.uint8, device=x0.device)
    run = sa.Run(problem, x0, seed=seed, T0=T0, rho=rho, n_stages=n_stages, steps_per_stage=steps_per_stage,
                 trace=trace, trace_every=trace_every, refresh_every=refresh_every)
    stats = run.stats()
    run.close()
    X, delta, flags = trace_rows(trace)
    return X, improving_labels(delta, flags), stats


def train(model: "sa.Mlp", X, y, *, epochs: int, batch: int, lr: float, seed: int, log=None):
    """Minibatch Adam over shuffled rows; returns the per-epoch mean losses."""
    import torch
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    M = X.shape[0]
    losses = []
    loss_buf = torch.zeros(1, dtype=torch.float32, device=X.device)
    for ep in range(epochs):
        perm = torch.randperm(M, generator=g, device=X.device)
        acc = torch.zeros(1, dtype=torch.float32, device=X.device)
        nb = 0
        for b0 in range(0, M, batch):
            idx = perm[b0:b0 + batch]
            model.train_step(X.index_select(0, idx).contiguous(), y.index_select(0, idx).contiguous(), lr,
                             loss=loss_buf)
            acc += loss_buf
            nb += 1
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"[train] epoch {ep}: mean batch loss {losses[-1]:.4f}")
    return losses
