"""The proposal network's GPU kernels (bf16 MFMA, float32 accumulation)
against the float64 reference of oracle/mlp_reference.py, through the C ABI.

Every comparison is element by element.  Inputs and weights are bf16 on both
sides, so products are exact; what differs is float32 accumulation (about
1e-6 relative), the bf16 rounding of the hidden activations (one bf16 ulp,
2^-8 relative, where float32 and float64 pre-activations round to different
sides of a bf16 boundary), and in training the bf16 rounding of dZ before the
dW1 product (2^-9 relative per term).  Hence the bounds, stated per element:
  logit_r:   2^-8 * l1_r,                 l1_r = sum_h |a_rh| |w2_h|
  dW1[k,h]:  2^-8 * sum_r |X_rk| |w2_h| (|dlogit_r| + l1_r / n)
  dw2[h]:    2^-8 * sum_r |a_rh| (|dlogit_r| + l1_r / n)
  db2:       2^-8 * sum_r (|dlogit_r| + l1_r / n)
(the l1_r / n term covers the change of dlogit_r = (sigmoid(logit_r) - y_r)/n
under the logit's own error, at most a quarter of it over n).  The Adam
update is checked separately from the gradient: the reference applies
mlp_reference.adam in float64 to the GPU's own float32 gradients, so what is
compared is the update's float32 arithmetic, bounded per element by
t * (2^-20 * lr + 2^-22 * |w|) after t steps."""
import numpy as np
import pytest

from oracle import mlp_reference as M
from oracle.learned import logits as oracle_logits

pytestmark = pytest.mark.gpu


def _params(rng, scale=0.3):
    W1 = rng.normal(size=(32, 256)) * scale
    w2 = rng.normal(size=256) * scale / 4
    return W1, w2, 0.25


def _rows(rng, n):
    X = rng.normal(size=(n, 32))
    X[:, 24:31] = 0
    X[:, 31] = 1
    X[:, :7] = rng.integers(0, 2, size=(n, 7))
    return M.bf16(X)


def _tensor_bf16(X):
    import torch
    return torch.from_numpy(np.asarray(X, dtype=np.float32)).to(torch.bfloat16).cuda()


@pytest.mark.parametrize("n", [1, 15, 16, 1000, 4099])
def test_forward_matches_reference(n):
    import torch
    from paper_2506_19866_amd import sa
    rng = np.random.default_rng(n)
    W1, w2, b2 = _params(rng)
    X = _rows(rng, n)
    net = sa.Mlp(sa.pack_mlp_params(W1, w2, b2))
    got = net.forward(_tensor_bf16(X)).cpu().numpy().astype(np.float64)
    model = {"W1": W1.astype(np.float32), "w2": w2.astype(np.float32), "b2": b2}
    ref = oracle_logits(model, X)
    a = M.bf16(np.maximum(X @ M.bf16(W1.astype(np.float32)), 0))
    l1 = np.abs(a) @ np.abs(M.bf16(w2.astype(np.float32)))
    assert np.all(np.abs(got - ref) <= 4e-3 * l1 + 1e-5), np.max(np.abs(got - ref))
    net.close()
    torch.cuda.synchronize()


def _ref_grads(W1, w2, b2, X, y):
    W1b, w2b = M.bf16(W1.astype(np.float32)), M.bf16(w2.astype(np.float32))
    g = M.grads(X, y, W1b, np.zeros(256), w2b, float(np.float32(b2)), round_hidden=True)
    return np.concatenate([g["W1"].reshape(-1), g["W2"], [g["b2"]]]), \
        M.loss(X, y, W1b, np.zeros(256), w2b, float(np.float32(b2)), round_hidden=True)


def _grad_bounds(W1, w2, b2, X, y):
    """Per-element bounds of the GPU gradient's deviation from the reference
    (module docstring)."""
    W1b, w2b = M.bf16(W1.astype(np.float32)), M.bf16(w2.astype(np.float32))
    n = X.shape[0]
    _, Hb, logit = M.forward(X, W1b, np.zeros(256), w2b, float(np.float32(b2)), round_hidden=True)
    dlogit = (1.0 / (1.0 + np.exp(-logit)) - y) / n
    l1 = np.abs(Hb) @ np.abs(w2b)
    s = np.abs(dlogit) + l1 / n
    eps = 2.0 ** -8
    bw1 = eps * np.outer(np.abs(X).T @ s, np.abs(w2b))       # [32, 256]
    bw2 = eps * (np.abs(Hb).T @ s)
    bb2 = eps * s.sum()
    return np.concatenate([bw1.reshape(-1), bw2, [bb2]]) + 1e-12


@pytest.mark.parametrize("n", [1, 33, 512, 70001])
def test_gradients_match_reference(n):
    import torch
    from paper_2506_19866_amd import sa
    rng = np.random.default_rng(100 + n)
    W1, w2, b2 = _params(rng)
    X = _rows(rng, n)
    y = (rng.random(n) < 0.3).astype(np.float32)
    net = sa.Mlp(sa.pack_mlp_params(W1, w2, b2))
    g, loss = net.gradients(_tensor_bf16(X), torch.from_numpy(y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    ref, ref_loss = _ref_grads(W1, w2, b2, X, y)
    bound = _grad_bounds(W1, w2, b2, X, y)
    err = np.abs(g - ref)
    for name, sl in (("W1", slice(0, 8192)), ("w2", slice(8192, 8448)), ("b2", slice(8448, 8449))):
        worst = int(np.argmax(err[sl] / bound[sl]))
        assert np.all(err[sl] <= bound[sl]), (name, worst, g[sl][worst], ref[sl][worst], bound[sl][worst])
    # features 24..30 are zero in every row: their W1 gradients are exactly zero on both sides
    assert np.all(g[24 * 256:31 * 256] == 0) and np.all(ref[24 * 256:31 * 256] == 0)
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * abs(ref_loss) + 1e-6
    # deterministic: the partials are reduced in a fixed order
    g2, _ = net.gradients(_tensor_bf16(X), torch.from_numpy(y).cuda())
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)
    net.close()


@pytest.mark.parametrize("n,steps", [(3000, 4), (70001, 3)])
def test_adam_steps_match_reference(n, steps):
    """Several sa_mlp_train_step calls against mlp_reference.adam (beta1 0.9,
    beta2 0.999, eps 1e-8) fed with the GPU's own gradients at each step: the
    moments, the bias corrections at t = 1..steps and the update arithmetic,
    element by element."""
    import torch
    from paper_2506_19866_amd import sa
    rng = np.random.default_rng(300 + n)
    W1, w2, b2 = _params(rng)
    X = _rows(rng, n)
    y = (rng.random(n) < 0.4).astype(np.float32)
    xt, yt = _tensor_bf16(X), torch.from_numpy(y).cuda()
    flat = sa.pack_mlp_params(W1, w2, b2)
    net = sa.Mlp(flat)
    lr = 2e-3
    ref = {"p": flat.astype(np.float32).astype(np.float64)}
    state = {}
    for t in range(1, steps + 1):
        g, _ = net.gradients(xt, yt)               # the gradient train_step reduces, bit for bit
        net.train_step(xt, yt, lr)
        M.adam(ref, {"p": g.cpu().numpy().astype(np.float64)}, state, lr=lr)
        got = net.params().astype(np.float64)
        bound = t * (2.0 ** -20 * lr + 2.0 ** -22 * np.abs(ref["p"]))
        err = np.abs(got - ref["p"])
        worst = int(np.argmax(err / bound))
        assert np.all(err <= bound), (t, worst, got[worst], ref["p"][worst], bound[worst])
        # the steps are not trivial: most weights moved by a sizeable part of lr at this step
        if t == 1:
            assert np.mean(np.abs(got - flat) > 0.5 * lr) > 0.5
    net.close()


def test_adam_step_and_fragment_refresh():
    import torch
    from paper_2506_19866_amd import sa
    rng = np.random.default_rng(7)
    W1, w2, b2 = _params(rng)
    n = 3000
    X = _rows(rng, n)
    y = (rng.random(n) < 0.4).astype(np.float32)
    flat = sa.pack_mlp_params(W1, w2, b2)
    net = sa.Mlp(flat)
    assert np.array_equal(net.params(), flat)
    lr = 1e-3
    loss = net.train_step(_tensor_bf16(X), torch.from_numpy(y).cuda(), lr)
    new = net.params().astype(np.float64)
    ref_g, ref_loss = _ref_grads(W1, w2, b2, X, y)
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * abs(ref_loss) + 1e-6
    # the first Adam step moves each weight by lr * g / (|g| + eps'): +-lr where g is clearly non-zero
    step = new - flat.astype(np.float64)
    big = np.abs(ref_g) > 0.05 * np.max(np.abs(ref_g))
    assert np.allclose(step[big], -lr * np.sign(ref_g[big]), rtol=1e-3, atol=1e-6)
    assert np.all(np.abs(step) <= lr * (1 + 1e-3))
    # the forward pass uses the updated weights
    p = sa.unpack_mlp_params(new)
    got = net.forward(_tensor_bf16(X[:257])).cpu().numpy().astype(np.float64)
    ref = oracle_logits(p, X[:257])
    a = M.bf16(np.maximum(X[:257] @ M.bf16(p["W1"]), 0))
    assert np.all(np.abs(got - ref) <= 4e-3 * (np.abs(a) @ np.abs(M.bf16(p["w2"]))) + 1e-5)
    # set_params restores the start and resets Adam: the same step again
    net.set_params(flat)
    net.train_step(_tensor_bf16(X), torch.from_numpy(y).cuda(), lr)
    assert np.array_equal(net.params().astype(np.float64), new)
    net.close()


def test_training_learns_a_separable_rule():
    import torch
    from paper_2506_19866_amd import sa
    rng = np.random.default_rng(11)
    W1, w2, _ = _params(rng, scale=0.1)
    n = 8192
    X = _rows(rng, n)
    y = (X[:, 8] - X[:, 9] > 0).astype(np.float32)
    net = sa.Mlp(sa.pack_mlp_params(W1, w2, 0.0))
    xt, yt = _tensor_bf16(X), torch.from_numpy(y).cuda()
    first = float(net.gradients(xt, yt)[1].item())
    for _ in range(150):
        loss = net.train_step(xt, yt, 3e-3)
    last = float(loss.item())
    assert last < 0.35 * first, (first, last)
    acc = ((net.forward(xt) > 0).float() == yt).float().mean().item()
    assert acc > 0.95
    net.close()
