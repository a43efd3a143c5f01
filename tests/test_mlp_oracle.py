"""The float64 screen reference against finite differences, closed forms and
library routines (torch CPU autograd, torch's bfloat16 cast, torch Adam)."""
import numpy as np
import torch

from oracle import mlp_ref
from workloads import mlp_init


def small_params(seed=3, dims=(32, 16, 16, 16, 12)):
    return [(W.astype(np.float64), b.astype(np.float64) + 0.01 * np.arange(len(b)))
            for W, b in mlp_init(seed, dims)]


def batch(seed=4, B=5):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 32))
    y = (rng.random((B, 8)) < 0.5).astype(float)
    m = (rng.random((B, 8)) < 0.8).astype(float)
    h = rng.dirichlet(np.ones(4), size=B)
    return X, y, m, h


def total_loss(params, X, y, m, h):
    _, z = mlp_ref.forward(params, X)
    return mlp_ref.loss(z, y, m, h)[0]


def test_bf16_round_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10 ** rng.uniform(-30, 30, size=5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -3.0e38, 1e-40]])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp_ref.bf16_round(x)
    assert np.array_equal(got, want)


def test_gradients_match_central_differences():
    params = small_params()
    X, y, m, h = batch()
    acts, z = mlp_ref.forward(params, X)
    _, dz = mlp_ref.loss(z, y, m, h)
    grads = mlp_ref.backward(params, acts, dz)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for li, (W, bv) in enumerate(params):
        for which, P, G in ((0, W, grads[li][0]), (1, bv, grads[li][1])):
            for _ in range(12):
                idx = tuple(rng.integers(0, s) for s in P.shape)
                old = P[idx]
                P[idx] = old + eps
                lp = total_loss(params, X, y, m, h)
                P[idx] = old - eps
                lm = total_loss(params, X, y, m, h)
                P[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - G[idx]) <= 1e-6 * max(1.0, abs(fd)), (li, which, idx, fd, G[idx])


def test_gradients_match_torch_autograd():
    params = small_params(dims=(32, 256, 256, 256, 12))
    X, y, m, h = batch(B=17)
    acts, z = mlp_ref.forward(params, X)
    L, dz = mlp_ref.loss(z, y, m, h)
    grads = mlp_ref.backward(params, acts, dz)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    t = torch.tensor(X)
    for i, (W, b) in enumerate(tp):
        t = t @ W.T + b
        if i < len(tp) - 1:
            t = torch.relu(t)
    zs, zh = t[:, :8], t[:, 8:12]
    bce = torch.nn.functional.binary_cross_entropy_with_logits(zs, torch.tensor(y), reduction="none")
    Lt = ((torch.tensor(m) * bce).sum() + ((zh - torch.tensor(h)) ** 2).sum()) / X.shape[0]
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-12
    for (gW, gb), (W, b) in zip(grads, tp):
        assert np.allclose(gW, W.grad.numpy(), rtol=1e-10, atol=1e-13)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_single_linear_layer_l2_closed_form():
    """One linear layer, L2 loss on all outputs: dL/dW = (2/B) (y - t)^T x."""
    rng = np.random.default_rng(5)
    W = rng.normal(size=(4, 32))
    b = rng.normal(size=4)
    X = rng.normal(size=(6, 32))
    T = rng.normal(size=(6, 4))
    acts, z = mlp_ref.forward([(W, b)], X)
    dz = 2.0 * (z - T) / 6
    (gW, gb), = mlp_ref.backward([(W, b)], acts, dz)
    assert np.allclose(gW, (2.0 / 6) * (X @ W.T + b - T).T @ X)
    assert np.allclose(gb, (2.0 / 6) * (X @ W.T + b - T).sum(0))


def test_adam_matches_torch():
    params = small_params()
    X, y, m, h = batch()
    state = {}
    tp = [torch.tensor(p, requires_grad=True) for W, b in params for p in (W, b)]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(3):
        acts, z = mlp_ref.forward(params, X)
        _, dz = mlp_ref.loss(z, y, m, h)
        grads = mlp_ref.backward(params, acts, dz)
        opt.zero_grad()
        for k, (gW, gb) in enumerate(grads):
            tp[2 * k].grad = torch.tensor(gW)
            tp[2 * k + 1].grad = torch.tensor(gb)
        opt.step()
        params = mlp_ref.adam_step(params, grads, state, lr=1e-2)
    for k, (W, b) in enumerate(params):
        assert np.allclose(W, tp[2 * k].detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(b, tp[2 * k + 1].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_hand_worked():
    """Neuron F=3, b=2 (dmax 3), o=2, w=(2,-1,0), bias -5, T=(1,3,5), ReLU."""
    X = mlp_ref.features([3], [2], [2], [1], [[2, -1, 0, 0, 0, 0, 0, 0]], [-5],
                         [[1, 3, 5, 0, 0, 0, 0]])[0]
    want = np.zeros(32)
    want[0:3] = [2 / 8, -1 / 8, 0]
    want[8:11] = [6 / 32, -3 / 32, 0]
    want[16] = -5 / 16
    want[17:24] = [1 / 32, 3 / 32, 5 / 32, 5 / 32, 5 / 32, 5 / 32, 5 / 32]
    want[24] = (-5 + 6) / 32
    want[25] = (-5 - 3) / 32
    want[26] = 2 / 4
    want[28] = 1.0
    want[30] = 3 / 8
    want[31] = 1.0
    assert np.array_equal(X, want)


def test_labels_binning():
    y, m, h = mlp_ref.labels([2, 3, 2], [1, 1, 2], [1, 3, 2], [0b10, 0b101, 0b11],
                             [[1, 3, 0, 0, 0, 0, 0, 0], [1, 1, 1, 1, 1, 1, 1, 1], [2, 4, 4, 6, 0, 0, 0, 0]])
    assert list(m[0]) == [1, 1, 0, 0, 0, 0, 0, 0] and list(y[0]) == [0, 1, 0, 0, 0, 0, 0, 0]
    assert list(y[1]) == [1, 0, 1, 0, 0, 0, 0, 0]
    assert list(h[0]) == [0.25, 0.75, 0, 0]
    assert list(h[1]) == [0.25, 0.25, 0.25, 0.25]
    assert list(h[2]) == [2 / 16, 4 / 16, 4 / 16, 6 / 16]
