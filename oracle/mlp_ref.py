"""float64 NumPy reference of the learned screen -- TEST INFRASTRUCTURE ONLY.

The screen is a plain multilayer perceptron 32 -> 256 -> 256 -> 256 -> 12
with ReLU hidden layers.  Output columns 0..7 are per-input support logits,
columns 8..11 predict the 4-bin output histogram (fractions of all rows).

Loss, averaged over the batch of size B:

    L = (1/B) sum_i sum_{j<8} m_ij * BCE(z_ij, y_ij)
      + (1/B) sum_i sum_{v<4} (z_i,8+v - h_iv)^2

BCE is binary cross-entropy on logits; m masks inputs j >= F.  The squared
(L2) error on the histogram columns is the same kind of regression loss the
paper minimises by gradient descent in its multi-output regression
formulation (its Methodology section, the loss summed over outputs of the
squared difference from the targets).  Optimiser: Adam with bias correction
(Kingma and Ba), fp32 master weights on the device.

Everything here is written out directly (matrix products are the only library
primitive) so it can be checked line by line; BF16 rounding, where a test asks
for it, is round-to-nearest-even on the float32 bit pattern.
"""
from __future__ import annotations

import numpy as np

DIMS = (32, 256, 256, 256, 12)
N_SUP = 8
N_HIST = 4


# ----------------------------------------------------------------- numerics
def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64.
    The input is first rounded to float32, as on the device."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out.astype(np.float64)


# ----------------------------------------------------------------- features
def features(F, b, o, act, w, bias, thr) -> np.ndarray:
    """Screen input features [n, 32] from neuron descriptors.

    0..7   w_j / 8                      (0 for j >= F)
    8..15  w_j * (2^b - 1) / 32         largest contribution of input j
    16     bias / 16
    17..23 t_k / 32 for k < 2^o - 1, then the last used threshold repeated
    24     (bias + sum_j max(w_j, 0) * (2^b - 1)) / 32   largest pre-activation
    25     (bias + sum_j min(w_j, 0) * (2^b - 1)) / 32   smallest pre-activation
    26     b / 4
    27..29 one-hot of o in {1, 2, 3}
    30     F / 8
    31     act
    """
    n = len(F)
    X = np.zeros((n, 32), np.float64)
    for i in range(n):
        f, bb, oo = int(F[i]), int(b[i]), int(o[i])
        dmax = (1 << bb) - 1
        ws = [int(w[i][j]) if j < f else 0 for j in range(8)]
        for j in range(8):
            X[i, j] = ws[j] / 8.0
            X[i, 8 + j] = ws[j] * dmax / 32.0
        X[i, 16] = int(bias[i]) / 16.0
        K = (1 << oo) - 1
        for k in range(7):
            X[i, 17 + k] = int(thr[i][min(k, K - 1)]) / 32.0
        X[i, 24] = (int(bias[i]) + sum(max(v, 0) for v in ws) * dmax) / 32.0
        X[i, 25] = (int(bias[i]) + sum(min(v, 0) for v in ws) * dmax) / 32.0
        X[i, 26] = bb / 4.0
        X[i, 27 + (oo - 1)] = 1.0
        X[i, 30] = f / 8.0
        X[i, 31] = float(act[i])
    return X


def labels(F, b, o, support, hist):
    """Targets: support bits y [n, 8], valid-input mask m [n, 8] and the
    4-bin histogram as fractions of 2^(F*b) rows [n, 4].  With o = 1 the bins
    are {0, 1} (bins 2, 3 zero); with o = 2 they are q itself; with o = 3
    bin v holds codes 2v and 2v + 1."""
    n = len(F)
    y = np.zeros((n, 8))
    m = np.zeros((n, 8))
    h = np.zeros((n, 4))
    for i in range(n):
        f = int(F[i])
        rows = float(1 << (f * int(b[i])))
        for j in range(8):
            m[i, j] = 1.0 if j < f else 0.0
            y[i, j] = float((int(support[i]) >> j) & 1) if j < f else 0.0
        hh = [int(v) for v in hist[i]]
        oo = int(o[i])
        if oo == 1:
            bins = [hh[0], hh[1], 0, 0]
        elif oo == 2:
            bins = hh[:4]
        else:
            bins = [hh[0] + hh[1], hh[2] + hh[3], hh[4] + hh[5], hh[6] + hh[7]]
        h[i] = np.array(bins, dtype=np.float64) / rows
    return y, m, h


# ----------------------------------------------------------------- network
def forward(params, X, bf16=False):
    """params: list of (W [out, in], b [out]).  Returns (acts, z): acts[l] is
    the input of layer l (acts[0] = X), z the logits.  With bf16=True every
    GEMM operand (inputs, hidden activations, weights) is rounded to bf16 and
    accumulation is exact (float64), as a reference for a bf16 kernel that
    accumulates in fp32; biases stay fp32."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    h = rnd(X)
    acts = [h]
    for li, (W, bvec) in enumerate(params):
        z = h @ rnd(W).T + np.asarray(bvec, np.float64)[None, :]
        if li < len(params) - 1:
            h = rnd(np.maximum(z, 0.0))
            acts.append(h)
        else:
            return acts, z
    raise ValueError("empty network")


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(z, y, m, h):
    """Returns (L, dL/dz) for logits z [B, 12]."""
    B = z.shape[0]
    zs = z[:, :N_SUP]
    zh = z[:, N_SUP:N_SUP + N_HIST]
    bce = softplus(zs) - y * zs
    L = (np.sum(m * bce) + np.sum((zh - h) ** 2)) / B
    dz = np.zeros_like(z)
    dz[:, :N_SUP] = m * (sigmoid(zs) - y) / B
    dz[:, N_SUP:N_SUP + N_HIST] = 2.0 * (zh - h) / B
    return L, dz


def backward(params, acts, dz, bf16=False):
    """Gradients [(dW, db)] of the loss through the network given dL/dz.
    With bf16=True the GEMM operands of the backward pass (weights, stored
    activations and the incoming gradients) are rounded to bf16, matching a
    kernel that keeps gradients in bf16 between layers and accumulates in
    fp32."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    grads = [None] * len(params)
    g = rnd(dz)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        a = acts[li]
        grads[li] = (g.T @ a, np.sum(g, axis=0))
        if li > 0:
            gin = g @ rnd(W)
            g = rnd(gin * (acts[li] > 0))
    return grads


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; state = {'t': int, 'm': [...], 'v': [...]}."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(W), np.zeros_like(bv)] for W, bv in params]
        state["v"] = [[np.zeros_like(W), np.zeros_like(bv)] for W, bv in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for li, ((W, bv), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for k, (p, g) in enumerate(((W, gW), (bv, gb))):
            m = state["m"][li][k] = beta1 * state["m"][li][k] + (1 - beta1) * g
            v = state["v"][li][k] = beta2 * state["v"][li][k] + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out
