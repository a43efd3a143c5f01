"""Layered networks of neurons evaluated by the neuron definition itself --
TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Signals 0 .. P-1 are primary input codes; signal P + i is the output code of
neuron i.  Neuron i reads its input j (j < F_i) from signal fanin[i][j] and
takes that code modulo 2^b_i; its output is q of the definition: the integer
weighted sum plus bias, the activation, and the count of thresholds reached
(ties count as reached).  This is the per-row semantics the truth tables
hold, applied to one row per sample, so evaluating a network through its
tables must give the same codes.  Neurons must be in topological order
(every fanin signal below P + i).  Plain NumPy, vectorised over samples only.
"""
from __future__ import annotations

import numpy as np


def evaluate(ns, fanin, n_inputs: int, inputs) -> np.ndarray:
    """Output codes uint8 [batch, n] for primary input codes uint8 [batch, P]."""
    inputs = np.asarray(inputs)
    batch = inputs.shape[0]
    n = len(ns)
    sig = np.zeros((batch, n_inputs + n), np.int64)
    sig[:, :n_inputs] = inputs
    for i in range(n):
        F, b, o = int(ns.F[i]), int(ns.b[i]), int(ns.o[i])
        src = np.asarray(fanin[i][:F], np.int64)
        assert (src >= 0).all() and (src < n_inputs + i).all(), "not in topological order"
        x = sig[:, src] & ((1 << b) - 1)
        a = int(ns.bias[i]) + x @ ns.w[i, :F].astype(np.int64)
        if int(ns.act[i]) == 1:
            a = np.maximum(a, 0)
        K = (1 << o) - 1
        q = (a[:, None] >= ns.thr[i, :K].astype(np.int64)[None, :]).sum(1)
        sig[:, n_inputs + i] = q
    return sig[:, n_inputs:].astype(np.uint8)


# ---------------------------------------------------------------- sampling
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def splitmix64(seed: int, k) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number k >= 1
    of the stream seeded with ``seed`` -- the finaliser (xor-shift 30,
    multiply, xor-shift 27, multiply, xor-shift 31) of seed + k * gamma, all
    modulo 2^64 (NumPy uint64 arithmetic wraps)."""
    k = np.asarray(k, np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & (2**64 - 1)) + k * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def draws(seed: int, first: int, count: int, n_inputs: int) -> np.ndarray:
    """Raw input bytes uint8 [count, n_inputs] of draws first .. first+count-1:
    input j of draw d is byte j % 8 (little-endian) of SplitMix64 output
    d * Q + j // 8 + 1, Q = ceil(n_inputs / 8)."""
    Q = (n_inputs + 7) // 8
    d = np.arange(first, first + count, dtype=np.uint64)
    k = d[:, None] * np.uint64(Q) + np.arange(Q, dtype=np.uint64)[None, :] + np.uint64(1)
    z = splitmix64(seed, k)  # [count, Q]
    by = np.stack([(z >> np.uint64(8 * t)) & np.uint64(0xFF) for t in range(8)], axis=-1)  # [count, Q, 8]
    return by.reshape(count, Q * 8)[:, :n_inputs].astype(np.uint8)


def reader_masks(ns, fanin, n_inputs: int) -> np.ndarray:
    """Per primary input: 2^b - 1 when every neuron reading it takes b
    digits, else 0xFF (no readers, or readers of different b)."""
    seen = [set() for _ in range(n_inputs)]
    for i in range(len(ns)):
        for src in list(fanin[i])[: int(ns.F[i])]:
            if src < n_inputs:
                seen[src].add(int(ns.b[i]))
    return np.array([(1 << next(iter(s))) - 1 if len(s) == 1 else 0xFF for s in seen], np.uint8)


def sample(ns, fanin, n_inputs: int, targets: dict, seed: int, first: int, count: int):
    """Rejection sampling: the draws (in draw order) whose evaluation puts
    value v on signal s for every (s, v) in targets, and their inputs reduced
    by reader_masks.  Returns (draw numbers int64 [k], inputs uint8 [k, P])."""
    x = draws(seed, first, count, n_inputs) & reader_masks(ns, fanin, n_inputs)[None, :]
    out = evaluate(ns, fanin, n_inputs, x)
    sig = np.concatenate([x, out], axis=1)
    keep = np.ones(count, bool)
    for s, v in targets.items():
        keep &= sig[:, s] == v
    idx = np.nonzero(keep)[0]
    return (first + idx).astype(np.int64), x[idx]
