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
