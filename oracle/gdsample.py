"""Gradient-descent sampling of a transformed CNF (the paper's Section on
the probabilistic model: Table 1, the sigmoid embedding, the L2 loss, GD,
hardening and the satisfiable / non-redundant filter) -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The circuit is what the transformation (``oracle/transform.py``) returns:
expressions in the order found, each a truth table over its variables.

* Probabilistic value of an expression: the multilinear extension of its
  table, P = sum over rows r of t(r) * prod_j (p_j if digit j of r is 1 else
  1 - p_j), the probability that the table outputs 1 when its inputs are
  independent with probabilities p_j.  For the gates of Table 1 this is the
  table's formula (NOT 1 - p, AND p1 p2, OR 1 - (1-p1)(1-p2), XOR and XNOR).
  dP/dp_j = P(table with digit j fixed to 1) - P(digit j fixed to 0).
* Variables: primary inputs take P = sigmoid(V) (V: one row of logits per
  sample, given, one column per primary input in ascending index); intermediate variables take their expression's value; a
  variable whose expression is a constant (kind PO) takes that constant
  unless it is also a primary input.
* Loss per sample: sum over auxiliary outputs of (P - 1)^2 and over
  constant expressions whose variable is a primary input of (P - c)^2.
* GD: V <- V - lr * dL/dV, dL/dV = dL/dP * P (1 - P), iterations given.
* Hardening: primary input = 1 where V > 0; other variables from their
  tables on hard values (constants for PO).  A sample is valid when the hard
  assignment satisfies every clause of the CNF; solutions are the distinct
  primary-input vectors of valid samples.

Plain NumPy in float64, vectorised over samples only.
"""
from __future__ import annotations

import numpy as np


def table_bits(e) -> np.ndarray:
    n = len(e.vars)
    return np.array([(e.table >> r) & 1 for r in range(1 << n)], np.float64)


def multilinear(bits: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Multilinear extension of a table (bits [2^k]) at p [batch, k]."""
    k = p.shape[1]
    out = np.zeros(p.shape[0])
    for r in range(1 << k):
        if bits[r] == 0:
            continue
        w = np.ones(p.shape[0])
        for j in range(k):
            w = w * (p[:, j] if (r >> j) & 1 else 1.0 - p[:, j])
        out += w
    return out


def multilinear_grad(bits: np.ndarray, p: np.ndarray) -> np.ndarray:
    """dP/dp_j [batch, k]: extension with digit j = 1 minus with digit j = 0."""
    k = p.shape[1]
    g = np.zeros_like(p)
    for j in range(k):
        hi = p.copy()
        hi[:, j] = 1.0
        lo = p.copy()
        lo[:, j] = 0.0
        g[:, j] = multilinear(bits, hi) - multilinear(bits, lo)
    return g


class Circuit:
    def __init__(self, clauses, transform_result):
        self.clauses = clauses
        PO, PI, IV, exprs = transform_result
        self.pi = sorted(PI)  # one logit column per primary input, ascending index
        self.exprs = exprs
        self.pi_set = set(PI)

    def forward(self, V):
        """Probabilities of every variable (dict var -> [batch]) and the list
        of (probability, target) loss terms."""
        P = {x: 1.0 / (1.0 + np.exp(-V[:, q])) for q, x in enumerate(self.pi)}
        terms = []
        for e in self.exprs:
            bits = table_bits(e)
            if e.kind == "IV":
                p = np.stack([P[x] for x in e.vars], 1) if e.vars else np.zeros((V.shape[0], 0))
                P[e.out] = multilinear(bits, p)
            elif e.kind == "PO":
                c = float(bits[0])
                if e.out in self.pi_set:
                    terms.append((e, e.out, c))
                else:
                    P[e.out] = np.full(V.shape[0], c)
            else:  # AUX: its conjunction must be 1
                terms.append((e, None, 1.0))
        return P, terms

    def loss_and_grad(self, V):
        P, terms = self.forward(V)
        L = np.zeros(V.shape[0])
        G = {x: np.zeros(V.shape[0]) for x in P}
        for e, var, c in terms:
            if var is not None:
                L += (P[var] - c) ** 2
                G[var] += 2.0 * (P[var] - c)
            else:
                p = np.stack([P[x] for x in e.vars], 1)
                y = multilinear(table_bits(e), p)
                L += (y - 1.0) ** 2
                d = multilinear_grad(table_bits(e), p)
                for j, x in enumerate(e.vars):
                    G[x] += 2.0 * (y - 1.0) * d[:, j]
        for e in reversed(self.exprs):  # chain rule through intermediate variables
            if e.kind != "IV" or not e.vars:
                continue
            p = np.stack([P[x] for x in e.vars], 1)
            d = multilinear_grad(table_bits(e), p)
            for j, x in enumerate(e.vars):
                G[x] += G[e.out] * d[:, j]
        dV = np.stack([G[x] * P[x] * (1.0 - P[x]) for x in self.pi], 1)
        return L, dV

    def descend(self, V, lr: float, iters: int):
        V = V.astype(np.float64).copy()
        for _ in range(iters):
            _, dV = self.loss_and_grad(V)
            V -= lr * dV
        return V

    def harden(self, V) -> dict:
        H = {x: (V[:, q] > 0).astype(np.int64) for q, x in enumerate(self.pi)}
        for e in self.exprs:
            if e.kind == "IV":
                r = np.zeros(V.shape[0], np.int64)
                for j, x in enumerate(e.vars):
                    r |= H[x] << j
                H[e.out] = np.array([(e.table >> int(v)) & 1 for v in r], np.int64)
            elif e.kind == "PO" and e.out not in self.pi_set:
                H[e.out] = np.full(V.shape[0], e.table & 1)
        return H

    def valid(self, H) -> np.ndarray:
        ok = np.ones(len(next(iter(H.values()))), bool)
        for c in self.clauses:
            sat = np.zeros_like(ok)
            for lit in c:
                x = abs(lit)
                sat |= (H[x] == 1) if lit > 0 else (H[x] == 0)
            ok &= sat
        return ok


def sample(clauses, transform_result, V0, lr=10.0, iters=5):
    """Returns (final logits, validity per sample, distinct valid PI vectors
    as a set of tuples)."""
    C = Circuit(clauses, transform_result)
    V = C.descend(V0, lr, iters)
    H = C.harden(V)
    ok = C.valid(H)
    pis = np.stack([H[x] for x in C.pi], 1) if C.pi else np.zeros((V.shape[0], 0), np.int64)
    uniq = {tuple(int(b) for b in pis[i]) for i in np.nonzero(ok)[0]}
    return V, ok, uniq
