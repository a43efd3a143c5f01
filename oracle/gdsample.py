"""Gradient-descent sampling of a transformed CNF (the paper's Methodology:
the transformation's simplified expressions turned into a circuit of logical
operators, Table 1's probabilistic operators, the sigmoid embedding, the L2
loss, GD, hardening and the satisfiable / non-redundant filter) -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The circuit is what the transformation (``oracle/transform.py``) returns:
expressions in the order found, each a truth table over its variables.

* Simplify (Algorithm 1 appends the simplified expression): the table is
  restricted to its support (the variables it depends on).  A parity of two
  or more support variables is Table 1's XOR chained over them in ascending
  index (its complement ends the chain with XNOR); any other function is
  its minimal sum of products (``oracle.sop.canonical_cover``: fewest terms,
  then fewest literals, then the smallest sorted list of term keys), written
  as an OR chain of the terms in key order, each an AND chain of its
  literals in ascending index, a negative literal being NOT of its
  variable.  For the two multiplexers of Fig. 1 this is exactly the
  generated module's OR(AND(s, a), AND(NOT(s), b)).
* Probabilistic model: every operator replaced by its Table 1 counterpart
  (NOT 1 - p, AND p1 p2, OR 1 - (1 - p1)(1 - p2), XOR, XNOR); derivatives by
  the chain rule through the operators with Table 1's derivatives, as
  automatic differentiation of the generated module does.  A variable read
  twice by an expression (a multiplexer's select) collects the derivative
  of both reads.
* Variables: primary inputs take P = sigmoid(V) (V: one row of logits per
  sample, one column per primary input in the transformation's order of
  entry, which is the input order of the Fig. 1 module); intermediate
  variables take their expression's value; a variable whose expression is a
  constant (kind PO) takes that constant unless it is also a primary input.
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

from oracle import sop

# ---------------------------------------------------------------- Table 1
# value and the two partial derivatives of each binary operator


def op_not(p):
    return 1.0 - p


def op_and(p1, p2):
    return p1 * p2, p2, p1


def op_or(p1, p2):
    return 1.0 - (1.0 - p1) * (1.0 - p2), 1.0 - p2, 1.0 - p1


def op_xor(p1, p2):
    return (1.0 - p1) * p2 + p1 * (1.0 - p2), 1.0 - 2.0 * p2, 1.0 - 2.0 * p1


def op_xnor(p1, p2):
    return p1 * p2 + (1.0 - p1) * (1.0 - p2), 2.0 * p2 - 1.0, 2.0 * p1 - 1.0


BINARY = {"AND": op_and, "OR": op_or, "XOR": op_xor, "XNOR": op_xnor}

# ------------------------------------------------------------- Simplify
# A form is a tree of tuples: ("VAR", x), ("CONST", c), ("NOT", f) or
# (op, f1, f2) with op one of AND, OR, XOR, XNOR.


def restrict(table: int, vars_, keep):
    """The table as a function of the variables ``keep`` alone (every other
    variable is outside its support, so any value of it will do: 0)."""
    pos = [vars_.index(x) for x in keep]
    t = 0
    for r in range(1 << len(keep)):
        row = 0
        for i, p in enumerate(pos):
            row |= ((r >> i) & 1) << p
        t |= ((table >> row) & 1) << r
    return t


def chain(op, items):
    f = items[0]
    for g in items[1:]:
        f = (op, f, g)
    return f


def simplify(e):
    """The form of an expression record (``vars``, ``table``, ``support``)."""
    S = list(e.support)
    k = len(S)
    t = restrict(e.table, e.vars, S)
    if k == 0:
        return ("CONST", t & 1)
    parity = sum(bin(r).count("1") % 2 << r for r in range(1 << k))
    full = (1 << (1 << k)) - 1
    if k >= 2 and t in (parity, full & ~parity):
        leaves = [("VAR", x) for x in S]
        f = chain("XOR", leaves[:-1])
        return ("XOR" if t == parity else "XNOR", f, leaves[-1])
    terms = []
    for care, value in sop.canonical_cover(t, k):
        lits = [("VAR", S[j]) if (value >> j) & 1 else ("NOT", ("VAR", S[j])) for j in range(k) if (care >> j) & 1]
        terms.append(chain("AND", lits) if lits else ("CONST", 1))
    if not terms:
        return ("CONST", 0)
    return chain("OR", terms)


def form_value(f, P, batch):
    op = f[0]
    if op == "VAR":
        return P[f[1]]
    if op == "CONST":
        return np.full(batch, float(f[1]))
    if op == "NOT":
        return op_not(form_value(f[1], P, batch))
    return BINARY[op](form_value(f[1], P, batch), form_value(f[2], P, batch))[0]


def form_backward(f, P, batch, adj, G):
    """Adds adj * d(form)/dP[x] to G[x] for every variable x the form reads."""
    op = f[0]
    if op == "VAR":
        G[f[1]] = G[f[1]] + adj
    elif op == "NOT":
        form_backward(f[1], P, batch, -adj, G)
    elif op != "CONST":
        _, d1, d2 = BINARY[op](form_value(f[1], P, batch), form_value(f[2], P, batch))
        form_backward(f[1], P, batch, adj * d1, G)
        form_backward(f[2], P, batch, adj * d2, G)


def form_vars(f):
    if f[0] == "VAR":
        return {f[1]}
    if f[0] == "CONST":
        return set()
    return set().union(*(form_vars(g) for g in f[1:]))


class Circuit:
    def __init__(self, clauses, transform_result):
        self.clauses = clauses
        PO, PI, IV, exprs = transform_result
        self.pi = list(PI)  # one logit column per primary input, in order of entry
        self.exprs = exprs
        self.forms = [simplify(e) for e in exprs]
        self.pi_set = set(PI)

    def forward(self, V):
        """Probabilities of every variable (dict var -> [batch]) and the list
        of (form, variable, target) loss terms."""
        B = V.shape[0]
        P = {x: 1.0 / (1.0 + np.exp(-V[:, q])) for q, x in enumerate(self.pi)}
        terms = []
        for e, f in zip(self.exprs, self.forms):
            if e.kind == "IV":
                P[e.out] = form_value(f, P, B)
            elif e.kind == "PO":
                c = float(e.table & 1)
                if e.out in self.pi_set:
                    terms.append((None, e.out, c))
                else:
                    P[e.out] = np.full(B, c)
            else:  # AUX: its conjunction must be 1
                terms.append((f, None, 1.0))
        return P, terms

    def loss_and_grad(self, V):
        B = V.shape[0]
        P, terms = self.forward(V)
        L = np.zeros(B)
        G = {x: np.zeros(B) for x in P}
        for f, var, c in terms:
            if var is not None:
                L += (P[var] - c) ** 2
                G[var] = G[var] + 2.0 * (P[var] - c)
            else:
                y = form_value(f, P, B)
                L += (y - 1.0) ** 2
                form_backward(f, P, B, 2.0 * (y - 1.0), G)
        for e, f in zip(reversed(self.exprs), reversed(self.forms)):  # chain rule through intermediates
            if e.kind == "IV":
                form_backward(f, P, B, G[e.out], G)
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
