"""Pins of the GD-sampling oracle (CPU): Table 1's probabilistic operators
and derivatives, the multiplexer of the chain-rule example (closed form of
its extension and of dL/dx13), finite differences of the whole gradient,
and the sampled solutions of the Fig. 1 CNF against all its solutions found
by brute force."""
import itertools
import json
import pathlib

import numpy as np

from oracle import gdsample as G
from oracle import transform as T

GOLDEN = pathlib.Path(__file__).parent / "golden"


class E:  # a bare expression: variables and table
    def __init__(self, vars_, table, kind="IV", out=0):
        self.vars, self.table, self.kind, self.out = vars_, table, kind, out


def tbl(fn, k):
    return sum(int(bool(fn(*[(r >> j) & 1 for j in range(k)]))) << r for r in range(1 << k))


def test_table1_operators_and_derivatives():
    rng = np.random.default_rng(1)
    p = rng.random((200, 2))
    p1, p2 = p[:, 0], p[:, 1]
    cases = {  # Table 1: output, derivative w.r.t. P1, w.r.t. P2
        "and": (tbl(lambda a, b: a & b, 2), p1 * p2, p2, p1),
        "or": (tbl(lambda a, b: a | b, 2), 1 - (1 - p1) * (1 - p2), 1 - p2, 1 - p1),
        "xor": (tbl(lambda a, b: a ^ b, 2), (1 - p1) * p2 + p1 * (1 - p2), 1 - 2 * p2, 1 - 2 * p1),
        "xnor": (tbl(lambda a, b: 1 - (a ^ b), 2), p1 * p2 + (1 - p1) * (1 - p2), 2 * p2 - 1, 2 * p1 - 1),
    }
    for name, (t, y, d1, d2) in cases.items():
        bits = G.table_bits(E([1, 2], t))
        assert np.allclose(G.multilinear(bits, p), y), name
        g = G.multilinear_grad(bits, p)
        assert np.allclose(g[:, 0], d1) and np.allclose(g[:, 1], d2), name
    bits = G.table_bits(E([1], tbl(lambda a: 1 - a, 1)))  # NOT: 1 - P1, derivative -1
    assert np.allclose(G.multilinear(bits, p[:, :1]), 1 - p1)
    assert np.allclose(G.multilinear_grad(bits, p[:, :1])[:, 0], -1.0)


def test_chain_rule_example_multiplexer():
    """x10 = (x9 and x13) or (not x9 and x14) with L = (x10 - 1)^2: the
    extension is x9 x13 + (1 - x9) x14, so dL/dx13 = 2 (x10 - 1) x9."""
    rng = np.random.default_rng(2)
    p = rng.random((100, 3))  # columns x9, x13, x14
    bits = G.table_bits(E([9, 13, 14], tbl(lambda s, a, b: (s & a) | ((1 - s) & b), 3)))
    x9, x13, x14 = p[:, 0], p[:, 1], p[:, 2]
    y = G.multilinear(bits, p)
    assert np.allclose(y, x9 * x13 + (1 - x9) * x14)
    dL = 2 * (y - 1) * G.multilinear_grad(bits, p)[:, 1]
    assert np.allclose(dL, 2 * (y - 1) * x9)


def fig1():
    g = json.loads((GOLDEN / "fig1_cnf.json").read_text())
    C = T.parse_dimacs(g["dimacs"])
    return C, T.transform(C)


def test_gradient_matches_finite_differences():
    C, R = fig1()
    circ = G.Circuit(C, R)
    rng = np.random.default_rng(3)
    V = rng.normal(0, 1.5, (5, len(circ.pi)))
    L, dV = circ.loss_and_grad(V)
    h = 1e-6
    for q in range(V.shape[1]):
        Vp, Vm = V.copy(), V.copy()
        Vp[:, q] += h
        Vm[:, q] -= h
        fd = (circ.loss_and_grad(Vp)[0] - circ.loss_and_grad(Vm)[0]) / (2 * h)
        assert np.allclose(fd, dV[:, q], atol=1e-6), q
    # only the constrained path's inputs (x6, x13, x14) move the loss
    pi = circ.pi
    free = [q for q, x in enumerate(pi) if x in (1, 11, 12)]
    assert np.allclose(dV[:, free], 0.0)


def test_fig1_samples_are_solutions():
    """Every kept solution satisfies the CNF; with 1000 samples GD finds all
    32 assignments of the six primary inputs that force x10 = 1."""
    C, R = fig1()
    V0 = np.random.default_rng(0).normal(0, 1, (1000, len(R[1])))
    V, ok, uniq = G.sample(C, R, V0, lr=10.0, iters=5)
    pi = R[1]
    brute = set()
    for bits in itertools.product([0, 1], repeat=len(pi)):
        H = {x: np.array([b]) for x, b in zip(pi, bits)}
        circ = G.Circuit(C, R)
        Vb = np.array([[1.0 if b else -1.0 for b in bits]])
        H = circ.harden(Vb)
        if circ.valid(H)[0]:
            brute.add(bits)
    assert len(brute) == 32
    assert uniq <= brute and len(uniq) == 32
