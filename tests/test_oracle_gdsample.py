"""Pins of the GD-sampling oracle (CPU).

* Table 1's operators: at 0/1 inputs they are the Boolean gates, at any
  inputs they are the probability that the gate outputs 1 for independent
  inputs (computed here by summing over the input combinations), and their
  derivatives agree with central finite differences.
* Simplify: the forms of the Fig. 1 CNF are exactly the gates of the
  figure's generated module (x5 and x10 = OR(AND(s, a), AND(NOT(s), b)),
  the NOTs and buffers), the primary inputs come in the module's order, and
  a function with two minimal covers gets the one the tie rule names.
* The chain-rule example: the composition gives dx10/dx13 =
  x9 (1 - (1 - x9) x14); with the select inverted it gives the printed
  (1 - x9 x14)(1 - x9), so the printed equation is this composition with
  the multiplexer's select taken the other way round.
* Finite differences of the whole gradient, zero gradient on the
  unconstrained inputs, and the Fig. 1 samples against all solutions of the
  CNF found by brute force over every assignment of its 14 variables.
"""
import itertools
import json
import pathlib

import numpy as np

from oracle import gdsample as G
from oracle import sop
from oracle import transform as T

GOLDEN = pathlib.Path(__file__).parent / "golden"


class E:  # a bare expression record: variables, table, support
    def __init__(self, vars_, table, kind="IV", out=0):
        self.vars, self.table, self.kind, self.out = vars_, table, kind, out
        self.support = [vars_[j] for j in T.support(table, len(vars_))]


def tbl(fn, k):
    return sum(int(bool(fn(*[(r >> j) & 1 for j in range(k)]))) << r for r in range(1 << k))


def prob_one(fn, p):
    """P(fn = 1) for independent inputs with P(input j = 1) = p[:, j]."""
    k = p.shape[1]
    out = np.zeros(p.shape[0])
    for bits in itertools.product([0, 1], repeat=k):
        if fn(*bits):
            w = np.ones(p.shape[0])
            for j, bj in enumerate(bits):
                w = w * (p[:, j] if bj else 1.0 - p[:, j])
            out += w
    return out


def test_table1_operators_are_gate_probabilities():
    rng = np.random.default_rng(1)
    p = rng.random((300, 2))
    gates = {"AND": lambda a, b: a & b, "OR": lambda a, b: a | b, "XOR": lambda a, b: a ^ b,
             "XNOR": lambda a, b: 1 - (a ^ b)}
    h = 1e-6
    for name, fn in gates.items():
        op = G.BINARY[name]
        for a, b in itertools.product([0.0, 1.0], repeat=2):
            assert op(np.array([a]), np.array([b]))[0][0] == fn(int(a), int(b)), name
        y, d1, d2 = op(p[:, 0], p[:, 1])
        assert np.allclose(y, prob_one(fn, p)), name
        fd1 = (op(p[:, 0] + h, p[:, 1])[0] - op(p[:, 0] - h, p[:, 1])[0]) / (2 * h)
        fd2 = (op(p[:, 0], p[:, 1] + h)[0] - op(p[:, 0], p[:, 1] - h)[0]) / (2 * h)
        assert np.allclose(d1, fd1, atol=1e-7) and np.allclose(d2, fd2, atol=1e-7), name
    assert np.allclose(G.op_not(p[:, 0]), prob_one(lambda a: 1 - a, p[:, :1]))
    V = {1: p[:, 0]}
    g = {1: np.zeros(300)}
    G.form_backward(("NOT", ("VAR", 1)), V, 300, np.ones(300), g)
    assert np.allclose(g[1], -1.0)  # Table 1: dP_y/dP_1 = -1


def fig1():
    g = json.loads((GOLDEN / "fig1_cnf.json").read_text())
    C = T.parse_dimacs(g["dimacs"])
    return C, T.transform(C)


def V_(x):
    return ("VAR", x)


def mux(s, a, b):  # the generated module's form
    return ("OR", ("AND", V_(s), V_(a)), ("AND", ("NOT", V_(s)), V_(b)))


def test_fig1_forms_are_the_generated_module():
    """Fig. 1(c): x2 = NOT(x1), x3 = x2, x4 = x3, x5 = OR(AND(x4, x11),
    AND(NOT(x4), x12)), x7 = x6, x8 = x7, x9 = NOT(x8), x10 = OR(AND(x9,
    x13), AND(NOT(x9), x14)); outputs = x10, constrained to 1.  Inputs
    x1, x11, x12, x6, x13, x14 in the module's order (the module's x7 in
    the input list is x6: the variable x7 is computed from it)."""
    C, R = fig1()
    circ = G.Circuit(C, R)
    got = {e.out: f for e, f in zip(circ.exprs, circ.forms) if e.kind == "IV"}
    want = {2: ("NOT", V_(1)), 3: V_(2), 4: V_(3), 5: mux(4, 11, 12), 7: V_(6), 8: V_(7), 9: ("NOT", V_(8)),
            10: mux(9, 13, 14)}
    assert got == want
    aux = [f for e, f in zip(circ.exprs, circ.forms) if e.kind == "AUX"]
    assert aux == [V_(10)]
    assert circ.pi == [1, 11, 12, 6, 13, 14]


def test_chain_rule_example():
    """L = (x10 - 1)^2 over x10 = OR(AND(x9, x13), AND(NOT(x9), x14)):
    x10 = 1 - (1 - x9 x13)(1 - (1 - x9) x14) and
    dL/dx13 = 2 (x10 - 1) x9 (1 - (1 - x9) x14).  The same composition with
    the select inverted gives the printed 2 (x10 - 1)(1 - x9 x14)(1 - x9).
    Neither equals the multilinear extension x9 x13 + (1 - x9) x14 (exact
    probability of the multiplexer): the composition falls short of it by
    x9 (1 - x9) x13 x14, because the select is read twice."""
    rng = np.random.default_rng(2)
    p = rng.random((200, 3))
    x9, x13, x14 = p[:, 0], p[:, 1], p[:, 2]
    P = {9: x9, 13: x13, 14: x14}
    for f, y_want, d_want in (
            (mux(9, 13, 14), 1 - (1 - x9 * x13) * (1 - (1 - x9) * x14), x9 * (1 - (1 - x9) * x14)),
            (mux(9, 14, 13), 1 - (1 - x9 * x14) * (1 - (1 - x9) * x13), (1 - x9 * x14) * (1 - x9))):
        y = G.form_value(f, P, 200)
        assert np.allclose(y, y_want)
        g = {x: np.zeros(200) for x in P}
        G.form_backward(f, P, 200, 2.0 * (y - 1.0), g)
        assert np.allclose(g[13], 2.0 * (y - 1.0) * d_want)
    y = G.form_value(mux(9, 13, 14), P, 200)
    exact = prob_one(lambda s, a, b: (s & a) | ((1 - s) & b), p)
    assert np.allclose(exact - y, x9 * (1 - x9) * x13 * x14)


def test_read_once_forms_are_exact_probabilities():
    """Where every support variable is read once (AND/OR/NAND/NOR chains,
    parities) the composed form is the probability that the expression is 1
    for independent inputs."""
    rng = np.random.default_rng(5)
    p = rng.random((100, 4))
    fns = [lambda a, b, c, d: a & b & (1 - c), lambda a, b, c, d: a | (1 - b) | d,
           lambda a, b, c, d: 1 - (a & b & c & d), lambda a, b, c, d: a ^ b ^ c ^ d,
           lambda a, b, c, d: 1 - (a ^ c ^ d)]
    for fn in fns:
        e = E([1, 2, 3, 4], tbl(fn, 4))
        f = G.simplify(e)
        P = {x: p[:, j] for j, x in enumerate([1, 2, 3, 4])}
        assert np.allclose(G.form_value(f, P, 100), prob_one(fn, p))


def test_simplify_forms_and_tie_rule():
    """Parity becomes an XOR chain (XNOR for its complement), a constant a
    CONST, a variable outside the support is dropped, and among the two
    minimal covers of b xor c or a b / a c (K-map bits a b c d = row bits
    3 2 1 0) the tie rule takes the one whose sorted term keys come first:
    (c NOT b), (c a), (NOT c b)."""
    e = E([3, 5, 7], tbl(lambda a, b, c: a ^ b ^ c, 3))
    assert G.simplify(e) == ("XOR", ("XOR", V_(3), V_(5)), V_(7))
    e = E([3, 5], tbl(lambda a, b: 1 - (a ^ b), 2))
    assert G.simplify(e) == ("XNOR", V_(3), V_(5))
    assert G.simplify(E([3, 5], 0)) == ("CONST", 0)
    assert G.simplify(E([3, 5], 0xF)) == ("CONST", 1)
    e = E([3, 5, 7], tbl(lambda a, b, c: a & c, 3))  # x5 outside the support
    assert G.simplify(e) == ("AND", V_(3), V_(7))
    cover = sop.canonical_cover(0xFC3C, 4)
    assert cover == [(0b0110, 0b0010), (0b1010, 0b1010), (0b0110, 0b0100)]
    assert sop.minimal_cost(0xFC3C, 4)[0] == (3, 6)
    e = E([1, 2, 3, 4], 0xFC3C)
    assert G.simplify(e) == ("OR", ("OR", ("AND", V_(2), ("NOT", V_(3))), ("AND", V_(2), V_(4))),
                             ("AND", ("NOT", V_(2)), V_(3)))


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
    free = [q for q, x in enumerate(circ.pi) if x in (1, 11, 12)]
    assert np.allclose(dV[:, free], 0.0)
    # dL/dV13 = 2 (x10 - 1) x9 (1 - (1 - x9) x14) P13 (1 - P13)
    P, _ = circ.forward(V)
    q13 = circ.pi.index(13)
    want = 2 * (P[10] - 1) * P[9] * (1 - (1 - P[9]) * P[14]) * P[13] * (1 - P[13])
    assert np.allclose(dV[:, q13], want)


def test_fig1_samples_are_solutions():
    """Every kept solution satisfies the CNF; with 1000 samples GD finds all
    32 primary-input assignments of the CNF's solutions, which a brute force
    over all 2^14 assignments of its variables lists clause by clause."""
    C, R = fig1()
    pi = R[1]
    brute = set()
    for bits in itertools.product([0, 1], repeat=14):
        val = {x + 1: bits[x] for x in range(14)}
        if all(any((val[abs(l)] == 1) == (l > 0) for l in c) for c in C):
            brute.add(tuple(val[x] for x in pi))
    assert len(brute) == 32
    V0 = np.random.default_rng(0).normal(0, 1, (1000, len(pi)))
    V, ok, uniq = G.sample(C, R, V0, lr=10.0, iters=5)
    assert uniq <= brute and len(uniq) == 32
