"""Pins of the Algorithm 1 oracle (CPU): the paper's worked example, its
Fig. 1 CNF and circuit, the Tseitin signatures of the primary gates (each
recognised as its own function, computed here directly from the gate), the
under-specified OR of the text, unit clauses, and the support of the
recorded tables."""
import itertools
import json
import pathlib
import random

import pytest

from oracle import transform as T

GOLDEN = pathlib.Path(__file__).parent / "golden"


def table_of(fn, vars_):
    """Truth table over vars_ (slot j = digit j) of fn(assignment dict)."""
    t = 0
    for r in range(1 << len(vars_)):
        a = {x: (r >> j) & 1 for j, x in enumerate(vars_)}
        t |= int(bool(fn(a))) << r
    return t


def test_worked_example_mux():
    """The four clauses over x4, x107, x108, x5 define
    x5 = (x107 and x4) or (x108 and not x4); no other variable works."""
    C = [[-4, -107, 5], [-4, 107, -5], [4, -108, 5], [4, 108, -5]]
    PO, PI, IV, E = T.transform(C)
    assert IV == [5] and sorted(PI) == [4, 107, 108] and PO == []
    (e,) = E
    assert e.out == 5 and e.vars == [4, 107, 108] and (e.first, e.last) == (0, 3)
    assert e.table == table_of(lambda a: (a[107] and a[4]) or (a[108] and not a[4]), e.vars)
    sc = C
    for v in (4, 107, 108):
        others = [x for x in [4, 5, 107, 108] if x != v]
        f = T.find_expression(v, sc, others)
        g = T.find_expression(-v, sc, others)
        assert f != (~g) & ((1 << (1 << 3)) - 1)


def test_fig1_cnf_circuit():
    g = json.loads((GOLDEN / "fig1_cnf.json").read_text())
    C = T.parse_dimacs(g["dimacs"])
    assert len(C) == 21
    PO, PI, IV, E = T.transform(C)
    assert PI == g["primary_inputs_in_module_order"]
    assert IV == g["intermediate"]
    gate = {
        "not": lambda a, x: not a[x[0]],
        "buf": lambda a, x: a[x[0]],
        "mux": lambda a, x: (a[x[0]] and a[x[1]]) or (not a[x[0]] and a[x[2]]),
    }
    by_out = {e.out: e for e in E if e.kind == "IV"}
    for out, spec in g["gates"].items():
        kind, *ins = spec.split()
        ins = [int(x) for x in ins]
        e = by_out[int(out)]
        assert sorted(e.support) == sorted(ins), out
        assert e.table == table_of(lambda a: gate[kind](a, ins), e.vars), out
    # x10 = 1: the unit clause left over becomes an auxiliary output on x10
    (aux,) = [e for e in E if e.kind == "AUX"]
    assert PO == [0] and aux.vars == [10] and aux.table == 0b10


def gate_signature(kind, ins, f):
    """The Tseitin clauses of a gate, as the equations of the transformation
    section give them."""
    if kind == "not":
        return [[f, ins[0]], [-f, -ins[0]]]
    if kind == "or":
        return [[-f] + ins] + [[f, -x] for x in ins]
    if kind == "and":
        return [[f] + [-x for x in ins]] + [[-f, x] for x in ins]
    if kind == "nor":  # OR with the output inverted
        return [[f] + ins] + [[-f, -x] for x in ins]
    if kind == "nand":
        return [[-f] + [-x for x in ins]] + [[f, x] for x in ins]
    if kind in ("xor", "xnor"):
        # XNOR(ins, f) for xor (f = XOR(ins)); XOR(ins, f) for xnor:
        # the clauses exclude every assignment of odd (xor) / even parity
        allv = ins + [f]
        bad_parity = 1 if kind == "xor" else 0
        cl = []
        for bits in itertools.product([0, 1], repeat=len(allv)):
            if sum(bits) % 2 == bad_parity:
                cl.append([-x if b else x for x, b in zip(allv, bits)])
        return cl
    raise ValueError(kind)


GATES = {
    "not": lambda v: not v[0],
    "or": lambda v: any(v),
    "and": lambda v: all(v),
    "nor": lambda v: not any(v),
    "nand": lambda v: not all(v),
    "xor": lambda v: sum(v) % 2 == 1,
    "xnor": lambda v: sum(v) % 2 == 0,
}


@pytest.mark.parametrize("kind", sorted(GATES))
def test_gate_signatures_are_recognised(kind):
    rng = random.Random(hash(kind) & 0xFFFF)
    for n in ([1] if kind == "not" else [2, 3, 4]):
        ins = rng.sample(range(1, 9), n)
        f = 20  # highest index: tried first
        C = gate_signature(kind, ins, f)
        rng.shuffle(C)
        PO, PI, IV, E = T.transform(C)
        assert IV == [f] and sorted(PI) == sorted(ins), (kind, n)
        (e,) = E
        assert e.table == table_of(lambda a: GATES[kind]([a[x] for x in ins]), e.vars)
        assert sorted(e.support) == sorted(ins)


def test_under_specified_or_and_unit_clauses():
    # x3 = x1 or x2 with x3 = 1: only (x1 or x2) remains -> auxiliary output
    PO, PI, IV, E = T.transform([[1, 2]])
    assert PO == [0] and sorted(PI) == [1, 2] and IV == []
    assert E[0].kind == "AUX" and E[0].table == table_of(lambda a: a[1] or a[2], [1, 2])
    # a unit clause on a fresh variable: v = 1 is forced, a constant output
    PO, PI, IV, E = T.transform([[-7]])
    assert PO == [7] and E[0].kind == "PO" and E[0].vars == [] and E[0].table == 0  # f = False: x7 = 0


def test_support_drops_unused_inputs():
    # x5 = x1 and x2, written with a redundant x3 literal pair: (x3 or -x3) is
    # excluded, so use a clause set where x3 cancels: f = x1 x2 (x3 or not x3)
    C = [[-5, 1], [-5, 2], [5, -1, -2, 3], [5, -1, -2, -3]]
    PO, PI, IV, E = T.transform(C)
    (e,) = E
    assert e.out == 5 and e.vars == [1, 2, 3] and sorted(e.support) == [1, 2]
