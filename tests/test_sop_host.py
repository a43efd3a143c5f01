"""Host minimiser (tt_sop_minimize, CPU): minimal cost equal to the
oracle's exhaustive search for every 3-variable function and random
4-variable ones, covers equivalent to the table and made of implicants for
random tables of up to 10 variables, the K-map text in the template's
layout.  No GPU is used."""
import random

import numpy as np

import paper_2502_08673_amd as tt
from oracle import sop


def words_of(t, n):
    nw = max(1, (1 << n) // 64)
    return [(t >> (64 * w)) & ((1 << 64) - 1) for w in range(nw)]


def cover_table(terms, n):
    got = 0
    for care, value in terms:
        for r in range(1 << n):
            if (r & care) == value:
                got |= 1 << r
    return got


def check_equiv(t, n, terms):
    assert cover_table(terms, n) == t
    for care, value in terms:  # every term is an implicant
        assert all((t >> r) & 1 for r in range(1 << n) if (r & care) == value)


def test_all_three_variable_functions_are_minimal():
    for t in range(256):
        terms, lits, exact = tt.sop_minimize(words_of(t, 3), 3)
        assert exact
        check_equiv(t, 3, terms)
        assert (len(terms), lits) == sop.minimal_cost(t, 3)[0], hex(t)


def test_random_four_variable_functions_are_minimal():
    rng = random.Random(11)
    for t in [0xFEE8, 0xFC3C, 0xFFC0, 0x6996, 0, 0xFFFF] + [rng.getrandbits(16) for _ in range(150)]:
        terms, lits, exact = tt.sop_minimize(words_of(t, 4), 4)
        assert exact
        check_equiv(t, 4, terms)
        assert (len(terms), lits) == sop.minimal_cost(t, 4)[0], hex(t)


def test_larger_tables_are_covered_by_implicants():
    rng = random.Random(12)
    for n in (5, 6, 7, 8, 10):
        for density in (0.1, 0.5, 0.9):
            t = sum(int(rng.random() < density) << r for r in range(1 << n))
            terms, lits, exact = tt.sop_minimize(words_of(t, n), n, node_budget=200000)
            check_equiv(t, n, terms)
            assert lits == sum(bin(c).count("1") for c, _ in terms)


def test_kmap_text_layout():
    txt = tt.kmap_text(0xFEE8).splitlines()
    cells = sop.kmap_cells()
    for i, line in enumerate(txt[1:5]):
        bits = [int(x) for x in line.split()[1:]]
        assert bits == [(0xFEE8 >> c) & 1 for c in cells[i]]


def test_tie_rule_picks_the_canonical_cover():
    """Among covers of equal cost the host minimiser returns the one the
    oracle's tie rule names (smallest sorted list of term keys), in key
    order: every 3-variable function, random 4- and 5-variable ones, and
    the two-plane K-map example whose plane 0 has two minimal covers."""
    rng = random.Random(21)
    cases = [(t, 3) for t in range(256)] + [(0xFC3C, 4), (0xFEE8, 4)]
    cases += [(rng.getrandbits(16), 4) for _ in range(120)] + [(rng.getrandbits(32), 5) for _ in range(30)]
    for t, n in cases:
        terms, _, exact = tt.sop_minimize(words_of(t, n), n)
        assert exact
        assert terms == sop.canonical_cover(t, n), (hex(t), n)


def gates_to_form(gates, vars_):
    """The oracle's form tree of a tt_simplify gate program (digit j is the
    variable vars_[j])."""
    temps = {}

    def opd(o):
        f = temps[o & 0xFFFF] if o & tt.OPD_TEMP else ("VAR", vars_[o & 0xFFFF])
        return ("NOT", f) if o & tt.OPD_NEG else f

    names = {tt.GATE_AND: "AND", tt.GATE_OR: "OR", tt.GATE_XOR: "XOR", tt.GATE_XNOR: "XNOR"}
    root = None
    for i, g in enumerate(gates):
        op, a, b, dst = int(g["op"]), int(g["a"]), int(g["b"]), int(g["dst"])
        if op == tt.GATE_CONST:
            f = ("CONST", a)
        elif op == tt.GATE_COPY:
            f = opd(a)
        else:
            f = (names[op], opd(a), opd(b))
        if dst == -1:
            assert i == len(gates) - 1
            root = f
        else:
            assert dst == i
            temps[dst] = f
    return root


class _Rec:
    def __init__(self, vars_, table):
        from oracle import transform as T
        self.vars, self.table = vars_, table
        self.support = [vars_[j] for j in T.support(table, len(vars_))]


def test_simplify_forms_equal_the_oracle():
    """tt_simplify's gate program, read back as a tree, is the oracle's
    Simplify form (support restriction, XOR/XNOR chains for parity, the
    canonical minimal SOP as OR/AND chains) for every function of up to 3
    variables, random 4- and 5-variable ones, and functions whose support
    skips digits."""
    from oracle import gdsample as G
    rng = random.Random(22)
    cases = [(t, n) for n in range(4) for t in range(1 << (1 << n))]
    cases += [(rng.getrandbits(16), 4) for _ in range(150)] + [(rng.getrandbits(32), 5) for _ in range(40)]
    # digits 0 and 2 of 4 only (the others are outside the support)
    cases += [(sum(((r & 1) ^ ((r >> 2) & 1)) << r for r in range(16)), 4),
              (sum(((r & 1) | ((r >> 3) & 1)) << r for r in range(16)), 4)]
    for t, n in cases:
        vars_ = [3 * j + 5 for j in range(n)]
        gates, exact = tt.simplify(words_of(t, n), n)
        assert exact
        assert gates_to_form(gates, vars_) == G.simplify(_Rec(vars_, t)), (hex(t), n)


def test_simplify_of_parity_and_mux():
    g, _ = tt.simplify([0x96], 3)  # x0 ^ x1 ^ x2
    assert [int(x) for x in g["op"]] == [tt.GATE_XOR, tt.GATE_XOR]
    g, _ = tt.simplify([0x69], 3)  # its complement: XNOR last
    assert [int(x) for x in g["op"]] == [tt.GATE_XOR, tt.GATE_XNOR]
    mux = sum(((r & 1) & ((r >> 1) & 1) | (1 - (r & 1)) & ((r >> 2) & 1)) << r for r in range(8))
    g, _ = tt.simplify([mux], 3)
    assert gates_to_form(g, [9, 13, 14]) == ("OR", ("AND", ("VAR", 9), ("VAR", 13)),
                                             ("AND", ("NOT", ("VAR", 9)), ("VAR", 14)))
