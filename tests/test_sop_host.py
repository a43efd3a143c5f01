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
