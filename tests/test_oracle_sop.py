"""Pins of the minimal-SOP oracle (CPU): the threshold function 'at least two
of four' (all six pairs, all essential), a hand-worked two-plane example,
constants, a single variable, parity (no merging possible), and the cost of
a brute-force check that every prime is an implicant."""
from oracle import sop


def tbl(fn, n):
    return sum(int(bool(fn(r))) << r for r in range(1 << n))


def test_at_least_two_of_four():
    t = tbl(lambda r: bin(r).count("1") >= 2, 4)
    assert t == 0xFEE8
    (terms, lits), cover = sop.minimal_cost(t, 4)
    assert (terms, lits) == (6, 12)
    assert sorted(cover) == sorted(((1 << i) | (1 << j), (1 << i) | (1 << j))
                                   for i in range(4) for j in range(i + 1, 4))


def test_hand_worked_planes():
    """q(r) for a = x0 + 2 x1 - 1 (x0 = digits 0-1, x1 = digits 2-3), ReLU,
    thresholds 1, 3, 5: q = 0,0,1,1, 1,1,2,2, 2,2,3,3, 3,3,3,3.  With
    a = r3, b = r2, c = r1, d = r0: plane 1 = a or (b and c) (2 terms, 3
    literals); plane 0 = (b xor c) or (a and b) (3 terms, 6 literals)."""
    q = [0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3]
    p0 = sum((v & 1) << r for r, v in enumerate(q))
    p1 = sum(((v >> 1) & 1) << r for r, v in enumerate(q))
    assert (p0, p1) == (0xFC3C, 0xFFC0)
    assert sop.minimal_cost(p1, 4)[0] == (2, 3)
    assert sop.minimal_cost(p0, 4)[0] == (3, 6)


def test_constants_variable_and_parity():
    assert sop.minimal_cost(0, 3)[0] == (0, 0)
    assert sop.minimal_cost(0xFF, 3)[0] == (1, 0)
    assert sop.minimal_cost(tbl(lambda r: (r >> 2) & 1, 3), 3)[0] == (1, 1)
    par = tbl(lambda r: bin(r).count("1") % 2, 4)
    assert sop.minimal_cost(par, 4)[0] == (8, 32)  # every minterm is prime


def test_primes_are_maximal_implicants():
    import random
    rng = random.Random(4)
    for _ in range(20):
        t = rng.getrandbits(16)
        P = sop.primes(t, 4)
        imp = set(sop.implicants(t, 4))
        assert set(P) <= imp and sop.covers(P, t, 4)


def test_kmap_cells_follow_the_template():
    cells = sop.kmap_cells()
    assert cells[0] == [0, 1, 3, 2] and [row[0] for row in cells] == [0, 4, 12, 8]
    assert sorted(c for row in cells for c in row) == list(range(16))


def test_canonical_cover_against_every_implicant_subset():
    """For every 3-variable table: the canonical cover covers the table, has
    the minimal cost, and no cover made of ANY implicants (prime or not) of
    that cost has a smaller sorted list of term keys; it comes sorted by key."""
    from itertools import combinations
    for t in range(256):
        cov = sop.canonical_cover(t, 3)
        (terms, lits), _ = sop.minimal_cost(t, 3)
        assert sop.covers(cov, t, 3) and len(cov) == terms
        assert sum(bin(c).count("1") for c, _ in cov) == lits
        keys = [sop.term_key(c, 3) for c in cov]
        assert keys == sorted(keys)
        imp = sop.implicants(t, 3)
        for sub in combinations(imp, terms):
            if sum(bin(c).count("1") for c, _ in sub) == lits and sop.covers(sub, t, 3):
                assert keys <= sorted(sop.term_key(c, 3) for c in sub), hex(t)
