"""Minimal sum-of-products of a truth table by exhaustive search -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A cube is (care, value): it covers row r iff (r & care) == value; its
literals are the set bits of care (variable j positive when bit j of value
is 1).  Cost of a cover = (number of cubes, number of literals), compared
in that order.  A minimum-cost cover can always be built from prime
implicants (Quine), so the search runs over subsets of primes in order of
size; plain loops, practical for up to four variables.
"""
from __future__ import annotations

from itertools import combinations, product


def implicants(table: int, n: int):
    """Every cube whose rows all carry a 1."""
    out = []
    for care in range(1 << n):
        for value in range(1 << n):
            if value & ~care:
                continue
            rows = [r for r in range(1 << n) if (r & care) == value]
            if all((table >> r) & 1 for r in rows):
                out.append((care, value))
    return out


def primes(table: int, n: int):
    """Implicants not contained in another implicant (a cube A lies inside B
    when B's care bits are a subset of A's and they agree there)."""
    imp = implicants(table, n)
    def inside(a, b):
        return a != b and (b[0] & ~a[0]) == 0 and (a[1] & b[0]) == b[1]
    return [a for a in imp if not any(inside(a, b) for b in imp)]


def covers(cubes, table: int, n: int) -> bool:
    got = 0
    for care, value in cubes:
        for r in range(1 << n):
            if (r & care) == value:
                got |= 1 << r
    return got == table


def minimal_cost(table: int, n: int):
    """(terms, literals) of a minimum cover and one such cover."""
    if table == 0:
        return (0, 0), []
    P = primes(table, n)
    for k in range(1, len(P) + 1):
        best = None
        for sub in combinations(P, k):
            if covers(sub, table, n):
                lits = sum(bin(c).count("1") for c, _ in sub)
                if best is None or lits < best[0]:
                    best = (lits, list(sub))
        if best is not None:
            return (k, best[0]), best[1]
    raise AssertionError("primes always cover the table")


def kmap_cells(n: int = 4):
    """Cell layout of a four-variable Karnaugh map in the preamble's
    template: rows x1x2 and columns x3x4 in Gray order 00, 01, 11, 10; the
    cell holds row number 8 x1 + 4 x2 + 2 x3 + x4 (x1 the most significant
    digit of r)."""
    gray = [0, 1, 3, 2]
    return [[8 * (g1 >> 1) + 4 * (g1 & 1) + 2 * (g2 >> 1) + (g2 & 1) for g2 in gray] for g1 in gray]
