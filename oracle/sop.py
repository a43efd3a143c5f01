"""Minimal sum-of-products of a truth table by exhaustive search -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A cube is (care, value): it covers row r iff (r & care) == value; its
literals are the set bits of care (variable j positive when bit j of value
is 1).  Cost of a cover = (number of cubes, number of literals), compared
in that order.  A minimum-cost cover can always be built from prime
implicants (Quine: enlarging an implicant to a prime drops literals and
keeps the cover), so the search runs over subsets of primes in order of
size.

Minimal covers are not unique (the two-plane K-map example of this project
has two).  ``canonical_cover`` fixes one: among the covers of least cost,
the one whose list of term keys, sorted, is lexicographically smallest,
where a term's key lists its literals in ascending variable order, literal
(j, positive) coded 2j and (j, negative) coded 2j + 1.  The cover is returned
sorted by term key: this is the order in which the Simplify step of the
transformation writes the terms of an expression (for the multiplexers of
the paper's Fig. 1 it gives OR(AND(s, a), AND(NOT(s), b)), the order of the
figure's generated module).

Plain loops; practical up to about ten variables with few primes.
"""
from __future__ import annotations

from itertools import combinations


def implicants(table: int, n: int):
    """Every cube whose rows all carry a 1: for each care mask, a value is
    excluded when some row with a 0 agrees with it on the cared digits."""
    zeros = [r for r in range(1 << n) if not (table >> r) & 1]
    out = []
    for care in range(1 << n):
        bad = {r & care for r in zeros}
        for value in range(1 << n):
            if value & ~care or value in bad:
                continue
            out.append((care, value))
    return out


def primes(table: int, n: int):
    """Implicants from which no literal can be dropped (an implicant inside a
    larger one can always drop a literal the larger one lacks and remain an
    implicant, so this is the usual definition of a prime implicant)."""
    imp = set(implicants(table, n))
    out = []
    for care, value in sorted(imp):
        if not any((care >> j) & 1 and (care & ~(1 << j), value & ~(1 << j)) in imp for j in range(n)):
            out.append((care, value))
    return out


def covers(cubes, table: int, n: int) -> bool:
    got = 0
    for care, value in cubes:
        for r in range(1 << n):
            if (r & care) == value:
                got |= 1 << r
    return got == table


def term_key(cube, n: int) -> tuple:
    """Literals of a cube in ascending variable order: 2j for x_j, 2j + 1 for
    NOT x_j."""
    care, value = cube
    return tuple(2 * j + (0 if (value >> j) & 1 else 1) for j in range(n) if (care >> j) & 1)


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


def canonical_cover(table: int, n: int):
    """The minimal cover picked by the tie rule above, sorted by term key.
    The constant 0 has no term; the constant 1 one term with no literal."""
    if table == 0:
        return []
    P = primes(table, n)
    for k in range(1, len(P) + 1):
        best = None
        for sub in combinations(P, k):
            if covers(sub, table, n):
                lits = sum(bin(c).count("1") for c, _ in sub)
                keys = sorted(term_key(c, n) for c in sub)
                if best is None or (lits, keys) < best[:2]:
                    best = (lits, keys, sub)
        if best is not None:
            return sorted(best[2], key=lambda c: term_key(c, n))
    raise AssertionError("primes always cover the table")


def kmap_cells(n: int = 4):
    """Cell layout of a four-variable Karnaugh map in the preamble's
    template: rows x1x2 and columns x3x4 in Gray order 00, 01, 11, 10; the
    cell holds row number 8 x1 + 4 x2 + 2 x3 + x4 (x1 the most significant
    digit of r)."""
    gray = [0, 1, 3, 2]
    return [[8 * (g1 >> 1) + 4 * (g1 & 1) + 2 * (g2 >> 1) + (g2 & 1) for g2 in gray] for g1 in gray]
