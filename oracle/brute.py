"""Pure-Python brute force for tiny neurons -- TEST INFRASTRUCTURE ONLY.

A second, independent reading of the enumeration definition, written without
bit shifts or the C oracle's loops: input vectors come from
``itertools.product`` (whose first element varies slowest, so it is reversed
to make input 0 the least significant digit), the row index is rebuilt by
positional arithmetic, planes are assembled as Python big integers and the
support is decided by comparing every pair of input vectors that differ in one
position.  Cost grows as 2^(F*b) * F * 2^b: use only for F*b <= 12.
"""
from __future__ import annotations

import itertools
from collections import Counter


def neuron_codes(F, b, o, act, w, bias, thr):
    """dict row -> q for one neuron."""
    base = 2 ** b
    K = 2 ** o - 1
    codes = {}
    for xs in itertools.product(range(base), repeat=F):
        x = xs[::-1]  # x[0] is input 0, the least significant digit
        row = sum(x[j] * base ** j for j in range(F))
        a = int(bias) + sum(int(w[j]) * x[j] for j in range(F))
        if act == 1:
            a = max(a, 0)
        codes[row] = sum(1 for k in range(K) if a >= int(thr[k]))
    return codes


def planes_words(F, b, o, codes):
    """List of o planes, each a list of 64-bit words (little-endian rows)."""
    rows = 2 ** (F * b)
    nwords = max(1, rows // 64)
    out = []
    for p in range(o):
        big = 0
        for r in range(rows):
            if (codes[r] >> p) & 1:
                big += 2 ** r
        out.append([(big >> (64 * i)) & (2 ** 64 - 1) for i in range(nwords)])
    return out


def hist(codes):
    c = Counter(codes.values())
    return [c.get(v, 0) for v in range(8)]


def support(F, b, codes):
    base = 2 ** b
    s = 0
    vecs = list(itertools.product(range(base), repeat=F))

    def row(x):
        return sum(x[j] * base ** j for j in range(F))

    for j in range(F):
        hit = False
        for xs in vecs:
            x = list(xs[::-1])
            q0 = codes[row(x)]
            for v in range(base):
                if v == x[j]:
                    continue
                y = list(x)
                y[j] = v
                if codes[row(y)] != q0:
                    hit = True
                    break
            if hit:
                break
        if hit:
            s |= 1 << j
    return s


def brute(F, b, o, act, w, bias, thr):
    codes = neuron_codes(F, b, o, act, w, bias, thr)
    return {
        "codes": codes,
        "planes": planes_words(F, b, o, codes),
        "hist": hist(codes),
        "support": support(F, b, codes),
    }


def kmap4(plane_word):
    """Render a 16-row single-word plane as the 4-variable Karnaugh map of the
    paper's preamble: rows are x1x2 and columns x3x4, both in Gray order
    00, 01, 11, 10, and the cell for (x1, x2, x3, x4) is row index
    8*x1 + 4*x2 + 2*x3 + x4, so x1 is the most significant row bit."""
    gray = [(0, 0), (0, 1), (1, 1), (1, 0)]
    grid = []
    for (x1, x2) in gray:
        line = []
        for (x3, x4) in gray:
            cell = 8 * x1 + 4 * x2 + 2 * x3 + x4
            line.append((plane_word >> cell) & 1)
        grid.append(line)
    return grid
