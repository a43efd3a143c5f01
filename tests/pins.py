"""Checks that pin the CPU oracle to facts other than itself.

Each check takes an oracle library handle so the same suite can be run
against deliberately broken copies of the oracle (see
``test_oracle_mutants.py``).  Sources of truth used here:

* hand-worked tables in ``tests/golden/kmap_examples.json``;
* closed forms (digit-sum polynomial coefficients, binomial sums);
* a generating-function histogram and a sum-set support test, two exact
  algorithms that never enumerate rows;
* an independent pure-Python brute force for tiny neurons;
* invariants: histogram mass, monotonicity, zero weights, digit complement,
  shift and scale equivalences, ReLU as a no-op for positive thresholds.
"""
from __future__ import annotations

import json
import math
import os
from collections import defaultdict

import numpy as np

import oracle
from oracle import brute
from workloads.gen import _empty, random_neurons, cfg0, cfg3, subset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kmap_examples.json")


def one_neuron(F, b, o, act, w, bias, thr):
    ns = _empty(1, "one")
    ns.F[0], ns.b[0], ns.o[0], ns.act[0] = F, b, o, act
    ns.w[0, : len(w)] = w
    ns.bias[0] = bias
    ns.thr[0, : len(thr)] = thr
    return ns


def q_of(a, act, thr_used):
    if act == 1:
        a = max(a, 0)
    return sum(1 for t in thr_used if a >= t)


# ---------------------------------------------------------------- golden
def check_golden(lib):
    data = json.load(open(GOLDEN))
    for ex in data["examples"]:
        ns = one_neuron(ex["F"], ex["b"], ex["o"], ex["act"], ex["w"], ex["bias"], ex["thr"])
        r = oracle.enumerate(ns, lib=lib)
        got = [int(x) for x in r["planes"]]
        want = [int(x, 16) for x in ex["planes"]]
        assert got == want, (ex["name"], [hex(x) for x in got])
        assert list(r["hist"][0]) == ex["hist"], (ex["name"], r["hist"][0])
        assert int(r["support"][0]) == ex["support"], (ex["name"], r["support"][0])
        if "codes" in ex:
            assert list(oracle.codes(ns, lib=lib)) == ex["codes"], ex["name"]
        for p in range(ex["o"]):
            key = f"kmap_plane{p}"
            if key in ex:
                assert brute.kmap4(got[p]) == ex[key], (ex["name"], key)
    cf = data["closed_forms"]["unit_weights_F6_b2_T4_8_12"]
    ns = one_neuron(6, 2, 2, 1, [1] * 6, 0, [4, 8, 12])
    assert list(oracle.enumerate(ns, lib=lib)["hist"][0]) == cf["hist"]


# ----------------------------------------------------------- closed forms
def check_digit_sum_closed_form(lib):
    """Unit weights, zero bias: a is the digit sum, so the number of rows with
    a = s is the coefficient of z^s in (1 + z + ... + z^(2^b - 1))^F."""
    for F, b, thr in [(6, 2, [4, 8, 12]), (5, 3, [3, 9, 17]), (8, 1, [2, 5, 7]), (4, 4, [10, 20, 30])]:
        poly = np.array([1], dtype=object)
        for _ in range(F):
            poly = np.convolve(poly, np.array([1] * (1 << b), dtype=object))
        want = [0] * 8
        for s, c in enumerate(poly):
            want[q_of(s, 1, thr)] += int(c)
        ns = one_neuron(F, b, 2, 1, [1] * F, 0, thr)
        assert list(oracle.enumerate(ns, lib=lib)["hist"][0]) == want, (F, b)


def check_binomial_closed_form(lib):
    """b = 1, unit weights, one threshold t: sum_{k >= t} C(F, k) ones."""
    for F in range(1, 9):
        for t in range(0, F + 2):
            ns = one_neuron(F, 1, 1, 0, [1] * F, 0, [t])
            h = oracle.enumerate(ns, lib=lib)["hist"][0]
            ones = sum(math.comb(F, k) for k in range(max(t, 0), F + 1))
            assert int(h[1]) == ones and int(h[0]) == (1 << F) - ones, (F, t)


# ------------------------------------------ generating function / sum-set
def gf_distribution(F, b, w, bias):
    """Multiset of pre-activations a over all 2^(F*b) rows, by convolving the
    per-input value distributions (no row is enumerated)."""
    dist = {int(bias): 1}
    for j in range(F):
        nxt = defaultdict(int)
        for a, c in dist.items():
            for x in range(1 << b):
                nxt[a + int(w[j]) * x] += c
        dist = nxt
    return dist


def gf_hist(F, b, o, act, w, bias, thr):
    K = (1 << o) - 1
    h = [0] * 8
    for a, c in gf_distribution(F, b, w, bias).items():
        h[q_of(a, act, [int(t) for t in thr[:K]])] += c
    return h


def sumset_support(F, b, o, act, w, bias, thr):
    """Input j is in the support iff for some value s of the other inputs'
    weighted sum (plus bias) the code changes as x_j runs over its values."""
    K = (1 << o) - 1
    tu = [int(t) for t in thr[:K]]
    s = 0
    for j in range(F):
        others = [int(w[k]) for k in range(F) if k != j]
        rest = gf_distribution(F - 1, b, others, bias)
        for a0 in rest:
            qs = {q_of(a0 + int(w[j]) * x, act, tu) for x in range(1 << b)}
            if len(qs) > 1:
                s |= 1 << j
                break
    return s


def check_generating_function(lib, n_random=60, n_big=2):
    ns = random_neurons(seed=7, n=n_random, max_fb=16, wmax=127, bias_max=400)
    r = oracle.enumerate(ns, lib=lib)
    for i in range(len(ns)):
        args = (int(ns.F[i]), int(ns.b[i]), int(ns.o[i]), int(ns.act[i]), ns.w[i], int(ns.bias[i]), ns.thr[i])
        assert list(r["hist"][i]) == gf_hist(*args), i
        assert int(r["support"][i]) == sumset_support(*args), i
    big = subset(cfg3(), list(range(n_big)))
    r = oracle.enumerate(big, lib=lib)
    for i in range(len(big)):
        args = (8, 3, 2, 1, big.w[i], int(big.bias[i]), big.thr[i])
        assert list(r["hist"][i]) == gf_hist(*args), i
        assert int(r["support"][i]) == sumset_support(*args), i


# ----------------------------------------------------------- brute force
def check_brute_force(lib, n=150, seed=11, max_fb=10):
    ns = random_neurons(seed=seed, n=n, max_fb=max_fb)
    r = oracle.enumerate(ns, lib=lib)
    for i in range(len(ns)):
        F, b, o = int(ns.F[i]), int(ns.b[i]), int(ns.o[i])
        bf = brute.brute(F, b, o, int(ns.act[i]), ns.w[i], int(ns.bias[i]), ns.thr[i])
        off = int(r["word_off"][i])
        W = max(1, (1 << (F * b)) // 64)
        for p in range(o):
            got = [int(x) for x in r["planes"][off + p * W: off + (p + 1) * W]]
            assert got == bf["planes"][p], (i, p)
        assert list(r["hist"][i]) == bf["hist"], i
        assert int(r["support"][i]) == bf["support"], i


# ------------------------------------------------------------ invariants
def _codes_by_neuron(ns, lib):
    c = oracle.codes(ns, lib=lib)
    out, off = [], 0
    for i in range(len(ns)):
        R = 1 << (int(ns.F[i]) * int(ns.b[i]))
        out.append(c[off: off + R])
        off += R
    return out


def check_invariants(lib):
    ns = random_neurons(seed=23, n=80, max_fb=14)
    base = cfg0()
    for s in (ns, base):
        r = oracle.enumerate(s, lib=lib)
        codes = _codes_by_neuron(s, lib)
        for i in range(len(s)):
            F, b = int(s.F[i]), int(s.b[i])
            R = 1 << (F * b)
            assert int(r["hist"][i].sum()) == R
            rows = np.arange(R, dtype=np.int64)
            dmax = (1 << b) - 1
            for j in range(F):
                wj = int(s.w[i, j])
                xj = (rows >> (j * b)) & dmax
                lo = rows[xj < dmax]
                step = codes[i][lo + (1 << (j * b))].astype(int) - codes[i][lo].astype(int)
                if wj >= 0:
                    assert (step >= 0).all(), (i, j)  # non-decreasing in x_j
                if wj <= 0:
                    assert (step <= 0).all(), (i, j)
                if wj == 0:
                    assert not (int(r["support"][i]) >> j) & 1
    # digit complement: (-w, bias + sum w_j (2^b-1)) at row ~r equals (w, bias) at r
    ns = random_neurons(seed=31, n=60, max_fb=12, wmax=100, bias_max=200)
    comp = _empty(len(ns), "comp")
    for f in ("F", "b", "o", "act", "thr"):
        getattr(comp, f)[:] = getattr(ns, f)
    comp.w[:] = -ns.w.astype(np.int16)
    dm = (1 << ns.b.astype(np.int64)) - 1
    comp.bias[:] = ns.bias.astype(np.int64) + (ns.w.astype(np.int64) * dm[:, None]).sum(1)
    c0, c1 = _codes_by_neuron(ns, lib), _codes_by_neuron(comp, lib)
    for i in range(len(ns)):
        R = 1 << (int(ns.F[i]) * int(ns.b[i]))
        assert np.array_equal(c0[i], c1[i][(R - 1) - np.arange(R)]), i
    # shift (identity activation) and positive scale
    ns = random_neurons(seed=37, n=60, max_fb=12, wmax=40, bias_max=100, acts=(0,))
    sh = subset(ns, np.arange(len(ns)))
    sh.bias[:] = ns.bias.astype(np.int32) + 57
    sh.thr[:] = ns.thr + 57
    sc = subset(ns, np.arange(len(ns)))
    sc.w[:] = ns.w * 3
    sc.bias[:] = ns.bias.astype(np.int32) * 3
    sc.thr[:] = ns.thr * 3
    a, b_, c = oracle.codes(ns, lib=lib), oracle.codes(sh, lib=lib), oracle.codes(sc, lib=lib)
    assert np.array_equal(a, b_) and np.array_equal(a, c)
    # ReLU changes nothing when every used threshold is positive
    pos = subset(cfg0(), np.arange(64))
    ident = subset(pos, np.arange(64))
    ident.act[:] = 0
    assert np.array_equal(oracle.codes(pos, lib=lib), oracle.codes(ident, lib=lib))


def check_layout(lib):
    ns = random_neurons(seed=41, n=40, max_fb=12)
    word_off, total = oracle.offsets(ns, lib=lib)
    acc = 0
    for i in range(len(ns)):
        assert int(word_off[i]) == acc
        acc += int(ns.o[i]) * max(1, (1 << (int(ns.F[i]) * int(ns.b[i]))) // 64)
    assert total == acc
    r = oracle.enumerate(ns, lib=lib)
    for i in range(len(ns)):
        R = 1 << (int(ns.F[i]) * int(ns.b[i]))
        if R < 64:
            for p in range(int(ns.o[i])):
                assert int(r["planes"][int(word_off[i]) + p]) >> R == 0


ALL_CHECKS = [
    check_golden,
    check_digit_sum_closed_form,
    check_binomial_closed_form,
    check_generating_function,
    check_brute_force,
    check_invariants,
    check_layout,
]
