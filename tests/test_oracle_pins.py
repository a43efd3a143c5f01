"""The CPU oracle against hand-worked tables, closed forms, exact non-enumerating
algorithms, an independent brute force and invariants (no GPU)."""
import numpy as np
import pytest

import pins
from workloads import cfg0, cfg1, cfg2, cfg3


def test_golden_examples(oracle_lib):
    pins.check_golden(oracle_lib)


def test_digit_sum_closed_form(oracle_lib):
    pins.check_digit_sum_closed_form(oracle_lib)


def test_binomial_closed_form(oracle_lib):
    pins.check_binomial_closed_form(oracle_lib)


def test_generating_function_and_sumset(oracle_lib):
    pins.check_generating_function(oracle_lib)


def test_brute_force_tiny(oracle_lib):
    pins.check_brute_force(oracle_lib)


@pytest.mark.slow
def test_brute_force_up_to_12_bits(oracle_lib):
    pins.check_brute_force(oracle_lib, n=40, seed=13, max_fb=12)


def test_invariants(oracle_lib):
    pins.check_invariants(oracle_lib)


def test_layout(oracle_lib):
    pins.check_layout(oracle_lib)


def test_unused_slots_ignored(oracle_lib):
    """Weights beyond F and thresholds beyond 2^o - 1 do not matter."""
    import oracle
    from workloads import random_neurons, subset
    ns = random_neurons(seed=5, n=50, max_fb=10)
    junk = subset(ns, np.arange(len(ns)))
    for i in range(len(ns)):
        junk.w[i, int(ns.F[i]):] = 99
        junk.thr[i, (1 << int(ns.o[i])) - 1:] = -12345
    a = oracle.enumerate(ns, lib=oracle_lib)
    b = oracle.enumerate(junk, lib=oracle_lib)
    for k in ("planes", "hist", "support"):
        assert np.array_equal(a[k], b[k])


# ----------------------------------------------------------- generator
def test_generator_cfg0_distribution():
    """cfg0 weights: pruned Gaussian with sigma 3 -- the zero fraction is
    P(|x| < 1) = erf(1 / (3 sqrt 2)) = 0.2611; clip to [-7, 7]."""
    ns = cfg0()
    w = ns.w[:, :6]
    assert len(ns) == 64 and (ns.F == 6).all() and (ns.b == 2).all() and (ns.o == 2).all()
    assert np.abs(w).max() <= 7
    big = np.concatenate([cfg0(seed=s).w[:, :6].ravel() for s in range(100, 140)])
    assert abs((big == 0).mean() - 0.2611) < 0.015
    assert (ns.bias >= -8).all() and (ns.bias <= 8).all()
    assert (ns.thr[:, :3] == [4, 8, 12]).all()


def test_generator_cfg1_structure():
    ns = cfg1()
    assert len(ns) == 448
    assert list(np.bincount(ns.layer)) == [256, 128, 64]
    for i in range(len(ns)):
        fi = ns.fanin[i, :6]
        assert len(set(fi.tolist())) == 6
        limit = 256 if ns.layer[i] == 0 else (256 if ns.layer[i] == 1 else 128)
        assert fi.max() < limit


def test_generator_cfg2_distribution():
    ns = cfg2()
    fb = ns.F.astype(int) * ns.b.astype(int)
    assert len(ns) == 8192 and fb.max() <= 16 and ns.F.min() >= 3 and ns.F.max() <= 8
    assert abs(ns.total_rows() / len(ns) - 8349.3) / 8349.3 < 0.1
    live = np.arange(8)[None, :] < ns.F[:, None]
    wz = (ns.w[live] == 0).mean()
    # 30% zeroed plus round(N(0,3)) == 0 (about 0.13 of the rest)
    assert 0.33 < wz < 0.43
    for i in range(0, len(ns), 97):
        K = (1 << int(ns.o[i])) - 1
        t = ns.thr[i, :K]
        assert (np.diff(t) > 0).all() and t[0] >= 1 and t[0] <= 8


def test_generator_cfg3_shape():
    ns = cfg3()
    assert len(ns) == 512 and (ns.F == 8).all() and (ns.b == 3).all()
    assert np.abs(ns.w.astype(int)).max() <= 15
    assert ns.total_rows() == 512 * (1 << 24)


def test_generator_is_seeded():
    a, b = cfg2(), cfg2()
    for f in ("F", "b", "o", "w", "bias", "thr"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
