"""Seeded generators for the synthetic neuron workloads.

A neuron is the tuple (F, b, o, act, w[0..F-1], bias, t[0..2^o-2]):
F inputs of b unsigned bits each, int8 weights, an int16 bias, an activation
(0 = identity, 1 = ReLU) and 2^o - 1 non-decreasing int32 thresholds of an
o-bit output quantiser.  Unused weight slots (j >= F) and unused threshold
slots (k >= 2^o - 1) are zero.

Weight distribution of the small workloads follows the pruned Gaussian drawn
in the paper's preamble (the ``gaussprune`` density: a normal density whose
mass on |x| < 1 is removed, with the second argument as the standard
deviation).  We sample the real value, zero it when |x| < 1, then round half
to even and clip.  Pruning before rounding is the only reading under which
the prune is not a no-op.

Every generator takes an explicit seed; workload k uses
``numpy.random.Generator(PCG64(CONFIG_SEED_BASE + k))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

CONFIG_SEED_BASE = 20250212
MAX_F = 8
MAX_T = 7


@dataclass
class NeuronSet:
    F: np.ndarray  # uint8 [n]
    b: np.ndarray  # uint8 [n]
    o: np.ndarray  # uint8 [n]
    act: np.ndarray  # uint8 [n]
    w: np.ndarray  # int8 [n, 8]
    bias: np.ndarray  # int16 [n]
    thr: np.ndarray  # int32 [n, 7]
    name: str = ""
    # optional structure (layered workload): fan-in index sets and layer id
    fanin: Optional[np.ndarray] = None  # int32 [n, 8], -1 where unused
    layer: Optional[np.ndarray] = None  # int32 [n]
    meta: dict = field(default_factory=dict)

    def __len__(self) -> int:
        return int(self.F.shape[0])

    def rows(self) -> np.ndarray:
        """Number of truth-table rows 2^(F*b) per neuron (uint64)."""
        return np.left_shift(np.uint64(1), (self.F.astype(np.uint64) * self.b.astype(np.uint64)))

    def total_rows(self) -> int:
        return int(sum(1 << (int(f) * int(bb)) for f, bb in zip(self.F, self.b)))


def _empty(n: int, name: str) -> NeuronSet:
    return NeuronSet(
        F=np.zeros(n, np.uint8),
        b=np.zeros(n, np.uint8),
        o=np.zeros(n, np.uint8),
        act=np.ones(n, np.uint8),
        w=np.zeros((n, MAX_F), np.int8),
        bias=np.zeros(n, np.int16),
        thr=np.zeros((n, MAX_T), np.int32),
        name=name,
    )


def _pruned_gauss(rng: np.random.Generator, shape, sigma: float, clip: int) -> np.ndarray:
    x = rng.normal(0.0, sigma, size=shape)
    r = np.clip(np.rint(x), -clip, clip)
    r[np.abs(x) < 1.0] = 0.0
    return r.astype(np.int8)


def _fixed_thresholds(ns: NeuronSet, t) -> None:
    for i in range(len(ns)):
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = t[:k]


def cfg0(seed: int = CONFIG_SEED_BASE + 0) -> NeuronSet:
    """One layer of 64 neurons, F=6, b=2 (4096 rows), pruned-Gaussian int8
    weights (sigma 3, |x|<1 zeroed, clip +-7), bias U{-8..8}, ReLU, 2-bit
    output with thresholds {4, 8, 12}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 64
    ns = _empty(n, "cfg0")
    ns.F[:] = 6
    ns.b[:] = 2
    ns.o[:] = 2
    ns.act[:] = 1
    ns.w[:, :6] = _pruned_gauss(rng, (n, 6), 3.0, 7)
    ns.bias[:] = rng.integers(-8, 9, size=n)
    _fixed_thresholds(ns, [4, 8, 12])
    return ns


def cfg1(seed: int = CONFIG_SEED_BASE + 1) -> NeuronSet:
    """Three-layer sparse MLP 256 -> 128 -> 64 neurons (448 neurons), each
    with F=6 distinct fan-in indices drawn uniformly without replacement from
    the previous layer (256 primary 2-bit inputs feed layer 1); weights,
    bias, activation and thresholds as in cfg0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    widths = [256, 128, 64]
    n = sum(widths)
    ns = _empty(n, "cfg1")
    ns.F[:] = 6
    ns.b[:] = 2
    ns.o[:] = 2
    ns.act[:] = 1
    ns.fanin = np.full((n, MAX_F), -1, np.int32)
    ns.layer = np.zeros(n, np.int32)
    prev = 256  # primary inputs
    i = 0
    for li, wdt in enumerate(widths):
        for _ in range(wdt):
            ns.fanin[i, :6] = rng.choice(prev, size=6, replace=False)
            ns.layer[i] = li
            i += 1
        prev = wdt
    ns.w[:, :6] = _pruned_gauss(rng, (n, 6), 3.0, 7)
    ns.bias[:] = rng.integers(-8, 9, size=n)
    _fixed_thresholds(ns, [4, 8, 12])
    ns.meta["widths"] = widths
    ns.meta["primary_inputs"] = 256
    return ns


def _cfg2_like(rng: np.random.Generator, n: int, name: str) -> NeuronSet:
    """Uneven neurons: F ~ U{3..8}, b ~ U{1,2,3}, redrawn until F*b <= 16;
    o ~ U{1,2,3}; w = clip(round(N(0,3)), +-7) then each weight zeroed
    independently with probability 0.3; bias U{-8..8}; thresholds
    t_k = k*s with a per-neuron step s ~ U{1..8}; ReLU."""
    ns = _empty(n, name)
    F = rng.integers(3, 9, size=n)
    b = rng.integers(1, 4, size=n)
    bad = F * b > 16
    while bad.any():
        m = int(bad.sum())
        F[bad] = rng.integers(3, 9, size=m)
        b[bad] = rng.integers(1, 4, size=m)
        bad = F * b > 16
    ns.F[:] = F
    ns.b[:] = b
    ns.o[:] = rng.integers(1, 4, size=n)
    ns.act[:] = 1
    wr = np.clip(np.rint(rng.normal(0.0, 3.0, size=(n, MAX_F))), -7, 7)
    wr[rng.random(size=(n, MAX_F)) < 0.3] = 0
    wr[np.arange(MAX_F)[None, :] >= F[:, None]] = 0
    ns.w[:] = wr.astype(np.int8)
    ns.bias[:] = rng.integers(-8, 9, size=n)
    step = rng.integers(1, 9, size=n)
    for i in range(n):
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = step[i] * np.arange(1, k + 1)
    return ns


def cfg2(seed: int = CONFIG_SEED_BASE + 2, n: int = 8192) -> NeuronSet:
    rng = np.random.Generator(np.random.PCG64(seed))
    return _cfg2_like(rng, n, "cfg2")


def cfg3(seed: int = CONFIG_SEED_BASE + 3, n: int = 512) -> NeuronSet:
    """Large neurons: F=8, b=3 (2^24 rows each), w = clip(round(N(0,4)),
    +-15) without pruning, bias U{-8..8}, ReLU, 2-bit output {4, 8, 12}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = _empty(n, "cfg3")
    ns.F[:] = 8
    ns.b[:] = 3
    ns.o[:] = 2
    ns.act[:] = 1
    ns.w[:] = np.clip(np.rint(rng.normal(0.0, 4.0, size=(n, 8))), -15, 15).astype(np.int8)
    ns.bias[:] = rng.integers(-8, 9, size=n)
    _fixed_thresholds(ns, [4, 8, 12])
    return ns


def cfg4_train(n: int = 200_000, seed: int = CONFIG_SEED_BASE + 40) -> NeuronSet:
    rng = np.random.Generator(np.random.PCG64(seed))
    return _cfg2_like(rng, n, "cfg4_train")


def cfg4_screen(n: int = 100_000, seed: int = CONFIG_SEED_BASE + 41) -> NeuronSet:
    rng = np.random.Generator(np.random.PCG64(seed))
    return _cfg2_like(rng, n, "cfg4_screen")


def make_config(k: int, **kw) -> NeuronSet:
    return {0: cfg0, 1: cfg1, 2: cfg2, 3: cfg3}[k](**kw)


def random_neurons(
    seed: int,
    n: int,
    F=(1, 8),
    b=(1, 4),
    o=(1, 3),
    max_fb: int = 12,
    wmax: int = 127,
    bias_max: int = 300,
    acts=(0, 1),
    zero_frac: float = 0.2,
) -> NeuronSet:
    """Generic random neurons for parity and edge-case tests: uniform shapes
    with F*b <= max_fb, weights uniform in [-wmax, wmax] (a fraction zeroed),
    bias uniform in [-bias_max, bias_max], random sorted thresholds (ties
    allowed, some <= 0), and both activations."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = _empty(n, f"random{seed}")
    for i in range(n):
        while True:
            f = int(rng.integers(F[0], F[1] + 1))
            bb = int(rng.integers(b[0], b[1] + 1))
            if f * bb <= max_fb:
                break
        oo = int(rng.integers(o[0], o[1] + 1))
        ns.F[i], ns.b[i], ns.o[i] = f, bb, oo
        ns.act[i] = int(rng.choice(acts))
        wv = rng.integers(-wmax, wmax + 1, size=f)
        wv[rng.random(size=f) < zero_frac] = 0
        ns.w[i, :f] = wv
        ns.bias[i] = int(rng.integers(-bias_max, bias_max + 1))
        k = (1 << oo) - 1
        span = int(wmax * ((1 << bb) - 1) * f / 2 + bias_max) + 1
        t = np.sort(rng.integers(-span // 4, span + 1, size=k))
        if rng.random() < 0.2 and k > 1:  # force a tie
            j = int(rng.integers(0, k - 1))
            t[j + 1] = t[j]
        ns.thr[i, :k] = t
    return ns


def network_fanin(ns: NeuronSet) -> np.ndarray:
    """Fan-in of a layered set (cfg1) as signal indices: signals 0 .. P - 1
    are the primary inputs, signal P + i is neuron i's output; layer 0 reads
    primary inputs, layer l the outputs of layer l - 1.  int32 [n, 8], -1
    where unused."""
    P = int(ns.meta["primary_inputs"])
    starts = np.concatenate([[0], np.cumsum(ns.meta["widths"])]).astype(np.int64)
    out = np.full((len(ns), MAX_F), -1, np.int32)
    for i in range(len(ns)):
        li = int(ns.layer[i])
        base = 0 if li == 0 else P + int(starts[li - 1])
        F = int(ns.F[i])
        out[i, :F] = base + ns.fanin[i, :F]
    return out


def subset(ns: NeuronSet, idx) -> NeuronSet:
    idx = np.asarray(idx)
    out = NeuronSet(
        F=ns.F[idx].copy(), b=ns.b[idx].copy(), o=ns.o[idx].copy(), act=ns.act[idx].copy(),
        w=ns.w[idx].copy(), bias=ns.bias[idx].copy(), thr=ns.thr[idx].copy(),
        name=f"{ns.name}[sub]",
    )
    if ns.fanin is not None:
        out.fanin = ns.fanin[idx].copy()
    if ns.layer is not None:
        out.layer = ns.layer[idx].copy()
    return out


def concat(sets) -> NeuronSet:
    sets = list(sets)
    return NeuronSet(
        F=np.concatenate([s.F for s in sets]), b=np.concatenate([s.b for s in sets]),
        o=np.concatenate([s.o for s in sets]), act=np.concatenate([s.act for s in sets]),
        w=np.concatenate([s.w for s in sets]), bias=np.concatenate([s.bias for s in sets]),
        thr=np.concatenate([s.thr for s in sets]), name="+".join(s.name for s in sets),
    )


def mlp_init(seed: int, dims=(32, 256, 256, 256, 12)):
    """Initial screen weights: W_l ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)) as
    float32 [out, in], biases zero.  These are random draws only; both the
    device trainer and the reference start from the same arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for i in range(len(dims) - 1):
        lim = float(np.sqrt(6.0 / dims[i]))
        W = rng.uniform(-lim, lim, size=(dims[i + 1], dims[i])).astype(np.float32)
        params.append((W, np.zeros(dims[i + 1], np.float32)))
    return params


_GATE_KINDS = ("not", "and", "or", "nand", "nor", "xor", "xnor", "mux")


def _gate_clauses(kind, ins, f):
    """Tseitin clauses of one gate with output variable f (the gate
    signatures of the transformation section)."""
    if kind == "not":
        return [[f, ins[0]], [-f, -ins[0]]]
    if kind == "and":
        return [[f] + [-x for x in ins]] + [[-f, x] for x in ins]
    if kind == "or":
        return [[-f] + list(ins)] + [[f, -x] for x in ins]
    if kind == "nand":
        return [[-f] + [-x for x in ins]] + [[f, x] for x in ins]
    if kind == "nor":
        return [[f] + list(ins)] + [[-f, -x] for x in ins]
    if kind in ("xor", "xnor"):
        a, b = ins
        if kind == "xor":  # f = a xor b: forbid the assignments of odd parity of (a, b, f)
            return [[-a, -b, -f], [a, b, -f], [a, -b, f], [-a, b, f]]
        return [[-a, -b, f], [a, b, f], [a, -b, -f], [-a, b, -f]]
    if kind == "mux":  # f = (s and a) or (not s and b)
        s, a, b = ins
        return [[-s, -a, f], [-s, a, -f], [s, -b, f], [s, b, -f]]
    raise ValueError(kind)


def tseitin_instances(seed: int, n_inst: int, n_in=(4, 12), n_gates=(8, 64), window: int = 12):
    """Random combinational circuits written as CNF (Tseitin clauses gate by
    gate, then a unit clause forcing the last gate's output to 1), the
    synthetic stand-in for the paper's SAT benchmark instances.  Primary
    inputs are variables 1 .. n_in, gate k's output is n_in + k; each gate
    draws its kind uniformly and its inputs among the last ``window``
    signals.  Returns a list of (n_vars, clauses)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_inst):
        ni = int(rng.integers(n_in[0], n_in[1] + 1))
        ng = int(rng.integers(n_gates[0], n_gates[1] + 1))
        clauses = []
        for k in range(ng):
            f = ni + k + 1
            kind = _GATE_KINDS[int(rng.integers(len(_GATE_KINDS)))]
            arity = {"not": 1, "xor": 2, "xnor": 2, "mux": 3}.get(kind, int(rng.integers(2, 4)))
            pool = np.arange(max(1, f - window), f)
            if len(pool) < arity:
                kind, arity = "not", 1
            ins = [int(x) for x in rng.choice(pool, size=arity, replace=False)]
            clauses.extend(_gate_clauses(kind, ins, f))
        clauses.append([ni + ng])
        out.append((ni + ng, clauses))
    return out
