"""Two-level minimisation of planes enumerated on the device: the host
minimiser (tt_sop_minimize) reads planes that tt_enumerate wrote and copied
back.  The hand-worked K-map examples and every small random neuron
(at most 4 row bits) get the oracle's minimal cost and its canonical cover;
planes of the 3-layer network's neurons (12 row bits) get covers equal to
the device plane and made of implicants."""
import json
import os

import numpy as np
import pytest

import paper_2502_08673_amd as tt
from gpu_util import host_u64, note
from oracle import sop
from workloads import cfg1, random_neurons, subset
from pins import one_neuron

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kmap_examples.json")


def device_planes(ns):
    """Every plane of every neuron, enumerated on the device: a list of
    (neuron, plane, row bits, words)."""
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = torch.zeros(total, dtype=torch.int64, device="cuda")
    note(f"enumerate {ns.name} n={len(ns)} for minimisation")
    tt.enumerate(desc, tables, total_words=total)
    torch.cuda.synchronize()
    words = host_u64(tables, 0, total)
    out = []
    for i in range(len(ns)):
        n = int(ns.F[i]) * int(ns.b[i])
        W = max(1, (1 << n) // 64)
        for p in range(int(ns.o[i])):
            at = int(desc["word_off"][i]) + p * W
            out.append((i, p, n, words[at:at + W].copy()))
    return out


def as_int(words, n):
    t = 0
    for w, x in enumerate(words):
        t |= int(x) << (64 * w)
    return t & ((1 << (1 << n)) - 1)


def cover_rows(terms, n):
    r = np.arange(1 << n, dtype=np.uint32)
    got = np.zeros(1 << n, bool)
    for care, value in terms:
        got |= (r & care) == value
    return got


def plane_rows(words, n):
    bits = np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little").astype(bool)
    return bits[: 1 << n]


def test_hand_worked_examples_from_device_planes():
    data = json.load(open(GOLDEN))
    for ex in data["examples"][:2]:  # A (2-of-4) and B (two 2-bit inputs)
        ns = one_neuron(ex["F"], ex["b"], ex["o"], ex["act"], ex["w"], ex["bias"], ex["thr"])
        for _, p, n, words in device_planes(ns):
            assert int(words[0]) == int(ex["planes"][p], 16)
            terms, lits, exact = tt.sop_minimize(words, n)
            t = as_int(words, n)
            assert exact and terms == sop.canonical_cover(t, n)
            assert (len(terms), lits) == sop.minimal_cost(t, n)[0]
    # A: the six two-literal pairs; B plane 1: a + b c (3 literals), plane 0:
    # b xor c + a b (three terms, six literals)
    ns = one_neuron(4, 1, 1, 1, [1, 1, 1, 1], 0, [2])
    terms, lits, _ = tt.sop_minimize(device_planes(ns)[0][3], 4)
    assert len(terms) == 6 and lits == 12 and all(bin(c).count("1") == 2 for c, _ in terms)
    ns = one_neuron(2, 2, 2, 1, [1, 2], -1, [1, 3, 5])
    (_, _, _, w0), (_, _, _, w1) = device_planes(ns)
    assert tt.sop_minimize(w1, 4)[:2][1] == 3 and len(tt.sop_minimize(w1, 4)[0]) == 2
    assert len(tt.sop_minimize(w0, 4)[0]) == 3 and tt.sop_minimize(w0, 4)[1] == 6


def test_small_random_neurons_minimal_and_canonical():
    ns = random_neurons(71, 300, F=(1, 4), b=(1, 2), max_fb=4, wmax=7, bias_max=12)
    n_checked = 0
    for _, _, n, words in device_planes(ns):
        terms, lits, exact = tt.sop_minimize(words, n)
        t = as_int(words, n)
        assert exact
        assert (len(terms), lits) == sop.minimal_cost(t, n)[0]
        assert terms == sop.canonical_cover(t, n)
        n_checked += 1
    assert n_checked >= 300


def test_network_neuron_planes_covered_by_implicants():
    ns = subset(cfg1(), list(range(0, 448, 28)))  # 16 neurons across the three layers
    for i, p, n, words in device_planes(ns):
        assert n == 12
        terms, lits, exact = tt.sop_minimize(words, n, node_budget=100000)
        on = plane_rows(words, n)
        assert np.array_equal(cover_rows(terms, n), on), (i, p)
        r = np.arange(1 << n, dtype=np.uint32)
        for care, value in terms:  # every term is an implicant of the plane
            assert on[(r & care) == value].all(), (i, p, care, value)
        assert lits == sum(bin(c).count("1") for c, _ in terms)
