"""Pins of the network-evaluation oracle (CPU): the arithmetic evaluation of
a layered network against lookups in the C oracle's packed tables (two
independent paths to the same codes), a hand-worked two-layer example, and
the modulo-2^b reading of input codes."""
import numpy as np

import oracle
from oracle import lutnet
from workloads import cfg1, network_fanin
from workloads.gen import NeuronSet, _empty


def lookup(planes, word_off, F, b, o, row):
    W = max(1, (1 << (F * b)) // 64)
    q = 0
    for p in range(o):
        q |= int((int(planes[int(word_off) + p * W + (row >> 6)]) >> (row & 63)) & 1) << p
    return q


def test_cfg1_arithmetic_matches_table_lookups():
    ns = cfg1()
    ref = oracle.enumerate(ns, hist=False, support=False)
    rng = np.random.default_rng(5)
    P = 256
    inputs = rng.integers(0, 4, size=(64, P)).astype(np.uint8)
    sig_fanin = [f[:6] for f in network_fanin(ns)]
    # layer 0 reads inputs, layer l the outputs of layer l - 1
    assert sig_fanin[0].max() < P and P <= sig_fanin[300].min() and sig_fanin[300].max() < P + 256
    assert sig_fanin[400].min() >= P + 256
    out = lutnet.evaluate(ns, sig_fanin, P, inputs)
    for s in range(0, 64, 7):
        sig = list(inputs[s]) + [None] * len(ns)
        for i in range(len(ns)):
            row = 0
            for j, src in enumerate(sig_fanin[i]):
                row |= (int(sig[src]) & 3) << (2 * j)
            sig[P + i] = lookup(ref["planes"], ref["word_off"][i], 6, 2, 2, row)
        assert list(out[s]) == sig[P:], s


def test_hand_worked_two_layer_network():
    """Neuron 0: F=4, b=1, w=1, bias 0, one threshold 2 (q = at least two of
    four bits set).  Neuron 1: F=2, b=2, w=(1, 2), bias -1, ReLU,
    T={1,3,5}, reading primary input 4 and neuron 0: a = x0 + 2 q0 - 1."""
    ns = _empty(2, "hand")
    ns.F[:] = [4, 2]
    ns.b[:] = [1, 2]
    ns.o[:] = [1, 2]
    ns.act[:] = [1, 1]
    ns.w[0, :4] = 1
    ns.w[1, :2] = [1, 2]
    ns.bias[:] = [0, -1]
    ns.thr[0, 0] = 2
    ns.thr[1, :3] = [1, 3, 5]
    fanin = [[0, 1, 2, 3], [4, 5]]
    inputs = np.array([[0, 0, 0, 0, 0], [1, 1, 0, 0, 3], [1, 0, 0, 0, 3], [1, 1, 1, 1, 2], [0, 1, 0, 1, 1]],
                      np.uint8)
    # q0: 0, 1, 0, 1, 1;  a1 = x4 + 2 q0 - 1: -1, 4, 2, 3, 2  ->  q1: 0, 2, 1, 2, 1
    out = lutnet.evaluate(ns, fanin, 5, inputs)
    assert out[:, 0].tolist() == [0, 1, 0, 1, 1]
    assert out[:, 1].tolist() == [0, 2, 1, 2, 1]


def test_codes_are_read_modulo_two_to_the_b():
    ns = _empty(1, "mod")
    ns.F[0], ns.b[0], ns.o[0], ns.act[0] = 1, 2, 2, 0
    ns.w[0, 0] = 1
    ns.thr[0, :3] = [1, 2, 3]
    out = lutnet.evaluate(ns, [[0]], 1, np.array([[5], [7], [4]], np.uint8))
    assert out[:, 0].tolist() == [1, 3, 0]  # 5 -> 1, 7 -> 3, 4 -> 0


# ------------------------------------------------------------ sampling pins
def test_splitmix64_published_outputs():
    import json
    import pathlib
    g = json.loads((pathlib.Path(__file__).parent / "golden" / "splitmix64_vectors.json").read_text())
    for st in g["streams"]:
        want = [int(v) for v in st["first_outputs"]]
        got = lutnet.splitmix64(st["seed"], np.arange(1, len(want) + 1))
        assert [int(v) for v in got] == want


def test_draws_layout_and_continuation():
    """Draw d's bytes are the little-endian bytes of outputs d Q + 1 ...;
    a stream read in two pieces equals one read."""
    n_inputs = 13  # Q = 2, the second output only partly used
    a = lutnet.draws(99, 0, 10, n_inputs)
    b = lutnet.draws(99, 4, 6, n_inputs)
    assert a.shape == (10, 13) and np.array_equal(a[4:], b)
    z = [int(v) for v in lutnet.splitmix64(99, [2 * 7 + 1, 2 * 7 + 2])]
    row = [(z[0] >> (8 * t)) & 0xFF for t in range(8)] + [(z[1] >> (8 * t)) & 0xFF for t in range(5)]
    assert list(a[7]) == row
    # bytes are close to uniform: each bit set about half the time
    big = lutnet.draws(1, 0, 4000, 64)
    frac = np.unpackbits(big, axis=1).mean()
    assert abs(frac - 0.5) < 0.01


def test_reader_masks_hand_case():
    ns = _empty(3, "masks")
    ns.F[:] = [2, 1, 2]
    ns.b[:] = [2, 3, 2]
    ns.o[:] = [1, 1, 1]
    m = lutnet.reader_masks(ns, [[0, 1], [1], [0, 3]], 4)
    # input 0: b=2 (neurons 0, 2); input 1: b=2 and b=3; input 2: none; input 3: b=2 (neuron 2)
    assert list(m) == [3, 0xFF, 0xFF, 3]


def test_sample_partitions_draws_by_target_value():
    """Every draw is kept for exactly one value of a target signal; a target
    on a primary input keeps exactly the draws with that (reduced) input."""
    ns = cfg1()
    fanin = [f[:6] for f in network_fanin(ns)]
    P, n = 256, len(ns)
    seen = []
    for v in range(4):
        d, x = lutnet.sample(ns, fanin, P, {P + n - 1: v}, seed=3, first=100, count=600)
        assert (np.diff(d) > 0).all()
        seen.append(d)
    allv = np.sort(np.concatenate(seen))
    assert np.array_equal(allv, np.arange(100, 700))
    d_all, x_all = lutnet.sample(ns, fanin, P, {}, seed=3, first=100, count=600)
    assert np.array_equal(d_all, np.arange(100, 700))
    m = lutnet.reader_masks(ns, fanin, P)  # every reader takes 2 digits; unread inputs stay whole bytes
    assert set(np.unique(m)) <= {3, 0xFF} and (m == 3).sum() > 200
    assert np.array_equal(x_all, lutnet.draws(3, 100, 600, P) & m)
    d, x = lutnet.sample(ns, fanin, P, {17: 2, 40: 1}, seed=3, first=100, count=600)
    sel = (x_all[:, 17] == 2) & (x_all[:, 40] == 1)
    assert np.array_equal(d, d_all[sel]) and np.array_equal(x, x_all[sel])
