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
