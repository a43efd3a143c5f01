"""GPU parity: networks evaluated through their enumerated tables
(tt_lutnet_eval) against the oracle's arithmetic evaluation, bit for bit."""
import numpy as np
import pytest

import paper_2502_08673_amd as tt
from gpu_util import device_tables, note
from oracle import lutnet
from workloads import cfg1, network_fanin, random_neurons

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run(ns, fanin, n_inputs, inputs, tables_from="plan"):
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    if tables_from == "plan":
        with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT) as plan:
            plan.launch(tables)
            torch.cuda.synchronize()
    else:
        tt.enumerate(desc, tables, total_words=total)
    x = torch.from_numpy(inputs).cuda()
    out = torch.full((inputs.shape[0], len(ns)), 0xEE, dtype=torch.uint8, device="cuda")
    note(f"lutnet {ns.name} n={len(ns)} batch={inputs.shape[0]}")
    tt.lutnet_eval(desc, fanin, n_inputs, tables, total, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_cfg1_network_through_tables():
    """The 256 -> 128 -> 64 network; input codes over the whole byte range
    (read modulo 4)."""
    ns = cfg1()
    fanin = network_fanin(ns)
    inputs = np.random.default_rng(7).integers(0, 256, size=(3000, 256)).astype(np.uint8)
    got = run(ns, fanin, 256, inputs)
    want = lutnet.evaluate(ns, [f[:6] for f in fanin], 256, inputs)
    assert np.array_equal(got, want)
    assert len(np.unique(want[:, -64:])) > 1  # the last layer is not constant


def test_cfg1_network_full_batch_sampled():
    """The benchmark's launch: the cfg1 network through a tt_lutnet handle on
    2^18 samples of 256 input codes U{0..3} (its seed); every 16th sample's
    448 outputs against the oracle, bit for bit."""
    ns = cfg1()
    fanin = network_fanin(ns)
    P, B = 256, 1 << 18
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    tt.enumerate(desc, tables, total_words=total)
    inputs = np.random.Generator(np.random.PCG64(20250212 + 101)).integers(0, 4, size=(B, P)).astype(np.uint8)
    x = torch.from_numpy(inputs).cuda()
    out = torch.full((B, len(ns)), 0xEE, dtype=torch.uint8, device="cuda")
    note(f"lutnet cfg1 full batch B={B}")
    with tt.Lutnet(desc, fanin, P, tables, total) as net:
        net.run(x, out)
        torch.cuda.synchronize()
    rows = np.arange(0, B, 16)
    want = lutnet.evaluate(ns, [f[:6] for f in fanin], P, inputs[rows])
    assert np.array_equal(out.cpu().numpy()[rows], want)


def test_random_network_mixed_shapes():
    """A random DAG of neurons of every shape (F*b up to 16, all o, both
    activations), each reading primary inputs and earlier neurons, output
    codes wider than the reader's digits included; ragged batch; tables
    from the one-shot call."""
    ns = random_neurons(seed=81, n=120, max_fb=16, wmax=20, bias_max=30)
    rng = np.random.default_rng(82)
    P = 40
    fanin = np.full((len(ns), 8), -1, np.int32)
    for i in range(len(ns)):
        F = int(ns.F[i])
        fanin[i, :F] = rng.integers(0, P + i, size=F)
    inputs = rng.integers(0, 256, size=(777, P)).astype(np.uint8)
    got = run(ns, fanin, P, inputs, tables_from="oneshot")
    want = lutnet.evaluate(ns, [fanin[i, :int(ns.F[i])] for i in range(len(ns))], P, inputs)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("F,o,P,B", [((1, 2), (1, 1), 37, 65), ((3, 5), (1, 2), 64, 128),
                                     ((7, 7), (3, 3), 13, 200), ((1, 8), (1, 3), 5, 1)])
def test_network_shapes_and_odd_rows(F, o, P, B):
    """Networks whose largest F and o take each form of the single-launch
    kernel (fan-in reads and planes per neuron), rows of odd byte counts (no
    dword staging), ragged and one-sample batches."""
    ns = random_neurons(seed=100 + P, n=53, F=F, o=o, max_fb=16)
    rng = np.random.default_rng(P)
    fanin = np.full((len(ns), 8), -1, np.int32)
    for i in range(len(ns)):
        f = int(ns.F[i])
        fanin[i, :f] = rng.integers(0, P + i, size=f)
    inputs = rng.integers(0, 256, size=(B, P)).astype(np.uint8)
    got = run(ns, fanin, P, inputs, tables_from="oneshot")
    want = lutnet.evaluate(ns, [fanin[i, :int(ns.F[i])] for i in range(len(ns))], P, inputs)
    assert np.array_equal(got, want)


def test_handle_reused_across_batches():
    """One tt_lutnet handle evaluates several batches (ragged sizes, another
    stream) with the results of the one-shot call and of the oracle."""
    ns = cfg1()
    fanin = network_fanin(ns)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    tt.enumerate(desc, tables, total_words=total)
    rng = np.random.default_rng(11)
    side = torch.cuda.Stream()
    with tt.Lutnet(desc, fanin, 256, tables, total) as net:
        torch.cuda.synchronize()
        for B, stream in ((1000, None), (77, side), (64, None)):
            inputs = rng.integers(0, 256, size=(B, 256)).astype(np.uint8)
            x = torch.from_numpy(inputs).cuda()
            out = torch.full((B, len(ns)), 0xEE, dtype=torch.uint8, device="cuda")
            note(f"lutnet handle batch={B}")
            net.run(x, out, stream=stream)
            torch.cuda.synchronize()
            want = lutnet.evaluate(ns, [f[:6] for f in fanin], 256, inputs)
            assert np.array_equal(out.cpu().numpy(), want)


def test_empty_batch_is_a_no_op():
    ns = cfg1()
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    x = torch.zeros((0, 256), dtype=torch.uint8, device="cuda")
    out = torch.zeros((0, len(ns)), dtype=torch.uint8, device="cuda")
    tt.lutnet_eval(desc, network_fanin(ns), 256, tables, total, x, out)
    torch.cuda.synchronize()


def test_wide_network_takes_the_per_level_path():
    """More signals per sample than a block keeps in LDS (6000 inputs + 300
    neurons): one launch per level, signals in global memory."""
    ns = random_neurons(seed=91, n=300, max_fb=12)
    rng = np.random.default_rng(92)
    P = 6000
    fanin = np.full((len(ns), 8), -1, np.int32)
    for i in range(len(ns)):
        F = int(ns.F[i])
        fanin[i, :F] = rng.integers(0, P + i, size=F)
    inputs = rng.integers(0, 256, size=(70, P)).astype(np.uint8)
    got = run(ns, fanin, P, inputs)
    want = lutnet.evaluate(ns, [fanin[i, :int(ns.F[i])] for i in range(len(ns))], P, inputs)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ sampling
def _cfg1_handle():
    ns = cfg1()
    fanin = network_fanin(ns)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    tt.enumerate(desc, tables, total_words=total)
    return ns, fanin, tt.Lutnet(desc, fanin, 256, tables, total), tables


def _found(net, targets, seed, first, n, max_found, count=None):
    fi = torch.full((max_found, net.n_inputs), 0xEE, dtype=torch.uint8, device="cuda")
    fd = torch.full((max_found,), -1, dtype=torch.int64, device="cuda")
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
    note(f"lutnet sample targets={targets} seed={seed} first={first} draws={n} max_found={max_found}")
    net.sample(targets, seed, first, n, fi, fd, count)
    torch.cuda.synchronize()
    return fi.cpu().numpy(), fd.cpu().numpy(), int(count.item())


def test_sample_without_targets_keeps_every_draw():
    """Every draw kept: the device draws equal the oracle's SplitMix64 draws
    (reduced to the readers' digits), each draw exactly once."""
    ns, fanin, net, _ = _cfg1_handle()
    with net:
        fi, fd, c = _found(net, {}, seed=12345, first=7, n=1000, max_found=1000)
    assert c == 1000
    order = np.argsort(fd)
    assert np.array_equal(fd[order], np.arange(7, 1007))
    want_d, want_x = lutnet.sample(ns, [f[:6] for f in fanin], 256, {}, 12345, 7, 1000)
    assert np.array_equal(fi[order], want_x)


def test_sample_with_output_targets_matches_oracle():
    """Targets on two last-layer neurons and one input; the kept set, each
    kept draw's inputs and the count equal the oracle's; a second call
    continues the stream and adds to the count."""
    ns, fanin, net, _ = _cfg1_handle()
    f6 = [f[:6] for f in fanin]
    P, n = 256, len(ns)
    pilot = lutnet.evaluate(ns, f6, P, lutnet.draws(1, 0, 2000, P) & lutnet.reader_masks(ns, f6, P))
    v1 = int(np.bincount(pilot[:, n - 1]).argmax())
    v2 = int(np.bincount(pilot[:, n - 5]).argmax())
    targets = {P + n - 1: v1, P + n - 5: v2, 3: 1}
    with net:
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        fi, fd, c1 = _found(net, targets, seed=77, first=0, n=3000, max_found=3000, count=count)
        want_d, want_x = lutnet.sample(ns, f6, P, targets, 77, 0, 3000)
        assert 0 < c1 == len(want_d) < 3000
        order = np.argsort(fd[:c1])
        assert np.array_equal(fd[:c1][order], want_d)
        assert np.array_equal(fi[:c1][order], want_x)
        assert (fd[c1:] == -1).all()
        fi2, fd2, c2 = _found(net, targets, seed=77, first=3000, n=1500, max_found=3000, count=count)
    want2, _ = lutnet.sample(ns, f6, P, targets, 77, 3000, 1500)
    assert c2 == c1 + len(want2)
    assert np.array_equal(np.sort(fd2[c1:c2]), want2)


def test_sample_places_beyond_max_found_are_not_written():
    ns, fanin, net, _ = _cfg1_handle()
    f6 = [f[:6] for f in fanin]
    with net:
        fi, fd, c = _found(net, {}, seed=5, first=0, n=500, max_found=100)
    assert c == 500
    want_d, want_x = lutnet.sample(ns, f6, 256, {}, 5, 0, 500)
    assert len(set(fd.tolist())) == 100 and set(fd.tolist()) <= set(want_d.tolist())
    assert np.array_equal(fi, want_x[fd])


@pytest.mark.parametrize("P", [13, 600])
def test_sample_draw_widths(P):
    """Input rows that are not a whole number of 8-byte draws (13 bytes: two
    draws, the second cut to 5 bytes, several rows per wave pass) and rows
    of more than 64 draws (600 bytes: a lane takes two of a row's draws):
    every draw kept, equal to the oracle's."""
    ns = random_neurons(seed=140 + P, n=53, max_fb=12, wmax=20, bias_max=30)
    rng = np.random.default_rng(P + 1)
    fanin = np.full((len(ns), 8), -1, np.int32)
    for i in range(len(ns)):
        f = int(ns.F[i])
        fanin[i, :f] = rng.integers(0, P + i, size=f)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    tt.enumerate(desc, tables, total_words=total)
    with tt.Lutnet(desc, fanin, P, tables, total) as net:
        fi, fd, c = _found(net, {}, seed=99, first=3, n=300, max_found=300)
    assert c == 300
    order = np.argsort(fd)
    assert np.array_equal(fd[order], np.arange(3, 303))
    _, want_x = lutnet.sample(ns, [fanin[i, :int(ns.F[i])] for i in range(len(ns))], P, {}, 99, 3, 300)
    assert np.array_equal(fi[order], want_x)


def test_sample_rejects_a_per_level_network():
    ns = random_neurons(seed=91, n=300, max_fb=12)
    rng = np.random.default_rng(92)
    P = 6000
    fanin = np.full((len(ns), 8), -1, np.int32)
    for i in range(len(ns)):
        fanin[i, :int(ns.F[i])] = rng.integers(0, P + i, size=int(ns.F[i]))
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    with tt.Lutnet(desc, fanin, P, tables, total) as net:
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(tt.TTError):
            net.sample({}, 1, 0, 64, None, None, count)
