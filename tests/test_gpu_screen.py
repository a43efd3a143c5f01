"""GPU parity of the learned screen: BF16 layer kernels, loss, Adam, features
and labels against the float64 reference; the screening pipeline (reduced
enumeration, exact check, fallback) against the CPU oracle, bit for bit."""
import math

import numpy as np
import pytest

import oracle
import paper_2502_08673_amd as tt
from gpu_util import note
from oracle import mlp_ref
from workloads import cfg4_train, concat, mlp_init, random_neurons, subset

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def bf16_bits(x64):
    """bf16 bit patterns (as int16) of values already representable in bf16."""
    f = np.asarray(x64, np.float32)
    return torch.from_numpy((f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()


def from_bf16(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def rnd(shape, seed, scale=1.0):
    return mlp_ref.bf16_round(np.random.default_rng(seed).normal(size=shape) * scale)


@pytest.mark.parametrize("B,K,N,relu", [(70, 32, 256, 1), (256, 256, 256, 1), (33, 256, 12, 0), (1, 17, 5, 1)])
def test_forward_layer(B, K, N, relu):
    X, W = rnd((B, K), 1), rnd((N, K), 2, 0.2)
    bias = np.random.default_rng(3).normal(size=N).astype(np.float32)
    ref = X @ W.T + bias.astype(np.float64)
    if relu:
        ref = np.maximum(ref, 0)
    yf = torch.empty((B, N), dtype=torch.float32, device="cuda")
    yb = torch.empty((B, N), dtype=torch.int16, device="cuda")
    note(f"mlp forward {B}x{K}x{N}")
    tt.mlp_forward(bf16_bits(X), B, bf16_bits(W), torch.from_numpy(bias).cuda(), relu, y_bf16=yb, y_f32=yf)
    torch.cuda.synchronize()
    scale = np.abs(X) @ np.abs(W).T + np.abs(bias)
    err = np.abs(yf.cpu().numpy() - ref)
    assert (err <= 1e-6 * scale + 1e-7).all()  # fp32 accumulation of bf16 products
    # bf16 output: within one bf16 rounding of the exact value
    assert (np.abs(from_bf16(yb) - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-6 * scale + 1e-30).all()


@pytest.mark.parametrize("B,IN,OUT", [(96, 256, 12), (300, 32, 256), (5, 64, 40), (4096, 256, 256),
                                      (1000, 256, 256), (4096, 256, 12), (4096, 32, 256), (77, 256, 256)])
def test_backward_layer(B, IN, OUT):
    dY, W = rnd((B, OUT), 4, 0.01), rnd((OUT, IN), 5, 0.1)
    X = mlp_ref.bf16_round(np.maximum(np.random.default_rng(6).normal(size=(B, IN)), 0))
    dx = torch.empty((B, IN), dtype=torch.int16, device="cuda")
    dw = torch.empty((OUT, IN), dtype=torch.float32, device="cuda")
    db = torch.empty(OUT, dtype=torch.float32, device="cuda")
    scratch = torch.empty(tt.mlp_scratch_floats(B, max(IN, OUT)), dtype=torch.float32, device="cuda")
    note(f"mlp backward {B}x{IN}x{OUT}")
    tt.mlp_backward(bf16_bits(dY), B, bf16_bits(W), bf16_bits(X), relu_mask=True, dx=dx, dw=dw, db=db,
                    scratch=scratch)
    torch.cuda.synchronize()
    ref_dx = (dY @ W) * (X > 0)
    ref_dw = dY.T @ X
    ref_db = dY.sum(0)
    s_dx = (np.abs(dY) @ np.abs(W))
    assert (np.abs(from_bf16(dx) - ref_dx) <= 2.0 ** -8 * np.abs(ref_dx) + 1e-6 * s_dx + 1e-30).all()
    assert (np.abs(dw.cpu().numpy() - ref_dw) <= 1e-6 * (np.abs(dY).T @ np.abs(X)) + 1e-9).all()
    assert (np.abs(db.cpu().numpy() - ref_db) <= 1e-6 * np.abs(dY).sum(0) + 1e-9).all()


def test_loss_and_gradient():
    B = 517
    rng = np.random.default_rng(8)
    z = (rng.normal(size=(B, 12)) * 3).astype(np.float32)
    y = (rng.random((B, 8)) < 0.5).astype(np.float32)
    m = (rng.random((B, 8)) < 0.8).astype(np.float32)
    h = rng.dirichlet(np.ones(4), size=B).astype(np.float32)
    L, dz = mlp_ref.loss(z.astype(np.float64), y, m, h)
    dzt = torch.empty((B, 12), dtype=torch.int16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    scratch = torch.empty(64, dtype=torch.float32, device="cuda")
    tt.mlp_loss(torch.from_numpy(z).cuda(), B, torch.from_numpy(y).cuda(), torch.from_numpy(m).cuda(),
                torch.from_numpy(h).cuda(), dzt, loss, scratch)
    torch.cuda.synchronize()
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    assert (np.abs(from_bf16(dzt) - dz) <= 2.0 ** -8 * np.abs(dz) + 1e-9).all()


def test_adam_multi_equals_separate_steps():
    """One tt_adam_step_multi launch over tensors of uneven sizes gives the
    bits of one tt_adam_step per tensor, over several steps."""
    rng = np.random.default_rng(12)
    sizes = [1, 255, 256, 4097, 12, 65536 + 3]
    mk = lambda: [torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda() for n in sizes]
    p0 = mk()
    pa, pb_ = [t.clone() for t in p0], [t.clone() for t in p0]
    ma, va = [torch.zeros_like(t) for t in p0], [torch.zeros_like(t) for t in p0]
    mb, vb = [torch.zeros_like(t) for t in p0], [torch.zeros_like(t) for t in p0]
    ba = [torch.zeros(t.numel(), dtype=torch.int16, device="cuda") for t in p0]
    bb = [torch.zeros(t.numel(), dtype=torch.int16, device="cuda") for t in p0]
    bb[1] = None
    for step in range(1, 4):
        grads = mk()
        note(f"adam multi step {step}")
        for k in range(len(sizes)):
            tt.adam_step(pa[k], grads[k], ma[k], va[k], ba[k] if k != 1 else None, 3e-3, 0.9, 0.999, 1e-8, step)
        group = tt.AdamGroup(pb_, grads, mb, vb, bb)
        group.step(3e-3, 0.9, 0.999, 1e-8, step)
        torch.cuda.synchronize()
        for k in range(len(sizes)):
            assert torch.equal(pa[k], pb_[k]) and torch.equal(ma[k], mb[k]) and torch.equal(va[k], vb[k]), k
            if k != 1:
                assert torch.equal(ba[k], bb[k]), k


def test_adam_matches_reference():
    rng = np.random.default_rng(9)
    p = rng.normal(size=1000).astype(np.float32)
    state = {}
    tp = torch.from_numpy(p.copy()).cuda()
    m = torch.zeros_like(tp)
    v = torch.zeros_like(tp)
    pb = torch.empty(1000, dtype=torch.int16, device="cuda")
    ref = [(p.astype(np.float64), np.zeros(1))]
    for step in range(1, 4):
        g = (rng.normal(size=1000) * 0.1).astype(np.float32)
        tt.adam_step(tp, torch.from_numpy(g).cuda(), m, v, pb, 1e-2, 0.9, 0.999, 1e-8, step)
        ref = mlp_ref.adam_step(ref, [(g.astype(np.float64), np.zeros(1))], state, lr=1e-2)
    torch.cuda.synchronize()
    assert np.allclose(tp.cpu().numpy(), ref[0][0], rtol=1e-5, atol=1e-6)
    assert np.array_equal(from_bf16(pb), mlp_ref.bf16_round(tp.cpu().numpy()))


def test_features_and_labels_exact():
    ns = concat([cfg4_train(n=3000, seed=123), random_neurons(seed=4, n=200, max_fb=16, wmax=120, bias_max=500)])
    c = tt.screen.candidates(ns)
    note("features / labels")
    data = tt.screen.exact_labels(c)
    torch.cuda.synchronize()
    X_ref = mlp_ref.features(ns.F, ns.b, ns.o, ns.act, ns.w, ns.bias, ns.thr)
    assert np.array_equal(from_bf16(data["X"]), mlp_ref.bf16_round(X_ref))
    ref = oracle.enumerate(ns)
    assert np.array_equal(data["support"].cpu().numpy(), ref["support"])
    assert np.array_equal(data["hist"].cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
    y, m, h = mlp_ref.labels(ns.F, ns.b, ns.o, ref["support"], ref["hist"])
    assert np.array_equal(data["y"].cpu().numpy(), y.astype(np.float32))
    assert np.array_equal(data["m"].cpu().numpy(), m.astype(np.float32))
    assert np.array_equal(data["h"].cpu().numpy(), h.astype(np.float32))


def test_network_forward_backward_match_reference():
    """Whole network, one batch: logits and weight gradients against the
    float64 reference with bf16 operands (tolerances from bf16 rounding of
    the hidden activations, 2^-8 relative per layer)."""
    params = mlp_init(11, mlp_ref.DIMS)
    net = tt.screen.ScreenNet(params, max_batch=512)
    B = 384
    rng = np.random.default_rng(12)
    X = rnd((B, 32), 13)
    y = (rng.random((B, 8)) < 0.5).astype(np.float32)
    m = (rng.random((B, 8)) < 0.8).astype(np.float32)
    h = rng.dirichlet(np.ones(4), size=B).astype(np.float32)
    Xt = bf16_bits(X)
    note("network forward/backward")
    net.forward(Xt, B)
    tt.mlp_loss(net.z, B, torch.from_numpy(y).cuda(), torch.from_numpy(m).cuda(), torch.from_numpy(h).cuda(),
                net.dz, net.loss, net.scratch)
    net.backward(Xt, B)
    torch.cuda.synchronize()
    p64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    acts, z = mlp_ref.forward(p64, X, bf16=True)
    L, dz = mlp_ref.loss(z, y, m, h)
    grads = mlp_ref.backward(p64, acts, dz, bf16=True)
    zg = net.z[:B].cpu().numpy()
    assert np.linalg.norm(zg - z) <= 2e-2 * np.linalg.norm(z)
    assert abs(net.loss.item() - L) <= 1e-2 * abs(L)
    for l in range(4):
        gw = net.gW[l].cpu().numpy()
        rw = grads[l][0]
        cos = float((gw * rw).sum() / (np.linalg.norm(gw) * np.linalg.norm(rw) + 1e-30))
        assert cos >= 0.999, (l, cos)
        assert np.linalg.norm(gw - rw) <= 5e-2 * np.linalg.norm(rw), l


@pytest.mark.parametrize("n", [1, 128, 129, 1000])
def test_fused_inference_matches_layers_and_reference(n):
    """tt_mlp_infer (one launch, activations on chip) against four
    tt_mlp_forward calls and the float64 reference with bf16 operands:
    ragged row counts, several blocks."""
    params = mlp_init(31, mlp_ref.DIMS)
    net = tt.screen.ScreenNet(params, max_batch=1024)
    X = rnd((n, 32), 32)
    Xt = bf16_bits(X)
    note(f"fused inference n={n}")
    zi = net.infer(Xt, n).cpu().numpy().copy()
    net.forward(Xt, n)
    torch.cuda.synchronize()
    zl = net.z[:n].cpu().numpy()
    p64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    _, z = mlp_ref.forward(p64, X, bf16=True)
    assert np.isfinite(zi).all()
    assert np.linalg.norm(zi - z) <= 2e-2 * np.linalg.norm(z)
    # same roundings, summation order aside: hidden values may differ by one bf16 step
    assert np.abs(zi - zl).max() <= 2.0 ** -5 * max(1.0, float(np.abs(zl).max()))
    assert np.linalg.norm(zi - zl) <= 1e-2 * np.linalg.norm(zl)


# --------------------------------------------------------------- screening
def check_screen_against_oracle(ns, runner, ref):
    torch.cuda.synchronize()
    assert runner.status.item() == 0
    assert np.array_equal(runner.support.cpu().numpy(), ref["support"])
    assert np.array_equal(runner.hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
    mask = runner.mask.cpu().numpy()
    acc = runner.accept.cpu().numpy()
    F = ns.F.astype(int)
    covers = (ref["support"] & ~mask) == 0
    nothing_skipped = mask == ((1 << F) - 1)
    assert np.array_equal(acc.astype(bool), covers | nothing_skipped)  # exact check == ground truth
    full = torch.empty_like(runner.tables)
    runner.expand(full)
    torch.cuda.synchronize()
    assert np.array_equal(full.cpu().numpy().view(np.uint64), ref["planes"])


@pytest.mark.parametrize("seed", [21, 22])
def test_screen_with_forced_masks(seed):
    """Arbitrary predicted supports (too small, too large, empty, full):
    outputs always equal the oracle; acceptance equals 'covers the true
    support'."""
    ns = concat([cfg4_train(n=2500, seed=seed), random_neurons(seed=seed, n=300, max_fb=16, wmax=60, bias_max=200)])
    ref = oracle.enumerate(ns)
    c = tt.screen.candidates(ns)
    runner = tt.screen.ScreenRunner(c)
    rng = np.random.default_rng(seed)
    F = ns.F.astype(int)
    choices = [ref["support"].astype(int),                                   # exact support
               ref["support"].astype(int) | rng.integers(0, 256, len(ns)),   # supersets
               rng.integers(0, 256, len(ns)),                                 # random
               np.zeros(len(ns), int), (1 << F) - 1]
    for k, mk in enumerate(choices):
        mk = (mk & ((1 << F) - 1)).astype(np.uint8)
        note(f"screen forced mask set {k}")
        runner.screened(force_mask=torch.from_numpy(mk).cuda())
        check_screen_against_oracle(ns, runner, ref)


def test_screen_with_network_logits():
    ns = cfg4_train(n=4000, seed=77)
    ref = oracle.enumerate(ns)
    c = tt.screen.candidates(ns)
    net = tt.screen.ScreenNet(mlp_init(5, mlp_ref.DIMS), max_batch=4096)
    data = tt.screen.exact_labels(c)
    logits = tt.screen.predict(net, data["X"], c.n)
    runner = tt.screen.ScreenRunner(c)
    for tau in (0.5, 0.1):
        note(f"screen with logits tau={tau}")
        runner.screened(logits=logits, tau=tau)
        check_screen_against_oracle(ns, runner, ref)


def test_training_learns_support():
    """A short training run on the device: the loss falls and the support
    prediction beats chance by a wide margin on held-out neurons."""
    train_ns = cfg4_train(n=40000, seed=5)
    test_ns = cfg4_train(n=8000, seed=6)
    ctr, cte = tt.screen.candidates(train_ns), tt.screen.candidates(test_ns)
    dtr, dte = tt.screen.exact_labels(ctr), tt.screen.exact_labels(cte)
    net = tt.screen.ScreenNet(mlp_init(7, mlp_ref.DIMS), max_batch=8192)
    note("train")
    losses = tt.screen.train(net, dtr, epochs=30, batch=1024, lr=2e-3, seed=1)
    print(f"[train] losses {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    logits = tt.screen.predict(net, dte["X"], cte.n)
    acc = tt.screen.support_accuracy(logits, dte["y"], dte["m"], 0.5)
    print(f"[train] held-out {acc}", flush=True)
    assert acc["bit_accuracy"] > 0.95, acc


def test_screen_infer_from_descriptors_matches_feature_path():
    """tt_screen_infer (features computed in the inference kernel) gives the
    logits of tt_screen_features + tt_mlp_infer bit for bit; gated, it writes
    exactly the rows of the wave-pass candidates (host mirror of the gate)."""
    from paper_2502_08673_amd import screen as sc
    ns = concat([cfg4_train(n=1500, seed=61), random_neurons(seed=62, n=300, max_fb=16, wmax=127, bias_max=300)])
    c = sc.candidates(ns)
    net = sc.ScreenNet(mlp_init(63, mlp_ref.DIMS), max_batch=c.n)
    for n in (1, 255, 257, 1000, c.n):
        X = torch.empty((n, 32), dtype=torch.int16, device="cuda")
        sc.screen_features(c.d_desc, n, X)
        want = net.infer(X, n).clone()
        note(f"screen_infer n={n}")
        got = torch.full((n, 12), 7.0, dtype=torch.float32, device="cuda")
        net.infer_desc(c.d_desc, n, False, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), n
        got.fill_(7.0)
        net.infer_desc(c.d_desc, n, True, got)
        torch.cuda.synchronize()
        gate = torch.from_numpy(sc.wave_pass_candidates(c.desc[:n])).cuda()
        assert torch.equal(got[gate], want[gate]), n
        assert bool((got[~gate] == 7.0).all()), n


def test_gated_inference_many_chunks_and_spans():
    """Gated tt_screen_infer on 280 000 candidates, over a third of them
    taken: the compacted list has 547 spans of 512 candidates (two per thread
    in the inference blocks' prefix sums) and more 128-row chunks than one
    block per CU takes at once, so blocks take several; the taken rows equal
    the feature path's logits bit for bit and no other row is written."""
    from paper_2502_08673_amd import screen as sc
    ns = random_neurons(seed=64, n=280000, max_fb=16, wmax=127, bias_max=300)
    c = sc.candidates(ns)
    n = c.n
    net = sc.ScreenNet(mlp_init(65, mlp_ref.DIMS), max_batch=n)
    X = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    sc.screen_features(c.d_desc, n, X)
    want = net.infer(X, n).clone()
    got = torch.full((n, 12), 7.0, dtype=torch.float32, device="cuda")
    note(f"screen_infer gated n={n}")
    net.infer_desc(c.d_desc, n, True, got)
    torch.cuda.synchronize()
    gate = torch.from_numpy(sc.wave_pass_candidates(c.desc)).cuda()
    assert int(gate.sum()) > 128 * 512  # more chunks than any one-block-per-CU grid here
    assert torch.equal(got[gate], want[gate])
    assert bool((got[~gate] == 7.0).all())


def test_trained_screen_gain_over_plain_and_trivial():
    """What the trained network gains: on unseen candidates its support
    prediction on the candidates it screens is at least 99 % right per bit,
    and the learned screen is exact (support, histogram and expanded tables
    equal plain full enumeration) with fewer row-evaluations than both plain
    enumeration and the zero-weight rule.  Times of all paths are printed
    (on this distribution the zero-weight rule is the faster screen)."""
    from paper_2502_08673_amd import screen as sc
    tr = sc.candidates(cfg4_train(n=60000, seed=31))
    dtr = sc.exact_labels(tr)
    net = sc.ScreenNet(mlp_init(33, mlp_ref.DIMS), max_batch=30000)
    note("train for A/B")
    sc.train(net, dtr, epochs=30, batch=2048, lr=2e-3, seed=2)
    c = sc.candidates(cfg4_train(n=30000, seed=32))
    d = sc.exact_labels(c)
    tau = 0.3
    logits = sc.predict(net, d["X"], c.n)
    gi = torch.from_numpy(np.nonzero(sc.wave_pass_candidates(c.desc))[0]).cuda()
    acc = sc.support_accuracy(logits.index_select(0, gi), d["y"].index_select(0, gi), d["m"].index_select(0, gi), tau)
    runner = sc.ScreenRunner(c)
    learned = sc.LearnedScreen(net, runner, tau)
    full = torch.empty_like(runner.tables)
    costs, times = {}, {}
    times["plain"] = sc.timed(runner.plain, 3)
    trivial = sc.nonzero_weight_mask(c)
    for name, fn in (("trivial", lambda: runner.screened(force_mask=trivial)), ("learned", learned)):
        times[name] = sc.timed(fn, 3)
        torch.cuda.synchronize()
        assert torch.equal(runner.support, d["support"]) and torch.equal(runner.hist, d["hist"]), name
        runner.expand(full)
        torch.cuda.synchronize()
        assert torch.equal(full, d["tables"]), name
        assert runner.status.item() == 0
        costs[name] = sc.row_cost(c, runner.mask.cpu().numpy(), runner.accept.cpu().numpy())
    plain_rows = c.ns.total_rows()
    print(f"[screen A/B] accuracy {acc} rows plain {plain_rows} trivial {costs['trivial']} "
          f"learned {costs['learned']} times_ms {times}", flush=True)
    assert acc["bit_accuracy"] >= 0.99, acc
    assert costs["learned"] < costs["trivial"] < plain_rows


def test_device_descriptor_enumerate_and_support():
    """The per-neuron device-descriptor kernels (one workgroup per neuron)
    against the oracle, including skipped neurons and a rejected one."""
    ns = concat([cfg4_train(n=1500, seed=55), random_neurons(seed=56, n=300, max_fb=16, wmax=127, bias_max=400)])
    ref = oracle.enumerate(ns)
    c = tt.screen.candidates(ns)
    tables = torch.zeros(c.total_words, dtype=torch.int64, device="cuda")
    sup = torch.zeros(c.n, dtype=torch.uint8, device="cuda")
    hist = torch.zeros(c.n * 8, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    note("enumerate_device / support_device")
    tt.enumerate_device(c.d_desc, c.n, tables, status=status)
    tt.support_device(c.d_desc, c.n, tables, support_out=sup, hist=hist, status=status)
    torch.cuda.synchronize()
    assert status.item() == 0
    assert np.array_equal(tables.cpu().numpy().view(np.uint64), ref["planes"])
    assert np.array_equal(sup.cpu().numpy(), ref["support"])
    assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
    # active mask: only odd neurons rewritten
    tables2 = torch.zeros_like(tables)
    active = torch.from_numpy((np.arange(c.n) % 2).astype(np.uint8)).cuda()
    tt.enumerate_device(c.d_desc, c.n, tables2, active=active, status=status)
    torch.cuda.synchronize()
    got = tables2.cpu().numpy().view(np.uint64)
    for i in (0, 1, 2, 3, c.n - 1):
        off, W = int(c.desc["word_off"][i]), max(1, (1 << (int(ns.F[i]) * int(ns.b[i]))) // 64)
        span = slice(off, off + int(ns.o[i]) * W)
        want = ref["planes"][span] if i % 2 else np.zeros(int(ns.o[i]) * W, np.uint64)
        assert np.array_equal(got[span], want), i
    # a descriptor beyond the table buffer is skipped and flagged
    bad = c.desc.copy()
    bad["word_off"][3] = c.total_words
    dbad = tt.device_descriptors(bad)
    status.zero_()
    tt.enumerate_device(dbad, c.n, tables2, status=status)
    torch.cuda.synchronize()
    assert status.item() & 1
