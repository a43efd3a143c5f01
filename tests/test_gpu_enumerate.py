"""GPU parity: the HIP enumerator, support, histogram and pack kernels,
called through the C ABI, against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import paper_2502_08673_amd as tt
from gpu_util import check_canary, device_tables, host_u64, note
from workloads import cfg0, cfg1, cfg2, cfg3, concat, random_neurons, subset

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def run_gpu(ns, mode="plain", tune=None, flags=None, want_hist=True):
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda") if want_hist else None
    note(f"enumerate {ns.name} n={len(ns)} rows={ns.total_rows()} mode={mode} tune={tune}")
    if mode == "plain":
        tt.enumerate(desc, tables, total_words=total, hist=hist)
    else:
        fl = flags if flags is not None else (tt.TT_PLAN_PERSISTENT | tt.TT_PLAN_GRAPH)
        with tt.Plan(desc, total, tune=tune, flags=fl) as plan:
            plan.launch(tables, hist)
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    check_canary(tables, total)
    return desc, total, tables, hist


def assert_matches_oracle(ns, desc, tables, total, hist=None):
    ref = oracle.enumerate(ns)
    assert np.array_equal(ref["word_off"], desc["word_off"]), "layout differs"
    got = host_u64(tables, 0, total)
    if not np.array_equal(got, ref["planes"]):
        bad = np.nonzero(got != ref["planes"])[0]
        raise AssertionError(f"{len(bad)} table words differ, first at {bad[:8]}")
    if hist is not None:
        h = hist.cpu().numpy().reshape(-1, 8).astype(np.uint32)
        assert np.array_equal(h, ref["hist"]), "histogram differs"
    return ref


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_cfg0(mode):
    ns = cfg0()
    desc, total, tables, hist = run_gpu(ns, mode)
    assert_matches_oracle(ns, desc, tables, total, hist)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_cfg1(mode):
    ns = cfg1()
    desc, total, tables, hist = run_gpu(ns, mode)
    assert_matches_oracle(ns, desc, tables, total, hist)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_cfg2_uneven_batch(mode):
    ns = cfg2()
    desc, total, tables, hist = run_gpu(ns, mode)
    assert_matches_oracle(ns, desc, tables, total, hist)


@pytest.mark.parametrize("seed", [101, 102])
def test_random_shapes_and_edge_values(seed):
    """All (F, b, o), both activations, full int8 weights (large mask tables),
    ties and thresholds <= 0, rows from 2 to 2^16."""
    ns = concat([random_neurons(seed=seed, n=300, max_fb=16),
                 random_neurons(seed=seed + 1, n=60, F=(1, 2), b=(1, 2), max_fb=4)])
    for mode in ("plain", "batched"):
        desc, total, tables, hist = run_gpu(ns, mode)
        assert_matches_oracle(ns, desc, tables, total, hist)


def test_ragged_chunks_and_tiles():
    """Chunk sizes that do not divide the word count, partial tiles."""
    ns = concat([subset(cfg2(n=700), np.arange(700)), random_neurons(seed=5, n=37, F=(5, 5), b=(4, 4), max_fb=20)])
    for tune in ({"chunk_words": 96, "blocks_per_cu": 1, "waves": 4, "nontemporal": 0, "tile_neurons": 32},
                 {"chunk_words": 224, "blocks_per_cu": 3, "waves": 8, "nontemporal": 1, "tile_neurons": 8},
                 {"chunk_words": 64, "blocks_per_cu": 2, "waves": 4, "nontemporal": 0, "tile_neurons": 16}):
        desc, total, tables, hist = run_gpu(ns, "batched", tune=tune)
        assert_matches_oracle(ns, desc, tables, total, hist)


def test_histogram_counts_at_largest_items():
    """Fused histogram where the per-lane counts are largest: every row of the
    ReLU neurons with thresholds <= 0 reaches every threshold.  Wide tables
    (F=8, b=3: one wave per 256 words) and the tile kernel's largest items
    (F*b = 16: a whole 1024-word table per item, 4 waves), mixed with
    ordinary neurons of the same shapes."""
    wide = random_neurons(seed=77, n=6, F=(8, 8), b=(3, 3), o=(3, 3), max_fb=24, wmax=15, bias_max=8, acts=(1,))
    tile = random_neurons(seed=78, n=6, F=(4, 4), b=(4, 4), o=(3, 3), max_fb=16, wmax=15, bias_max=8, acts=(1,))
    ns = concat([wide, tile])
    for i in (0, 1, 2, 6, 7, 8):
        ns.thr[i, :7] = np.array([-60, -50, -40, -30, -20, -10, 0], dtype=ns.thr.dtype)
    for tune in ({"chunk_words": 65536, "blocks_per_cu": 1, "waves": 4, "nontemporal": 1, "tile_neurons": 8},
                 {"chunk_words": 65536, "blocks_per_cu": 1, "waves": 4, "nontemporal": 0, "tile_neurons": 32}):
        desc, total, tables, hist = run_gpu(ns, "batched", tune=tune)
        assert_matches_oracle(ns, desc, tables, total, hist)
        h = hist.cpu().numpy().reshape(-1, 8).astype(np.uint64)
        assert (h[:3, 7] == 1 << 24).all() and (h[6:9, 7] == 1 << 16).all()


def test_wide_and_tile_groups_mixed():
    """Wide groups (2^12 or more words per plane) beside tile groups in one
    plan.  The first wide tables sit at even word offsets (16-byte stores);
    a one-word table then puts the next ones at odd offsets (8-byte stores);
    every o; persistent and static plans and the one-shot call; tables,
    histogram and support against the oracle."""
    wide_a = [random_neurons(seed=402 + k, n=1, F=(6, 6), b=(3, 3), o=(k, k), max_fb=18, wmax=15, bias_max=40)
              for k in (1, 2, 3)]
    one = random_neurons(seed=401, n=1, F=(2, 2), b=(1, 1), o=(1, 1), max_fb=2)
    wide_b = [random_neurons(seed=410 + k, n=1, F=(5, 5), b=(4, 4), o=(k, k), max_fb=20, wmax=9, bias_max=40)
              for k in (3, 1, 2)]
    tile = random_neurons(seed=403, n=20, F=(3, 8), b=(1, 4), max_fb=16)
    ns = concat(wide_a + [one] + wide_b + [tile])
    ref = oracle.enumerate(ns)
    wide = (ns.F.astype(int) * ns.b.astype(int)) >= 18
    assert {int(x) % 2 for x in ref["word_off"][wide]} == {0, 1}
    for mode, flags in (("plain", None), ("batched", tt.TT_PLAN_PERSISTENT | tt.TT_PLAN_GRAPH), ("batched", 0)):
        desc, total, tables, hist = run_gpu(ns, mode, flags=flags)
        assert_matches_oracle(ns, desc, tables, total, hist)
        sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
        tt.support(desc, tables, support_out=sup)
        torch.cuda.synchronize()
        assert np.array_equal(sup.cpu().numpy(), ref["support"]), mode
    with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT) as plan:
        assert plan.info()["wide_neurons"] == int(wide.sum())


def test_large_rows_sampled():
    """cfg3 shape (F=8, b=3, 2^24 rows, 2 GiB of tables) in the launch
    configuration the benchmark times; sampled neurons compared with the
    oracle, full histogram of every sampled neuron."""
    import os
    ns = cfg3()
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    cache = os.path.join(os.path.dirname(tt.__file__), "tune_cache.txt")
    tune = tt.autotune(desc, tables, cache_path=cache)  # the benchmark's launch shape
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda")
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    note(f"cfg3 full size, tune {tune}")
    sup_scan = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    with tt.Plan(desc, total, tune=tune, flags=tt.TT_PLAN_PERSISTENT) as plan:
        plan.launch(tables, hist)
        plan.support_enumerated(tables, support_out=sup)  # the benchmark step
        plan.support(tables, support_out=sup_scan)        # every digit from the tables
        torch.cuda.synchronize()
    check_canary(tables, total)
    assert torch.equal(sup, sup_scan)
    pick = [0, 1, 137, 255, 256, 400, 510, 511]
    sub = subset(ns, pick)
    ref = oracle.enumerate(sub)
    W = 1 << 18
    h = hist.cpu().numpy().reshape(-1, 8).astype(np.uint32)
    sp = sup.cpu().numpy()
    for k, i in enumerate(pick):
        off = int(desc["word_off"][i])
        got = host_u64(tables, off, off + 2 * W)
        want = ref["planes"][int(ref["word_off"][k]): int(ref["word_off"][k]) + 2 * W]
        assert np.array_equal(got, want), f"neuron {i} differs"
        assert np.array_equal(h[i], ref["hist"][k])
        assert sp[i] == ref["support"][k], f"neuron {i} support"
    assert (h.sum(1) == (1 << 24)).all()
    # every input with zero weight is outside the support (at any size)
    zero_w = (ns.w[:, :8] == 0).astype(np.uint8)
    zero_bits = (zero_w << np.arange(8, dtype=np.uint8)).sum(1).astype(np.uint8)
    assert not np.any(sp & zero_bits)


def test_largest_neurons():
    """The largest tables the ABI allows with F <= 8, b <= 4: F = 7, b = 4
    (2^28 rows, 2^22 words per plane), 1- and 3-bit outputs, through a plan
    (with histogram and support) and through the one-shot call; every word
    compared with the oracle."""
    ns = random_neurons(seed=301, n=2, F=(7, 7), b=(4, 4), o=(1, 3), max_fb=28, wmax=9, bias_max=40,
                        acts=(1,), zero_frac=0.2)
    ns.o[:] = [1, 3]
    ns.w[0, :7] = [3, -2, 5, 0, 4, 1, 0]  # input 6 (the top digit) never matters
    ns.bias[0] = -10
    ns.thr[0, 0] = 40
    ref = oracle.enumerate(ns)
    for mode in ("batched", "plain"):
        desc, total, tables, hist = run_gpu(ns, mode, flags=tt.TT_PLAN_PERSISTENT)
        assert np.array_equal(ref["word_off"], desc["word_off"])
        assert np.array_equal(host_u64(tables, 0, total), ref["planes"]), mode
        assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"]), mode
        sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
        tt.support(desc, tables, support_out=sup)
        torch.cuda.synchronize()
        assert np.array_equal(sup.cpu().numpy(), ref["support"]), mode
    assert ref["support"][0] == 0b0110111 and ref["hist"][0, 1] > 0


def test_empty_and_single():
    desc = tt.descriptors(cfg0())[:0]
    tables = torch.zeros(4, dtype=torch.int64, device="cuda")
    tt.enumerate(desc, tables, total_words=0)
    ns = random_neurons(seed=9, n=1, F=(1, 1), b=(1, 1), max_fb=1)
    desc, total, tables, hist = run_gpu(ns, "plain")
    assert_matches_oracle(ns, desc, tables, total, hist)


def test_repeat_is_deterministic():
    ns = cfg2(n=2000)
    desc, total, t1, _ = run_gpu(ns, "batched")
    _, _, t2, _ = run_gpu(ns, "plain")
    assert torch.equal(t1[:total], t2[:total])


def test_graph_replays_match_eager():
    ns = cfg2(n=1500)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    ref = oracle.enumerate(ns)
    tables = device_tables(total)
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda")
    note("graph replays")
    with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT | tt.TT_PLAN_GRAPH) as plan:
        for rep in range(4):
            tables[:total].fill_(int(np.int64(rep * 7919 - 3)))
            hist.fill_(rep + 1)
            torch.cuda.synchronize()
            plan.launch(tables, hist)
            torch.cuda.synchronize()
            assert np.array_equal(host_u64(tables, 0, total), ref["planes"]), rep
            assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"]), rep
            _ = (torch.arange(1000, device="cuda") * 3).sum().item()  # eager work between replays
    check_canary(tables, total)


@pytest.mark.parametrize("flags", ["eager", "graph", "static"])
def test_plan_step_whole_step(flags):
    """tt_plan_step (enumeration + histogram + support of the plan's own
    tables), eager and replayed from one captured graph, persistent and
    static (one launch per group), against the oracle on every replay, with
    eager work and poisoned outputs between replays and a recapture when the
    output pointers change."""
    ns = concat([cfg2(n=1500), random_neurons(seed=641, n=3, F=(6, 6), b=(3, 3), max_fb=18)])
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    ref = oracle.enumerate(ns)
    fl = 0 if flags == "static" else tt.TT_PLAN_PERSISTENT | (tt.TT_PLAN_GRAPH if flags == "graph" else 0)
    bufs = [(device_tables(total), torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda"),
             torch.zeros(len(ns), dtype=torch.uint8, device="cuda")) for _ in range(2)]
    note(f"plan step {flags}")
    with tt.Plan(desc, total, flags=fl) as plan:
        for rep in range(5):
            tables, hist, sup = bufs[rep // 3]  # third replay on: new pointers
            tables[:total].fill_(int(np.int64(rep * 7919 - 3)))
            hist.fill_(rep + 1)
            sup.fill_(0xEE)
            torch.cuda.synchronize()
            plan.step(tables, hist, sup)
            torch.cuda.synchronize()
            assert np.array_equal(host_u64(tables, 0, total), ref["planes"]), rep
            assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"]), rep
            assert np.array_equal(sup.cpu().numpy(), ref["support"]), rep
            _ = (torch.arange(1000, device="cuda") * 3).sum().item()  # eager work between replays
    for tables, _, _ in bufs:
        check_canary(tables, total)


# ---------------------------------------------------------------- support
def upload_oracle_tables(ns):
    ref = oracle.enumerate(ns)
    t = device_tables(ref["total_words"])
    t[: ref["total_words"]] = torch.from_numpy(ref["planes"].view(np.int64)).cuda()
    return ref, t


@pytest.mark.parametrize("which", ["cfg0", "cfg2", "random"])
def test_support_and_hist_from_oracle_tables(which):
    ns = {"cfg0": cfg0, "cfg2": lambda: cfg2(n=3000),
          "random": lambda: random_neurons(seed=77, n=400, max_fb=16)}[which]()
    ref, t = upload_oracle_tables(ns)
    desc = tt.descriptors(ns)
    tt.layout(desc)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda")
    note(f"support {which} n={len(ns)}")
    tt.support(desc, t, support_out=sup, hist=hist)
    torch.cuda.synchronize()
    assert np.array_equal(sup.cpu().numpy(), ref["support"])
    assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
    sup.fill_(0xEE)
    tt.support(desc, t, support_out=sup)  # support only: checks planned on the device
    torch.cuda.synchronize()
    assert np.array_equal(sup.cpu().numpy(), ref["support"])


def test_support_far_word_bits():
    """Neurons with more words than one support chunk (2^11), so row bits
    beyond the chunk are checked across chunks; includes inputs that matter
    only through their top bit and inputs with zero weight."""
    ns = random_neurons(seed=91, n=12, F=(6, 8), b=(3, 3), max_fb=21, zero_frac=0.25)
    big = subset(cfg3(), [3, 4])
    b4 = random_neurons(seed=92, n=6, F=(5, 6), b=(4, 4), o=(1, 3), max_fb=22, zero_frac=0.3)  # 4-bit far digits
    ns = concat([ns, big, b4])
    ns.w[0, :] = 0
    ns.w[0, ns.F[0] - 1] = 1  # only the most significant input matters
    ns.bias[0] = 0
    ns.thr[0, :] = 0
    ns.thr[0, : (1 << int(ns.o[0])) - 1] = 7
    ref, t = upload_oracle_tables(ns)
    desc = tt.descriptors(ns)
    tt.layout(desc)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    note(f"support far bits n={len(ns)}")
    tt.support(desc, t, support_out=sup)
    torch.cuda.synchronize()
    assert np.array_equal(sup.cpu().numpy(), ref["support"])


def test_pack_matches_oracle_planes():
    ns = concat([cfg2(n=500), random_neurons(seed=12, n=100, max_fb=14)])
    codes = oracle.codes(ns)
    ref = oracle.from_codes(ns, codes)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    dc = torch.from_numpy(codes).cuda()
    note(f"pack n={len(ns)}")
    tt.pack(desc, dc, tables)
    torch.cuda.synchronize()
    check_canary(tables, total)
    assert np.array_equal(host_u64(tables, 0, total), ref["planes"])
    # arbitrary codes (not from a neuron): high bits beyond o are ignored
    rng = np.random.default_rng(4)
    junk = rng.integers(0, 256, size=codes.shape, dtype=np.uint8)
    ref2 = oracle.from_codes(ns, junk)
    tt.pack(desc, torch.from_numpy(junk).cuda(), tables)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda")
    tt.support(desc, tables, support_out=sup, hist=hist)
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(tables, 0, total), ref2["planes"])
    assert np.array_equal(sup.cpu().numpy(), ref2["support"])
    assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref2["hist"])


def test_autotune_returns_valid_config(tmp_path):
    ns = cfg2(n=800)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    cache = str(tmp_path / "tune.txt")
    note("autotune")
    best = tt.autotune(desc, tables, cache_path=cache)
    assert best["waves"] in (4, 8) and best["chunk_words"] % 32 == 0
    again = tt.autotune(desc, tables, cache_path=cache)  # served from the cache
    assert again == best
    d2, total2, t2, h2 = run_gpu(ns, "batched", tune=best)
    assert_matches_oracle(ns, d2, t2, total2, h2)


def test_plan_support_and_hist_match_oracle():
    """Support through a plan's prepared work lists, after the plan's own
    enumeration, on mixed shapes including neurons with far word bits."""
    ns = concat([cfg2(n=600), random_neurons(seed=93, n=10, F=(7, 8), b=(3, 3), max_fb=24, zero_frac=0.3),
                 subset(cfg3(), [7])])
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    hist = torch.zeros(len(ns) * 8, dtype=torch.int32, device="cuda")
    ref = oracle.enumerate(ns)
    note(f"plan support n={len(ns)}")
    with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT) as plan:
        for rep in range(2):
            sup.fill_(0xEE)
            hist.fill_(-1)
            plan.launch(tables)
            plan.support(tables, support_out=sup, hist=hist)
            torch.cuda.synchronize()
            assert np.array_equal(sup.cpu().numpy(), ref["support"]), rep
            assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"]), rep
        plan.support(tables, hist=hist)  # histogram only
        torch.cuda.synchronize()
        assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
        for rep in range(2):
            sup.fill_(0xEE)
            plan.support(tables, support_out=sup)  # support only
            torch.cuda.synchronize()
            assert np.array_equal(sup.cpu().numpy(), ref["support"]), rep
        for rep in range(2):  # zero-weight inputs settled without reading the tables
            sup.fill_(0xEE)
            hist.fill_(-1)
            plan.support_enumerated(tables, support_out=sup, hist=hist if rep else None)
            torch.cuda.synchronize()
            assert np.array_equal(sup.cpu().numpy(), ref["support"]), rep
            if rep:
                assert np.array_equal(hist.cpu().numpy().reshape(-1, 8).astype(np.uint32), ref["hist"])
    check_canary(tables, total)


def test_plan_support_enumerated_saturated_and_zero_weights():
    """Support of a plan's own tables when inputs of nonzero weight still
    never matter (saturation: every row reaches the top threshold, or the
    sum stays below the first) beside zero-weight inputs, in tile and wide
    groups, against the oracle."""
    ns = concat([random_neurons(seed=611, n=24, F=(4, 8), b=(2, 3), max_fb=16, zero_frac=0.4),
                 random_neurons(seed=612, n=6, F=(7, 8), b=(3, 3), max_fb=24, wmax=15, bias_max=40,
                                zero_frac=0.4)])
    for i in range(0, len(ns), 3):  # saturated: q constant although weights are nonzero
        ns.act[i] = 0
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = -100000 if i % 2 == 0 else 100000
    for i in range(1, len(ns), 5):  # one input matters only at the extreme rows
        f = int(ns.F[i])
        ns.w[i, :f] = 1
        ns.act[i] = 0
        ns.bias[i] = 0
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = f * ((1 << int(ns.b[i])) - 1)
    ref = oracle.enumerate(ns)
    assert (ref["support"] == 0).any() and (ref["support"] != 0).any()
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    note(f"plan support_enumerated saturated n={len(ns)}")
    with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT) as plan:
        plan.launch(tables)
        sup.fill_(0xEE)
        plan.support_enumerated(tables, support_out=sup)
        torch.cuda.synchronize()
    check_canary(tables, total)
    assert np.array_equal(sup.cpu().numpy(), ref["support"])


def test_support_from_parameters_matches_oracle():
    """Support of a plan's own tables decided from the parameters (subset-sum
    bitset, no table read) against the oracle's table-based support: random
    shapes, weights, biases, thresholds (ties, <= 0, identity and ReLU),
    saturated neurons, weight ranges that fill 1 to 4 bitset registers (sums
    up to 7 * 128 * 15), and both sides of the 64- and 512-value limits of
    the one-wave forms."""
    sets = [random_neurons(seed=620 + s, n=500, max_fb=14, wmax=127, bias_max=300) for s in range(3)]
    sets.append(random_neurons(seed=630, n=400, max_fb=12, wmax=7, bias_max=20, zero_frac=0.3))
    big = random_neurons(seed=631, n=6, F=(4, 6), b=(4, 4), o=(1, 3), max_fb=24, wmax=127, bias_max=3000)
    big.w[:, :6] = np.where(np.arange(6)[None, :] % 2 == 0, -128, 127)[:, :6].astype(np.int8)
    for i in range(len(big)):
        f = int(big.F[i])
        big.w[i, f:] = 0
        k = (1 << int(big.o[i])) - 1
        big.thr[i, :k] = np.sort(np.random.default_rng(632 + i).integers(-4000, 4000, size=k))
    top = random_neurons(seed=633, n=1, F=(7, 7), b=(4, 4), o=(2, 2), max_fb=28, wmax=127, bias_max=100)
    top.w[0, :7] = [-128, 127, -128, 127, 100, -90, 3]
    top.thr[0, :3] = [-500, 7, 900]
    # sums spanning 511 and 512 values: the two sides of the one-wave path's limit
    edge = random_neurons(seed=634, n=8, F=(5, 5), b=(1, 1), o=(2, 3), max_fb=8, wmax=127, bias_max=50)
    for i in range(len(edge)):
        edge.w[i, :5] = [127, -127, 127, -127, 3 + (i % 2)]
        edge.act[i] = i % 2
        k = (1 << int(edge.o[i])) - 1
        edge.thr[i, :k] = np.sort(np.random.default_rng(635 + i).integers(-300, 300, size=k))
    # sums spanning 63 and 64 values: the two sides of the one-register path's limit
    edge64 = random_neurons(seed=636, n=8, F=(3, 3), b=(1, 1), o=(2, 3), max_fb=3, wmax=63, bias_max=20)
    for i in range(len(edge64)):
        edge64.w[i, :3] = [31 + (i % 2), -31, 1] if i < 4 else [-1, 31, -(31 + (i % 2))]
        edge64.act[i] = (i // 2) % 2
        k = (1 << int(edge64.o[i])) - 1
        edge64.thr[i, :k] = np.sort(np.random.default_rng(637 + i).integers(-70, 70, size=k))
    ns = concat(sets + [cfg2(n=400), big, top, edge, edge64])
    for i in range(0, 400, 7):  # saturated: q constant although weights are nonzero
        ns.act[i] = 0
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = -1000000 if i % 2 else 1000000
    ref = oracle.enumerate(ns, hist=False, support=True)
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    sup = torch.zeros(len(ns), dtype=torch.uint8, device="cuda")
    note(f"support from parameters n={len(ns)} total_words={total}")
    with tt.Plan(desc, total, flags=tt.TT_PLAN_PERSISTENT) as plan:
        plan.launch(tables)
        for rep in range(2):
            sup.fill_(0xEE)
            plan.support_enumerated(tables, support_out=sup)
            torch.cuda.synchronize()
            got = sup.cpu().numpy()
            bad = np.nonzero(got != ref["support"])[0]
            assert len(bad) == 0, (rep, bad[:8], got[bad[:8]], ref["support"][bad[:8]])
    check_canary(tables, total)
    assert np.array_equal(host_u64(tables, 0, total), ref["planes"])


def test_weight_minus_128_largest_mask_tables():
    """Weights of -128 (the int8 minimum) on the digits that span the low six
    row bits at b = 4: the mask table then holds 15*128 + 3*128 + 2 entries,
    the largest any neuron has.  Tile groups (F*b <= 16), a wide group
    (F = 5, b = 4: 2^14 words per plane) and the device-descriptor kernel,
    against the oracle."""
    tile = random_neurons(seed=501, n=4, F=(3, 4), b=(4, 4), o=(1, 3), max_fb=16, wmax=127, bias_max=300)
    wide = random_neurons(seed=502, n=2, F=(5, 5), b=(4, 4), o=(2, 3), max_fb=20, wmax=127, bias_max=300)
    ns = concat([tile, wide])
    for i in range(len(ns)):
        ns.w[i, 0] = -128
        ns.w[i, 1] = -128 if i % 2 == 0 else 127
        ns.bias[i] = 2000
        ns.act[i] = i % 2
        k = (1 << int(ns.o[i])) - 1
        ns.thr[i, :k] = np.linspace(-1500, 2500, k).astype(np.int32)
    ref = oracle.enumerate(ns)
    assert (np.count_nonzero(ref["hist"], axis=1) > 1).all()
    for mode, flags in (("plain", None), ("batched", tt.TT_PLAN_PERSISTENT)):
        desc, total, tables, hist = run_gpu(ns, mode, flags=flags)
        assert_matches_oracle(ns, desc, tables, total, hist)
    small = subset(ns, range(len(tile)))
    sref = oracle.enumerate(small)
    desc = tt.descriptors(small)
    total = tt.layout(desc)
    d_desc = tt.device_descriptors(desc)
    tables = device_tables(total)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    note(f"enumerate_device w=-128 n={len(small)}")
    tt.enumerate_device(d_desc, len(small), tables, total_words=total, status=status)
    torch.cuda.synchronize()
    check_canary(tables, total)
    assert int(status.item()) == 0
    assert np.array_equal(host_u64(tables, 0, total), sref["planes"])
