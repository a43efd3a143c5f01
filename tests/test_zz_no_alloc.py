"""tt_enumerate_noalloc (the enumeration for callers that cannot allocate
device memory) against tt_enumerate on the same descriptors, bit for bit,
on consecutive calls that share the library's fixed scratch: a large mixed
batch, then a smaller one (stale contents of the first call must not leak
into the second), then inputs at and beyond the scratch limit."""
import numpy as np
import pytest

import oracle
import paper_2502_08673_amd as tt
from gpu_util import check_canary, device_tables, host_u64, note
from workloads import cfg0, cfg2, concat, random_neurons

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _both(ns, want_hist=True):
    """Tables and histograms of tt_enumerate and tt_enumerate_noalloc."""
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    out = []
    for name, fn in (("tt_enumerate", tt.enumerate), ("tt_enumerate_noalloc", tt.enumerate_noalloc)):
        tables = device_tables(total)
        hist = None
        if want_hist:
            hist = torch.full((len(ns) * 8,), -1, dtype=torch.int32, device="cuda")
        note(f"{name} {ns.name} n={len(ns)} rows={ns.total_rows()} hist={want_hist}")
        fn(desc, tables, total_words=total, hist=hist)
        torch.cuda.synchronize()
        check_canary(tables, total)
        out.append((host_u64(tables, 0, total), None if hist is None else hist.cpu().numpy()))
    (t0, h0), (t1, h1) = out
    if not np.array_equal(t0, t1):
        bad = np.nonzero(t0 != t1)[0]
        raise AssertionError(f"{len(bad)} table words differ, first at {bad[:8]}")
    if want_hist:
        assert np.array_equal(h0, h1), "histograms differ"
    return t1, h1


def _big_mixed():
    wide = random_neurons(20250212 + 701, 4, F=(6, 6), b=(3, 3), max_fb=18)  # 2^18 rows: wide kernel
    wide.w[0, :2] = -128
    small = random_neurons(20250212 + 702, 300, max_fb=12)
    small.w[:3, :2] = -128
    return concat([cfg2(), wide, small])


def test_noalloc_matches_enumerate_on_consecutive_calls():
    _both(_big_mixed())
    ns = cfg0()
    tables, hist = _both(ns)  # smaller input into the same scratch
    ref = oracle.enumerate(ns)
    assert np.array_equal(tables, ref["planes"])
    assert np.array_equal(hist.reshape(-1, 8).astype(np.uint32), ref["hist"])
    _both(random_neurons(20250212 + 703, 17, max_fb=10), want_hist=False)


def _lut_heavy(n):
    """F=2, b=4 neurons with both weights -128: the largest mask table a
    neuron can have (2306 entries), so n of them need about 18 KiB each."""
    ns = random_neurons(20250212 + 704, n, F=(2, 2), b=(4, 4), o=(2, 2), max_fb=8)
    ns.w[:, :2] = -128
    ns.act[:] = 0
    ns.bias[:] = 0
    ns.thr[:, :3] = np.array([-3000, -1500, -200])
    return ns


def test_noalloc_limit():
    _both(_lut_heavy(1000))  # about 18 MiB of mask tables: fits
    ns = _lut_heavy(2000)    # about 37 MiB: beyond the scratch
    desc = tt.descriptors(ns)
    total = tt.layout(desc)
    tables = device_tables(total)
    note(f"tt_enumerate_noalloc beyond the scratch limit n={len(ns)}")
    with pytest.raises(tt.TTError) as ei:
        tt.enumerate_noalloc(desc, tables, total_words=total)
    assert ei.value.status == tt.TT_ESCRATCH
    torch.cuda.synchronize()
    check_canary(tables, total)
    from gpu_util import POISON
    assert (tables[:total].cpu().numpy() == POISON).all(), "a rejected call wrote tables"
