"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and validates descriptors without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2502_08673_amd as tt
from workloads import cfg0, cfg2, random_neurons

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tt_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = tt.lib()
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_descriptor_layout_matches_header():
    assert tt.NEURON_DTYPE.itemsize == 64
    off = {k: tt.NEURON_DTYPE.fields[k][1] for k in tt.NEURON_DTYPE.names}
    assert off == {"w": 0, "thr": 8, "bias": 36, "F": 38, "b": 39, "o": 40, "act": 41, "pad": 42,
                   "word_off": 48, "reserved": 56}


def test_strerror_and_version():
    L = tt.lib()
    assert L.tt_strerror(0) == b"success"
    assert L.tt_strerror(-1) == b"invalid argument"
    assert L.tt_strerror(-5) == b"device is not gfx950"
    assert L.tt_strerror(-99) == b"unknown status"
    assert tt.version() >> 16 == 1


def test_words_per_plane():
    assert tt.words_per_plane(6, 2) == 64
    assert tt.words_per_plane(2, 2) == 1
    assert tt.words_per_plane(8, 3) == 1 << 18
    assert tt.words_per_plane(8, 4) == 0  # F*b = 32 > 30
    assert tt.words_per_plane(0, 2) == 0
    assert tt.words_per_plane(9, 1) == 0


def test_layout_is_prefix_sum_of_planes():
    ns = random_neurons(seed=3, n=100, max_fb=20)
    d = tt.descriptors(ns)
    total = tt.layout(d)
    acc = 0
    for i in range(len(d)):
        assert int(d["word_off"][i]) == acc
        acc += int(d["o"][i]) * max(1, (1 << (int(d["F"][i]) * int(d["b"][i]))) // 64)
    assert total == acc


@pytest.mark.parametrize("field,value,status", [
    ("F", 0, tt.TT_EINVAL), ("F", 9, tt.TT_EINVAL), ("b", 0, tt.TT_EINVAL), ("b", 5, tt.TT_EINVAL),
    ("o", 0, tt.TT_EINVAL), ("o", 4, tt.TT_EINVAL), ("act", 2, tt.TT_EINVAL),
])
def test_validate_rejects_bad_fields(field, value, status):
    d = tt.descriptors(cfg0())
    d[field][5] = value
    with pytest.raises(tt.TTError) as e:
        tt.validate(d)
    assert e.value.status == status


def test_validate_rejects_too_many_rows():
    d = tt.descriptors(cfg0())
    d["F"][0], d["b"][0] = 8, 4  # 32 bits
    with pytest.raises(tt.TTError) as e:
        tt.validate(d)
    assert e.value.status == tt.TT_ERANGE


def test_validate_rejects_decreasing_thresholds_but_ignores_unused():
    d = tt.descriptors(cfg0())
    d["thr"][3, :3] = [4, 8, 6]
    with pytest.raises(tt.TTError):
        tt.validate(d)
    d = tt.descriptors(cfg0())
    d["thr"][3, 3:] = [-5, 100, -7, 3]  # slots beyond 2^o - 1 are ignored
    d["thr"][4, :3] = [4, 4, 4]        # ties are allowed
    tt.validate(d)


def test_null_and_negative_arguments():
    L = tt.lib()
    assert L.tt_validate(None, 3) == tt.TT_EINVAL
    assert L.tt_validate(None, 0) == tt.TT_OK
    assert L.tt_validate(None, -1) == tt.TT_EINVAL
    assert L.tt_layout(None, 0, None) == tt.TT_EINVAL
    d = tt.descriptors(cfg0())
    # Entry points reject bad arguments before any device work.
    assert L.tt_enumerate(d.ctypes.data, -1, None, 0, None, None) == tt.TT_EINVAL
    assert L.tt_enumerate(d.ctypes.data, len(d), None, 10, None, None) == tt.TT_EINVAL
    assert L.tt_enumerate_noalloc(d.ctypes.data, -1, None, 0, None, None) == tt.TT_EINVAL
    assert L.tt_enumerate_noalloc(d.ctypes.data, len(d), None, 10, None, None) == tt.TT_EINVAL
    assert L.tt_enumerate_noalloc(d.ctypes.data, 0, None, 0, None, None) == tt.TT_OK
    assert L.tt_support(d.ctypes.data, len(d), None, 10, None, None, None) == tt.TT_EINVAL
    assert L.tt_pack(d.ctypes.data, len(d), None, 10, None, 10, None) == tt.TT_EINVAL
    assert L.tt_plan_create(d.ctypes.data, len(d), 0, None, 0, None) == tt.TT_EINVAL
    assert L.tt_plan_launch(None, None, None, None) == tt.TT_EINVAL
    assert L.tt_plan_destroy(None) == tt.TT_OK
    assert L.tt_autotune(d.ctypes.data, len(d), None, 0, None, None) == tt.TT_EINVAL
    # n = 0 is a no-op that needs no device
    assert L.tt_enumerate(d.ctypes.data, 0, None, 0, None, None) == tt.TT_OK


def test_table_ranges_are_checked_before_device_work():
    L = tt.lib()
    d = tt.descriptors(cfg2(n=64))
    total = tt.layout(d)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.tt_enumerate(d.ctypes.data, len(d), fake, total - 1, None, None) == tt.TT_ERANGE
    d2 = d.copy()
    d2["word_off"][7] = d2["word_off"][6]  # overlapping tables
    assert L.tt_enumerate(d2.ctypes.data, len(d2), fake, total, None, None) == tt.TT_EINVAL
    assert L.tt_support(d.ctypes.data, len(d), fake, total - 1, fake, None, None) == tt.TT_ERANGE
    assert L.tt_enumerate_noalloc(d.ctypes.data, len(d), fake, total - 1, None, None) == tt.TT_ERANGE
    assert L.tt_enumerate_noalloc(d2.ctypes.data, len(d2), fake, total, None, None) == tt.TT_EINVAL
    codes_needed = sum(1 << (int(f) * int(b)) for f, b in zip(d["F"], d["b"]))
    assert L.tt_pack(d.ctypes.data, len(d), fake, codes_needed - 1, fake, total, None) == tt.TT_ERANGE


def test_noalloc_rejects_inputs_beyond_its_scratch_before_device_work():
    L = tt.lib()
    ns = random_neurons(20250212 + 704, 2000, F=(2, 2), b=(4, 4), o=(2, 2), max_fb=8)
    ns.w[:, :2] = -128  # largest mask table: 2306 entries of 8 bytes per neuron
    d = tt.descriptors(ns)
    total = tt.layout(d)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the size check fails first
    assert L.tt_enumerate_noalloc(d.ctypes.data, len(d), fake, total, None, None) == tt.TT_ESCRATCH
    assert tt.TT_ESCRATCH == -6 and "scratch" in L.tt_strerror(tt.TT_ESCRATCH).decode()


def test_mlp_backward_checks_its_scratch_size():
    L = tt.lib()
    a = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    need = tt.mlp_scratch_floats(4096, 256)
    assert need >= 32 * (256 * 256 + 256)
    assert L.tt_mlp_backward(a, 4096, 256, a, 256, a, 1, None, a, a, a, need - 1, None) == tt.TT_ERANGE
    assert L.tt_mlp_backward(a, 4096, 256, a, 256, None, 0, None, a, None, a, need, None) == tt.TT_EINVAL  # no x
    assert L.tt_mlp_backward(a, 0, 256, a, 256, a, 1, a, None, None, None, 0, None) == tt.TT_EINVAL


def test_screen_inference_and_plan_queries_check_arguments():
    L = tt.lib()
    a = ctypes.c_void_p(0x1000)      # aligned, never dereferenced: validation fails first
    odd = ctypes.c_void_p(0x1008)    # not 16-byte aligned
    ws = [a, None, a, None, a, None, a, None]
    assert L.tt_mlp_infer(a, 0, *ws, a, None) == tt.TT_OK           # nothing to do, no device
    assert L.tt_mlp_infer(a, -1, *ws, a, None) == tt.TT_EINVAL
    assert L.tt_mlp_infer(None, 5, *ws, a, None) == tt.TT_EINVAL    # no features
    assert L.tt_mlp_infer(a, 5, *ws, None, None) == tt.TT_EINVAL    # no logits
    assert L.tt_mlp_infer(odd, 5, *ws, a, None) == tt.TT_EINVAL     # misaligned features
    assert L.tt_screen_infer(a, 0, 1, *ws, a, None, None) == tt.TT_OK       # nothing to do, no device
    assert L.tt_screen_infer(a, -1, 0, *ws, a, None, None) == tt.TT_EINVAL
    assert L.tt_screen_infer(a, 5, 2, *ws, a, None, None) == tt.TT_EINVAL   # gated is 0 or 1
    assert L.tt_screen_infer(None, 5, 1, *ws, a, None, None) == tt.TT_EINVAL  # no descriptors
    assert L.tt_screen_infer(odd, 5, 1, *ws, a, None, None) == tt.TT_EINVAL   # misaligned descriptors
    assert L.tt_screen_infer(a, 5, 1, *ws, None, None, None) == tt.TT_EINVAL  # no logits
    assert L.tt_screen_infer(a, 5, 0, odd, *ws[1:], a, None, None) == tt.TT_EINVAL  # misaligned weights
    assert L.tt_screen_infer(a, 5, 1, *ws, a, ctypes.c_void_p(0x1002), None) == tt.TT_EINVAL  # misaligned list
    assert L.tt_screen_infer_work_bytes(0) == 0 and L.tt_screen_infer_work_bytes(1 << 22) == 0
    assert L.tt_screen_infer_work_bytes(1000) == 4 * (2 * 512 + 2)
    bad_w = [a, None, None, None, a, None, a, None]                 # W2 missing
    assert L.tt_mlp_infer(a, 5, *bad_w, a, None) == tt.TT_EINVAL
    bad_b = [a, odd, a, None, a, None, a, None]                     # misaligned bias
    assert L.tt_mlp_infer(a, 5, *bad_b, a, None) == tt.TT_EINVAL
    n = ctypes.c_int(-1)
    assert L.tt_plan_wide_neurons(None, ctypes.byref(n)) == tt.TT_EINVAL


def test_lutnet_checks_fanin_before_device_work():
    L = tt.lib()
    d = tt.descriptors(cfg0())
    total = tt.layout(d)
    fake = ctypes.c_void_p(0x1000)
    fan = np.full((len(d), 8), -1, np.int32)
    fan[:, :6] = np.arange(6)  # every neuron reads primary inputs 0..5
    ok_args = (d.ctypes.data, len(d), fan.ctypes.data, 6, fake, total, fake, 0, fake, None)
    assert L.tt_lutnet_eval(*ok_args) == tt.TT_OK  # batch 0: nothing to do
    bad = fan.copy()
    bad[3, 2] = 6 + 3  # neuron 3 reading itself
    assert L.tt_lutnet_eval(d.ctypes.data, len(d), bad.ctypes.data, 6, fake, total, fake, 5, fake, None) == \
        tt.TT_EINVAL
    bad = fan.copy()
    bad[0, 0] = -1
    assert L.tt_lutnet_eval(d.ctypes.data, len(d), bad.ctypes.data, 6, fake, total, fake, 5, fake, None) == \
        tt.TT_EINVAL
    assert L.tt_lutnet_eval(d.ctypes.data, len(d), None, 6, fake, total, fake, 5, fake, None) == tt.TT_EINVAL
    assert L.tt_lutnet_eval(d.ctypes.data, len(d), fan.ctypes.data, 6, fake, total - 1, fake, 5, fake, None) == \
        tt.TT_ERANGE


def test_lutnet_handle_checks_and_empty_network():
    L = tt.lib()
    d = tt.descriptors(cfg0())
    total = tt.layout(d)
    fake = ctypes.c_void_p(0x1000)
    fan = np.full((len(d), 8), -1, np.int32)
    fan[:, :6] = np.arange(6)
    h = ctypes.c_void_p()
    assert L.tt_lutnet_create(d.ctypes.data, len(d), fan.ctypes.data, 6, fake, total, None, None) == tt.TT_EINVAL
    bad = fan.copy()
    bad[5, 0] = 6 + 5  # reads itself
    assert L.tt_lutnet_create(d.ctypes.data, len(d), bad.ctypes.data, 6, fake, total, None,
                              ctypes.byref(h)) == tt.TT_EINVAL
    assert h.value is None
    assert L.tt_lutnet_create(d.ctypes.data, len(d), fan.ctypes.data, 6, None, total, None,
                              ctypes.byref(h)) == tt.TT_EINVAL
    assert L.tt_lutnet_create(d.ctypes.data, len(d), fan.ctypes.data, 6, fake, total - 1, None,
                              ctypes.byref(h)) == tt.TT_ERANGE
    # an empty network needs no device: its handle evaluates nothing
    assert L.tt_lutnet_create(None, 0, None, 6, None, 0, None, ctypes.byref(h)) == tt.TT_OK
    assert h.value is not None
    assert L.tt_lutnet_run(h, fake, 10, fake, None) == tt.TT_OK
    assert L.tt_lutnet_run(h, fake, -1, fake, None) == tt.TT_EINVAL
    assert L.tt_lutnet_run(None, fake, 10, fake, None) == tt.TT_EINVAL
    assert L.tt_lutnet_destroy(h) == tt.TT_OK
    assert L.tt_lutnet_destroy(None) == tt.TT_OK


def test_lutnet_sample_argument_checks():
    L = tt.lib()
    fake = ctypes.c_void_p(0x1000)
    sig = np.array([0], np.int32)
    val = np.array([1], np.uint8)
    assert L.tt_lutnet_sample(None, None, None, 0, 1, 0, 10, fake, fake, 4, fake, None) == tt.TT_EINVAL
    h = ctypes.c_void_p()
    assert L.tt_lutnet_create(None, 0, None, 6, None, 0, None, ctypes.byref(h)) == tt.TT_OK
    # an empty network has nothing to sample
    assert L.tt_lutnet_sample(h, sig.ctypes.data, val.ctypes.data, 1, 1, 0, 10, fake, fake, 4, fake, None) == \
        tt.TT_EINVAL
    assert L.tt_lutnet_destroy(h) == tt.TT_OK


def test_cnf_transform_argument_checks():
    L = tt.lib()
    fake = ctypes.c_void_p(0x1000)

    def call(inst, n_inst=None):
        lits, coff, ioff, nv = tt.cnf_csr(inst)
        return L.tt_cnf_transform(lits.ctypes.data if len(lits) else None, coff.ctypes.data, ioff.ctypes.data,
                                  len(nv) if n_inst is None else n_inst, nv.ctypes.data, fake, fake, fake, fake,
                                  None)

    assert L.tt_cnf_transform(None, None, None, 0, None, None, None, None, None, None) == tt.TT_OK
    assert call([(3, [[1, 2], [-3]])], n_inst=-1) == tt.TT_EINVAL
    assert call([(2, [[1, 3]])]) == tt.TT_EINVAL        # variable beyond n_vars
    assert call([(3, [[1, -1, 2]])]) == tt.TT_EINVAL    # tautology
    assert call([(3, [[1], []])]) == tt.TT_EINVAL       # empty clause
    assert call([(40000, [[1]])]) == tt.TT_EINVAL       # too many variables for one instance


def test_gd_and_sop_argument_checks():
    L = tt.lib()
    h = ctypes.c_void_p()
    cls = np.zeros(4, np.uint8)
    assert L.tt_gd_create(None, None, 0, 3, None, 0, cls.ctypes.data, None, None) == tt.TT_EINVAL
    assert L.tt_gd_create(None, None, -1, 3, None, 0, cls.ctypes.data, None, ctypes.byref(h)) == tt.TT_EINVAL
    assert L.tt_gd_create(None, None, 0, 3, None, 0, None, None, ctypes.byref(h)) == tt.TT_EINVAL
    # an expression over more variables than a transformation records
    rec = np.zeros(1, tt.CNF_EXPR_DTYPE)
    rec["kind"], rec["out"], rec["n_vars"] = tt.TT_CNF_IV, 9, 13
    cls = np.zeros(10, np.uint8)
    assert L.tt_gd_create(None, None, 0, 9, rec.ctypes.data, 1, cls.ctypes.data, None,
                          ctypes.byref(h)) == tt.TT_EINVAL
    assert L.tt_gd_run(None, None, 1, 1.0, 1, None, None, None) == tt.TT_EINVAL
    assert L.tt_gd_run_from(None, None, None, 1, 1.0, 1, None, None, None) == tt.TT_EINVAL
    assert L.tt_gd_unique(None, None, None, 1, None, None, None) == tt.TT_EINVAL
    assert L.tt_gd_destroy(None) == tt.TT_OK
    plane = np.zeros(1, np.uint64)
    nt, nl, ex = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.tt_sop_minimize(plane.ctypes.data, 13, 0, 0, None, None, ctypes.byref(nt), ctypes.byref(nl),
                             ctypes.byref(ex)) == tt.TT_EINVAL
    assert L.tt_sop_minimize(None, 3, 0, 0, None, None, ctypes.byref(nt), ctypes.byref(nl),
                             ctypes.byref(ex)) == tt.TT_EINVAL
    assert L.tt_sop_minimize(plane.ctypes.data, 3, 0, 0, None, None, ctypes.byref(nt), ctypes.byref(nl),
                             ctypes.byref(ex)) == tt.TT_OK and nt.value == 0
    buf = ctypes.create_string_buffer(64)
    assert L.tt_kmap_text(plane.ctypes.data, buf, 64) == tt.TT_EINVAL
