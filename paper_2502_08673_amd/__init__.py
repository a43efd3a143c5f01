"""Python binding of libtt.so, the MI355X truth-table enumeration library.

Argument marshalling only: every step runs in the library's HIP kernels.
Descriptors travel as a NumPy structured array in host memory (dtype
``NEURON_DTYPE``, 64 bytes per neuron, the layout of ``struct tt_neuron``);
tables, histograms, supports and codes are torch tensors in device memory
(tables as int64 holding the uint64 bit patterns).  Streams default to the
current torch stream.  If libtt.so has not been built, importing works but
every call raises ``RuntimeError``; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# TT_LIBRARY selects another build of the same library (the host-sanitizer
# build libtt_san.so for CPU runs of the host-side tests).
LIB_PATH = os.environ.get("TT_LIBRARY") or os.path.join(PKG, "libtt.so")

NEURON_DTYPE = np.dtype(
    {
        "names": ["w", "thr", "bias", "F", "b", "o", "act", "pad", "word_off", "reserved"],
        "formats": [("i1", 8), ("<i4", 7), "<i2", "u1", "u1", "u1", "u1", ("u1", 6), "<u8", "<u8"],
        "offsets": [0, 8, 36, 38, 39, 40, 41, 42, 48, 56],
        "itemsize": 64,
    }
)

TT_OK, TT_EINVAL, TT_ERANGE, TT_EHIP, TT_ENOMEM, TT_ENOTSUP, TT_ESCRATCH = 0, -1, -2, -3, -4, -5, -6
TT_NOALLOC_SCRATCH_BYTES = 32 << 20
TT_PLAN_PERSISTENT = 1
TT_PLAN_GRAPH = 2
TT_PLAN_TIMING = 4


class TTError(RuntimeError):
    def __init__(self, status: int, where: str, hip: int = 0):
        self.status = status
        lib = _lib_or_none()
        text = lib.tt_strerror(status).decode() if lib else str(status)
        super().__init__(f"{where}: {text} (status {status}, hip error {hip})")


class TTTune(ctypes.Structure):
    _fields_ = [("chunk_words", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("waves", ctypes.c_int), ("nontemporal", ctypes.c_int), ("tile_neurons", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def _lib_or_none():
    return _LIB


def lib():
    """The loaded libtt.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950). "
                "There is no CPU fallback.")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        L.tt_strerror.restype = ctypes.c_char_p
        L.tt_strerror.argtypes = [i32]
        L.tt_last_hip_error.restype = i32
        L.tt_version.restype = i32
        L.tt_device_check.restype = i32
        L.tt_words_per_plane.restype = u64
        L.tt_words_per_plane.argtypes = [i32, i32]
        L.tt_validate.argtypes = [vp, i32]
        L.tt_layout.argtypes = [vp, i32, ctypes.POINTER(u64)]
        L.tt_enumerate.argtypes = [vp, i32, vp, u64, vp, vp]
        L.tt_enumerate_noalloc.argtypes = [vp, i32, vp, u64, vp, vp]
        L.tt_pack.argtypes = [vp, i32, vp, u64, vp, u64, vp]
        L.tt_support.argtypes = [vp, i32, vp, u64, vp, vp, vp]
        L.tt_plan_create.argtypes = [vp, i32, u64, ctypes.POINTER(TTTune), ctypes.c_uint, ctypes.POINTER(vp)]
        L.tt_plan_launch.argtypes = [vp, vp, vp, vp]
        L.tt_plan_destroy.argtypes = [vp]
        L.tt_plan_info.argtypes = [vp, ctypes.POINTER(TTTune), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
        L.tt_autotune.argtypes = [vp, i32, vp, u64, ctypes.c_char_p, ctypes.POINTER(TTTune)]
        L.tt_plan_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)]
        L.tt_plan_support.argtypes = [vp, vp, vp, vp, vp]
        L.tt_plan_support_enumerated.argtypes = [vp, vp, vp, vp, vp]
        L.tt_plan_step.argtypes = [vp, vp, vp, vp, vp]
        L.tt_plan_wide_neurons.argtypes = [vp, ctypes.POINTER(i32)]
        for name in ("tt_validate", "tt_layout", "tt_enumerate", "tt_enumerate_noalloc", "tt_pack", "tt_support", "tt_plan_create",
                     "tt_plan_launch", "tt_plan_destroy", "tt_plan_info", "tt_autotune", "tt_plan_kernel_times",
                     "tt_plan_support", "tt_plan_support_enumerated", "tt_plan_wide_neurons", "tt_plan_step"):
            getattr(L, name).restype = i32
        sz = ctypes.c_size_t
        fl = ctypes.c_float
        L.tt_enumerate_device.argtypes = [vp, i32, vp, vp, u64, vp, vp]
        L.tt_support_device.argtypes = [vp, i32, vp, u64, vp, vp, vp, vp]
        L.tt_screen_features.argtypes = [vp, i32, vp, vp]
        L.tt_screen_labels.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.tt_mlp_forward.argtypes = [vp, i32, i32, vp, vp, i32, i32, vp, vp, vp]
        L.tt_mlp_infer.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.tt_lutnet_eval.argtypes = [vp, i32, vp, i32, vp, u64, vp, i32, vp, vp]
        L.tt_lutnet_create.argtypes = [vp, i32, vp, i32, vp, u64, vp, ctypes.POINTER(vp)]
        L.tt_lutnet_run.argtypes = [vp, vp, i32, vp, vp]
        L.tt_lutnet_destroy.argtypes = [vp]
        L.tt_lutnet_sample.argtypes = [vp, vp, vp, i32, u64, u64, i32, vp, vp, i32, vp, vp]
        L.tt_cnf_transform.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.tt_cnf_create.argtypes = [vp, vp, vp, i32, vp, vp, ctypes.POINTER(vp)]
        L.tt_cnf_run.argtypes = [vp, vp, vp, vp, vp, vp]
        L.tt_cnf_destroy.argtypes = [vp]
        L.tt_gd_create.argtypes = [vp, vp, i32, i32, vp, i32, vp, vp, ctypes.POINTER(vp)]
        L.tt_gd_inputs.argtypes = [vp, ctypes.POINTER(i32)]
        L.tt_gd_input_vars.argtypes = [vp, vp]
        L.tt_simplify.argtypes = [vp, i32, i32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.tt_gd_run.argtypes = [vp, vp, i32, fl, i32, vp, vp, vp]
        L.tt_gd_run_from.argtypes = [vp, vp, vp, i32, fl, i32, vp, vp, vp]
        L.tt_gd_sample_unique.argtypes = [vp, vp, vp, i32, fl, i32, vp, vp, vp, vp, vp]
        L.tt_gd_unique.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.tt_gd_destroy.argtypes = [vp]
        L.tt_gd_kernel.argtypes = [vp, ctypes.POINTER(i32)]
        L.tt_gd_set_kernel.argtypes = [vp, i32]
        L.tt_sop_minimize.argtypes = [vp, i32, ctypes.c_long, i32, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
        L.tt_kmap_text.argtypes = [vp, ctypes.c_char_p, i32]
        L.tt_mlp_backward.argtypes = [vp, i32, i32, vp, i32, vp, i32, vp, vp, vp, vp, sz, vp]
        L.tt_mlp_scratch_floats.argtypes = [i32, i32]
        L.tt_mlp_scratch_floats.restype = sz
        L.tt_mlp_loss.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.tt_adam_step.argtypes = [vp, vp, vp, vp, vp, sz, fl, fl, fl, fl, i32, vp]
        L.tt_adam_step_multi.argtypes = [i32, vp, vp, vp, vp, vp, vp, fl, fl, fl, fl, i32, vp]
        L.tt_cast_bf16.argtypes = [vp, vp, sz, vp]
        L.tt_screen_work_bytes.argtypes = [i32]
        L.tt_screen_work_bytes.restype = sz
        L.tt_screen_run.argtypes = [vp, i32, vp, fl, vp, vp, u64, vp, vp, vp, vp, vp, vp, vp]
        L.tt_screen_infer.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.tt_screen_infer_work_bytes.argtypes = [i32]
        L.tt_screen_infer_work_bytes.restype = ctypes.c_size_t
        L.tt_screen_expand.argtypes = [vp, i32, vp, vp, vp, vp]
        for name in ("tt_enumerate_device", "tt_support_device", "tt_screen_features", "tt_screen_labels",
                     "tt_mlp_forward", "tt_mlp_infer", "tt_lutnet_eval", "tt_lutnet_create", "tt_lutnet_run",
                     "tt_lutnet_destroy", "tt_lutnet_sample", "tt_cnf_transform",
                     "tt_cnf_create", "tt_cnf_run", "tt_cnf_destroy", "tt_gd_create", "tt_gd_inputs", "tt_gd_input_vars", "tt_simplify",
                     "tt_gd_run", "tt_gd_run_from", "tt_gd_sample_unique", "tt_gd_unique", "tt_gd_kernel", "tt_gd_set_kernel", "tt_gd_destroy", "tt_sop_minimize", "tt_kmap_text", "tt_mlp_backward", "tt_mlp_loss",
                     "tt_adam_step", "tt_adam_step_multi", "tt_cast_bf16",
                     "tt_screen_run", "tt_screen_infer", "tt_screen_expand"):
            getattr(L, name).restype = i32
        _LIB = L
        _register_extras(L)
    return _LIB


_EXTRA_REGISTRARS = []


def _register_extras(L):
    for f in _EXTRA_REGISTRARS:
        f(L)


def check(status: int, where: str):
    if status != TT_OK:
        raise TTError(status, where, lib().tt_last_hip_error())


# ------------------------------------------------------------------ helpers
def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _desc_arr(desc) -> np.ndarray:
    desc = np.ascontiguousarray(desc)
    if desc.dtype != NEURON_DTYPE:
        raise TypeError("descriptors must use NEURON_DTYPE")
    return desc


def descriptors(ns) -> np.ndarray:
    """Pack a workloads.NeuronSet into host descriptors (word_off zero)."""
    n = len(ns)
    d = np.zeros(n, NEURON_DTYPE)
    d["w"] = ns.w
    d["thr"] = ns.thr
    d["bias"] = ns.bias
    d["F"], d["b"], d["o"], d["act"] = ns.F, ns.b, ns.o, ns.act
    return d


def version() -> int:
    return lib().tt_version()


def device_check() -> None:
    check(lib().tt_device_check(), "tt_device_check")


def words_per_plane(F: int, b: int) -> int:
    return int(lib().tt_words_per_plane(F, b))


def validate(desc) -> None:
    desc = _desc_arr(desc)
    check(lib().tt_validate(_ptr(desc), len(desc)), "tt_validate")


def layout(desc) -> int:
    """Fill desc['word_off'] in place with the canonical layout; return total words."""
    desc = _desc_arr(desc)
    total = ctypes.c_uint64(0)
    check(lib().tt_layout(_ptr(desc), len(desc), ctypes.byref(total)), "tt_layout")
    return int(total.value)


def enumerate(desc, tables, total_words=None, hist=None, stream=None) -> None:
    desc = _desc_arr(desc)
    tw = tables.numel() if total_words is None else total_words
    check(lib().tt_enumerate(_ptr(desc), len(desc), _ptr(tables), tw, _ptr(hist), _stream(stream)),
          "tt_enumerate")


def enumerate_noalloc(desc, tables, total_words=None, hist=None, stream=None) -> None:
    """tt_enumerate with the library's fixed device scratch instead of an
    allocation (raises TTError with TT_ESCRATCH when the input does not fit)."""
    desc = _desc_arr(desc)
    tw = tables.numel() if total_words is None else total_words
    check(lib().tt_enumerate_noalloc(_ptr(desc), len(desc), _ptr(tables), tw, _ptr(hist), _stream(stream)),
          "tt_enumerate_noalloc")


def pack(desc, codes, tables, stream=None) -> None:
    desc = _desc_arr(desc)
    check(lib().tt_pack(_ptr(desc), len(desc), _ptr(codes), codes.numel(), _ptr(tables), tables.numel(),
                        _stream(stream)), "tt_pack")


def support(desc, tables, support_out=None, hist=None, stream=None) -> None:
    desc = _desc_arr(desc)
    check(lib().tt_support(_ptr(desc), len(desc), _ptr(tables), tables.numel(), _ptr(support_out), _ptr(hist),
                           _stream(stream)), "tt_support")


class Plan:
    """Batched enumeration plan (persistent work queue, optional hipGraph)."""

    def __init__(self, desc, total_words: int, tune: Optional[dict] = None,
                 flags: int = TT_PLAN_PERSISTENT | TT_PLAN_GRAPH):
        desc = _desc_arr(desc)
        self._h = ctypes.c_void_p()
        t = None
        if tune is not None:
            t = TTTune(**tune)
        check(lib().tt_plan_create(_ptr(desc), len(desc), total_words, ctypes.byref(t) if t else None, flags,
                                   ctypes.byref(self._h)), "tt_plan_create")

    def launch(self, tables, hist=None, stream=None) -> None:
        check(lib().tt_plan_launch(self._h, _ptr(tables), _ptr(hist), _stream(stream)), "tt_plan_launch")

    def support(self, tables, support_out=None, hist=None, stream=None) -> None:
        check(lib().tt_plan_support(self._h, _ptr(tables), _ptr(support_out), _ptr(hist), _stream(stream)),
              "tt_plan_support")

    def step(self, tables, hist=None, support_out=None, stream=None) -> None:
        """Enumeration (+ histogram) then the support of the plan's own tables
        (tt_plan_step); with TT_PLAN_GRAPH, the whole step replays as one graph."""
        check(lib().tt_plan_step(self._h, _ptr(tables), _ptr(hist), _ptr(support_out), _stream(stream)),
              "tt_plan_step")

    def support_enumerated(self, tables, support_out=None, hist=None, stream=None) -> None:
        """Support of tables holding this plan's own enumeration (zero-weight
        inputs settled without reading the tables)."""
        check(lib().tt_plan_support_enumerated(self._h, _ptr(tables), _ptr(support_out), _ptr(hist),
                                               _stream(stream)), "tt_plan_support_enumerated")

    def kernel_times_ms(self, max_count: int = 256) -> list:
        """Durations of the enumeration kernel of the launches since the last
        call (plans created with TT_PLAN_TIMING)."""
        buf = (ctypes.c_float * max_count)()
        cnt = ctypes.c_int()
        check(lib().tt_plan_kernel_times(self._h, buf, max_count, ctypes.byref(cnt)), "tt_plan_kernel_times")
        return [float(buf[i]) for i in range(cnt.value)]

    def info(self) -> dict:
        t = TTTune()
        ni, ng, grid = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().tt_plan_info(self._h, ctypes.byref(t), ctypes.byref(ni), ctypes.byref(ng), ctypes.byref(grid)),
              "tt_plan_info")
        nwide = ctypes.c_int()
        check(lib().tt_plan_wide_neurons(self._h, ctypes.byref(nwide)), "tt_plan_wide_neurons")
        d = t.as_dict()
        d.update(n_items=ni.value, n_groups=ng.value, grid=grid.value, wide_neurons=nwide.value)
        return d

    def close(self) -> None:
        if self._h:
            check(lib().tt_plan_destroy(self._h), "tt_plan_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h and _LIB is not None:
                _LIB.tt_plan_destroy(self._h)
        except Exception:
            pass


def autotune(desc, tables, cache_path: Optional[str] = None) -> dict:
    desc = _desc_arr(desc)
    t = TTTune()
    check(lib().tt_autotune(_ptr(desc), len(desc), _ptr(tables), tables.numel(),
                            cache_path.encode() if cache_path else None, ctypes.byref(t)), "tt_autotune")
    return t.as_dict()


# ------------------------------------------------------ device descriptors
def device_descriptors(desc):
    """Device copy of host descriptors (uint8 tensor of n * 64 bytes)."""
    import torch
    desc = _desc_arr(desc)
    return torch.from_numpy(desc.view(np.uint8).copy()).cuda()


def enumerate_device(d_desc, n, tables, total_words=None, active=None, status=None, stream=None) -> None:
    tw = tables.numel() if total_words is None else total_words
    check(lib().tt_enumerate_device(_ptr(d_desc), n, _ptr(active), _ptr(tables), tw, _ptr(status), _stream(stream)),
          "tt_enumerate_device")


def support_device(d_desc, n, tables, support_out=None, hist=None, status=None, stream=None) -> None:
    check(lib().tt_support_device(_ptr(d_desc), n, _ptr(tables), tables.numel(), _ptr(support_out), _ptr(hist),
                                  _ptr(status), _stream(stream)), "tt_support_device")


def screen_features(d_desc, n, x, stream=None) -> None:
    check(lib().tt_screen_features(_ptr(d_desc), n, _ptr(x), _stream(stream)), "tt_screen_features")


def screen_labels(d_desc, n, support_in, hist_in, y, m, h, stream=None) -> None:
    check(lib().tt_screen_labels(_ptr(d_desc), n, _ptr(support_in), _ptr(hist_in), _ptr(y), _ptr(m), _ptr(h),
                                 _stream(stream)), "tt_screen_labels")


def mlp_forward(x, batch, w, bias, relu, y_bf16=None, y_f32=None, stream=None) -> None:
    out, inp = w.shape
    check(lib().tt_mlp_forward(_ptr(x), batch, inp, _ptr(w), _ptr(bias), out, int(relu), _ptr(y_bf16),
                               _ptr(y_f32), _stream(stream)), "tt_mlp_forward")


def lutnet_eval(desc, fanin, n_inputs, tables, total_words, inputs, out, stream=None) -> None:
    """Network outputs through the tables (tt_lutnet_eval): fanin int32
    [n, 8] of signal indices (host), inputs uint8 [batch, n_inputs] and out
    uint8 [batch, n] on the device."""
    fanin = np.ascontiguousarray(fanin, np.int32)
    assert fanin.shape == (len(desc), 8)
    batch = int(inputs.shape[0]) if len(desc) else 0
    check(lib().tt_lutnet_eval(_ptr(desc), len(desc), fanin.ctypes.data, int(n_inputs), _ptr(tables),
                               int(total_words), _ptr(inputs), batch, _ptr(out), _stream(stream)),
          "tt_lutnet_eval")


TT_GD_INTERPRETED, TT_GD_COMPILED = 0, 1
TT_CNF_IV, TT_CNF_PO, TT_CNF_AUX = 1, 2, 3
TT_CNF_CLS_PI, TT_CNF_CLS_IV, TT_CNF_CLS_PO = 1, 2, 4
TT_CNF_MAX_VARS = 12
CNF_EXPR_DTYPE = np.dtype([("out", "<i4"), ("kind", "<i4"), ("first", "<i4"), ("last", "<i4"),
                           ("n_vars", "<i4"), ("support", "<u4"), ("vars", "<i4", (12,)), ("pad", "<i4", (14,)),
                           ("table", "<u8", (64,))])
assert CNF_EXPR_DTYPE.itemsize == 640


def cnf_csr(instances):
    """Host CSR arrays for tt_cnf_transform from a list of (n_vars, clauses)
    with clauses lists of DIMACS literals."""
    lits, coff, ioff, nvars = [], [0], [0], []
    for nv, clauses in instances:
        for c in clauses:
            lits.extend(c)
            coff.append(len(lits))
        ioff.append(len(coff) - 1)
        nvars.append(nv)
    return (np.asarray(lits, np.int32), np.asarray(coff, np.int32), np.asarray(ioff, np.int32),
            np.asarray(nvars, np.int32))


def cnf_transform(lits, clause_off, inst_off, n_vars, var_class, expr, n_expr, status, stream=None) -> None:
    """CNF instances to circuits (tt_cnf_transform): host CSR int32 arrays
    (see cnf_csr); device outputs var_class uint8 [sum(n_vars + 1)], expr
    uint8 [n_clauses * 640] (CNF_EXPR_DTYPE records), n_expr and status int32
    [n_inst]."""
    n_inst = len(n_vars)
    check(lib().tt_cnf_transform(lits.ctypes.data if len(lits) else None, clause_off.ctypes.data,
                                 inst_off.ctypes.data, n_inst, n_vars.ctypes.data, _ptr(var_class), _ptr(expr),
                                 _ptr(n_expr), _ptr(status), _stream(stream)), "tt_cnf_transform")


class Cnf:
    """Staged CNF instances (tt_cnf_create / run / destroy)."""

    def __init__(self, lits, clause_off, inst_off, n_vars, stream=None):
        self._h = ctypes.c_void_p()
        self.n_inst = len(n_vars)
        check(lib().tt_cnf_create(lits.ctypes.data if len(lits) else None, clause_off.ctypes.data,
                                  inst_off.ctypes.data, self.n_inst, n_vars.ctypes.data, _stream(stream),
                                  ctypes.byref(self._h)), "tt_cnf_create")

    def run(self, var_class, expr, n_expr, status, stream=None) -> None:
        assert self._h.value is not None, "closed"
        check(lib().tt_cnf_run(self._h, _ptr(var_class), _ptr(expr), _ptr(n_expr), _ptr(status), _stream(stream)),
              "tt_cnf_run")

    def close(self) -> None:
        if self._h.value is not None:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib().tt_cnf_destroy(h), "tt_cnf_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def sop_minimize(plane_words, n_vars, node_budget=0, max_terms=4096):
    """Minimal sum of products of one plane on the host (tt_sop_minimize):
    returns (terms as (care, value) pairs, literals, exact)."""
    words = np.ascontiguousarray(plane_words, np.uint64)
    care = np.zeros(max_terms, np.uint32)
    value = np.zeros(max_terms, np.uint32)
    nt, nl, ex = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().tt_sop_minimize(words.ctypes.data, int(n_vars), int(node_budget), max_terms, care.ctypes.data,
                                value.ctypes.data, ctypes.byref(nt), ctypes.byref(nl), ctypes.byref(ex)),
          "tt_sop_minimize")
    t = min(nt.value, max_terms)
    return [(int(c), int(v)) for c, v in zip(care[:t], value[:t])], int(nl.value), bool(ex.value)


GATE_DTYPE = np.dtype([("op", np.int32), ("a", np.int32), ("b", np.int32), ("dst", np.int32)])
GATE_CONST, GATE_COPY, GATE_AND, GATE_OR, GATE_XOR, GATE_XNOR = range(6)
OPD_TEMP, OPD_NEG = 1 << 16, 1 << 17


def simplify(table_words, n_vars, max_gates=1 << 15):
    """Simplify of one expression table on the host (tt_simplify): returns
    (gates as a GATE_DTYPE array, exact)."""
    words = np.ascontiguousarray(table_words, np.uint64)
    gates = np.zeros(max_gates, GATE_DTYPE)
    ng, ex = ctypes.c_int32(), ctypes.c_int32()
    check(lib().tt_simplify(words.ctypes.data, int(n_vars), max_gates, gates.ctypes.data, ctypes.byref(ng),
                            ctypes.byref(ex)), "tt_simplify")
    return gates[: ng.value].copy(), bool(ex.value)


def kmap_text(plane_word) -> str:
    """The four-variable Karnaugh map of a one-word plane (tt_kmap_text)."""
    w = np.array([plane_word], np.uint64)
    buf = ctypes.create_string_buffer(512)
    check(lib().tt_kmap_text(w.ctypes.data, buf, 512), "tt_kmap_text")
    return buf.value.decode()


class GdSampler:
    """GD sampling of one transformed CNF instance (tt_gd_*): clauses as a
    list of DIMACS literal lists, the instance's expression records
    (CNF_EXPR_DTYPE) and class bytes from the transformation (host)."""

    def __init__(self, clauses, n_vars, expr_records, var_class, stream=None):
        lits, coff, _, _ = cnf_csr([(n_vars, clauses)])
        recs = np.ascontiguousarray(expr_records)
        cls = np.ascontiguousarray(var_class, np.uint8)
        assert len(cls) == n_vars + 1
        self._h = ctypes.c_void_p()
        check(lib().tt_gd_create(lits.ctypes.data if len(lits) else None, coff.ctypes.data, len(clauses), int(n_vars),
                                 recs.ctypes.data if len(recs) else None, len(recs), cls.ctypes.data,
                                 _stream(stream), ctypes.byref(self._h)), "tt_gd_create")
        n = ctypes.c_int32()
        check(lib().tt_gd_inputs(self._h, ctypes.byref(n)), "tt_gd_inputs")
        self.n_pi = int(n.value)
        self.words = (self.n_pi + 63) // 64
        pv = np.zeros(max(self.n_pi, 1), np.int32)
        check(lib().tt_gd_input_vars(self._h, pv.ctypes.data), "tt_gd_input_vars")
        self.pi_vars = [int(x) for x in pv[: self.n_pi]]

    @property
    def kernel(self) -> int:
        """TT_GD_COMPILED (the circuit's own kernel) or TT_GD_INTERPRETED."""
        k = ctypes.c_int32()
        check(lib().tt_gd_kernel(self._h, ctypes.byref(k)), "tt_gd_kernel")
        return int(k.value)

    @kernel.setter
    def kernel(self, k: int) -> None:
        check(lib().tt_gd_set_kernel(self._h, int(k)), "tt_gd_set_kernel")

    def run(self, V, lr, iters, valid, solution, stream=None) -> None:
        check(lib().tt_gd_run(self._h, _ptr(V), int(V.shape[0]), float(lr), int(iters), _ptr(valid), _ptr(solution),
                              _stream(stream)), "tt_gd_run")

    def run_from(self, V0, V, lr, iters, valid, solution, stream=None) -> None:
        """Initial logits V0 (read only), final logits into V (None: not kept)."""
        check(lib().tt_gd_run_from(self._h, _ptr(V0), _ptr(V), int(V0.shape[0]),
                                   float(lr), int(iters), _ptr(valid), _ptr(solution), _stream(stream)),
              "tt_gd_run_from")

    def sample_unique(self, V0, V, lr, iters, valid, solution, first, count, stream=None) -> None:
        """run_from, then unique, in fewer passes (the compiled kernel does the
        filter's first pass)."""
        check(lib().tt_gd_sample_unique(self._h, _ptr(V0), _ptr(V), int(V0.shape[0]), float(lr), int(iters),
                                        _ptr(valid), _ptr(solution), _ptr(first), _ptr(count), _stream(stream)),
              "tt_gd_sample_unique")

    def unique(self, valid, solution, first, count, stream=None) -> None:
        check(lib().tt_gd_unique(self._h, _ptr(valid), _ptr(solution), int(valid.shape[0]), _ptr(first), _ptr(count),
                                 _stream(stream)), "tt_gd_unique")

    def close(self) -> None:
        if self._h.value is not None:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib().tt_gd_destroy(h), "tt_gd_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Lutnet:
    """A reusable network handle (tt_lutnet_create / run / destroy): fanin
    int32 [n, 8] of signal indices (host); the device tables must not change
    while the handle is open."""

    def __init__(self, desc, fanin, n_inputs, tables, total_words, stream=None):
        fanin = np.ascontiguousarray(fanin, np.int32)
        assert fanin.shape == (len(desc), 8)
        self.n, self.n_inputs = len(desc), int(n_inputs)
        self._h = ctypes.c_void_p()
        check(lib().tt_lutnet_create(_ptr(desc), len(desc), fanin.ctypes.data, self.n_inputs, _ptr(tables),
                                     int(total_words), _stream(stream), ctypes.byref(self._h)), "tt_lutnet_create")

    def run(self, inputs, out, stream=None) -> None:
        """inputs uint8 [batch, n_inputs], out uint8 [batch, n], device."""
        assert self._h.value is not None, "closed"
        batch = int(inputs.shape[0])
        check(lib().tt_lutnet_run(self._h, _ptr(inputs), batch, _ptr(out), _stream(stream)), "tt_lutnet_run")

    def sample(self, targets, seed, first_draw, n_draws, found_inputs, found_draw, count, stream=None) -> None:
        """Rejection sampling (tt_lutnet_sample): targets {signal: value};
        found_inputs uint8 [max_found, n_inputs], found_draw int64
        [max_found] and count int32 [1] on the device (count is added to)."""
        assert self._h.value is not None, "closed"
        sig = np.ascontiguousarray(list(targets.keys()), np.int32)
        val = np.ascontiguousarray(list(targets.values()), np.uint8)
        max_found = int(found_inputs.shape[0]) if found_inputs is not None else 0
        check(lib().tt_lutnet_sample(self._h, sig.ctypes.data if len(sig) else None,
                                     val.ctypes.data if len(val) else None, len(sig), int(seed) & (2**64 - 1),
                                     int(first_draw), int(n_draws), _ptr(found_inputs), _ptr(found_draw), max_found,
                                     _ptr(count), _stream(stream)), "tt_lutnet_sample")

    def close(self) -> None:
        if self._h.value is not None:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib().tt_lutnet_destroy(h), "tt_lutnet_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def mlp_infer(x, n, weights, biases, logits, stream=None) -> None:
    """The whole screening network in one launch (tt_mlp_infer): weights and
    biases are the four layers' [out][in] bf16 and [out] fp32 tensors."""
    w1, w2, w3, w4 = weights
    b1, b2, b3, b4 = biases
    check(lib().tt_mlp_infer(_ptr(x), n, _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2), _ptr(w3), _ptr(b3), _ptr(w4),
                             _ptr(b4), _ptr(logits), _stream(stream)), "tt_mlp_infer")


def mlp_backward(dy, batch, w, x, relu_mask, dx=None, dw=None, db=None, scratch=None, stream=None) -> None:
    out, inp = w.shape
    check(lib().tt_mlp_backward(_ptr(dy), batch, out, _ptr(w), inp, _ptr(x), int(relu_mask), _ptr(dx), _ptr(dw),
                                _ptr(db), _ptr(scratch), scratch.numel() if scratch is not None else 0,
                                _stream(stream)), "tt_mlp_backward")


def mlp_scratch_floats(batch, dim) -> int:
    """Scratch floats of tt_mlp_backward / tt_mlp_loss for layers whose in and
    out are at most dim."""
    return int(lib().tt_mlp_scratch_floats(batch, dim))


def mlp_loss(z, batch, y, m, h, dz, loss, scratch, stream=None) -> None:
    check(lib().tt_mlp_loss(_ptr(z), batch, _ptr(y), _ptr(m), _ptr(h), _ptr(dz), _ptr(loss), _ptr(scratch),
                            _stream(stream)), "tt_mlp_loss")


def adam_step(p, g, m, v, p_bf16, lr, beta1, beta2, eps, step, stream=None) -> None:
    check(lib().tt_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(p_bf16), p.numel(), lr, beta1, beta2, eps,
                             step, _stream(stream)), "tt_adam_step")


class AdamGroup:
    """A fixed set of tensors updated by one tt_adam_step_multi launch (the
    host arrays of their device pointers are built once)."""

    def __init__(self, params, grads, ms, vs, p_bf16=None):
        k = len(params)
        if not 0 < k <= 8:
            raise ValueError("1 to 8 tensors")
        P = ctypes.c_void_p * k
        self._keep = (params, grads, ms, vs, p_bf16)
        self._p = P(*[t.data_ptr() for t in params])
        self._g = P(*[t.data_ptr() for t in grads])
        self._m = P(*[t.data_ptr() for t in ms])
        self._v = P(*[t.data_ptr() for t in vs])
        self._pb = P(*[(t.data_ptr() if t is not None else None) for t in p_bf16]) if p_bf16 else None
        self._n = (ctypes.c_size_t * k)(*[t.numel() for t in params])
        self.count = k

    def step(self, lr, beta1, beta2, eps, step, stream=None) -> None:
        check(lib().tt_adam_step_multi(self.count, self._p, self._g, self._m, self._v, self._pb, self._n, lr, beta1,
                                       beta2, eps, step, _stream(stream)), "tt_adam_step_multi")


def cast_bf16(x, y, stream=None) -> None:
    check(lib().tt_cast_bf16(_ptr(x), _ptr(y), x.numel(), _stream(stream)), "tt_cast_bf16")


def screen_work_bytes(n) -> int:
    return int(lib().tt_screen_work_bytes(n))


def screen_run(d_desc, n, logits, tau, tables, support_out, hist, work, force_mask=None, mask=None,
               accept=None, status=None, stream=None) -> None:
    """logits = force_mask = None: plain full enumeration of every candidate."""
    check(lib().tt_screen_run(_ptr(d_desc), n, _ptr(logits), float(tau), _ptr(force_mask), _ptr(tables),
                              tables.numel(), _ptr(support_out), _ptr(hist), _ptr(mask), _ptr(accept), _ptr(work),
                              _ptr(status), _stream(stream)), "tt_screen_run")


def screen_infer(d_desc, n, gated, weights, biases, logits, work=None, stream=None) -> None:
    """Features and network from device descriptors (tt_screen_infer);
    gated: only the candidates the wave pass takes, listed first in work
    (screen_infer_work_bytes(n) bytes; None: allocated in the call)."""
    w1, w2, w3, w4 = weights
    b1, b2, b3, b4 = biases
    check(lib().tt_screen_infer(_ptr(d_desc), n, int(gated), _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2), _ptr(w3),
                                _ptr(b3), _ptr(w4), _ptr(b4), _ptr(logits), _ptr(work), _stream(stream)),
          "tt_screen_infer")


def screen_infer_work_bytes(n: int) -> int:
    return int(lib().tt_screen_infer_work_bytes(int(n)))


def screen_expand(d_desc, n, work, screened, full, stream=None) -> None:
    check(lib().tt_screen_expand(_ptr(d_desc), n, _ptr(work), _ptr(screened), _ptr(full), _stream(stream)),
          "tt_screen_expand")
from . import screen  # noqa: E402,F401
