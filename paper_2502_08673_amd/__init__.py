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
LIB_PATH = os.path.join(PKG, "libtt.so")

NEURON_DTYPE = np.dtype(
    {
        "names": ["w", "thr", "bias", "F", "b", "o", "act", "pad", "word_off", "reserved"],
        "formats": [("i1", 8), ("<i4", 7), "<i2", "u1", "u1", "u1", "u1", ("u1", 6), "<u8", "<u8"],
        "offsets": [0, 8, 36, 38, 39, 40, 41, 42, 48, 56],
        "itemsize": 64,
    }
)

TT_OK, TT_EINVAL, TT_ERANGE, TT_EHIP, TT_ENOMEM, TT_ENOTSUP = 0, -1, -2, -3, -4, -5
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
        for name in ("tt_validate", "tt_layout", "tt_enumerate", "tt_pack", "tt_support", "tt_plan_create",
                     "tt_plan_launch", "tt_plan_destroy", "tt_plan_info", "tt_autotune", "tt_plan_kernel_times",
                     "tt_plan_support"):
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
        d = t.as_dict()
        d.update(n_items=ni.value, n_groups=ng.value, grid=grid.value)
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
