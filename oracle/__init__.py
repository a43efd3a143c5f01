"""The CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never imports,
links or executes anything here, and nothing here imports the product.

* ``tt_oracle.c``  -- plain C row loop (enumeration, packing, histogram,
  support), built into ``liboracle.so`` with gcc.
* ``brute.py``     -- an independent pure-Python brute force for tiny neurons.
* ``mlp_ref.py``   -- float64 NumPy reference of the screening MLP (forward,
  backward, losses, Adam).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


SAN_LIB = os.path.join(HERE, "liboracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(force: bool = True, out: str = LIB, defines=(), sanitize: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no intrinsics); with
    sanitize, with clang and AddressSanitizer + UndefinedBehaviorSanitizer
    into liboracle_san.so (the runtime shared with the library's sanitizer
    build, so both load into one process)."""
    if sanitize and out == LIB:
        out = SAN_LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    if sanitize:
        cmd = [CLANG, "-O1", "-g", "-fopenmp", "-shared", "-fPIC", "-Wall", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-shared-libasan",
               "-o", out + ".tmp", SRC]
    else:
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", out + ".tmp", SRC]
    cmd += [f"-D{d}" for d in defines]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def load(path: str = None):
    global _lib
    path = path or os.environ.get("ORACLE_LIBRARY") or LIB
    if path == LIB and _lib is not None:
        return _lib
    if not os.path.exists(path) or (path == LIB and os.path.getmtime(path) < os.path.getmtime(SRC)):
        build(force=True, out=path, sanitize=path == SAN_LIB)
    lib = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_offsets.argtypes = [ctypes.c_int, u8p, u8p, u8p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_enumerate.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 11 + [ctypes.c_int]
    lib.oracle_codes.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 8
    lib.oracle_from_codes.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 8
    lib.oracle_max_threads.restype = ctypes.c_int
    if path == LIB:
        _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _arrays(ns):
    F = np.ascontiguousarray(ns.F, np.uint8)
    b = np.ascontiguousarray(ns.b, np.uint8)
    o = np.ascontiguousarray(ns.o, np.uint8)
    act = np.ascontiguousarray(ns.act, np.uint8)
    w = np.ascontiguousarray(ns.w, np.int8)
    bias = np.ascontiguousarray(ns.bias, np.int16)
    thr = np.ascontiguousarray(ns.thr, np.int32)
    assert w.shape[1] == 8 and thr.shape[1] == 7
    return F, b, o, act, w, bias, thr


def offsets(ns, lib=None):
    lib = lib or load()
    F, b, o, *_ = _arrays(ns)
    n = len(F)
    word_off = np.zeros(n, np.uint64)
    total = np.zeros(1, np.uint64)
    lib.oracle_offsets(n, F.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                       b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                       o.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _p(word_off), _p(total))
    return word_off, int(total[0])


def enumerate(ns, planes=True, hist=True, support=True, nthreads=0, lib=None):
    """Planes (canonical layout), histogram [n, 8] and support bitmask [n]."""
    lib = lib or load()
    F, b, o, act, w, bias, thr = _arrays(ns)
    n = len(F)
    word_off, total = offsets(ns, lib)
    pl = np.zeros(total, np.uint64) if planes else None
    hi = np.zeros((n, 8), np.uint32) if hist else None
    su = np.zeros(n, np.uint8) if support else None
    rc = lib.oracle_enumerate(n, _p(F), _p(b), _p(o), _p(act), _p(w), _p(bias), _p(thr),
                              _p(word_off), _p(pl), _p(hi), _p(su), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_enumerate failed")
    return {"planes": pl, "hist": hi, "support": su, "word_off": word_off, "total_words": total}


def codes(ns, lib=None):
    """Concatenated per-row output codes (uint8), neuron i at the prefix sum of rows."""
    lib = lib or load()
    F, b, o, act, w, bias, thr = _arrays(ns)
    total = int(sum(1 << (int(f) * int(bb)) for f, bb in zip(F, b)))
    out = np.zeros(total, np.uint8)
    lib.oracle_codes(len(F), _p(F), _p(b), _p(o), _p(act), _p(w), _p(bias), _p(thr), _p(out))
    return out


def from_codes(ns, code_arr, lib=None):
    """Planes / histogram / support of given concatenated codes."""
    lib = lib or load()
    F, b, o, *_ = _arrays(ns)
    n = len(F)
    word_off, total = offsets(ns, lib)
    code_arr = np.ascontiguousarray(code_arr, np.uint8)
    pl = np.zeros(total, np.uint64)
    hi = np.zeros((n, 8), np.uint32)
    su = np.zeros(n, np.uint8)
    lib.oracle_from_codes(n, _p(F), _p(b), _p(o), _p(code_arr), _p(word_off), _p(pl), _p(hi), _p(su))
    return {"planes": pl, "hist": hi, "support": su, "word_off": word_off, "total_words": total}


def max_threads(lib=None) -> int:
    return int((lib or load()).oracle_max_threads())
