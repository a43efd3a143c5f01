"""Build libtt.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtt.so")
SOURCES = ["tt_api.hip", "tt_enum.hip", "tt_support.hip", "tt_mlp.hip", "tt_screen.hip", "tt_lutnet.hip", "tt_cnf.hip", "tt_gd.hip", "tt_gd_compile.hip", "tt_sop.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # Keep the compiler from forming packed fp32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


# Sources whose text decides what the autotuner measures: a signature of
# them is compiled in and keys the tune cache, so a kernel edit re-tunes.
KERNEL_SIG_SOURCES = ["tt_enum.hip", "tt_internal.h"]


def kernel_signature() -> str:
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SIG_SOURCES:
        with open(os.path.join(CSRC, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Host-only AddressSanitizer + UndefinedBehaviorSanitizer: each flag goes to
# the host compilation (device code is not instrumented).  The result,
# libtt_san.so, is for CPU runs of the host-side tests only.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-g"]
SAN_LIB = os.path.join(PKG, "libtt_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source to an object file, link libtt.so (libtt_san.so
    with host-side sanitizers).  Always rebuilds."""
    cc = hipcc()
    sig = f"-DTT_KERNEL_SIG=0x{kernel_signature()}ull"
    objdir = os.path.join(PKG, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    for s in srcs:
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        cmd = [cc, *HIPCC_FLAGS, *(SANITIZE_FLAGS if sanitize else []), sig, "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(s)
            sys.stderr.write("\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp"
    # hipRTC: the GD sampler compiles each circuit into a kernel of its own
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
