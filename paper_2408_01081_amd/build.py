"""Build the HIP library for gfx950 in-tree (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
CSRC = os.path.join(HERE, "csrc")
LIBNAME = "liblbm_hip.so"
SOURCES = ["lbm.hip", "lbm_tb_pa.hip", "lbm_tb_pb.hip", "lbm_tb_da.hip", "lbm_tb_db.hip",
           "lbm_tb_xa.hip", "lbm_tb_xb.hip", "lbm_tb_sp.hip", "lbm_batch.hip", "lbm_wop.hip",
           "sg.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the rounding sequence exactly as written (no FMA contraction)
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed (%d): %s" % (r.returncode, " ".join(cmd)))


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the
    shared library; the library is replaced only when all steps succeed."""
    from concurrent.futures import ThreadPoolExecutor
    out = os.path.join(HERE, LIBNAME)
    tag = "%d" % os.getpid()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, "%s.%s.o" % (src, tag))
        objs.append(obj)
        cmds.append([hipcc()] + compile_flags + ["-I", INCLUDE, "-I", CSRC, "-c", "-o", obj,
                                                 os.path.join(CSRC, src)])
    try:
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 4)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = out + ".tmp" + tag
        _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


# the files that define each profiled kernel's device code
KERNEL_SOURCES = {
    "k_tblock": ["lbm_tblock.hpp", "lbm_kernels.hpp", "lbm_step.hpp"],
    "k_step": ["lbm_step.hpp", "lbm_kernels.hpp"],
}


def kernel_hash(kname: str) -> str:
    """SHA-256 over the device sources of kernel `kname` and the build flags:
    identifies the kernel code that stored counter results belong to."""
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES[kname]:
        with open(os.path.join(CSRC, s), "rb") as fh:
            h.update(s.encode() + b"\0" + fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()


def source_hash(prefix: str = "") -> str:
    """SHA-256 over the HIP sources whose names start with `prefix` (all by
    default; "lbm" for the lattice kernels), the public headers and the build
    flags: identifies a kernel build for stored profiling results."""
    import hashlib
    h = hashlib.sha256()
    for s in sorted(os.listdir(CSRC)):
        if not s.startswith(prefix):
            continue
        with open(os.path.join(CSRC, s), "rb") as fh:
            h.update(s.encode() + b"\0" + fh.read())
    for s in sorted(os.listdir(INCLUDE)):
        if not s.startswith(prefix):
            continue
        with open(os.path.join(INCLUDE, s), "rb") as fh:
            h.update(s.encode() + b"\0" + fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()


if __name__ == "__main__":
    print(build(verbose=True))
