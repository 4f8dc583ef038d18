"""Build the gfx950 Q2X library (``libq2x.so``) in-tree with hipcc.

Every HIP source is compiled for gfx950 only.  The twelve tile-kernel
instantiation units (6 element kinds x 2 precisions) and the eight
receiving-side units (4 kinds x 2 precisions) are large, fully unrolled
translation units, so they compile in parallel.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libq2x.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]

# The FP32 tile kernels are scheduled for instruction-level parallelism: a
# tile's wave often has its SIMD to itself, and the default schedule (fewest
# registers) runs every ladder output's FMA chain to the end before the next.
# (Measured: FP32 gains a little everywhere; the FP64 kernels, whose registers
# double, lost a quarter of their speed, so they keep the default.)
TILE_FLAGS_F32 = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
# The receiving-side kernels take the same schedule in both precisions: they
# run at most three waves per SIMD, and each degree's FP64 dot products with
# L are independent of the next degree's ladder (measured: about a fifth
# faster in FP32 and a tenth in FP64 at p = 16, with no spills).
EVAL_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]

SIMPLE = ["q2x_api.hip", "q2x_bucket.hip", "q2x_dispatch.hip", "q2x_batch.hip", "q2x_m2m.hip", "q2x_near.hip",
          "q2x_peak.hip"]
INST = [(k, f) for k in range(6) for f in (0, 1)]
EVAL_INST = [(k, f) for k in range(4) for f in (0, 1)]


def _units():
    units = []
    for src in SIMPLE:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        units.append((obj, [os.path.join(CSRC, src)], []))
    for k, f in INST:
        obj = os.path.join(BUILD, f"q2x_inst_k{k}_f{f}.o")
        units.append((obj, [os.path.join(CSRC, "q2x_inst.hip")],
                      [f"-DQ2X_INST_KIND={k}", f"-DQ2X_INST_F32={f}"] + (TILE_FLAGS_F32 if f else [])))
    for k, f in EVAL_INST:
        obj = os.path.join(BUILD, f"q2x_eval_k{k}_f{f}.o")
        units.append((obj, [os.path.join(CSRC, "q2x_eval_inst.hip")],
                      [f"-DQ2X_INST_KIND={k}", f"-DQ2X_INST_F32={f}"] + EVAL_FLAGS))
    return units


def source_hash() -> str:
    """Short hash of the sources and compiler flags of the tile kernel (ties
    stored profiler figures of that kernel to the code they measured)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("q2x_tile.hpp", "q2x_internal.hpp", "q2x_inst.hip"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    # the flags without the include directory, an absolute path that depends
    # on where the tree is checked out
    flags, skip = [], False
    for f in COMMON + TILE_FLAGS_F32:
        if skip:
            skip = False
            continue
        if f == "-I":
            skip = True
            continue
        flags.append(f)
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def library_hash() -> str:
    """Hash of every source of the library (its build identity, q2x_build_id)."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp")))
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(HERE, "..", "include", "q2x.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _build_id_object(verbose) -> str:
    """The build-identity unit, compiled with the host compiler on every build."""
    obj = os.path.join(BUILD, "q2x_build_id.o")
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-fPIC", f'-DQ2X_BUILD_ID="{library_hash()}"', "-c",
           os.path.join(CSRC, "q2x_build_id.cpp"), "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(obj + ".tmp", obj)
    return obj


def _headers():
    return [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")] + \
        [os.path.join(HERE, "..", "include", "q2x.h")]


def _stale(obj, srcs):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(s) > t for s in list(srcs) + _headers())


def _build_id_stale(obj) -> bool:
    t = os.path.getmtime(obj)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(HERE, "..", "include", "q2x.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


def _compile(unit, verbose):
    obj, srcs, defs = unit
    cmd = [HIPCC] + COMMON + defs + ["-c", srcs[0], "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {srcs[0]} {defs}:\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = True, verbose: bool = False, jobs: int | None = None) -> str:
    """Compile (all units when force, else only stale ones) and link libq2x.so."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    todo = [u for u in units if force or _stale(u[0], u[1])]
    jobs = jobs or min(8, os.cpu_count() or 4)
    if todo:
        # largest units first
        todo.sort(key=lambda u: 0 if "inst" in u[0] else (1 if "eval" in u[0] else 2))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(lambda u: _compile(u, verbose), todo))
    objs = [u[0] for u in units]
    bid = os.path.join(BUILD, "q2x_build_id.o")
    fresh_id = not os.path.exists(bid) or _build_id_stale(bid)
    if fresh_id:
        _build_id_object(verbose)
    objs.append(bid)
    if todo or fresh_id or not os.path.exists(LIB):
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
