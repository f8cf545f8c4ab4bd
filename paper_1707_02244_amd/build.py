"""Build libcscirc.so for gfx950 with hipcc (in-tree, no JIT cache).

Each kernel length is compiled in its own translation unit so the objects
build in parallel; the runtime and the C ABI live in runtime.hip.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcscirc.so")

ROW_LENGTHS = [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]   # pass A (N2)
COL_LENGTHS = [4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]            # pass B (N1)
SOLVE_LOGN = list(range(7, 22))                                     # persistent solver, N = 2^L
BATCH_ALG = [0, 1]                                                  # persistent batched solver: ISTA, ADMM
COL2_LENGTHS = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]  # 2-D column pass (rows R)
ROW2_LENGTHS = [8, 16, 32, 64, 128, 256, 512, 1024, 2048]           # 2-D row pass (H = columns / 2)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(os.path.dirname(HERE), "include"),
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (p.returncode, " ".join(cmd), out))
    return out


def _stale(src, obj):
    """An object is stale when it is missing or older than its source, any
    header under csrc/ or the C ABI header."""
    if not os.path.exists(obj):
        return True
    deps = [src, os.path.join(os.path.dirname(HERE), "include", "cscirc.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    return max(os.path.getmtime(f) for f in deps) > os.path.getmtime(obj)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every unit (incremental: only stale objects) and link."""
    os.makedirs(BUILD, exist_ok=True)
    units = []
    for L in ROW_LENGTHS:
        units.append((os.path.join(CSRC, "inst_passA.hip"), os.path.join(BUILD, "passA_%d.o" % L), ["-DCS_LEN=%d" % L]))
    for L in COL_LENGTHS:
        units.append((os.path.join(CSRC, "inst_passB.hip"), os.path.join(BUILD, "passB_%d.o" % L), ["-DCS_LEN=%d" % L]))
    for L in SOLVE_LOGN:
        units.append((os.path.join(CSRC, "inst_solve.hip"), os.path.join(BUILD, "solve_%d.o" % L), ["-DCS_LOGN=%d" % L]))
        units.append((os.path.join(CSRC, "inst_solve.hip"), os.path.join(BUILD, "solve_tr_%d.o" % L),
                      ["-DCS_LOGN=%d" % L, "-DCS_TRACE=1"]))
    for A in BATCH_ALG:
        units.append((os.path.join(CSRC, "inst_bpersist.hip"), os.path.join(BUILD, "bpersist_%d.o" % A), ["-DCS_ALG=%d" % A]))
    for L in COL2_LENGTHS:
        units.append((os.path.join(CSRC, "inst2d_col.hip"), os.path.join(BUILD, "col2_%d.o" % L), ["-DCS_LEN=%d" % L]))
    for L in ROW2_LENGTHS:
        units.append((os.path.join(CSRC, "inst2d_row.hip"), os.path.join(BUILD, "row2_%d.o" % L), ["-DCS_LEN=%d" % L]))
    units.append((os.path.join(CSRC, "inst_direct.hip"), os.path.join(BUILD, "direct.o"), []))
    units.append((os.path.join(CSRC, "runtime.hip"), os.path.join(BUILD, "runtime.o"), []))
    units.append((os.path.join(CSRC, "runtime2d.hip"), os.path.join(BUILD, "runtime2d.o"), []))
    units.append((os.path.join(CSRC, "runtime_batch.hip"), os.path.join(BUILD, "runtime_batch.o"), []))
    units.sort(key=lambda u: ("solve" not in u[1] and "batch" not in u[1], -len(u[1])))
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo = [u for u in units if not incremental or _stale(u[0], u[1])]
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]) for src, obj, extra in todo]
        for f in futs:
            out = f.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
