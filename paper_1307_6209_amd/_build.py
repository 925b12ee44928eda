"""Compile the HIP sources under csrc/ into libsellcs.so for gfx950.

Every call recompiles (objects under _build/, then one shared library next
to this file). Run as ``python -m paper_1307_6209_amd._build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsellcs.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for the device code on purpose; the
# host pass of hipcc warns that it does not know the feature (harmless).
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-I" + os.path.join(ROOT, "include"),
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# spmv_combo.hip holds the launchers of one dtype combination (values, x,
# accumulation); it is compiled once per entry, as (launcher suffix, enumerator).
COMBO_SRC = "spmv_combo.hip"
COMBOS = [("f64_f64", "COMBO_F64_F64"), ("f32_f32", "COMBO_F32_F32"), ("f32_f64", "COMBO_F32_F64"),
          ("bf16_f32", "COMBO_BF16_F32"), ("bf16_f64", "COMBO_BF16_F64")]


def units(csrc: str = CSRC):
    """The compile units: (source, extra flags, object file name)."""
    out = []
    for src in sorted(glob.glob(os.path.join(csrc, "*.hip"))):
        name = os.path.basename(src)
        if name == COMBO_SRC:
            for lc, combo in COMBOS:
                out.append((src, ["-DSELL_COMBO=" + combo, "-DSELL_LC=" + lc], "spmv_%s.o" % lc))
        else:
            out.append((src, [], name + ".o"))
    return out


def _compile(unit) -> str:
    src, defs, name = unit
    obj = os.path.join(OBJ, name)
    cmd = [HIPCC, *CFLAGS, *defs, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    todo = units()
    jobs = jobs or min(len(todo), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, todo))
    tmp = LIB + ".tmp%d" % os.getpid()
    p = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp],
                       capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
