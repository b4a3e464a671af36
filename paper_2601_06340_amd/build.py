"""Build libbpm_hip.so (gfx950) from csrc/ with hipcc.

Every (precision, nx) march kernel is instantiated in its own translation unit
(generated under ``_build/gen``) so the units compile in parallel; the host
library (C ABI, server) and the setup kernels are separate units.  The link
produces ``paper_2601_06340_amd/libbpm_hip.so``.

Usage: python -m paper_2601_06340_amd.build [-j N] [--incremental]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libbpm_hip.so")

ARCH = "gfx950"
# -packed-fp32-ops: no v_pk_{add,mul,fma}_f32 anywhere in the library.
HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INC, "-I", CSRC]

# keep in sync with Limits<> in csrc/bpm_march.hpp
UNIFORM = {"float": range(6, 15), "double": range(6, 14)}
STAGED = {"float": range(15, 17), "double": range(14, 17)}
THREE_D_LOG2NX = range(8, 11)  # 3D envelopes: rows of nx = 256..1024
THREE_D_LOG2NY = range(4, 9)   # ny = 16..256 rows
MIXED = ("float", "double")
STRAIN_CLASSES = (0, 1, 2)   # none, polynomial, dislocation/table
POLY1_CLASS = 3              # polynomial without the X^2 term: FP32 per-size kernels only


def _gen_units() -> list[str]:
    os.makedirs(GEN, exist_ok=True)
    units = []

    def write(name, body):
        path = os.path.join(GEN, name)
        old = open(path).read() if os.path.exists(path) else None
        if old != body:
            with open(path, "w") as f:
                f.write(body)
        units.append(path)

    for sc in STRAIN_CLASSES:
        for t, rng in UNIFORM.items():
            for l2 in rng:
                write("march_%s_%d_sc%d.hip" % (t, l2, sc),
                      '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
                      "template hipError_t launch_uniform<%s, %d, %d>(const SolveDesc *, int, const char *, "
                      "char *, double *, hipStream_t);\n}\n" % (t, l2, sc))
        for t, rng in STAGED.items():
            for l2 in rng:
                write("march_staged_%s_%d_sc%d.hip" % (t, l2, sc),
                      '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
                      "template hipError_t launch_staged<%s, %d, %d>(const SolveDesc *, int, const char *, "
                      "char *, double *, hipStream_t);\n"
                      "template hipError_t launch_wide_T<%s, %d, %d, false, 9>(int, const WideArgs &, "
                      "hipStream_t, WideShape *);\n}\n" % (t, l2, sc, t, l2, sc))
        for t in MIXED:
            for l2x in THREE_D_LOG2NX:
                for l2y in THREE_D_LOG2NY:
                    write("march_3d_%s_%d_%d_sc%d.hip" % (t, l2x, l2y, sc),
                          '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
                          "template hipError_t launch_3d<%s, %d, %d, %d>(const SolveDesc *, int, const char *, "
                          "char *, double *, hipStream_t);\n"
                          "template hipError_t launch_wide_T<%s, %d, %d, true, %d>(int, const WideArgs &, "
                          "hipStream_t, WideShape *);\n}\n" % (t, l2x, l2y, sc, t, l2x + l2y, sc, l2x))
            write("march_mixed_%s_sc%d.hip" % (t, sc),
                  '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
                  "template hipError_t launch_mixed<%s, %d>(const SolveDesc *, int, const char *, char *, "
                  "double *, hipStream_t);\n}\n" % (t, sc))
    for l2 in UNIFORM["float"]:
        write("march_float_%d_sc%d.hip" % (l2, POLY1_CLASS),
              '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
              "template hipError_t launch_uniform<float, %d, %d>(const SolveDesc *, int, const char *, "
              "char *, double *, hipStream_t);\n}\n" % (l2, POLY1_CLASS))
    for t in MIXED:
        write("march_any_%s.hip" % t,
              '#include "bpm_march_kernels.hpp"\nnamespace bpm {\n'
              "template hipError_t launch_any<%s>(const SolveDesc *, int, const char *, char *, "
              "double *, hipStream_t);\n}\n" % t)
    return units


def _up_to_date(obj: str) -> bool:
    """The object exists and is newer than every file its dependency list names."""
    dep = obj + ".d"
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    t = os.path.getmtime(obj)
    text = open(dep).read().replace("\\\n", " ")
    files = text.split(":", 1)[1].split() if ":" in text else []
    return bool(files) and all(os.path.exists(f) and os.path.getmtime(f) <= t for f in files)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and _up_to_date(obj):
        return obj
    cmd = ["hipcc"] + HIPFLAGS + ["-MMD", "-MF", obj + ".d", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, "\n".join(errs)))
    return obj


def build(jobs: int | None = None, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every unit and link the library (incremental: only the units
    whose object is older than a file it depends on)."""
    t0 = time.time()
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in ("bpm_setup.hip", "bpm_td.hip", "bpm_api.cpp", "bpm_server.cpp",
                                            "bpm_tune.cpp", "bpm_noalloc.hip")]
    srcs += _gen_units()
    # largest units first
    srcs.sort(key=lambda s: ("_any_" not in s, "mixed" not in s,
                            not any(("_%d_" % k) in s for k in (12, 13, 14, 15, 16))))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.0f s (%d units, -j%d)" % (LIB, time.time() - t0, len(srcs), jobs))
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--incremental", action="store_true", help="rebuild only out-of-date units")
    a = ap.parse_args()
    try:
        build(a.j, incremental=a.incremental)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
