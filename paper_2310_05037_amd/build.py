"""Build librawalign.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librawalign.so")

SOURCES = ["dtw_single.hip", "dtw_multi.hip", "dtw_antidiag.hip", "dtw_plan.hip", "dtw_bnb.hip", "dtw_global.hip",
           "dtw_band.hip", "dtw_path.hip", "dtw_noalloc.hip", "dtw_pipe.hip",
           "rawalign_abi.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # min-plus arithmetic must not be contracted or reassociated
    "-ffp-contract=off", "-fno-fast-math",
    # no packed FP32 instructions (v_pk_*_f32); the DP does not use them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


# Issue-rate probe behind the roofline peak (bench.py --valu-rate); a library
# of its own, not part of librawalign.
PROBE_SOURCE = "valu_probe.hip"
PROBE_LIB = os.path.join(PKG, "libvaluprobe.so")


def build_probe(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-shared", "-x", "hip", os.path.join(CSRC, PROBE_SOURCE), "-o", tmp]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        sys.stderr.write("\n".join(ln for ln in p.stdout.splitlines() if "packed-fp32-ops" not in ln) + "\n")
        raise RuntimeError(f"hipcc failed on {PROBE_SOURCE}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return PROBE_LIB


def build(verbose: bool = True, out: str = LIB, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    t0 = time.time()
    procs = []
    for src in SOURCES:
        obj = out + "." + src + ".o"
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc, *HIPCC_FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, p in procs:
        log, _ = p.communicate()
        lines = [ln for ln in log.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            sys.stderr.write("\n".join(lines) + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
    tmp = out + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f}s")
    return out


if __name__ == "__main__":
    build()
    build_probe()
