"""Builds the HIP library ``libdg.so`` in-tree for gfx950.

Usage: ``python -m paper_1211_0582_amd.build`` (or ``build()`` from Python).
Host-only setup code is compiled with g++, everything that touches HIP with
hipcc; the kernel file is compiled once per order N = 1..9 and precision
group so the objects build in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdg.so")
ORDERS = range(1, 10)

ARCH = os.environ.get("DG_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

# Packed FP32 instructions are switched off for every device compile.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]


def _embed_rtc_source() -> str:
    """C++ file holding the text of rtc_kernel.hpp (the kernel template that
    run-time compiled systems are built from) as kRtcKernelSource."""
    text = open(os.path.join(CSRC, "rtc_kernel.hpp"), encoding="utf-8").read()
    if ")DGRTC\"" in text:
        raise RuntimeError("rtc_kernel.hpp contains the raw-string delimiter")
    out = os.path.join(BUILD, "rtc_source.cpp")
    body = 'extern const char kRtcKernelSource[];\nconst char kRtcKernelSource[] = R"DGRTC(' + text + ')DGRTC";\n'
    if not os.path.exists(out) or open(out, encoding="utf-8").read() != body:
        with open(out, "w", encoding="utf-8") as f:
            f.write(body)
    return out


def _jobs():
    jobs = []
    for name in ("host_refelem.cpp", "host_mesh.cpp"):
        src = os.path.join(CSRC, name)
        jobs.append(([CXX, *HOST_FLAGS, "-c", src, "-o", os.path.join(BUILD, name + ".o")], name))
    src = _embed_rtc_source()
    jobs.append(([CXX, *HOST_FLAGS, "-c", src, "-o", os.path.join(BUILD, "rtc_source.o")], "rtc_source.cpp"))
    for name in ("api.cpp", "batch.cpp", "rtc.cpp", "lserk.hip", "noalloc.hip", "diag.hip"):
        src = os.path.join(CSRC, name)
        lang = ["-x", "hip"] if name.endswith(".cpp") else []
        jobs.append(([HIPCC, *HIP_FLAGS, *lang, "-c", src, "-o", os.path.join(BUILD, name + ".o")], name))
    for n in ORDERS:
        for g in (0, 1, 2):   # precision groups: FP64, FP32, split 16-bit
            src = os.path.join(CSRC, "rhs_inst.hip")
            jobs.append(([HIPCC, *HIP_FLAGS, f"-DDG_ORDER={n}", f"-DDG_GROUP={g}", "-c", src, "-o",
                          os.path.join(BUILD, f"rhs_n{n}_g{g}.o")], f"rhs_inst.hip N={n} group={g}"))
    return jobs


def _run(cmd_name):
    cmd, name = cmd_name
    p = subprocess.run(cmd, capture_output=True, text=True)
    return name, p.returncode, p.stdout + p.stderr, cmd


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source and links libdg.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    work = _jobs()
    n = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        results = list(ex.map(_run, work))
    bad = [r for r in results if r[1] != 0]
    for name, rc, out, cmd in results:
        if verbose or rc != 0:
            filtered = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
            if filtered:
                print(f"--- {name} (rc={rc})\n{filtered}", file=sys.stderr)
    if bad:
        raise RuntimeError("compilation failed: " + ", ".join(b[0] for b in bad))
    objs = [w[0][-1] for w in work]
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lhiprtc"]
    p = subprocess.run(link, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
