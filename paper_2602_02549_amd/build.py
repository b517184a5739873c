"""Build libozaki2.so (HIP for gfx950) in-tree with hipcc.

Usage:  python -m paper_2602_02549_amd.build   (or __graft_entry__.build())
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libozaki2.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

SOURCES = ["tables.cpp", "api.cpp", "scale.hip", "residue.hip", "gemm_i8.hip", "crt.hip",
           "plan.hip", "noalloc.hip", "complex.hip", "probe.hip"]

# -ffp-contract=off: every fused multiply-add in the library is an explicit
# fma(); the CRT and double-double code rely on single roundings elsewhere.
# Packed-FP32 instructions are disabled for all device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj)
        cmd = [cc, *FLAGS]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"[build] FAILED {src}\n{' '.join(cmd)}\n{text}\n")
        elif verbose and text.strip():
            sys.stderr.write(f"[build] {src}:\n{text}\n")
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = OUT + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout.decode(errors="replace"))
    os.replace(tmp, OUT)
    return OUT


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer: the flags apply
# to the host pass only (device code is built as usual and never launched by
# the host-only checks that load this variant).
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def build_host_sanitized(out_dir: str) -> str:
    """Build a copy of the library whose host code (argument checks, layouts,
    constant tables, workspace queries, caches) carries ASan and UBSan, into
    out_dir/libozaki2_hostsan.so.  Loading it needs the clang ASan runtime
    preloaded (asan_runtime()).  A test aid: the product build is build()."""
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w",
             "-fno-omit-frame-pointer", *HOST_SANITIZE]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(out_dir, src + ".san.o")
        objs.append(obj)
        cmd = [cc, *flags] + (["-x", "hip"] if src.endswith(".hip") else [])
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"sanitized build of {src} failed:\n" + out.decode(errors="replace"))
    lib = os.path.join(out_dir, "libozaki2_hostsan.so")
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", *HOST_SANITIZE,
           *objs, "-o", lib]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if p.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + p.stdout.decode(errors="replace"))
    return lib


def asan_runtime() -> str:
    """Path of the clang ASan runtime that the sanitized library links to."""
    out = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"],
                         stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True).stdout.strip()
    if out and os.path.isabs(out) and os.path.exists(out):
        return out
    base = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(base)) if os.path.isdir(base) else []:
        cand = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    raise RuntimeError("clang ASan runtime not found")


if __name__ == "__main__":
    print(build(verbose=True))
