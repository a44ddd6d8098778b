"""Builds libwtpic.so (HIP for gfx950) in-tree.

    python -m paper_1909_09613_amd.build

Every source is compiled with hipcc for gfx950 only.  Packed FP32 VALU
instructions are disabled (-packed-fp32-ops), and FP atomics use the
hardware instructions (-munsafe-fp-atomics: J is accumulated with FP64
global atomics, which is what the kernels intend).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwtpic.so")

# (source, object name, extra flags): the particle kernel is built once per
# precision policy, in parallel
SOURCES = [
    ("tables.cpp", "tables", []), ("runtime.cpp", "runtime", []),
    ("gpd.hip", "gpd32", ["-DWTPIC_GPD_POLICY=32"]), ("gpd.hip", "gpd64", ["-DWTPIC_GPD_POLICY=64"]),
    ("sort.hip", "sort", []), ("fields.hip", "fields", []), ("static_scratch.hip", "static_scratch", []),
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src, name, extra in SOURCES:
        obj = os.path.join(BUILD, name + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
