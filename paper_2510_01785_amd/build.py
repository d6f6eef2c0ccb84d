"""Build libshtx.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2510_01785_amd.build   (or call build()).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libshtx.so")
SOURCES = ["api.hip", "tables.hip", "ring_fft.hip", "legendre_valu.hip", "legendre_mfma.hip", "legendre_mfma64.hip",
           "legendre_bf16.hip", "layout.hip", "reorder.hip", "resize.hip"]
# Per-source flags.  The matrix-core kernels keep their accumulators in
# ordinary VGPRs (gfx950's unified register file): with AGPR accumulators the
# compiler copies them between the two register kinds around every
# contraction phase of the analysis kernel.
EXTRA = {"legendre_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "legendre_mfma64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "legendre_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions anywhere (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, jobs=None):
    """Compile every source and link libshtx.so; always rebuilds."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        text = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l
                         and "not a recognized feature" not in l)
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text + "\n")
        elif verbose and text.strip():
            print(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
