"""Build libtt.so (HIP for gfx950) in-tree with hipcc.

Usage: ``python -m paper_1910_02371_amd.build`` or ``build()`` from Python.
Object files go to ``paper_1910_02371_amd/_build/``; the shared library is
``paper_1910_02371_amd/libtt.so``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtt.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = [
    "solve.hip", "solve_fused_f32.hip", "solve_fused_bf16.hip",
    "stream_f32.hip", "stream_bf16.hip", "stream_f64.hip",
    "index.hip", "stream_host.hip", "vec.hip", "ccd.hip", "api.cpp", "noalloc.hip",
    "pcg_loop_f32.hip", "pcg_loop_bf16.hip", "pcg_loop_f64.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for device code: the compiler must
# not form v_pk_{add,mul,fma}_f32 (the host pass warns about the feature).
COMMON = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", f"-I{INCLUDE}",
]


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose=True, jobs=None, out=LIB, build_dir=BUILD, extra=()):
    """Compile every source and link ``out``; ``extra`` adds hipcc flags
    (for example -D knobs of the kernels)."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
