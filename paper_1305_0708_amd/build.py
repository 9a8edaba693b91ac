"""Build libheget.so for gfx950: generate the per-process kernels from their IRs,
compile every HIP translation unit with hipcc and link the shared library
in-tree (paper_1305_0708_amd/libheget.so)."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libheget.so")
ARCH = os.environ.get("HEGET_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 VALU forms are kept out of the generated code on purpose
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]

# device code only (host-side argument checks keep IEEE NaN semantics): the
# kernels' values are finite and the sign of a zero never reaches a result, so
# the compiler may drop the arithmetic on the structural zeros of fixed-helicity
# massless spinors and chiral couplings (x * 0 -> 0, x + 0 -> x); no
# reassociation is allowed, so compensated sums and the order of every other
# operation stay as written.  Every unit gets them, so that kernels sharing
# device code (the phase space) compile it alike.
GEN_FLAGS = ["-Xarch_device", "-fno-signed-zeros", "-Xarch_device", "-ffinite-math-only"]

PROCESSES = ("ee_mumu", "gg_ttbar_6f", "gg_ttbar_6f_bw", "gg_ttbar_6f_had", "ud_udhh_4b", "ud_udhhh", "ww_ww", "gg_4g", "gg_4g_ddm", "gg_5g_ddm",
             "gg_4g_cf", "gg_5g_cf", "gg_5g_split", "uu_ttg", "uu_ttgg", "uu_ttggg", "uu_ttggg_cf")


def generate_sources():
    sys.path.insert(0, ROOT)
    from paper_1305_0708_amd import codegen, processes
    os.makedirs(GEN, exist_ok=True)
    out = []
    for name in PROCESSES:
        proc = processes.by_name(name)
        out.append(codegen.generate(proc, GEN))
    return out


def _compile(src, force=False):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")] + \
        [os.path.join(os.path.dirname(CSRC), "..", "include", "heget.h")]
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
        return obj
    cmd = [HIPCC] + FLAGS + GEN_FLAGS + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(verbose=False, jobs=None, force=False):
    """Generate and compile every translation unit and link libheget.so; with
    force, recompile even objects newer than their sources."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = generate_sources() + [os.path.join(CSRC, "heget_abi.hip"), os.path.join(CSRC, "heget_server.hip"),
                                 os.path.join(CSRC, "heget_adaptive.hip")]
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, force), srcs))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
