"""Build the CPU lane emulator library (tests only): the library's host source
(heget_abi.hip) and generated kernels compiled as plain C++ for x86-64 against
the host stand-in of the HIP runtime (tests/emu/hip/hip_runtime.h), with
AddressSanitizer on every access, into tests/emu/_build/libheget_emu.so.

The product sources are copied unchanged except that their empty inline-asm
optimisation barriers (register-class constraints of the GPU) are dropped,
which changes no value.  The result exports the C ABI of include/heget.h;
tests load it in a child process with the sanitizer runtime preloaded.
"""
import concurrent.futures as cf
import glob
import hashlib
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1305_0708_amd", "csrc")
OUT = os.path.join(HERE, "_build")
SRC = os.path.join(OUT, "src")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-Wno-duplicate-decl-specifier", "-Wno-unused-result", "-w", "-I"]
LIB = os.path.join(OUT, "libheget_emu.so")

_ASM = re.compile(r'asm\s+volatile\s*\(\s*""\s*:[^;]*\)\s*;')


def asan_runtime():
    """path of the sanitizer runtime to preload into the child process"""
    r = subprocess.run([CXX, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        hits = glob.glob(os.path.join(os.path.dirname(os.path.dirname(CXX)), "lib", "clang", "*", "lib", "linux",
                                      "libclang_rt.asan-x86_64.so"))
        path = hits[0] if hits else ""
    return path


def _copy(name, dst_dir, edits=()):
    with open(os.path.join(CSRC, name)) as f:
        text = f.read()
    text, _ = _ASM.subn("(void)0;", text)
    for old, new in edits:
        if old not in text:
            raise ValueError(f"{name}: edit target not found")
        text = text.replace(old, new)
    dst = os.path.join(dst_dir, os.path.basename(name))
    os.makedirs(os.path.dirname(dst), exist_ok=True)
    with open(dst, "w") as f:
        f.write(text)
    return dst


def build(processes=("gg_4g", "gg_4g_ddm", "gg_5g_ddm"), force=False, abi_edits=(), out=None, root=None):
    """compile heget_abi and the named processes' generated kernels; abi_edits
    (old, new) are applied to the copy of heget_abi.hip, out names another
    build folder for such a variant and root another source tree"""
    global OUT, SRC, LIB, ROOT, CSRC
    if out:
        OUT, SRC, LIB = out, os.path.join(out, "src"), os.path.join(out, "libheget_emu.so")
    if root:
        ROOT, CSRC = root, os.path.join(root, "paper_1305_0708_amd", "csrc")
    flags = FLAGS[:FLAGS.index("-I")] + ["-I", HERE, "-I", SRC, "-I", os.path.join(ROOT, "include")]
    sys.path.insert(0, ROOT)
    from paper_1305_0708_amd import build as hb
    hb.generate_sources()
    if force and os.path.isdir(OUT):
        shutil.rmtree(OUT)
    os.makedirs(os.path.join(SRC, "gen"), exist_ok=True)
    for name in os.listdir(CSRC):
        if name.endswith(".hpp"):
            _copy(name, SRC)
    units = [_copy("heget_abi.hip", SRC, abi_edits)] + [_copy(os.path.join("gen", f"gen_{p}.hip"), os.path.join(SRC, "gen"))
                                             for p in processes]
    units.append(os.path.join(HERE, "lane_emu.cpp"))

    def compile_one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        with open(src, "rb") as f:
            stamp = hashlib.sha256(f.read()).hexdigest() + " ".join(flags)
        stamp_file = obj + ".stamp"
        if not force and os.path.exists(obj) and os.path.exists(stamp_file) and open(stamp_file).read() == stamp:
            return obj
        cmd = [CXX] + flags + ["-x", "c++", "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"emulator build failed for {src}:\n{r.stderr[-6000:]}")
        with open(stamp_file, "w") as f:
            f.write(stamp)
        return obj

    with cf.ThreadPoolExecutor(min(8, len(units))) as ex:
        objs = list(ex.map(compile_one, units))
    subprocess.run([CXX, "-shared", "-fsanitize=address", "-o", LIB] + objs, check=True)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
