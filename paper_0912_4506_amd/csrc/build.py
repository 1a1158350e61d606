"""Builds libjacobi.so (gfx950) in-tree with hipcc.

Each translation unit is compiled in parallel and the objects are linked into
paper_0912_4506_amd/libjacobi.so.  The library links the HIP runtime by its
SONAME (libamdhip64.so.7); when PyTorch is imported first, the runtime PyTorch
already loaded is the one the library uses.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libjacobi.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["tb_plain_f64.hip", "tb_plain_f32.hip", "tb_rhs_f64.hip", "tb_rhs_f32.hip",
           "tb_trace_f64.hip", "tb_trace_f32.hip", "tb_batch_f64.hip", "tb_batch_f32.hip",
           "tb_comp_f64.hip", "tb_comp_f32.hip",
           "kernels.hip", "lbm.hip", "api.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-ffp-contract=off",
    f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", HERE,
]


def _compile(src, verbose):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *lang, "-c", os.path.join(HERE, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is noise
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{err}")
    if verbose and err.strip():
        print(err, flush=True)
    return obj


def build(verbose=False, jobs=None):
    """Compile every source and link libjacobi.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


# Host sanitizers for the host code of api.cpp (argument checks, plans):
# each -fsanitize= goes to the host pass only (device code is built as usual)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(verbose=False):
    """A copy of the library whose host code (api.cpp) is built with
    AddressSanitizer and UndefinedBehaviorSanitizer, linked from the kernel
    objects of the normal build, at _build/san/libjacobi.so.  Load it into a
    process that preloads the compiler's ASan runtime (asan_runtime())."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        if src == "api.cpp":
            continue
        obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
        if not os.path.exists(obj):
            obj = _compile(src, verbose)
        objs.append(obj)
    san_dir = os.path.join(BUILD_DIR, "san")
    os.makedirs(san_dir, exist_ok=True)
    api_obj = os.path.join(san_dir, "api.cpp.o")
    cmd = [HIPCC, *COMMON, "-g", *SANITIZE, "-c", os.path.join(HERE, "api.cpp"), "-o", api_obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling api.cpp with sanitizers failed:\n{r.stderr}")
    out = os.path.join(san_dir, "libjacobi.so")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE, *objs, api_obj, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking the sanitized library failed:\n{r.stderr}")
    return out


def asan_runtime():
    """The compiler's shared ASan runtime (to preload)."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise FileNotFoundError("clang's libclang_rt.asan-x86_64.so not found")
    return os.path.realpath(path)


if __name__ == "__main__":
    print(build_sanitized(verbose=True) if "--sanitize" in sys.argv else build(verbose="-v" in sys.argv))
