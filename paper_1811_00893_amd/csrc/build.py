"""Build libwilson.so (HIP for gfx950) in-tree: paper_1811_00893_amd/libwilson.so.

Each source is compiled to an object in parallel, then linked with hipcc.  Packed FP32
instructions are disabled for device code (-target-feature -packed-fp32-ops).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libwilson.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["dslash.hip", "dslash_p64.hip", "dslash_p32.hip", "dslash_p16.hip", "dslash_p16l32.hip", "clover.hip", "blas.hip", "block.hip", "layout.hip", "layout_lab.hip", "runtime.cpp", "solver.cpp", "capi.cpp", "indexcheck.cpp"]
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-I", HERE, "-I", os.path.join(ROOT, "include")]
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


# the vector kernels give the same bits in both of their forms only without contraction
PER_SOURCE = {"blas.hip": ["-ffp-contract=off"]}


def resource_usage(src):
    """VGPRs and scratch bytes per lane of every kernel in one source, from the compiler's
    kernel-resource-usage remarks for the device code built with the library's flags."""
    import re
    cmd = (["hipcc", "-x", "hip"] + COMMON + DEVICE + PER_SOURCE.get(src, []) +
           ["--cuda-device-only", "-c", os.path.join(HERE, src), "-o", os.devnull,
            "-Rpass-analysis=kernel-resource-usage"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    usage, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]): (\d+)", line)
        if m and name:
            usage[name]["vgprs" if m.group(1) == "VGPRs" else "scratch"] = int(m.group(2))
    return usage


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = ["hipcc"] + lang + COMMON + DEVICE + PER_SOURCE.get(src, []) + ["-c", os.path.join(HERE, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


# The host code (runtime, solver, C ABI, index check) rebuilt with AddressSanitizer and
# UndefinedBehaviorSanitizer for the CPU tests; device code is never instrumented.
HOST_SOURCES = ["runtime.cpp", "solver.cpp", "capi.cpp", "indexcheck.cpp"]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
SAN_OUT = os.path.join(BUILD, "san", "libwilson_san.so")


def build_sanitized(verbose=False, jobs=4):
    """_build/san/libwilson_san.so: the host sources compiled with the sanitizers, linked
    with the device objects of the plain build (built first when missing).  It needs the
    sanitizer runtime preloaded (sanitizer_runtime()); only the CPU tests load it."""
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    dev_objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in dev_objs):
        build(verbose)

    def compile_san(src):
        obj = os.path.join(san, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", "-x", "hip"] + COMMON + DEVICE + SANITIZE + ["-c", os.path.join(HERE, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_san, HOST_SOURCES))
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", SAN_OUT + ".tmp"] + objs + dev_objs + SANITIZE
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_OUT + ".tmp", SAN_OUT)
    return SAN_OUT


def sanitizer_runtime():
    """The compiler's shared AddressSanitizer runtime (it carries the UndefinedBehavior
    handlers too), for LD_PRELOAD into a process that loads libwilson_san.so."""
    r = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/*/libclang_rt.asan*.so")
    return found[0] if found else None


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        build(verbose="-v" in sys.argv)
