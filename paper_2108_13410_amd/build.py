"""Build libz2h.so (HIP for gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instructions
disabled; the library links against the HIP runtime only.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libz2h.so")
ARCH = os.environ.get("Z2H_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"--offload-arch={ARCH}"]

SOURCES = ["z2h_kernels.hip", "z2h_host.cpp", "z2h_batch.cpp", "z2h_adjoint.cpp", "z2h_tune.cpp", "z2h_path.cpp",
           "z2h_krylov_kernels.hip", "z2h_krylov.cpp", "z2h_gates.hip", "z2h_circuit.cpp",
           "z2h_noalloc.cpp"]


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{r.stderr}")
    warn = [l for l in r.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
    if warn and verbose:
        print("\n".join(warn))
    return obj


# Translation units holding device code (kernels or device variables).  The
# others are host code only: the planner, launch sequences, batch and path
# engines, exact-solver host routines and gate-list builders.
DEVICE_SOURCES = ["z2h_kernels.hip", "z2h_krylov_kernels.hip", "z2h_gates.hip", "z2h_noalloc.cpp"]
HOST_SOURCES = [s for s in SOURCES if s not in DEVICE_SOURCES]
SANITIZE_DIR = os.path.join(BUILD, "sanitize")
SANITIZED_LIB = os.path.join(SANITIZE_DIR, "libz2h.so")
# AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
# (every -fsanitize= goes through -Xarch_host; no GPU code is instrumented).
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build_sanitized(verbose=False):
    """Host code of the library built with ASan and UBSan, linked with the
    device-code objects of build() (which must have run), into
    _build/sanitize/libz2h.so.  For CPU tests of the host-only entry points;
    load it with the clang ASan runtime preloaded (sanitizer_runtime())."""
    os.makedirs(SANITIZE_DIR, exist_ok=True)
    dev_objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in DEVICE_SOURCES]
    missing = [o for o in dev_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"device objects of the regular build are missing: {missing}")

    def one(src):
        obj = os.path.join(SANITIZE_DIR, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "-Wall",
               "-Wno-unused-function", *SANITIZE, "-x", "hip", "--offload-host-only", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized compile of {src} failed:\n{r.stderr}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(one, HOST_SOURCES))
    tmp = SANITIZED_LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *SANITIZE, "-Xarch_host", "-shared-libsan",
           *objs, *dev_objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SANITIZED_LIB)
    return SANITIZED_LIB


def sanitizer_runtime():
    """Path of the clang ASan runtime that must be preloaded into a process
    loading the sanitized library."""
    r = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not hits:
            raise RuntimeError("clang ASan runtime not found")
        path = hits[0]
    return path


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
