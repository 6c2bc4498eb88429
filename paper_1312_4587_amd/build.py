"""Build libfftpl.so in-tree with hipcc for gfx950.

Usage: python -m paper_1312_4587_amd.build   (or build() from Python).
With FFTPL_ROCTX=1 in the environment the build (and the loader) use
libfftpl_roctx.so instead: the same library with a roctx range around every
entry point (rocprofv3 --marker-trace shows them), linked against the roctx
library; the default build has none.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROCTX = os.environ.get("FFTPL_ROCTX") == "1"
LIB = os.path.join(HERE, "libfftpl_roctx.so" if ROCTX else "libfftpl.so")
OBJDIR = os.path.join(HERE, "_build_roctx" if ROCTX else "_build")
SOURCES = ["abi.hip", "band_scatter.hip", "density.hip", "driver.hip", "exchange.hip", "spectral_fft.hip", "spectral_gemm.hip",
           "wirelength.hip"]
ARCH = os.environ.get("FFTPL_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
] + (["-DFFTPL_ROCTX"] if ROCTX else [])
ROCM_LIB = "/opt/rocm/lib"
LINK_EXTRA = ([f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}", "-lrocprofiler-sdk-roctx"]
              if ROCTX else [])


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(src):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


STAMP = LIB + ".sources"


def sources_digest():
    """SHA-1 over the library's sources and its public header."""
    import hashlib
    h = hashlib.sha1()
    paths = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
             if f.endswith((".hip", ".hpp"))]
    paths.append(os.path.join(os.path.dirname(HERE), "include", "fftpl.h"))
    for p in paths:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def is_current():
    """True when libfftpl.so exists and was built from the sources as they are."""
    if not os.path.exists(LIB) or not os.path.exists(STAMP):
        return False
    with open(STAMP) as f:
        return f.read().strip() == sources_digest()


def ensure_built(verbose=False):
    """Build libfftpl.so unless it was built from the current sources."""
    if not is_current():
        build(verbose=verbose)
    return LIB


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, *LINK_EXTRA, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(STAMP, "w") as f:
        f.write(sources_digest() + "\n")
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
