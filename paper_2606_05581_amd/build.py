"""Build libmsk.so (the HIP/gfx950 walk library) in-tree with hipcc."""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmsk.so")
SOURCES = ["walk.hip", "psd.hip", "laplace.hip", "spectral.hip", "eigen.hip", "noalloc.hip", "kelvin.hip",
           "capi.cpp", "bvh_build.cpp", "symeig_host.cpp"]
LIBS = []

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # FP64 atomics as hardware instructions
    "-munsafe-fp-atomics",
    # IEEE division / square root in FP32 (the closest-point routine relies on it)
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    # never form packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def walk_sources_sha() -> str:
    """Revision of the walk kernels: a hash of their sources. Autotuner
    results and measured traffic records are keyed by it, so that any edit
    of the kernels invalidates them."""
    h = hashlib.sha256()
    for name in ("walk.hip", "msk_internal.h", "philox.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source into `out` (default: the in-tree libmsk.so);
    `defines` are extra NAME=VALUE macros (kernel tuning constants)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    rev = ['-DMSK_WALK_SRC_SHA="%s"' % walk_sources_sha()]
    cmd = ([hipcc] + HIPCC_FLAGS + rev + ["-D" + d for d in defines] + [os.path.join(CSRC, s) for s in SOURCES] +
           LIBS + ["-o", tmp])
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-6000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
