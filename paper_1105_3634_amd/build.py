"""Build libmlb.so (HIP for gfx950) in-tree with hipcc.

Float64 step kernels and all host code are compiled without floating-point
contraction; float32 kernels allow it.  Packed-FP32 instruction selection is
disabled for every device object.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmlb.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-Wno-unused-command-line-argument",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# extra compiler flags (e.g. -D tuning macros), space separated
COMMON += os.environ.get("MLB_HIPFLAGS", "").split()

# (source, extra flags)
UNITS = [
    ("step_f64.hip", ["-ffp-contract=off"]),
    ("step_f32.hip", ["-ffp-contract=fast"]),
    ("collide_f32.hip", ["-ffp-contract=fast"]),
    ("reduce.hip", ["-ffp-contract=off"]),
    ("spectral.hip", ["-ffp-contract=fast"]),
    ("cnn.hip", ["-ffp-contract=fast"]),
    ("closure.cpp", ["-ffp-contract=off", "-x", "hip"]),
    ("tables.cpp", ["-ffp-contract=off", "-x", "hip"]),
    ("api.cpp", ["-ffp-contract=off", "-x", "hip"]),
    ("stability.cpp", ["-ffp-contract=off"]),
]


def _compile(unit, verbose):
    src, extra = unit
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
