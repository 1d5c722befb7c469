"""Build the gfx950 shared library libcm.so in-tree with hipcc (and the small
accuracy probe of its FP64 elementary functions, libcm_fp64check.so)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcm.so")
SOURCES = ["api.cpp", "dg_kernels.hip", "reduce.hip", "mlp.hip", "filter.hip", "hevi.hip", "state.hip"]
CHECK_LIB = os.path.join(HERE, "libcm_fp64check.so")
CHECK_SOURCES = ["fp64_check.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-instruction accumulators in ordinary VGPRs: the fused network's
    # activations are read by vector instructions right after each product
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-command-line-argument", "-fvisibility=hidden",
]


def _compile(sources: list[str], out: str, extra: list[str] | None, verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + (extra or []) + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile every HIP/C++ source of the library for gfx950 (always
    rebuilds), and the FP64 accuracy probe.  ``extra`` adds compiler flags
    (e.g. ``-DCM_LIBM_THERMO``, library log/exp/sqrt/division in the
    thermodynamics) and ``out`` names another output file for such a
    variant; the probe is built only with the default library."""
    lib = _compile(SOURCES, out or LIB, extra, verbose)
    if out is None:
        _compile(CHECK_SOURCES, CHECK_LIB, extra, verbose)
    return lib


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--libm":
        print(build(verbose=True, extra=["-DCM_LIBM_THERMO"], out=os.path.join(HERE, "libcm_libm.so")))
    else:
        print(build(verbose=True))
