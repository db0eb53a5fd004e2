"""In-tree build of libtdbem.so with hipcc for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdbem.so")
SOURCES = ["api.hip", "k_tables.hip", "k_assemble.hip", "k_blocks.hip", "k_linalg.hip", "k_learned.hip", "k_batched.hip", "k_potential.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(verbose=False):
    """Compile every HIP source of csrc/ into libtdbem.so (always recompiles)."""
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["hipcc"] + FLAGS + srcs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-6000:])
    if verbose and res.stderr:
        print(res.stderr[-2000:])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_library(verbose=True))
