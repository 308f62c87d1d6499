"""Compile the HIP solver library for gfx950 (in-tree, no JIT cache).

``python -m paper_1410_1914_amd.build`` writes ``paper_1410_1914_amd/_liblbm.so``
(and the learned warm-start library when its sources exist)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
ARCH = os.environ.get("PAPER_AMD_ARCH", "gfx950")

# packed-FP32 instructions are kept out of every code object on purpose
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", f"-I{ROOT}"]

LIBS = {
    "_liblbm.so": ["prep.cpp", "kernels.hip", "engine.hip", "charz.hip", "d3q19.hip"],
    "_libunet.so": ["unet_kernels.hip", "unet_net.hip"],
}


def _compile(out, srcs, verbose):
    cmd = ["/opt/rocm/bin/hipcc", *HIP_FLAGS, *[os.path.join(CSRC, s) for s in srcs], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False):
    built = []
    for name, srcs in LIBS.items():
        if not all(os.path.exists(os.path.join(CSRC, s)) for s in srcs):
            continue
        out = os.path.join(HERE, name)
        _compile(out, srcs, verbose)
        built.append(out)
    return built


if __name__ == "__main__":
    for p in build(verbose="-q" not in sys.argv):
        print(p)
