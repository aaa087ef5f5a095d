"""Build libtd.so (HIP kernels for gfx950 + C++ runtime + C-ABI) in-tree,
and the kernel micro-benchmark driver kbench beside it.

Every HIP source is compiled for gfx950 with packed-FP32 instruction
selection disabled; host C++ sources are compiled by the same driver.
Objects go to _build/, the library to this package directory.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = ["k_noise.hip", "k_blend.hip", "k_conv.hip", "k_conv_bf16.hip", "k_gn.hip", "k_misc.hip",
               "k_laplace.hip", "k_train.hip"]
CPP_SOURCES = ["header.cpp", "model.cpp", "api.cpp", "profile.cpp", "train.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + HIP_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), "\n".join(noise)))
    return obj, noise


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = HIP_SOURCES + CPP_SOURCES
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, noise in results:
        if verbose and noise:
            print("\n".join(noise), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    # the kernel micro-benchmark driver (profiler runs), linked against the library
    kb = os.path.join(HERE, "kbench")
    cmd = [HIPCC] + COMMON + HIP_FLAGS + [os.path.join(CSRC, "kbench.cpp"), "-o", kb + ".tmp", "-L" + HERE, "-ltd",
                                          "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("kbench build failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(kb + ".tmp", kb)
    return LIB


if __name__ == "__main__":
    print(build())
