"""Build libba.so (the HIP kernels for gfx950 plus the host plan and C ABI).

    python -m paper_2506_04359_amd.build          # or __graft_entry__.build()

Compiles every time it is called.  Objects go to ``_build/`` beside this file;
the shared library lands in this package directory, where the binding loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libba.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

# gfx950 only; packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    obj = os.path.join(HERE, "_build")
    os.makedirs(obj, exist_ok=True)
    steps = [
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"),
                                                          "-o", os.path.join(obj, "kernels.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "pnp.hip"),
                                                          "-o", os.path.join(obj, "pnp.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "tri.hip"),
                                                          "-o", os.path.join(obj, "tri.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "pgo.hip"),
                                                          "-o", os.path.join(obj, "pgo.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "vi.hip"),
                                                          "-o", os.path.join(obj, "vi.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "map.hip"),
                                                          "-o", os.path.join(obj, "map.o")],
        [HIPCC, "-x", "hip"] + COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "api.cpp"),
                                                          "-o", os.path.join(obj, "api.o")],
        # the host plans are plain C++ (also built with the sanitizers by the tests)
        ["g++"] + COMMON + ["-c", os.path.join(CSRC, "plan.cpp"), "-o", os.path.join(obj, "plan.o")],
        ["g++"] + COMMON + ["-c", os.path.join(CSRC, "pgo_plan.cpp"), "-o", os.path.join(obj, "pgo_plan.o")],
    ]
    for cmd in steps:
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
    tmp = OUT + ".tmp"
    _run([HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp,
                                   os.path.join(obj, "kernels.o"), os.path.join(obj, "pnp.o"),
                                   os.path.join(obj, "tri.o"), os.path.join(obj, "pgo.o"),
                                   os.path.join(obj, "pgo_plan.o"), os.path.join(obj, "map.o"),
                                   os.path.join(obj, "vi.o"),
                                   os.path.join(obj, "api.o"),
                                   os.path.join(obj, "plan.o")])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
