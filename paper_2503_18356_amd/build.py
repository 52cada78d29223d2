"""Build librac.so (host C++ with g++, HIP kernels with hipcc for gfx950)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librac.so")

HOST_SRC = ["topology.cpp", "sampler.cpp"]
HIP_SRC = ["solver.hip", "sampler_device.hip", "kernels_f32_ss.hip", "kernels_f32_ts.hip", "kernels_f64_ss.hip",
           "kernels_f64_ts.hip", "kernels_f32_serve.hip", "server.hip", "kernels_f32_ss_tsit5.hip",
           "kernels_f32_ts_tsit5.hip", "kernels_f64_ss_tsit5.hip", "kernels_f64_ts_tsit5.hip",
           "postproc.hip", "ising.hip", "ceilings.hip", "kernels_f64_realn.hip",
           "kernels_f64_realn_tsit5.hip"]
# Packed FP32 instructions are kept out of every HIP object.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    cmds = []
    objs = []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SRC:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["hipcc", *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 1)) as ex:
        for r in ex.map(_run, cmds):
            if verbose and r.stderr:
                print(r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    build_c_demo()
    return LIB


C_DEMO_SRC = os.path.join(ROOT, "tests", "c_abi_demo.c")
C_DEMO = os.path.join(ROOT, "tests", "c_abi_demo")


def build_c_demo() -> str:
    """The plain C caller of the ABI that the tests run: C99 with gcc, the HIP
    runtime's C API and librac.so, found next to it at run time."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = C_DEMO + ".tmp"
    _run(["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
          "-I", INCLUDE, C_DEMO_SRC, "-L", HERE, "-lrac", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath,$ORIGIN/../paper_2503_18356_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"),
          "-o", tmp])
    os.replace(tmp, C_DEMO)
    return C_DEMO


if __name__ == "__main__":
    t = __import__("time").time()
    print(build(verbose="-v" in sys.argv), f"{__import__('time').time() - t:.1f}s")
