"""Build libmilrauv.so (HIP kernels for gfx950 + the C ABI host runtime)."""
import concurrent.futures as cf
import hashlib
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmilrauv.so")
SOURCES = ["env_kernels.hip", "est_kernels.hip", "learned_kernels.hip", "policy_kernels.hip",
           "pf_kernels.hip", "ppo_kernels.hip", "train_kernels.hip", "noalloc.hip", "abi.cpp",
           "learned_abi.cpp", "train_abi.cpp"]
ARCH = "gfx950"


def _flags(version: str):
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 (v_pk_*_f32) stays off: all FP32 math is scalar VALU
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # no implicit FMA contraction: fused multiply-adds are written out,
            # so every template instantiation (lane mapping) rounds identically
            "-ffp-contract=off",
            "-I", INCLUDE, "-I", CSRC, f'-DMIL_CODE_VERSION="{version}"',
            "-Wno-unused-command-line-argument"]


def code_version() -> str:
    h = hashlib.sha1()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    with open(os.path.join(INCLUDE, "mi_lrauv.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    version = code_version()
    flags = _flags(version)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    # rocBLAS and hipBLASLt serve the plain FP32 GEMMs of the networks' training form
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lrocblas", "-lhipblaslt", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
