"""Compile liblob.so (the HIP library behind include/lob.h) for gfx950, in-tree."""
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblob.so")
SOURCES = [os.path.join(CSRC, "lob_kernels.hip"), os.path.join(CSRC, "lob_small.hip"),
           os.path.join(CSRC, "lob_exec.hip"), os.path.join(CSRC, "lob_unsorted.hip"),
           os.path.join(CSRC, "lob_api.cpp"), os.path.join(CSRC, "lob_serve.cpp"),
           os.path.join(CSRC, "lob_windows.cpp")]
HEADERS = [os.path.join(CSRC, "lob_internal.h"), os.path.join(CSRC, "lob_ctx.h"),
           os.path.join(CSRC, "lob_device.h"), os.path.join(CSRC, "lob_lds_engine.h"),
           os.path.join(ROOT, "include", "lob.h")]
ARCH = os.environ.get("LOB_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def command(out):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # no packed fp32 instructions anywhere (the matcher is integer-only anyway)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # the matchers branch on wave-uniform values: keep those branches as
            # scalar branches instead of structurizing them into exec-masked flow
            "-mllvm", "-structurizecfg-skip-uniform-regions=true",
            # the execution reward is float64 arithmetic in a fixed order: no fused ops
            "-ffp-contract=off",
            # block layout for the matchers' many short uniform branches: I-cache aware
            # placement and more tail duplication (more fall-through paths)
            "-mllvm", "-enable-ext-tsp-block-placement",
            "-mllvm", "-tail-dup-placement-threshold=16", "-mllvm", "-tail-dup-size=16",
            "-mllvm", "-tail-dup-placement-aggressive-threshold=16",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            # the host-only sources go in as HIP too: a "-x c++" input makes hipcc
            # drop --offload-arch for the whole command
            SOURCES[0], SOURCES[1], SOURCES[2], SOURCES[3], "-x", "hip", SOURCES[4], SOURCES[5], SOURCES[6],
            "-o", out]


def up_to_date():
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(p) <= t for p in SOURCES + HEADERS)


def code_object_archs(lib):
    """Target names of the device code objects embedded in a built library."""
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    if not os.path.exists(objdump):
        return None
    with tempfile.TemporaryDirectory() as d:
        copy = os.path.join(d, "lib.so")
        shutil.copy(lib, copy)
        subprocess.run([objdump, "--offloading", copy], cwd=d, capture_output=True, text=True)
        return sorted({f.rsplit("--", 1)[-1] for f in os.listdir(d) if "hipv4-amdgcn" in f})


def build(force=True, verbose=False):
    """Always recompiles unless force=False and the library is newer than its sources."""
    if not force and up_to_date():
        return LIB
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building liblob.so")
    archs = code_object_archs(tmp)
    if archs is not None and archs != [ARCH]:
        os.remove(tmp)
        raise RuntimeError(f"liblob.so built for {archs}, expected [{ARCH!r}]")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
