"""Compile the HIP library for gfx950 (in-tree shared object)."""
import os
import shutil
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "eodabe.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "eodabe_kernels.hpp"), os.path.join(HERE, "csrc", "eodabe_tiles.hpp"),
        os.path.join(HERE, "csrc", "eodabe_mlp.hpp"), os.path.join(HERE, "csrc", "eodabe_apps.hpp"),
        os.path.join(ROOT, "include", "eodabe.h")]
OUT = os.path.join(HERE, "libeodabe.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # packed FP32 instructions stay off on this target (the compiler's host
    # pass warns that it does not know the feature; that is harmless)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build the EOD-ABE library)")


FAST_SRC = os.path.join(HERE, "csrc", "fastcall.c")
FAST_OUT = os.path.join(HERE, "_fastcall" + (sysconfig.get_config_var("EXT_SUFFIX") or ".so"))


def build_fastcall(verbose: bool = False) -> str:
    """Compile csrc/fastcall.c, the CPython entry for eodabe_factor (host C;
    it reaches the library through the address ctypes resolved)."""
    cc = os.environ.get("CC") or shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the CPython entry (gcc)")
    tmp = FAST_OUT + ".tmp"
    cmd = [cc, "-O2", "-shared", "-fPIC", "-I", sysconfig.get_paths()["include"], "-I", os.path.join(ROOT, "include"),
           FAST_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"C compiler failed ({res.returncode}):\n{res.stdout}{res.stderr}")
    os.replace(tmp, FAST_OUT)
    return FAST_OUT


def build(verbose: bool = False) -> str:
    """Compile csrc/eodabe.hip into libeodabe.so and the CPython entry
    (always recompiles)."""
    build_fastcall(verbose)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
