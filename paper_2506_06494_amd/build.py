"""Builds libjgs2.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjgs2.so")
SOURCES = ["solver.hip", "sweep.hip", "precompute.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # packed FP32 instructions are disabled for all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


BOUNDS_LIB = os.path.join(HERE, "libjgs2_bounds.so")


def build(verbose=False, bounds=False):
    """libjgs2.so, or with bounds=True libjgs2_bounds.so: the same sources
    with JGS2_BOUNDS_CHECK (index checks in the sweep kernels)."""
    lib = BOUNDS_LIB if bounds else LIB
    extra = ["-DJGS2_BOUNDS_CHECK"] if bounds else []
    suffix = ".bounds.o" if bounds else ".o"
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", suffix))
        cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0 or (verbose and out):
            sys.stdout.write(out.decode(errors="replace"))
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = lib + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lrocprofiler-sdk-roctx", "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


# Host-side sanitisers only (device code is built as usual): each -fsanitize
# goes right after -Xarch_host, so only the host pass is instrumented.
SAN_HOST = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined").split()
SAN_LIB = os.path.join(HERE, "libjgs2_san.so")
SAN_DRIVER = os.path.join(HERE, "abi_driver_san")


def build_sanitized(verbose=False):
    """libjgs2_san.so (host code under AddressSanitizer and UBSan) and the
    C driver tests/abi_driver.c linked against it."""
    root = os.path.dirname(HERE)
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".san.o"))
        cmd = ["hipcc", *FLAGS, *SAN_HOST, "-g", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *SAN_HOST, *objs, "-lrocprofiler-sdk-roctx",
           "-shared-libsan", "-o", SAN_LIB]
    subprocess.check_call(cmd)
    clang = "/opt/rocm/llvm/bin/clang"
    rt = os.path.dirname(subprocess.check_output(  # directory of the sanitiser runtimes
        [clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip())
    cmd = [clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-shared-libsan",
           "-I", os.path.join(root, "include"), os.path.join(root, "tests", "abi_driver.c"), SAN_LIB,
           "-Wl,-rpath," + HERE, "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath," + rt, "-lm", "-o", SAN_DRIVER]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return SAN_DRIVER


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose=True))
    elif "--bounds" in sys.argv:
        print(build(verbose=True, bounds=True))
    else:
        print(build(verbose=True))
