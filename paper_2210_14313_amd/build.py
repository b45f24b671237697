"""Build libsgmdi.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsgmdi.so")
# per-operation VALU ceiling probe (include/sgpeaks.h), a library of its own
PEAKS_LIB = os.path.join(PKG, "libsgpeaks.so")
PEAKS_SOURCE = "sg_peaks.hip"

FORWARD_UNITS = [f"sg_fwd_p{p}_{k}.hip" for p in (0, 1, 2) for k in ("k4", "k6", "k8", "g8")]
SOURCES = FORWARD_UNITS + ["sg_one_p0.hip", "sg_one_p1.hip", "sg_one_p2.hip", "sg_adj0.hip", "sg_adj1.hip", "sg_unrank.hip", "sg_points.hip",
           "sg_blocked.hip", "sg_oscq.hip", "sg_oscq_p1.hip", "sg_oscq_p2.hip", "sg_noalloc.hip", "sg_rules.cpp", "sg_counts.cpp", "sg_tuning.cpp",
           "sg_api.cpp"]

# Packed FP32 instructions are disabled for every device pass; contraction of
# a*b+c into FMAs is off so that compensated (two-sum) sequences keep their
# rounding; FMAs the kernels want are written explicitly.
# Machine-level loop-invariant code motion is off: it would hoist the
# hundreds of rule constants of the unrolled per-coordinate code out of the
# coordinate and work-queue loops into scalar registers and spill them to
# vector lanes (measured: 266 VGPRs instead of 100 for the K <= 6 kernel);
# rematerialising a constant inside the loop is one scalar move.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-disable-machine-licm",
             "-Wall", "-Werror", "-Wno-unused-function", "-Wno-unused-variable"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def host_cxx() -> str:
    for c in (os.environ.get("CXX"), shutil.which("g++"), shutil.which("c++"), shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("no host C++ compiler found")


def generate_tables(objdir: str, verbose: bool = False) -> None:
    """Write sg_tables.inc: the difference-rule records of every (rule, K)
    as C++ constants, produced by the library's own rule construction."""
    exe = os.path.join(objdir, "gen_tables")
    cmd = [host_cxx(), "-O2", "-std=c++17", "-Wall", "-Werror", "-I", INCLUDE, "-I", CSRC,
           os.path.join(CSRC, "gen_tables.cpp"),
           os.path.join(CSRC, "sg_rules.cpp"), "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compiling gen_tables failed")
    for args, name in (([], "sg_tables.inc"), (["device"], "sg_tables_dev.inc")):
        r = subprocess.run([exe] + args, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError("gen_tables failed")
        dst = os.path.join(objdir, name)
        if os.path.exists(dst) and open(dst).read() == r.stdout:
            continue   # unchanged: keep its timestamp
        tmp = dst + ".tmp"
        with open(tmp, "w") as f:
            f.write(r.stdout)
        os.replace(tmp, dst)


def build(verbose: bool = False, extra_flags=None, incremental: bool = False) -> str:
    """Compile every source and link libsgmdi.so next to this file.

    incremental=True skips objects newer than their source and every header
    (a development shortcut; the default always compiles everything)."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    generate_tables(objdir, verbose)
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith((".hpp", ".h"))]
    headers += [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE)]
    headers.append(os.path.join(objdir, "sg_tables.inc"))
    headers.append(os.path.join(objdir, "sg_tables_dev.inc"))

    peaks_header = os.path.join(INCLUDE, "sgpeaks.h")

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        deps = [peaks_header] if src == PEAKS_SOURCE else [h for h in headers if h != peaks_header]
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if all(os.path.getmtime(f) < t for f in [path] + deps):
                return obj
        cmd = [hipcc()] + HIP_FLAGS + (extra_flags or []) + ["-I", INCLUDE, "-I", CSRC, "-I", objdir, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"compiling {src} failed")
        return obj

    # the kernel units are independent: compile them in parallel
    workers = max(1, min(len(SOURCES) + 1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, SOURCES + [PEAKS_SOURCE]))
    for lib, lobjs in ((LIB, objs[:-1]), (PEAKS_LIB, objs[-1:])):
        tmp = lib + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + lobjs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"linking {os.path.basename(lib)} failed")
        os.replace(tmp, lib)
    return LIB


HOSTSAN_LIB = os.path.join(PKG, "_build", "libsgmdi_hostsan.so")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def build_host_sanitized(verbose: bool = False) -> str:
    """The host runtime (C ABI, counts, rules, plans) compiled with the host
    C++ compiler under AddressSanitizer and UndefinedBehaviorSanitizer,
    linked against a host stand-in for the HIP runtime calls and launchers
    that launch nothing (sg_host_stubs.cpp) instead of the HIP runtime.  CPU
    only; tests load it in a process that preloads the sanitizer runtimes."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(CSRC, f) for f in ("sg_api.cpp", "sg_counts.cpp", "sg_rules.cpp", "sg_tuning.cpp",
                                              "sg_host_stubs.cpp")]
    tmp = HOSTSAN_LIB + f".tmp{os.getpid()}"   # concurrent test workers each build their own
    cmd = ([host_cxx(), "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Werror", "-Wno-unused-function",
            "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE, "-I", CSRC, "-I", "/opt/rocm/include"] + SANITIZE + srcs +
           ["-Wl,--no-undefined", "-o", tmp])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compiling the sanitized host runtime failed")
    os.replace(tmp, HOSTSAN_LIB)
    return HOSTSAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
