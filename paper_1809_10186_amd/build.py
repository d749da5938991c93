"""Build libqcoll.so (all HIP sources in csrc/) for gfx950 with hipcc, in-tree.

Usage: python -m paper_1809_10186_amd.build  [--jobs J]
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqcoll.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed-FP32 instructions out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def compile_one(src):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


# Host-sanitized self-check (tests/host_check): the sources whose host code
# is the validation layer, the plan precompute, the autotune cache and the
# group / 1-D driver set-up are recompiled with AddressSanitizer and
# UndefinedBehaviorSanitizer on their host code only (device code is never
# built with a sanitizer); the kernel-heavy sources reuse the objects of
# build().  The driver is linked by clang++, which brings the sanitizer runtimes.
HOST_CHECK_SOURCES = ("qcoll_api.hip", "qcoll_plan.hip", "qcoll_group.hip", "qcoll_dg1d.hip", "qcoll_timing.hip",
                      "qcoll_noalloc.hip", "qcoll_dg.hip")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
HOST_CHECK_DIR = os.path.join(ROOT, "tests", "host_check")
HOST_CHECK_BIN = os.path.join(HOST_CHECK_DIR, "qcoll_host_check")
CLANGXX = os.environ.get("QCOLL_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def build_host_check(jobs=None):
    san = os.path.join(OBJ, "san")
    os.makedirs(san, exist_ok=True)

    def one(args):
        src, obj = args
        r = subprocess.run([HIPCC, *FLAGS, *SAN_FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (host sanitizers) failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    jobs_list = [(os.path.join(CSRC, f), os.path.join(san, f[:-4] + ".o")) for f in HOST_CHECK_SOURCES]
    jobs_list.append((os.path.join(HOST_CHECK_DIR, "qcoll_host_check.cpp"), os.path.join(san, "driver.o")))
    with ThreadPoolExecutor(jobs or min(len(jobs_list), os.cpu_count() or 4)) as ex:
        san_objs = list(ex.map(one, jobs_list))
    plain = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in sources()
             if os.path.basename(s) not in HOST_CHECK_SOURCES]
    for o in plain:
        if not os.path.exists(o):
            raise RuntimeError(f"{o} is missing: run build() first")
    cmd = [CLANGXX, "-fsanitize=address,undefined", "-o", HOST_CHECK_BIN + ".tmp", *san_objs, *plain,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host-check link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(HOST_CHECK_BIN + ".tmp", HOST_CHECK_BIN)
    return HOST_CHECK_BIN


if __name__ == "__main__":
    j = None
    if "--jobs" in sys.argv:
        j = int(sys.argv[sys.argv.index("--jobs") + 1])
    print(build(j))
    if "--host-check" in sys.argv:
        print(build_host_check(j))
