"""Build libkrux.so (the gfx950 HIP library behind include/krux.h) in-tree.

    python -m paper_1307_3519_amd.build [--jobs N]

Every .hip/.cpp file under csrc/ is compiled with hipcc for gfx950 (packed
fp32 instructions disabled) into build objects, then linked with rocBLAS.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkrux.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]
SOURCES = ["scan_f16_diag.hip", "scan_f16_miss.hip", "scan_f16_full.hip", "scan_f16_sums.hip",
           "scan_i8_diag.hip", "scan_i8_miss.hip", "scan_i8_full.hip", "scan_i8_sums.hip",
           "scan_cand.hip", "scan_tiled_f16.hip", "scan_tiled_i8.hip", "rank.hip", "prep.hip", "scan.hip", "sort.hip", "group.hip", "multi.hip", "multi_mfma.hip", "fp64.hip", "api.cpp"]


HEADERS = [os.path.join(CSRC, h) for h in ("kx_common.h", "kx_args.h", "kx_host.h", "radix.h", "multi_common.h",
                                            "scan_kernel.h", "scan_tiled.h")] + [
    os.path.join(HERE, "..", "include", "krux.h")]


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + HEADERS + [os.path.abspath(__file__)]
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def _compile(src, force=False):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, err))
    return obj


def build(jobs=None, force=False):
    """Compile (stale objects only unless force) and link libkrux.so."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--force", action="store_true")
    args = ap.parse_args()
    print(build(args.jobs, args.force))
    sys.exit(0)
