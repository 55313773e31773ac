"""Build step: generate the per-order kernels and compile libdgmax.so for gfx950.

    python -m paper_1104_4208_amd.build [--orders 1-8] [--jobs N]

Every HIP translation unit is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled (-Xclang -target-feature -Xclang -packed-fp32-ops)
and FMA contraction enabled; the shared library lands next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "generated")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdgmax.so")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-ffp-contract=fast",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


def _deps(src):
    """The source plus the generated kernel body it includes (same stem, .inc)."""
    inc = src[:-4] + ".inc"
    return [src, inc] if os.path.exists(inc) else [src]


def _compile(src, obj):
    newest = max(max(os.path.getmtime(d) for d in _deps(src)), _newest_header())
    if os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj, 0.0, ""
    t0 = time.time()
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    return obj, time.time() - t0, r.stderr


def _newest_header():
    paths = [os.path.join(CSRC, "launch.h"), os.path.join(CSRC, "dense.h"), os.path.join(HERE, "..", "include", "dgmax.h"),
             os.path.join(GEN, "frame.inc"), os.path.join(GEN, "tables.inc")]
    return max(os.path.getmtime(p) for p in paths if os.path.exists(p))


def build(orders=None, jobs=None, force=False, verbose=True):
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1104_4208_amd.gen import emit, tables

    orders = list(orders or range(1, tables.P_MAX + 1))
    units = emit.emit_all(GEN, orders)
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, "dgmax.hip"), os.path.join(CSRC, "dense.hip")] + units
    objs = [os.path.join(OBJ, os.path.basename(s).replace(".hip", ".o")) for s in srcs]
    if force:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    jobs = jobs or min(8, os.cpu_count() or 4)
    # largest orders first so the long compiles start early
    order = sorted(range(len(srcs)), key=lambda i: -sum(os.path.getsize(d) for d in _deps(srcs[i])))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, srcs[i], objs[i]): i for i in order}
        for f in cf.as_completed(futs):
            obj, dt, _ = f.result()
            if verbose and dt > 0:
                print(f"[build] {os.path.basename(obj)} {dt:.1f}s", flush=True)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr[-4000:]}")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"[build] linked {LIB}", flush=True)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--orders", default=None, help="e.g. 1-8 or 2,4,6")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args()
    orders = None
    if a.orders:
        if "-" in a.orders:
            lo, hi = a.orders.split("-")
            orders = range(int(lo), int(hi) + 1)
        else:
            orders = [int(v) for v in a.orders.split(",")]
    build(orders, a.jobs, a.force)


if __name__ == "__main__":
    main()
