"""Builds the gfx950 star-stencil library in-tree.

Compiles every source under csrc/ with hipcc for gfx950 and links
paper_2002_05983_amd/libstencil_mi355x.so.  Per-radius kernels are compiled
from one source with -DSTAR_R=<r>.  Objects are compiled in parallel.

  python -m paper_2002_05983_amd.build [--asm DIR]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libstencil_mi355x.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"

# Host-only translation units and (source, defines) device units.
HOST_UNITS = ["api.cpp", "plan.cpp", "tune.cpp", "lowp.cpp", "batch.cpp", "model.cpp"]
DEVICE_UNITS = [("naive.hip", {}), ("reduce.hip", {}), ("noalloc.hip", {})] + [("star2d.hip", {"STAR_R": r}) for r in range(1, 9)]
DEVICE_UNITS += [("star3d.hip", {"STAR_R": r}) for r in range(1, 9)]
DEVICE_UNITS += [("star3d_rows.hip", {"STAR_R": r}) for r in range(1, 9)]
DEVICE_UNITS += [("lowp3d.hip", {"STAR_R": r}) for r in (1, 2, 3, 4)] + [("lowp_util.hip", {})]
DEVICE_UNITS += [(f"batch{d}d.hip", {"STAR_R": r}) for d in (2, 3) for r in (1, 2, 3, 4)]

COMMON = ["-std=c++17", "-O3", "-fPIC", "-fvisibility=hidden", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-ffp-contract=off", "-fno-gpu-rdc",
          # no packed FP32 (v_pk_*_f32) instructions: plain VALU FP32 only
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # per-kernel register and scratch use, recorded next to each object
          "-Rpass-analysis=kernel-resource-usage"]
RESOURCE_FIELDS = ("VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]")


def _record_resources(obj: str, stderr: str):
    """Writes <obj>.resources: one line per kernel, its mangled name then
    VGPRs, AGPRs, scratch bytes per lane and occupancy (waves per SIMD), from
    the compiler's kernel-resource-usage remarks."""
    rows, cur = [], None
    for line in stderr.splitlines():
        if "Function Name: " in line:
            cur = {"name": line.split("Function Name: ", 1)[1].strip()}
            rows.append(cur)
        elif cur is not None:
            for f in RESOURCE_FIELDS:
                if f + ": " in line:
                    cur[f] = (line.split(f + ": ", 1)[1].split() or ["?"])[0]
    with open(obj + ".resources", "w") as fh:
        for r in rows:
            fh.write(" ".join([r["name"]] + [r.get(f, "?") for f in RESOURCE_FIELDS]) + "\n")


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _obj_name(src: str, defs: dict) -> str:
    stem = os.path.splitext(src)[0]
    suffix = "".join(f"_{k.lower()}{v}" for k, v in sorted(defs.items()))
    return f"{stem}{suffix}.o"


def _includes(path: str, seen: set) -> set:
    """The local headers `path` includes, directly or through other headers."""
    try:
        with open(path) as fh:
            text = fh.read()
    except OSError:
        return seen
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("#include") and '"' in line:
            name = line.split('"')[1]
            for d in (CSRC, INCLUDE):
                h = os.path.join(d, name)
                if os.path.exists(h) and h not in seen:
                    seen.add(h)
                    _includes(h, seen)
                    break
    return seen


def _stale(obj: str, src: str) -> bool:
    """An object is stale when older than its source or a header it includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *_includes(src, set())])


def build(verbose: bool = False, asm_dir: str | None = None, jobs: int | None = None,
          incremental: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds = []
    for src in HOST_UNITS:
        out = os.path.join(objdir, _obj_name(src, {}))
        cmds.append([hipcc, *COMMON, "-c", os.path.join(CSRC, src), "-o", out])
    for src, defs in DEVICE_UNITS:
        out = os.path.join(objdir, _obj_name(src, defs))
        cmd = [hipcc, *COMMON, *DEVICE, *[f"-D{k}={v}" for k, v in defs.items()],
               "-c", os.path.join(CSRC, src), "-o", out]
        if asm_dir:
            os.makedirs(asm_dir, exist_ok=True)
            cmd += ["-save-temps=obj"]
        cmds.append(cmd)

    def run(cmd):
        if incremental and "-c" in cmd and not _stale(cmd[-1], cmd[cmd.index("-c") + 1]):
            return cmd[-1]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode == 0 and "-Rpass-analysis=kernel-resource-usage" in cmd:
            _record_resources(cmd[cmd.index("-o") + 1], r.stderr)
        err = "\n".join(l for l in r.stderr.splitlines()
                        if "packed-fp32-ops" not in l and l.strip() and "remark:" not in l
                        and not l.lstrip().startswith(("Function Name", "VGPRs", "AGPRs",
                                                       "ScratchSize", "Dynamic Stack",
                                                       "Occupancy", "SGPRs", "LDS Size")))
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
        if err and verbose:
            print(err, file=sys.stderr)
        return cmd[-1]

    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(run, cmds))
    if asm_dir:
        for f in os.listdir(objdir):
            if f.endswith(".s") and "gfx950" in f:
                shutil.copy(os.path.join(objdir, f), asm_dir)
    tmp = LIB_PATH + ".tmp"
    run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None, help="copy the gfx950 assembly of each unit here")
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only units older than their source or a header")
    args = ap.parse_args()
    print(build(verbose=args.verbose, asm_dir=args.asm, incremental=args.incremental))
