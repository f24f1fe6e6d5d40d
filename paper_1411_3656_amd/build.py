"""Build libppf.so for gfx950 in-tree with hipcc.

Usage: python -m paper_1411_3656_amd.build [--jobs J] [--verbose]

Each source is compiled to an object in parallel, then linked into
paper_1411_3656_amd/libppf.so. Packed FP32 instructions are disabled for
all device code (-packed-fp32-ops).
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import pathlib
import shutil
import subprocess
import sys
import time

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = ROOT / "_build"
LIB = PKG / "libppf.so"

SOURCES = ["ppf_kernels.hip", "ppf_power.hip", "ppf_mfma.hip", "ppf_design.hip", "ppf_api.cpp", "ppf_server.cpp",
           "ppf_noalloc.hip", "ppf_widen.hip", "ppf_fourstep.hip"]
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libppf.so")


def _compile(src: str, verbose: bool, extra=(), bdir: pathlib.Path = BUILD) -> pathlib.Path:
    obj = bdir / (pathlib.Path(src).stem + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-x", "hip", "-c", str(CSRC / src), "-o", str(obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose:
        print(f"  {src}: {time.time() - t0:.1f}s", flush=True)
    # host-pass warnings about the packed-fp32 feature are expected noise
    return obj


def build(jobs: int = 4, verbose: bool = False, defines=(), out: pathlib.Path | None = None) -> pathlib.Path:
    """Compile and link; ``defines`` are extra -D flags, ``out`` another library path."""
    lib = pathlib.Path(out) if out else LIB
    bdir = BUILD if out is None else BUILD / lib.stem
    bdir.mkdir(parents=True, exist_ok=True)
    lib.parent.mkdir(parents=True, exist_ok=True)
    extra = [f"-D{d}" for d in defines]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, extra, bdir), SOURCES))
    tmp = lib.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link of libppf.so failed")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}", flush=True)
    if out is None:
        build_serve_bench(lib, verbose)
        build_copy_bench(verbose)
    return lib


def build_copy_bench(verbose: bool = False) -> pathlib.Path:
    """The copy yardstick of the HBM roofline (no library needed)."""
    exe = PKG / "ppf_copy_bench"
    tmp = exe.with_suffix(".tmp")
    cmd = [hipcc(), *COMMON, "-x", "hip", str(CSRC / "copy_bench.cpp"), "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build of ppf_copy_bench failed")
    os.replace(tmp, exe)
    if verbose:
        print(f"built {exe}", flush=True)
    return exe


def build_serve_bench(lib: pathlib.Path, verbose: bool = False) -> pathlib.Path:
    """The serving load generator, linked against the in-tree library."""
    exe = PKG / "ppf_serve_bench"
    tmp = exe.with_suffix(".tmp")
    cmd = [hipcc(), *COMMON, "-x", "hip", str(CSRC / "serve_bench.cpp"), "-x", "none", f"-L{lib.parent}", "-lppf",
           "-Wl,-rpath,$ORIGIN", "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build of ppf_serve_bench failed")
    os.replace(tmp, exe)
    if verbose:
        print(f"built {exe}", flush=True)
    return exe


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("-D", dest="defines", action="append", default=[], help="extra preprocessor define")
    ap.add_argument("--out", default=None, help="library path (default: in-tree libppf.so)")
    args = ap.parse_args()
    build(args.jobs, args.verbose, args.defines, args.out)


if __name__ == "__main__":
    main()
