"""Builds libfftcg.so (HIP, gfx950 only) in-tree.

Every source under ``csrc/`` is compiled with hipcc for ``--offload-arch=gfx950``;
the multi-pass and fused engine sources are compiled once per grid size and
boundary condition.  Objects go to ``_build/`` at the repository root and the library
to ``paper_1305_3625_amd/libfftcg.so``.

    python -m paper_1305_3625_amd.build [--jobs N]
"""

from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfftcg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CXXFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # code objects loadable by the HIP runtime bundled with PyTorch
    "-mcode-object-version=5",
    # packed FP32 instructions stay off (hand-written or compiler-made)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    f"-I{INC}", f"-I{CSRC}",
]


def engine_radix(m: int) -> int:
    """Largest radix of the multi-pass engine on an M x M grid.  Below
    M = 4096 a pass of one solve has too little work to fill the GPU with
    radix-16 threads; smaller radices spread it over four or two times as
    many threads at the cost of more LDS exchanges.  Radix 4 up to M = 256,
    radix 8 up to M = 2048 (it keeps most of radix 4's gain on single solves
    and is the better one with many solves batched), radix 16 from M = 4096
    on.  Solves/s of padded mixed solves batched 1 / 4 / 16 / 64 at a time
    (radix 4; 8; 16): L = 256: 482/1250/1037/2048; 423/1140/1894/2517;
    330/805/1051/1958.  L = 512: 336/570/849/807; 318/557/652/860;
    251/468/588/797.  L = 2048, one solve, per product (eps 1e-3): radix 16
    95.5 us, radix 8 117.9 us."""
    return 4 if m <= 256 else (8 if m <= 2048 else 16)


ENGINE_SIZES = [(m, 0, engine_radix(m)) for m in (2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192)] + \
               [(m, 1, engine_radix(m)) for m in (4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192)]

# (M, padded, largest radix) of the fused engine: on the smallest grids
# radix-4 or radix-8 stages spread a transform over more threads, which
# shortens each thread's chain of dependent loads (per product at M = 32:
# 8.7 us with radix 4 against 19.5 us with radix 16; M = 64 periodic: 14.8 us
# with radix 8 against 27.3 us; from M = 128 on radix 16 is as fast or faster)
FUSED_SIZES = [(m, 0, 4) for m in (2, 4, 8, 16, 32)] + [(64, 0, 8), (128, 0, 16), (256, 0, 16)] + \
              [(m, 1, 4) for m in (4, 8, 16, 32, 64)] + [(128, 1, 16), (256, 1, 16)]

SOURCES = ["fftcg_host.cpp", "common.hip", "fused.hip", "server.cpp", "greens.cpp"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and
                    "target-feature" not in l)
    if p.returncode != 0:
        raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + out)
    return out


def _jobs(build_dir, extra):
    obj = lambda name: os.path.join(build_dir, name + ".o")  # noqa: E731
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        yield [HIPCC, *CXXFLAGS, *extra, *lang, "-c", src, "-o", obj(os.path.splitext(s)[0])]
    for m, pad, maxr in ENGINE_SIZES:
        yield [HIPCC, *CXXFLAGS, *extra, f"-DFFTCG_M={m}", f"-DFFTCG_PAD={pad}", f"-DFFTCG_MAXR={maxr}", "-c",
               os.path.join(CSRC, "engine_inst.hip"), "-o", obj(f"engine_{m}_{pad}")]
    for m, pad, maxr in FUSED_SIZES:
        yield [HIPCC, *CXXFLAGS, *extra, f"-DFFTCG_M={m}", f"-DFFTCG_PAD={pad}", f"-DFFTCG_MAXR={maxr}", "-c",
               os.path.join(CSRC, "fused_inst.hip"), "-o", obj(f"fused_{m}_{pad}")]


# host-side sanitizers (device code is built as usual): -Xarch_host keeps
# each flag off the gfx950 compilation
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZE_LIB = os.path.join(BUILD, "asan", "libfftcg.so")


def build(jobs: int | None = None, verbose: bool = False, extra_flags=(), lib_path: str = LIB,
          build_dir: str = BUILD, sanitize: bool = False) -> str:
    """Compiles every source (always) and links lib_path.  extra_flags are
    passed to every compile (e.g. -D switches of tuning variants).  With
    sanitize, the host code is built with AddressSanitizer and
    UndefinedBehaviorSanitizer (default output _build/asan/libfftcg.so; the
    runtime must be preloaded, see tests/test_sanitize.py)."""
    if sanitize:
        extra_flags = list(extra_flags) + SANITIZE_FLAGS
        if lib_path == LIB:
            lib_path = SANITIZE_LIB
        if build_dir == BUILD:
            build_dir = os.path.join(BUILD, "asan_obj")
        os.makedirs(os.path.dirname(lib_path), exist_ok=True)
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds = list(_jobs(build_dir, list(extra_flags)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    objs = [c[-1] for c in cmds]
    tmp = lib_path + ".tmp"
    san = ["-fsanitize=address,undefined", "-shared-libsan"] if sanitize else []
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-fPIC", *san, "-o", tmp,
          *objs, "-lpthread"])
    os.replace(tmp, lib_path)
    return lib_path


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--sanitize", action="store_true",
                    help="host code with AddressSanitizer + UBSan, into _build/asan/libfftcg.so")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose, sanitize=a.sanitize))


if __name__ == "__main__":
    sys.exit(main())
