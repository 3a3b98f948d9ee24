"""Build step of the HIP library (``libsplotch.so``) for gfx950.

The library is compiled in-tree with hipcc; nothing is installed.  Flags:
gfx950 only, -O3, no floating-point contraction (the kernels write their
fused multiply-adds explicitly, so every kernel evaluates a sample with
the same operations), hardware float atomics, packed-FP32 code generation
disabled, and only the C ABI exported.
"""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SOURCES = [PKG / "csrc" / "render.hip", PKG / "csrc" / "nn.hip", PKG / "csrc" / "sort.hip"]
HEADERS = [PKG / "csrc" / "device.h", PKG / "csrc" / "kernels.h", PKG / "csrc" / "ordered.h",
           PKG / "csrc" / "sort.h"]
LIB = PKG / "libsplotch.so"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-munsafe-fp-atomics", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# libraries the link needs beyond the HIP runtime (roctx ranges of the
# render stages)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> Path:
    """Compile every HIP source into ``libsplotch.so`` (always recompiles):
    one object per source, compiled in parallel, then one link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    tmp = LIB.with_name(LIB.name + ".tmp")
    inc = [f"-I{ROOT / 'include'}", f"-I{PKG / 'csrc'}"]
    with tempfile.TemporaryDirectory() as d:
        objs = [Path(d) / (src.stem + ".o") for src in SOURCES]
        cmds = [[HIPCC, *FLAGS, *inc, "-c", "-o", str(o), str(src)]
                for src, o in zip(SOURCES, objs)]
        cmds = [[a for a in c if a != "-shared"] for c in cmds]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for fut in [ex.submit(subprocess.run, c, check=True) for c in cmds]:
                fut.result()
        link = [HIPCC, *FLAGS, "-o", str(tmp), *map(str, objs), *LIBS]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
