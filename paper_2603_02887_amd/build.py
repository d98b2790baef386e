"""Build libnxs.so (the HIP library behind the C ABI in include/nxs.h) in-tree.

    python -m paper_2603_02887_amd.build

compiles every csrc/*.hip for gfx950 with hipcc and links
paper_2603_02887_amd/libnxs.so.  Compilation always runs (no staleness
check), so a call after a source change always rebuilds.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libnxs.so"
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed-FP32 VALU forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
]
# per-file extra flags: the tile-key recipe must not be contracted into FMAs
EXTRA = {"project.hip": ["-ffp-contract=off"]}


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def _compile(src, obj):
    cmd = [hipcc(), *COMMON, *EXTRA.get(src.name, []), "-c", str(src), "-o", str(obj)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src.name}:\n{' '.join(cmd)}\n{res.stderr}")
    return obj


def build(verbose=False):
    """Compile all HIP sources and link libnxs.so; returns its path."""
    srcs = sorted(CSRC.glob("*.hip"))
    with tempfile.TemporaryDirectory(prefix="nxs_build_") as tmp:
        objs = [Path(tmp) / (s.stem + ".o") for s in srcs]
        with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
            list(ex.map(_compile, srcs, objs))
        out_tmp = LIB.with_suffix(".so.tmp")
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}",
               *map(str, objs), "-o", str(out_tmp)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stderr}")
        os.replace(out_tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
