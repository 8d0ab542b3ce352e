"""Build the HIP library libblocktransform.so in-tree for gfx950.

Every .hip file under csrc/ is compiled with hipcc (in parallel) and linked
into paper_1604_06236_amd/libblocktransform.so.  Packed FP32 instructions are
disabled in all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libblocktransform.so")
ARCH = os.environ.get("PYTORCH_ROCM_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _headers_mtime():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(ROOT, "include", "blocktransform.h"))
    return max(os.path.getmtime(h) for h in hs)


# translation units whose kernels stage data in LDS: the test build that poisons LDS
# (-DBT_POISON_LDS, libblocktransform_poison.so) recompiles these and reuses the others
POISON_SOURCES = ("bt_fused_m01_04.hip", "bt_fused_m05_08.hip", "bt_fused_m09_12.hip",
                  "bt_fused_m13_16.hip", "bt_fused_tuned.hip", "bt_fused_half.hip", "bt_ragged.hip",
                  "bt_decimated.hip")
POISON_LIB = os.path.join(PKG, "libblocktransform_poison.so")


def _compile(src: str, force: bool, poison: bool = False) -> str:
    out_dir = os.path.join(BUILD, "poison") if poison else BUILD
    obj = os.path.join(out_dir, os.path.basename(src)[:-4] + ".o")
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(src), _headers_mtime())):
        return obj
    cmd = [HIPCC] + CFLAGS + (["-DBT_POISON_LDS"] if poison else []) + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj


def _link(objs, lib):
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + sorted(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(force: bool = True, jobs: int | None = None, verbose: bool = False,
          poison: bool = False) -> str:
    """Compile all sources (every call recompiles unless force=False) and link.  With
    `poison`, also the LDS-poisoning test library."""
    os.makedirs(os.path.join(BUILD, "poison"), exist_ok=True)
    srcs = sources()
    jobs = jobs or int(os.environ.get("MAX_JOBS", "0")) or min(8, os.cpu_count() or 4)
    work = [(s, False) for s in srcs]
    if poison:
        work += [(s, True) for s in srcs if os.path.basename(s) in POISON_SOURCES]
    # the largest translation units first
    work.sort(key=lambda w: -os.path.getsize(w[0]))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda w: (w[0], w[1], _compile(w[0], force, w[1])), work))
    _link([o for s, p, o in objs if not p], LIB)
    if verbose:
        print(f"built {LIB}")
    if poison:
        poisoned = {os.path.basename(s) for s, p, o in objs if p}
        _link([o for s, p, o in objs if p] +
              [o for s, p, o in objs if not p and os.path.basename(s) not in poisoned], POISON_LIB)
        if verbose:
            print(f"built {POISON_LIB}")
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True, poison="--poison" in sys.argv)
