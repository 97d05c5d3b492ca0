"""Build the gfx950 HIP library ``libtplbm.so`` in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instructions
disabled.  The device assembly of each HIP source is also generated and
scanned by asm_check.py, which rejects scalar-memory writes of any kind.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtplbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-I", CSRC, "-I", os.path.join(ROOT, "include")]

SOURCES = ["d2q9.hip", "d2q9_march.hip", "layer_ref.hip", "stream_copy.hip", "tplbm_host.cpp"]
EXTRA_SOURCES = ["d1q3_batch.hip", "batch_noalloc.hip", "d3q19.hip", "d3q19_march.hip", "net.hip", "batch_host.cpp", "net_host.cpp", "theory_host.cpp"]


def _asm_scanner():
    import importlib.util

    spec = importlib.util.spec_from_file_location("tplbm_asm_check", os.path.join(HERE, "asm_check.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.scan


def _sources():
    out = []
    for s in SOURCES + EXTRA_SOURCES:
        if os.path.exists(os.path.join(CSRC, s)):
            out.append(s)
    return out


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", *COMMON, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    if src.endswith(".hip"):
        asm = os.path.join(BUILD, src + ".gfx950.s")
        r = subprocess.run([HIPCC, *COMMON, "--cuda-device-only", "-S", path, "-o", asm],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"device assembly of {src} failed:\n{r.stderr}")
        with open(asm) as fh:
            bad = _asm_scanner()(fh.read())
        if bad:
            raise RuntimeError(f"{src}: scalar-memory write instructions in device code: {set(bad)}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {', '.join(srcs)}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
