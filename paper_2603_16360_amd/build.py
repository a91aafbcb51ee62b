"""Compile libvj.so (HIP for gfx950) in-tree.

Every source under csrc/ (join_inst.hip once per row type and width,
build_inst.hip once per width) is
compiled by hipcc to an object in _build/, in
parallel, then linked into paper_2603_16360_amd/libvj.so.  Packed-fp32 VALU
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build", "libvj")
LIB = os.path.join(HERE, "libvj.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-but-set-variable", "-Wno-unused-result",
          "-fno-gpu-rdc"]


# join_inst.hip is compiled once per (row type, padded width)
JOIN_WIDTHS = (32, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
JOIN_TYPES = (("f32", "float"), ("u8", "uint8_t"), ("bf16", "uint16_t"), ("f8", "vj::f8e4m3"))


def sources() -> list[tuple[str, list[str], str]]:
    """(source, extra flags, object name) for every translation unit."""
    out = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp")):
            continue
        src = os.path.join(CSRC, f)
        if f == "build_inst.hip":
            for dp in JOIN_WIDTHS:
                out.append((src, [f"-DVJ_BUILD_DP={dp}"], f"build_rows_{dp}"))
        elif f == "join_inst.hip":
            for tag, ctype in JOIN_TYPES:
                for dp in JOIN_WIDTHS:
                    fn = f"launch_join_{tag}_{dp}"
                    out.append((src, [f"-DVJ_JOIN_ELEM={ctype}", f"-DVJ_JOIN_DP={dp}",
                                      f"-DVJ_JOIN_FN={fn}"], fn))
        else:
            out.append((src, [], f))
    return out


def _compile(unit, verbose: bool) -> str:
    src, flags, name = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *COMMON, *flags, "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src} {flags}:\n{res.stderr[-6000:]}")
    if verbose and res.stderr.strip():
        print(res.stderr[-3000:], file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
