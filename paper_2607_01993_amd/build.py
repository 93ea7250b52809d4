"""Build the HIP library libsilh.so for gfx950 in-tree (next to this file).

    python -m paper_2607_01993_amd.build            # or: python paper_2607_01993_amd/build.py

Every source is compiled on every call (objects go to paper_2607_01993_amd/_build/).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libsilh.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("SILH_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    # file: extra flags
    "silh_api.cpp": [],
    "silh_server.cpp": [],
    "k_index.hip": [],
    "k_phase1.hip": ["-ffp-contract=off"],
    "k_phase2_valu.hip": [],
    "k_rows.hip": [],
    "k_cohsep.hip": [],
    "silh_graph.cpp": [],
    # the sizes computed here repeat the host's floating-point steps exactly
    "k_graph.hip": ["-ffp-contract=off"],
    "silh_noalloc.hip": [],
    # MFMA results straight into VGPRs (no accumulator-register copies)
    "k_phase2_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}

# sources with instructions in inline asm whose wait states the compiler does
# not manage: their device assembly is kept from the compile and checked
# (asm_check.py); a hazard fails the build
CHECK_ASM = {"k_phase2_mfma.hip"}

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def _compile(src: str, extra) -> str:
    stem = os.path.splitext(src)[0]
    obj = os.path.join(BUILD, stem + ".o")
    # SILH_EXTRA_HIPFLAGS: extra compiler flags (tuning experiments)
    more = os.environ.get("SILH_EXTRA_HIPFLAGS", "").split()
    temps = os.path.join(BUILD, "temps_" + stem) if src in CHECK_ASM else None
    out = obj
    if temps:
        shutil.rmtree(temps, ignore_errors=True)
        os.makedirs(temps)
        out = os.path.join(temps, stem + ".o")
        more = more + ["-save-temps=obj"]
    cmd = [hipcc(), *COMMON, *extra, *more, "-c", os.path.join(CSRC, src), "-o", out]
    if src.endswith(".hip"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if temps:
        try:
            from . import asm_check
        except ImportError:  # run as a script from this directory
            import asm_check
        dev = [f for f in os.listdir(temps) if f.endswith(f"-{ARCH}.s")]
        if len(dev) != 1:
            raise RuntimeError(f"{src}: device assembly not found in {temps}")
        found = asm_check.check(os.path.join(temps, dev[0]))
        if found:
            raise RuntimeError(f"{src}: wait-state hazards in the device code:\n" + "\n".join(found[:20]))
        os.replace(out, obj)
        shutil.rmtree(temps, ignore_errors=True)
    warn = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln
                     and "unknown target feature" not in ln and ln.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False, out: str = OUT) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
