"""Build libtlrqmc.so in-tree for gfx950.

Host translation units (*.cpp) are compiled by ROCm's clang++ with OpenMP,
device translation units (*.hip) by hipcc for gfx950, and hipcc links the
shared library against the HIP runtime and rocBLAS.  Usage:
``python -m paper_2003_11183_amd.build``.
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtlrqmc.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HOST = [os.path.join(ROCM, "llvm", "bin", "clang++"), "-fopenmp", "-D__HIP_PLATFORM_AMD__",
        f"-I{os.path.join(ROCM, 'include')}"] + COMMON
# Machine-level loop-invariant code motion is off for the device code: it
# hoists every 64-bit constant of the special functions out of the sweep's
# row loop, which costs dozens of registers (and waves) for constants that
# are cheap to rematerialize with scalar moves inside the loop.
DEVICE = [os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-disable-machine-licm"] + COMMON


# Per-file device options.  The low-rank MFMA kernels and the sweep keep
# their matrix-core accumulators in ordinary VGPRs instead of AGPRs: the two
# share one register file, and the VGPR form needs fewer registers in total
# (more waves).  In the sweep it also removes the copies of the accumulators
# between AGPRs and VGPRs that the AGPR form makes at every block column.
FILE_FLAGS = {"kernels_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
              "kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in sources():
        obj = os.path.join(BUILD, src + ".o")
        cmd = (HOST if src.endswith(".cpp") else DEVICE + FILE_FLAGS.get(src, [])) + ["-c", os.path.join(CSRC, src),
                                                                             "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"compilation failed:\n{msg}")
    tmp = LIB + ".tmp"
    link = [os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-fopenmp"] + objs + [
        f"-L{os.path.join(ROCM, 'lib')}", "-lrocblas", "-lrocsolver",
        f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", f"-Wl,-rpath,{os.path.join(ROCM, 'llvm', 'lib')}",
        "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


PROBE_SRC = os.path.join(PKG, "probe", "issue_probe.hip")
PROBE = os.path.join(PKG, "probe", "issue_probe")


def build_probe(verbose: bool = False) -> str:
    """The issue probe behind bench.py's roofline model (an executable of
    its own, not part of the library): ``python bench.py --issue-probe``."""
    cmd = DEVICE + [PROBE_SRC, "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"issue probe build failed:\n{r.stdout}")
    os.replace(PROBE + ".tmp", PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
