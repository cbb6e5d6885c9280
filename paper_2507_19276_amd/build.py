"""Build libnqs.so (HIP for gfx950) in-tree: paper_2507_19276_amd/libnqs.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnqs.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["enumerate.hip", "order.hip", "nodes.hip", "psi.hip", "psi_bf16.hip", "energy.hip", "adjoint.hip", "unique.hip", "vmc.hip", "tensor_rnn.hip", "static_ws.hip",
           "runtime.cpp", "serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# MFMA accumulators in ordinary VGPRs: the epilogues read them directly
# instead of copying them out of the accumulation registers, and the kernels
# need fewer registers in total.
EXTRA = {src: ["-mllvm", "-amdgpu-mfma-vgpr-form"] for src in ("psi.hip", "psi_bf16.hip", "adjoint.hip")}


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
    bad = [src for src, p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError(f"hipcc failed for {bad}")
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
