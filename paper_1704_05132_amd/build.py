"""Build the HIP library libvns.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
SOURCES = ["vns_kernels.hip", "vns_mlp.hip", "vns_runtime.hip"]
PROBE_SOURCES = ["valu_probe.hip"]   # the VALU issue-rate probe behind the pricing kernels' peak
ARCH = os.environ.get("VNS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Werror=return-type",
    # packed FP32 instructions stay off for every HIP object of the project
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs: with the accumulator-register form the scorer's MFMAs all went
    # through one accumulator and ran one after another
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
]


def _link(hipcc, objs, out, verbose):
    tmp = out.with_name(out.name + ".tmp")
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(out)


def build(verbose: bool = False, jobs: int = 2) -> Path:
    """Compile libvns.so and the issue-rate probe libvaluprobe.so; returns the path of libvns.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = PKG / "libvns.so"
    objdir = ROOT / "_build"
    objdir.mkdir(exist_ok=True)
    objs, procs = [], []
    for src in SOURCES + PROBE_SOURCES:
        obj = objdir / (Path(src).stem + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{err}")
        if err and verbose:
            print(err, file=sys.stderr)
    _link(hipcc, objs[:len(SOURCES)], out, verbose)
    _link(hipcc, objs[len(SOURCES):], PKG / "libvaluprobe.so", verbose)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
