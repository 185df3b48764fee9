"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so with the system C compiler."""
from __future__ import annotations

import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent


def build(verbose: bool = False) -> Path:
    src = HERE / "vns_oracle.c"
    out = HERE / "liboracle.so"
    tmp = HERE / "liboracle.so.tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", str(src), "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
