"""Build the oracle's shared library with gcc (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(force: bool = True) -> str:
    out = os.path.join(HERE, "liboracle.so")
    src = os.path.join(HERE, "oracle.c")
    if (not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src)
            and os.path.exists(os.path.join(HERE, "liboracle_omp.so"))):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-Wextra", "-fPIC", "-shared", src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    # the multi-threaded enumeration of the benchmark's secondary CPU line
    out2 = os.path.join(HERE, "liboracle_omp.so")
    tmp2 = out2 + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-Wextra", "-fPIC", "-fopenmp", "-shared",
           os.path.join(HERE, "omp_enum.c"), "-o", tmp2]
    subprocess.run(cmd, check=True)
    os.replace(tmp2, out2)
    return out


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
