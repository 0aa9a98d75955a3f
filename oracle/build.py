"""Build the FP64 CPU oracle (test infrastructure) with gcc.

Floating-point contraction is disabled so every product and sum is rounded
exactly as written in tsne_oracle.c.  The target is generic x86-64-v3 so the
library built here also loads on the GPU hosts' CPUs.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "tsne_oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
