"""Build liboracle.so (plain C, FP64, no FMA contraction, OpenMP).
Test infrastructure: see nhdc_oracle.h."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")


def command(src, out):
    """The compiler command of the oracle library."""
    return ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared", "-I", HERE, src, "-lm", "-o", out]


def build():
    tmp = SO + ".tmp"
    cmd = command(os.path.join(HERE, "nhdc_oracle.c"), tmp)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + r.stderr)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build())
