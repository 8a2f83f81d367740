"""Build the C part of the CPU oracle (test infrastructure) with gcc."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "fast.c")]
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-I", _HERE] + srcs + ["-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
