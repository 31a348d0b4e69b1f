"""Build the multi-threaded CPU ruling-set baseline (plain C, gcc) into
cpu_baseline/libcpurs.so."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    out = os.path.join(HERE, "libcpurs.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
           os.path.join(HERE, "ruling_set.c"), "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
