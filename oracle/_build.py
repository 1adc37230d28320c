"""Compile the FP64 oracle (plain C) into a shared library next to its source.

Test infrastructure: the product build step compiles it too, so the oracle
exists wherever the tests run; nothing in the product path loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path():
    return os.path.join(HERE, "liboracle.so")


def build():
    src = os.path.join(HERE, "oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
