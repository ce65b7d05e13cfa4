"""Build the CPU oracle (plain C, gcc) into a shared library.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg load the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(out_path=LIB, defines=(), opt="-O2"):
    """Compile oracle.c with gcc; `defines` plants mistakes for pin tests."""
    cmd = ["gcc", opt, "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread", SRC, "-o", out_path]
    cmd += ["-D" + d for d in defines]
    subprocess.run(cmd, check=True)
    return out_path


if __name__ == "__main__":
    print(build())
