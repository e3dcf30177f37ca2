"""Build the C part of the oracle (test infrastructure only).

Compiles ``sgl_direct.c`` twice -- as double and as 80-bit long double -- into
``oracle/liboracle.so`` with gcc and OpenMP.  No fast-math: the oracle keeps
IEEE semantics.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "sgl_direct.c")
    objs = []
    for tag, extra in (("d", []), ("ld", ["-DORACLE_LONG_DOUBLE"])):
        obj = os.path.join(HERE, f"_sgl_direct_{tag}.o")
        cmd = ["gcc", "-O2", "-fPIC", "-fopenmp", "-std=c11", "-Wall", "-c", src, "-o", obj] + extra
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
