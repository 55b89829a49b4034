"""Build the CPU oracle library (test infrastructure only).

Compiles tfs_oracle.c three times (real, complex-step and x87 extended-precision
scalar types) with gcc and links them into oracle/liboracle.so.  -ffp-contract=off keeps every product and
sum rounded separately, as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.environ.get("TFS_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))


def build(verbose: bool = False, src: str = None, lib: str = None) -> str:
    src = src or os.path.join(HERE, "tfs_oracle.c")
    lib = lib or LIB
    objs = []
    for tag, defs in (("real", []), ("cplx", ["-DORC_COMPLEX"]), ("long", ["-DORC_LONG"])):
        obj = lib + f".{tag}.o"
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-Wno-unused-function", *defs, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
