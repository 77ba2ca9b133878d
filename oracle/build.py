"""Build step for the oracle's C core: gcc, FP64, OpenMP, no fast-math.

Test infrastructure only (see the package docstring).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False, sanitize=False, out=None):
    """Build liboracle.so in-tree, or with sanitize=True an ASan + UBSan
    build at `out` (load it with gcc's libasan preloaded)."""
    src = os.path.join(HERE, "z2h_oracle.c")
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c11", *opt, "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-shared", "-fPIC", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
