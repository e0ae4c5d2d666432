"""Build the reference oracle's shared library (test infrastructure).

The oracle is plain C compiled with gcc, FP64, without floating-point
contraction so that every operation rounds as written.
"""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: instrument with AddressSanitizer and UndefinedBehaviorSanitizer
    (load the library into a process started with libasan preloaded)."""
    srcs = sorted(glob.glob(os.path.join(HERE, "om_*.c")))
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           *san, "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
