"""Build the oracle's shared library (plain C, gcc) in place.

Test infrastructure: compiled by the build step next to the HIP library so the
checker is ready, but only tests, the smoke check and the CPU baseline load it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def _gcc(out: str, extra, verbose: bool) -> str:
    src = os.path.join(HERE, "cmc_oracle.c")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
           "-shared", *extra, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """liboracle.so (serial: the parity reference) and liboracle_omp.so (the
    same source with OpenMP, for the CPU baseline's all-core timing)."""
    out = _gcc(os.path.join(HERE, "liboracle.so"), ["-Wno-unknown-pragmas"], verbose)
    _gcc(os.path.join(HERE, "liboracle_omp.so"), ["-fopenmp"], verbose)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
