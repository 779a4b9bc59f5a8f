"""Build the CPU oracle shared libraries (test infrastructure only).

The oracle is compiled with strict IEEE evaluation (no FMA contraction) so
that its arithmetic follows the source exactly.  The same sources are built
twice: liborc.so runs sequentially; liborc_omp.so adds OpenMP over the node
loops of each sub-step (the all-cores CPU baseline and the long CPU pins).
Both give identical results.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
LIB_OMP = os.path.join(HERE, "liborc_omp.so")
SOURCES = ("mdf_oracle.c", "cnn_oracle.c")
FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def sources(src_dir: str = HERE):
    return [os.path.join(src_dir, f) for f in SOURCES if os.path.exists(os.path.join(src_dir, f))]


def compile_lib(out: str, srcs, openmp: bool, verbose: bool = False) -> str:
    extra = ["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"]
    cmd = ["gcc"] + FLAGS + extra + ["-o", out + ".tmp"] + list(srcs) + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    srcs = sources()
    compile_lib(LIB, srcs, False, verbose)
    compile_lib(LIB_OMP, srcs, True, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
