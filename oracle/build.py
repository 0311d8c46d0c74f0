"""Build step for the oracle's C Fourier transform (test infrastructure only).

Compiles ``oracle/fft.c`` with gcc into ``oracle/_oracle_fft.so``.  Only
``tests/``, the smoke check and the CPU-baseline leg of the benchmark use the
oracle; the product library never links it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fft.c")
LIB = os.path.join(HERE, "_oracle_fft.so")


def build(force=True):
    """Compile the oracle FFT.  With force=False an existing library is kept."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
