"""Build step for the oracle's C code (test infrastructure only).

Compiles ``oracle/fft.c`` with gcc into ``oracle/_oracle_fft.so`` and the MGP
integrands ``oracle/mgp.c`` into ``oracle/_oracle_mgp.so``.  Only
``tests/``, the smoke check and the CPU-baseline leg of the benchmark use the
oracle; the product library never links it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fft.c")
LIB = os.path.join(HERE, "_oracle_fft.so")
SRC_MGP = os.path.join(HERE, "mgp.c")
LIB_MGP = os.path.join(HERE, "_oracle_mgp.so")


def _compile(src, lib, force):
    if not force and os.path.exists(lib):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(force=True):
    """Compile the oracle's C libraries.  With force=False existing ones are
    kept.  Returns the FFT library's path."""
    _compile(SRC_MGP, LIB_MGP, force)
    return _compile(SRC, LIB, force)


def build_mgp(force=False):
    return _compile(SRC_MGP, LIB_MGP, force)


if __name__ == "__main__":
    print(build())
