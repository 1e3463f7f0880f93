"""Compile the C oracle (test infrastructure) with gcc into oracle/libckks_oracle.so."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "libckks_oracle.so")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Build the oracle library; always recompiles unless force is False and it exists."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", tmp, _SRC, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


if __name__ == "__main__":
    print(build_oracle())
