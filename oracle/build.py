"""Build the oracle's shared library (plain gcc, no GPU code)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rfim_oracle.c")
SRC_DEDISP = os.path.join(HERE, "dedisp_oracle.c")
LIB = os.path.join(HERE, "librfim_oracle.so")


def build_mutant(n: int, out_path: str) -> str:
    """Test-only: a copy of the oracle with planted mistake number ``n``."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", f"-DORACLE_MUTANT={n}",
                           "-o", out_path, SRC, SRC_DEDISP, "-lm"])
    return out_path


def build(force: bool = True) -> str:
    newest = max(os.path.getmtime(SRC), os.path.getmtime(SRC_DEDISP))
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, SRC, SRC_DEDISP, "-lm"])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
