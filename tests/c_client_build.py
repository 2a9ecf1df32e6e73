"""Compile tests/c_client.c (a plain C user of the library's C ABI) with gcc
into tests/_build/c_client, linked against the in-tree libzmc.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "c_client")
ROCM = "/opt/rocm"


def build() -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    pkg = os.path.join(ROOT, "paper_1902_07916_amd")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror",
           # the HIP runtime API header needs the platform named when the
           # compiler is not hipcc
           "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "c_client.c"), "-o", OUT,
           "-L" + pkg, "-lzmc", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1902_07916_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return OUT


if __name__ == "__main__":
    print(build())
