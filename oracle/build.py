"""Compile the CPU oracle (hive_oracle.c, hash_study.c) with gcc into
libhive_oracle.so.

Test infrastructure: building the checker is not using it.  Run as
`python -m oracle.build`."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(extra_flags: list[str] | None = None, out: str | None = None) -> str:
    out = out or os.path.join(HERE, "libhive_oracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           *(extra_flags or []), os.path.join(HERE, "hive_oracle.c"), os.path.join(HERE, "hash_study.c"),
           "-o", tmp]
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
