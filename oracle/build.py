"""Build the CPU oracle (test infrastructure) with the host C compiler.

``build()`` writes ``oracle/liboracle.so``; ``build(mutant="CONJ")`` writes a
copy with one planted mistake (``ORACLE_MUTANT_<name>``), which the tests use
to show that the oracle's pins catch that kind of mistake.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xeng_oracle.c")
MUTANTS = ("NIBBLE", "OFFSET", "INDEX", "CONJ", "DROP", "TLAST")
SHIFT_MUTANTS = ("SHIFT",)  # planted mistakes of the time-shifted mode only
FLAG_MUTANTS = ("FLAG",)    # planted mistakes of the flagged mode only
BEAM_MUTANTS = ("BEAMCONJ",)  # planted mistakes of the beamformer only


def lib_path(mutant: str | None = None, outdir: str | None = None, sanitize: bool = False) -> str:
    name = "liboracle.so" if not mutant else f"liboracle_mutant_{mutant.lower()}.so"
    if sanitize:
        name = name.replace(".so", "_san.so")
    return os.path.join(outdir or HERE, name)


def build(mutant: str | None = None, outdir: str | None = None, quiet: bool = True,
          sanitize: bool = False) -> str:
    """sanitize: a copy built with AddressSanitizer and UndefinedBehaviorSanitizer
    (load it with gcc's libasan preloaded, and ORACLE_LIBRARY naming it)."""
    out = lib_path(mutant, outdir, sanitize)
    cc = os.environ.get("CC", "gcc")
    cmd = [cc, "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", out + ".tmp", SRC]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-g"]
    if mutant:
        if mutant not in MUTANTS + SHIFT_MUTANTS + FLAG_MUTANTS + BEAM_MUTANTS:
            raise ValueError(f"unknown mutant {mutant}")
        cmd.insert(1, f"-DORACLE_MUTANT_{mutant}")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"oracle build failed: {' '.join(cmd)}")
    os.replace(out + ".tmp", out)
    if not quiet:
        print("built", out)
    return out


if __name__ == "__main__":
    build(quiet=False)
