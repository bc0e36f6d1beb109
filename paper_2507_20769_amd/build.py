"""Build the gfx950 library ``libmvf.so`` in-tree with hipcc.

Besides compiling, the build checks the device assembly of every kernel that
uses the register slot file: outside the slot-file inline asm the compiler
must not touch VGPRs at or above the slot-file base (an SGPR spill lane or any
other allocation there would corrupt interpreter state).
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmvf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["mvf_kernels.hip", "mvf_tape.cpp", "mvf_api.cpp", "mvf_bnb.cpp"]
DEVICE_SOURCES = ["mvf_kernels.hip"]
SLOT_BASE = 128
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17",
    "-ffp-contract=off",                                   # no contraction in round-to-nearest code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # loop-invariant code motion on machine code hoists constants (the exp/log
    # coefficients) and argument values out of the interpreter loops and keeps
    # them in SGPRs there; rematerialising them where used spills far less
    "-mllvm", "-disable-machine-licm",
    # branches on wave-uniform values (operand kinds, opcodes) stay plain scalar
    # branches instead of being restructured with execution-mask flow blocks
    "-mllvm", "-structurizecfg-skip-uniform-regions",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _check_slot_file(asm_text: str) -> list:
    problems = []
    for name, body in re.findall(r"\n(_Z\w+):(.*?)\.Lfunc_end", asm_text, flags=re.S):
        if "gpr_idx" not in body:
            continue
        outside = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", body, flags=re.S)
        for line in outside.split("\n"):
            code = line.split(";")[0]
            if any(int(v) >= SLOT_BASE for v in re.findall(r"\bv\[?(\d+)", code)):
                problems.append(f"{name}: {code.strip()}")
                break
    return problems


def build(verbose: bool = False, resource_report: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-fPIC", "-shared", *srcs, "-o", tmp]
    if resource_report:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmvf.so")
    if resource_report:
        sys.stderr.write(res.stderr)
    with tempfile.TemporaryDirectory() as td:
        for src in DEVICE_SOURCES:
            out = os.path.join(td, src + ".s")
            r = subprocess.run([HIPCC, *FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out],
                               capture_output=True, text=True)
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
                raise RuntimeError("hipcc -S failed")
            bad = _check_slot_file(open(out).read())
            if bad:
                os.unlink(tmp)
                raise RuntimeError("compiler-allocated VGPRs inside the slot file:\n" + "\n".join(bad))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_report="--resources" in sys.argv)
