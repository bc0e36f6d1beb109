"""The ISA checks build() applies to the compiled interpreter kernels."""
import os
import re
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2507_20769_amd import build as B  # noqa: E402

MODE = "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), {}"


def _kernel(lines):
    return "\n_ZN3mvf1kE:\n" + "\n".join("\t" + l for l in lines) + "\n.Lfunc_end0:\n"


def test_mode_switch_spacing_accepts_two_instructions():
    asm = _kernel([MODE.format(0), "v_mul_f64 v[0:1], v[2:3], v[4:5]", "v_add_f64 v[0:1], v[0:1], v[6:7]",
                   MODE.format(2)])
    assert B._check_mode_switches(asm) == []


def test_mode_switch_spacing_counts_nops():
    asm = _kernel([MODE.format(0), "s_nop 1", MODE.format(2)])
    assert B._check_mode_switches(asm) == []
    asm = _kernel([MODE.format(0), "s_nop 0", MODE.format(2)])
    assert len(B._check_mode_switches(asm)) == 1


def test_mode_switch_spacing_rejects_adjacent_switches():
    asm = _kernel([MODE.format(0), "v_mul_f64 v[0:1], v[2:3], v[4:5]", "; comment", ".LBB0_1:", MODE.format(2)])
    bad = B._check_mode_switches(asm)
    assert len(bad) == 1 and "1 wait states" in bad[0]


def test_mode_switch_spacing_ignores_other_registers():
    asm = _kernel([MODE.format(0), "s_setreg_imm32_b32 hwreg(HW_REG_TRAPSTS, 0, 1), 0", "v_nop",
                   "v_mov_b32 v0, v1", MODE.format(2)])
    assert B._check_mode_switches(asm) == []


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_interpreter_kernels_pass_the_isa_checks(tmp_path):
    out = str(tmp_path / "k.s")
    r = subprocess.run([B.HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(B.CSRC, "mvf_kernels.hip"),
                        "-o", out], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    text = open(out).read()
    assert len(re.findall(r"HW_REG_MODE", text)) > 100
    assert B._check_mode_switches(text) == []
    assert B._check_slot_file(text) == []
