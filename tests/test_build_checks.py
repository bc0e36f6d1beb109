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


def test_mode_switch_spacing_follows_loop_back_edges():
    # the switch at the loop head is two instructions after the one before the loop, but only one
    # after the switch at the end of the loop body when the branch goes back: a path the layout
    # order does not show
    asm = _kernel([MODE.format(2), "v_mov_b32 v0, v1", "v_mov_b32 v2, v3", ".LBB0_1:", MODE.format(0),
                   "v_mul_f64 v[0:1], v[2:3], v[4:5]", "v_add_f64 v[0:1], v[0:1], v[6:7]", MODE.format(2),
                   "s_cbranch_scc1 .LBB0_1", "s_endpgm"])
    bad = B._check_mode_switches(asm)
    assert len(bad) == 1 and "1 wait states" in bad[0]
    ok = _kernel([MODE.format(2), "v_mov_b32 v0, v1", "v_mov_b32 v2, v3", ".LBB0_1:", MODE.format(0),
                  "v_mul_f64 v[0:1], v[2:3], v[4:5]", "v_add_f64 v[0:1], v[0:1], v[6:7]", MODE.format(2),
                  "s_nop 0", "s_cbranch_scc1 .LBB0_1", "s_endpgm"])
    assert B._check_mode_switches(ok) == []


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("name", ["random", "mid"])
def test_generated_kernels_pass_the_mode_switch_check(tmp_path, name):
    # the run-time-compiled kernels differ per tape: compile the generated source of two tapes,
    # tangent mode and the (checkpointed) adjoint together, with the options the library gives
    # the run-time compiler, and check every switch pair on every path
    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    tape = {"random": lambda: I.random_small_tape(8, n=4, ops=120, n_con=2, con_ops=30, window=8),
            "mid": lambda: I.mid(1).tape}[name]()
    src = tmp_path / "g.hip"
    src.write_text(mvf.spec_source(tape, grad="auto", ckpt_budget=16))
    out = str(tmp_path / "g.s")
    r = subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S",
                        "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC, str(src), "-o", out],
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    text = open(out).read()
    kernels = [n for n, _ in B._kernel_bodies(text)]
    assert {"mvf_spec_bound", "mvf_spec_batch", "mvf_spec_bound_rev", "mvf_spec_batch_rev"} <= set(kernels)
    assert len(re.findall(r"HW_REG_MODE", text)) > 100
    assert B._check_mode_switches(text) == []
