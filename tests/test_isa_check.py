"""The static DPP-hazard check that the build runs on the device assembly:
planted hazards in small listings are found, safe listings pass, and the
assembly of the current build (when present) is clean."""
import glob
import os

import pytest

from paper_1808_04473_amd import build, isa_check

FMAC = "\tv_fmac_f32_dpp v5, -v1, v2 row_newbcast:3 row_mask:0xf bank_mask:0xf"


def asm(*body):
    return ["_Z1kv:", *body]


def inline(*body):
    return ["\t;;#ASMSTART", *body, "\t;;#ASMEND"]


def test_source_written_just_before_is_a_hazard():
    errs = isa_check.check_lines(asm("\tv_mov_b32_e32 v9, 0", "\ts_nop 4", "\tv_add_f32_e32 v1, v3, v4",
                                     *inline(FMAC)))
    assert len(errs) == 1 and "DPP source" in errs[0]


def test_two_wait_states_clear_the_source_hazard():
    for sep in (["\ts_nop 1"], ["\tv_mov_b32_e32 v7, v8", "\tv_mov_b32_e32 v9, v8"]):
        lines = asm("\ts_nop 4", "\tv_add_f32_e32 v1, v3, v4", *sep, *inline(FMAC))
        assert isa_check.check_lines(lines) == [], sep


def test_one_wait_state_is_not_enough():
    lines = asm("\ts_nop 4", "\tv_add_f32_e32 v1, v3, v4", "\ts_nop 0", *inline(FMAC))
    assert len(isa_check.check_lines(lines)) == 1


def test_register_ranges_and_modifiers():
    lines = asm("\ts_nop 4", "\tv_pk_mov_b32 v[0:1], v[4:5], v[4:5] op_sel:[0,1]",
                *inline("\tv_fmac_f32_dpp v5, |v1|, v2 row_newbcast:3 row_mask:0xf bank_mask:0xf"))
    assert len(isa_check.check_lines(lines)) == 1
    # a write of the accumulator or of src1 is not a DPP-source hazard
    lines = asm("\ts_nop 4", "\tv_add_f32_e32 v2, v3, v4", "\tv_add_f32_e32 v5, v3, v4", *inline(FMAC))
    assert isa_check.check_lines(lines) == []


def test_exec_write_needs_five_wait_states():
    lines = asm("\tv_cmpx_gt_f32_e32 vcc, 0, v3", "\ts_nop 2", *inline(FMAC))
    assert any("EXEC" in e for e in isa_check.check_lines(lines))
    lines = asm("\tv_cmpx_gt_f32_e32 vcc, 0, v3", "\ts_nop 4", *inline(FMAC))
    assert isa_check.check_lines(lines) == []


def test_block_label_without_wait_states():
    lines = asm("\ts_nop 4", ".LBB0_3:", *inline(FMAC))
    assert any("label" in e for e in isa_check.check_lines(lines))
    lines = asm(".LBB0_3:", *inline("\ts_nop 4", FMAC))
    assert isa_check.check_lines(lines) == []


def test_mfma_result_read():
    lines = asm("\tv_mfma_f32_16x16x4_f32 v[0:3], v8, v9, v[0:3]", "\ts_nop 7",
                *inline("\tv_fmac_f32_dpp v5, -v1, v2 row_newbcast:3 row_mask:0xf bank_mask:0xf"))
    assert any("MFMA" in e for e in isa_check.check_lines(lines))


def test_compiler_generated_dpp_is_not_checked():
    # the compiler inserts its own wait states; only inline assembly is checked
    lines = asm("\tv_add_f32_e32 v1, v3, v4",
                "\tv_mov_b32_dpp v7, v1 row_newbcast:3 row_mask:0xf bank_mask:0xf")
    assert isa_check.check_lines(lines) == []


def test_built_device_assembly_is_clean():
    files = [build.device_asm(s) for s in build.sources() if s.endswith(".hip")]
    files = [f for f in files if os.path.exists(f)]
    if not files:
        pytest.skip("no device assembly in the build folder (run python -m paper_1808_04473_amd.build)")
    for f in files:
        assert isa_check.check_file(f) == []
    # the factorisation's fused broadcasts are present in the forward kernels
    fwd = [f for f in files if "eq_forward" in f]
    assert fwd and "v_fmac_f32_dpp" in open(fwd[0]).read()
