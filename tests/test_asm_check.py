"""The build's wait-state check of the inline-asm DPP FMAs (asm_check.py) on
hand-written assembly: each hazard it guards against is caught, and the
safe forms pass."""
from paper_2607_01993_amd import asm_check

FMAC = "v_fmac_f32_dpp v1, {w}, {d} row_newbcast:0 row_mask:0xf bank_mask:0xf"


def run(tmp_path, body):
    p = tmp_path / "k.s"
    p.write_text("k:\n" + "".join(f"\t{ln}\n" if not ln.endswith(":") else f"{ln}\n" for ln in body))
    return asm_check.check(str(p))


def test_dpp_source_written_by_valu(tmp_path):
    assert len(run(tmp_path, ["v_mov_b32_e32 v5, v6", FMAC.format(w="v5", d="v2")])) == 1
    assert len(run(tmp_path, ["v_mov_b32_e32 v5, v6", "v_add_f32_e32 v9, v9, v9",
                              FMAC.format(w="v5", d="v2")])) == 1
    assert run(tmp_path, ["v_mov_b32_e32 v5, v6", "s_nop 1", FMAC.format(w="v5", d="v2")]) == []
    # loads and matrix-core writes are not vector-ALU writes of the source
    assert run(tmp_path, ["global_load_dword v5, v[2:3], off", FMAC.format(w="v5", d="v2")]) == []


def test_transcendental_result(tmp_path):
    assert len(run(tmp_path, ["v_sqrt_f32_e64 v2, |v3|", FMAC.format(w="v7", d="v2")])) == 1
    assert run(tmp_path, ["v_sqrt_f32_e64 v2, |v3|", "v_sqrt_f32_e64 v4, |v3|",
                          FMAC.format(w="v7", d="v2")]) == []
    assert run(tmp_path, ["v_sqrt_f32_e64 v2, |v3|", "s_nop 0", FMAC.format(w="v7", d="v2")]) == []


def test_register_ranges_and_branch_targets(tmp_path):
    assert len(run(tmp_path, ["v_mov_b64_e32 v[4:5], 0", FMAC.format(w="v5", d="v2")])) == 1
    # a branch target may follow any write
    assert len(run(tmp_path, [".LBB0_1:", FMAC.format(w="v8", d="v2")])) == 2
    assert run(tmp_path, [".LBB0_1:", "s_nop 1", FMAC.format(w="v8", d="v2")]) == []
