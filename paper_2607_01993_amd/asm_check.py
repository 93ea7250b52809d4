"""Build-time check of the wait states around the DPP FMAs written as inline
asm in k_phase2_mfma.hip.

The compiler inserts the wait states a hazard needs for the instructions it
emits itself, but not for those inside an asm statement.  Two hazards apply to
`v_fmac_f32_dpp` on gfx950:

* a DPP source VGPR written by a vector-ALU instruction needs two wait states
  before the DPP instruction reads it;
* the result of a transcendental vector-ALU instruction (`v_sqrt_f32` here)
  needs one wait state before a non-transcendental instruction reads it.

`check(path)` reads the device assembly of a build and reports every
`v_fmac_f32_dpp` whose sources were written too recently.  Each instruction
counts as one wait state and `s_nop N` as N + 1; a branch target counts as
written by an unknown transcendental instruction immediately before (any
predecessor may have written any register).
"""
from __future__ import annotations

import re
import sys

_TRANS = ("v_sqrt_", "v_rsq_", "v_rcp_", "v_exp_", "v_log_", "v_sin_", "v_cos_")
_ALL = frozenset(range(512))


def _vregs(tok: str) -> frozenset:
    tok = tok.strip("|-")
    m = re.fullmatch(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return frozenset(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.fullmatch(r"v(\d+)", tok)
    return frozenset({int(m.group(1))}) if m else frozenset()


def check(path: str) -> list[str]:
    """Return one message per hazard found in the assembly file at path."""
    found = []
    fn = "?"
    # recent instructions: (is_valu, is_trans, registers written, wait states)
    hist: list[tuple[bool, bool, frozenset, int]] = []
    with open(path) as f:
        for raw in f:
            line = raw.split(";")[0].strip()
            if not line:
                continue
            if line.endswith(":"):
                if line.startswith(".LBB"):
                    hist.append((True, True, _ALL, 1))
                elif not line.startswith("."):
                    fn, hist = line[:-1], []
                continue
            if line.startswith("."):
                continue
            parts = line.replace(",", " ").split()
            op = parts[0]
            if op == "s_nop":
                hist.append((False, False, frozenset(), int(parts[1], 0) + 1))
                continue
            if op.startswith("v_fmac_f32_dpp"):
                src0, src1 = _vregs(parts[2]), _vregs(parts[3])
                ws = 0
                for valu, trans, dst, w in reversed(hist):
                    if valu and (src0 & dst) and ws < 2:
                        found.append(f"{fn}: {line}: DPP source written {ws} wait states before")
                    if trans and ((src0 | src1) & dst) and ws < 1:
                        found.append(f"{fn}: {line}: transcendental result read {ws} wait states after")
                    ws += w
                    if ws >= 2:
                        break
            valu = op.startswith("v_") and not op.startswith("v_mfma")
            dst = _vregs(parts[1]) if valu and len(parts) > 1 else frozenset()
            hist.append((valu, op.startswith(_TRANS), dst, 1))
            del hist[:-8]
    return found


if __name__ == "__main__":
    msgs = check(sys.argv[1])
    print("\n".join(msgs) if msgs else "no hazards")
    sys.exit(1 if msgs else 0)
