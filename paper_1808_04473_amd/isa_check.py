"""Static check of the hand-written DPP instructions in the device assembly.

A DPP instruction reads its first source through the cross-lane DPP network.
On gfx9-family GPUs (gfx950 included) the hardware does not interlock that
read: two wait states must separate a VALU write of the VGPR from the DPP
read, and five a VALU write of EXEC from any DPP instruction; a matrix (MFMA)
result needs far more before any VALU reads it.  The compiler inserts these
for the DPP instructions it generates.  The fused row-broadcast FMACs of the
factorisation are inline assembly, so the compiler does not see their DPP
operand; this module verifies on the assembly of each build that none of
them reads a register written too recently.

Wait states are counted as the ISA does: one per instruction issued in
between, N + 1 for ``s_nop N``.  The walk back stops at a basic-block label,
where the requirement must already be met (a label can have predecessors
other than the fall-through).

    python -m paper_1808_04473_amd.isa_check <file.s> ...
"""
from __future__ import annotations

import re
import sys

DPP_SRC_WAIT = 2     # VALU writes VGPR -> DPP reads it
DPP_EXEC_WAIT = 5    # VALU writes EXEC -> any DPP instruction
MFMA_READ_WAIT = 19  # any MFMA result -> VALU read (largest pass count, conservative)

_REG = re.compile(r"^[-|]*(?:neg\()?\|?([va])(?:(\d+)|\[(\d+):(\d+)\])")


def _regs(operand: str) -> set[tuple[str, int]]:
    m = _REG.match(operand.strip())
    if not m:
        return set()
    kind = m.group(1)
    if m.group(2) is not None:
        return {(kind, int(m.group(2)))}
    return {(kind, r) for r in range(int(m.group(3)), int(m.group(4)) + 1)}


def _split(line: str) -> tuple[str, list[str]]:
    body = line.split(";")[0].strip()
    if not body:
        return "", []
    parts = body.split(None, 1)
    op = parts[0]
    if len(parts) == 1:
        return op, []
    # operands end where the first modifier (word with ':' or a bare keyword) starts
    ops = []
    for tok in parts[1].split(","):
        tok = tok.strip()
        ops.append(tok.split()[0] if tok else tok)
    return op, ops


def _wait_states(op: str, ops: list[str]) -> int:
    if op == "s_nop":
        return int(ops[0], 0) + 1 if ops else 1
    return 1


def _valu_writes(op: str, ops: list[str]) -> tuple[set[tuple[str, int]], bool]:
    """(VGPR/AGPR written, EXEC written) of a vector-ALU instruction."""
    if not op.startswith("v_") or not ops:
        return set(), False
    if op.startswith("v_cmpx"):
        return set(), True
    if op.startswith(("v_cmp", "v_readlane", "v_readfirstlane")):
        return set(), False
    return _regs(ops[0]), False


def check_lines(lines: list[str]) -> list[str]:
    """Returns one message per hazard found in the inline-assembly DPP
    instructions of the given assembly listing."""
    errors = []
    in_asm = False
    for n, raw in enumerate(lines):
        s = raw.strip()
        if s.startswith(";;#ASMSTART"):
            in_asm = True
            continue
        if s.startswith(";;#ASMEND"):
            in_asm = False
            continue
        if not in_asm:
            continue
        op, ops = _split(raw)
        if "_dpp" not in op or len(ops) < 2:
            continue
        src0 = _regs(ops[1])
        every = set()
        for o in ops[1:]:
            every |= _regs(o)
        waited = 0
        k = n - 1
        while k >= 0 and waited < MFMA_READ_WAIT:
            prev = lines[k].strip()
            if re.match(r"^[.\w]+:", prev) and not prev.startswith(";"):
                if waited < DPP_EXEC_WAIT:
                    errors.append(f"line {n + 1}: {s!r} follows block label {prev!r} "
                                  f"after only {waited} wait states")
                break
            pop, pops = _split(lines[k])
            if pop and not pop.startswith("."):
                wr, wexec = _valu_writes(pop, pops)
                if "mfma" in pop and wr & every:
                    errors.append(f"line {n + 1}: {s!r} reads an MFMA result of line {k + 1} "
                                  f"after {waited} wait states")
                elif waited < DPP_SRC_WAIT and wr & src0:
                    errors.append(f"line {n + 1}: {s!r} reads its DPP source written at line "
                                  f"{k + 1} ({prev!r}) after {waited} wait states")
                if wexec and waited < DPP_EXEC_WAIT:
                    errors.append(f"line {n + 1}: {s!r} follows an EXEC write at line {k + 1} "
                                  f"after {waited} wait states")
                waited += _wait_states(pop, pops)
            k -= 1
    return errors


def check_file(path: str) -> list[str]:
    with open(path) as f:
        return [f"{path}: {e}" for e in check_lines(f.read().split("\n"))]


def main(argv=None) -> int:
    errs = []
    for p in (argv if argv is not None else sys.argv[1:]):
        errs += check_file(p)
    for e in errs:
        print(e)
    return 1 if errs else 0


if __name__ == "__main__":
    sys.exit(main())
