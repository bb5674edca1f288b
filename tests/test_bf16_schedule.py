"""The BF16 leaf-GEMM schedule keeps the MFMA operand-read (WAR) rule.

A BF16 MFMA on gfx950 (v_mfma_f32_16x16x32_bf16: 8 passes; 32x32x16: 16
passes) reads its A and B source VGPRs while it runs; an instruction that
writes one of those VGPRs must not issue until enough independent
instructions (wait states) have passed, a number that grows with the op's
passes.  A build that let a VALU move overwrite the A operand 7 issue slots
after an 8-pass MFMA returned wrong products, so every group of BF16 MFMAs
ends with 16 wait states.  This test compiles the GEMM source for gfx950
(device assembly of this repository's own code, on the CPU) and checks, for
every BF16 and split-BF16 kernel (one-leaf and quad), that no VALU instruction writes a VGPR
read as A or B by an MFMA fewer than 16 wait states after that MFMA issued.
(LDS and memory loads write their VGPRs only when the data returns, after
the LDS or memory latency: the split-BF16 leaf-32 kernel issues an LDS read
into an A register right after the MFMA that reads it, and its products
match the oracle.)"""
import os
import re
import subprocess

import pytest

from paper_1906_08148_amd import build_lib

WAIT_STATES = 16


def _regs(op):
    out = set()
    for m in re.finditer(r"\bv\[(\d+):(\d+)\]", op):
        out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    for m in re.finditer(r"\bv(\d+)\b", op):
        out.add(int(m.group(1)))
    return out


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    out = tmp_path_factory.mktemp("asm") / "k_gemm.s"
    src = os.path.join(build_lib.CSRC, "k_gemm.hip")
    cmd = [build_lib.HIPCC, *build_lib.COMMON, "--cuda-device-only", "-S", src, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"hipcc unavailable: {r.stderr[:200]}")
    return out.read_text()


def _kernels(text, prec):
    for m in re.finditer(rf"^(_ZN5spamm(?:6k_gemm|11k_gemm_quad)ILi{prec}E\w+):", text, re.M):
        end = text.index(".Lfunc_end", m.end())
        yield m.group(1), [l.strip() for l in text[m.end():end].splitlines()
                           if l.strip() and not l.strip().startswith((";", ".", "/"))]


@pytest.mark.parametrize("prec", [2, 3])  # BF16, split BF16
def test_no_write_to_mfma_sources_within_the_wait_states(asm, prec):
    kernels = list(_kernels(asm, prec))
    assert kernels, "no BF16 kernel found"
    checked = 0
    for name, ins in kernels:
        for k, l in enumerate(ins):
            if not l.startswith("v_mfma"):
                continue
            ops = l.split(None, 1)[1].split(",")
            src = _regs(ops[1]) | _regs(ops[2])
            ws = 0
            for m in ins[k + 1:]:
                # the fall-through path of a conditional branch continues in
                # line; an unconditional branch or the end leaves it
                if ws >= WAIT_STATES or m.startswith(("s_branch", "s_endpgm", "s_setpc")):
                    break
                if m.startswith("s_nop"):
                    ws += int(m.split()[1]) + 1
                    continue
                if m.startswith("v_") and not m.startswith("v_mfma"):
                    dst = _regs(m.split(None, 1)[1].split(",")[0])
                    assert not (dst & src), f"{name}: '{m}' writes a source of '{l}' after {ws} wait states"
                ws += 1
            checked += 1
    assert checked > 0
