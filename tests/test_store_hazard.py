"""The 16-byte buffer stores of the block-transform kernels keep their offset in a
VGPR with a zero SGPR offset, so that the compiler's hazard check separates each
store from any rewrite of its data registers.  With the offset in an SGPR the
compiler leaves no wait state (the ISA exempts that form), and on gfx950 such
stores lost data under load.  This test compiles the schedules that use 16-byte
stores to gfx950 assembly (CPU only) and checks the emitted code."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1604_06236_amd import build as BLD

STORE = re.compile(r"\s+buffer_store_(dwordx3|dwordx4)\s+v\[(\d+):(\d+)\],\s*\S+,\s*s\[\d+:\d+\],\s*(\S+)")
VWRITE = re.compile(r"\s+v_\S+\s+(?:v\[(\d+):(\d+)\]|v(\d+))")


def _instructions(asm):
    return [ln for ln in asm.split("\n") if ln.startswith("\t") and not ln.strip().startswith((";", "."))]


def _check(asm):
    """(number of >8-byte buffer stores, violations)."""
    ins = _instructions(asm)
    n, bad = 0, []
    for i, ln in enumerate(ins):
        m = STORE.match(ln)
        if not m:
            continue
        n += 1
        lo, hi, soff = int(m.group(2)), int(m.group(3)), m.group(4)
        if soff.startswith("s"):
            bad.append(("SGPR offset", ln.strip()))
        nxt = VWRITE.match(ins[i + 1]) if i + 1 < len(ins) else None
        if nxt:
            a = int(nxt.group(3) or nxt.group(1))
            b = int(nxt.group(3) or nxt.group(2))
            if a <= hi and b >= lo:
                bad.append(("data rewritten by the next instruction", ln.strip()))
    return n, bad


def test_checker_flags_the_unsafe_form():
    unsafe = ("\tbuffer_store_dwordx4 v[60:63], v137, s[48:51], s76 offen\n"
              "\tv_mul_f32_e32 v60, v89, v165\n")
    safe = ("\tbuffer_store_dwordx4 v[60:63], v64, s[48:51], 0 offen\n"
            "\ts_nop 0\n"
            "\tv_mul_f32_e32 v60, v93, v177\n")
    assert sorted(k for k, _ in _check(unsafe)[1]) == ["SGPR offset", "data rewritten by the next instruction"]
    assert _check(safe) == (1, [])


@pytest.mark.skipif(shutil.which(BLD.HIPCC) is None and not os.path.exists(BLD.HIPCC), reason="no hipcc")
def test_wide_stores_have_no_sgpr_offset(tmp_path):
    src = os.path.join(BLD.CSRC, "bt_fused_tuned.hip")
    out = tmp_path / "tuned.s"
    r = subprocess.run([BLD.HIPCC] + BLD.CFLAGS + ["--cuda-device-only", "-S", src, "-o", str(out)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    n, bad = _check(out.read_text())
    assert n > 0, "the paired schedules should emit 16-byte stores"
    assert not bad, bad[:5]
