"""The HIP sources compile (for gfx950, to assembly) without a 16-byte vector-memory
store whose data registers the next two instruction slots overwrite.

On MI355X such a store has been seen to write the overwriting value into its
first dword now and then (float64 spectra with the low word of a real part
replaced by an index computed right after the store, at random lanes; the
results of the float64 plane pass at 128 points were then not reproducible).
The library holds each such store's data for two slots (fft.hpp,
hold_store_data); this test keeps that true for every kernel the compiler
emits.  CPU only (hipcc cross-compiles).
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0809_3739_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _regs(tok):
    tok = tok.strip(",")
    m = re.match(r"[va]\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"-?v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def hazards(asm: str):
    """(kernel, store, overwriting instruction) for every dwordx3/x4 vector-memory
    store whose data registers a VALU instruction writes within two slots."""
    lines = [l.strip() for l in asm.splitlines()]
    out, fn = [], None
    for k, l in enumerate(lines):
        m = re.match(r"^(_Z\w+):", l)
        if m:
            fn = m.group(1)
        if not re.match(r"(global|buffer|flat)_store_dwordx[34]\b", l):
            continue
        toks = l.split()
        data = _regs(toks[2]) if toks[0].startswith(("global", "flat")) else _regs(toks[1])
        slots = 0
        for l2 in lines[k + 1:k + 8]:
            if not l2 or l2.startswith((";", ".")) or l2.endswith(":"):
                continue
            parts = l2.split()
            slots += 1 + (int(parts[1]) if parts[0] == "s_nop" and len(parts) > 1 else 0)
            if slots > 2:
                break
            if parts[0].startswith("v_") and len(parts) > 1 and _regs(parts[1]) & data:
                out.append((fn, l, l2))
                break
    return out


def test_scanner_finds_a_planted_overwrite():
    asm = "_Zk:\n\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], 0 offen\n\tv_sub_u32_e32 v4, 0x68, v9\n"
    assert len(hazards(asm)) == 1
    held = "_Zk:\n\tbuffer_store_dwordx4 v[4:7], v1, s[0:3], 0 offen\n\ts_nop 1\n\tv_sub_u32_e32 v4, 0x68, v9\n"
    assert hazards(held) == []


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.timeout(900)
@pytest.mark.parametrize("src", ["prop.hip", "la.hip", "wsn.hip", "noalloc.hip", "api.hip"])
def test_no_store_data_overwrite(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}", "--cuda-device-only", "-S",
           os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    h = hazards(out.read_text())
    assert not h, f"{len(h)} stores, first: {h[0]}"
