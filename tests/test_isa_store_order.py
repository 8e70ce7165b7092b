"""The device code never issues a vector store wider than 64 bits whose data
registers a VALU instruction overwrites within the next few instructions.

On gfx950 such a 16-byte store has written the overwriting value in some
lanes (the last four of each group of sixteen): FP64 colour pairs stored
that way took the next direction's advection factor in place of A. The
kernels therefore store FP64 pairs and small state records in 8-byte pieces.
The check compiles the HIP sources to gfx950 assembly (as the library build
does) and scans every function. Register spills to scratch are 16-byte
stores of registers about to be reused, so a kernel that spills is allowed
only where the library refuses to launch it when it spills: the 64-VGPR
batch tile kernel (checked at batch creation)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1806_10589_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_10589_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
WINDOW = 12

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def _assembly(src, tmp_path):
    out = tmp_path / (os.path.basename(src) + ".s")
    # the library's own flags, less linking
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-Wall")]
    cmd = [HIPCC] + flags + ["-S", "--offload-device-only", src, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out.read_text().splitlines()


def _regs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _hazards(lines):
    """(function, kind, store, overwriting instruction) for every wide store
    whose data registers a VALU writes within WINDOW instructions."""
    instrs, func = [], None
    for line in lines:
        if re.match(r"^_Z\w+:", line):
            func = line.split(":")[0]
        s = line.strip()
        if s and not s.startswith((";", ".")) and not s.endswith(":"):
            instrs.append((func, s.split(";")[0].strip()))
    found = []
    for k, (f, s) in enumerate(instrs):
        m = re.match(r"(buffer|global|flat|scratch)_store_dwordx([34])\s", s)
        if not m:
            continue
        ops = [o.strip() for o in s.split(None, 1)[1].split(",")]
        data = _regs(ops[0] if m.group(1) == "buffer" else ops[1])
        for f2, t in instrs[k + 1:k + 1 + WINDOW]:
            op = t.split()[0]
            if op.startswith("v_") and not op.startswith(("v_cmp", "v_readfirstlane", "v_readlane")):
                if _regs(t.split()[1].rstrip(",")) & data:
                    found.append((f, m.group(1), s, t))
                    break
    return found


@pytest.mark.parametrize("src", ["engine.hip", "mlp.hip"])
def test_no_wide_store_has_its_data_overwritten_at_once(src, tmp_path):
    found = _hazards(_assembly(os.path.join(CSRC, src), tmp_path))
    direct = [h for h in found if h[1] != "scratch"]
    spills = [h for h in found if h[1] == "scratch" and "k_batch_tile8" not in h[0]]
    assert not direct, direct[:5]
    assert not spills, spills[:5]


def test_the_scan_sees_the_order_it_guards_against():
    # the order the FP64 colour step had: a 16-byte store, then a VALU
    # writing half of its data registers
    lines = ["_ZN4flbm1kEv:", "\tbuffer_store_dwordx4 v[6:9], v1, s[48:51], s20 offen nt",
             "\tv_fma_f64 v[6:7], v[2:3], s[0:1], 1.0", "\ts_endpgm"]
    assert len(_hazards(lines)) == 1
    lines[2] = "\tv_fma_f64 v[10:11], v[2:3], s[0:1], 1.0"
    assert not _hazards(lines)
    lines[1] = "\tbuffer_store_dwordx2 v[6:7], v1, s[48:51], s20 offen nt"
    lines[2] = "\tv_fma_f64 v[6:7], v[2:3], s[0:1], 1.0"
    assert not _hazards(lines)   # 8-byte stores are not affected
