"""Checks on the device code the build emits (CPU only: hipcc cross-compiles
the kernels to gfx950 assembly here).

Task dealing in the DTW engines must not let the compiler split a wave: a
fetch of the next task by lane 0 alone next to a lane-0 result store once
let the compiler send lanes 1-63 back round the task loop with their task
register reset to 0 while lane 0 waited outside, so they re-ran task 0
forever.  In the assembly that shows as a loop header whose first
instruction broadcasts (v_readfirstlane) a register that the code falling
into the header has just set to a constant.  Every kernel with a task loop
is checked for that shape.
"""
import os
import re
import subprocess

import pytest

from paper_1808_09617_amd import build as hipbuild


def split_deal_headers(asm: str, kernel_pattern: str):
    """{kernel: [(line, instruction)]} of loop headers of the suspicious shape."""
    out = {}
    for name in re.findall(r"^(_Z\S*" + kernel_pattern + r"\S*):", asm, re.M):  # pattern: non-capturing groups
        i = asm.index(name + ":")
        j = asm.index(".Lfunc_end", i)
        body = asm[i:j].splitlines()
        bad = []
        for n, line in enumerate(body):
            if "Loop Header" not in line:
                continue
            h = n
            while h > 0 and not body[h].startswith(".LBB"):
                h -= 1
            first = [x.strip() for x in body[n + 1:n + 8] if x.startswith("\t") and not x.strip().startswith(";")]
            if not first or not first[0].startswith("v_readfirstlane"):
                continue
            src = first[0].split(",")[-1].strip()
            before = [x.strip() for x in body[max(0, h - 25):h] if x.startswith("\t")]
            if any(re.match(r"v_mov_b32_e32 " + re.escape(src) + r", (-?\d+|s\d+)$", p) for p in before):
                bad.append((h, first[0]))
        out[name] = bad
    return out


def assembly(src_name: str, tmp_path) -> str:
    src = os.path.join(hipbuild.CSRC, src_name)
    out = os.path.join(str(tmp_path), src_name + ".s")
    cmd = [hipbuild.HIPCC, *hipbuild.CFLAGS, *hipbuild.EXTRA.get(src_name, []), "--cuda-device-only", "-S", src,
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


@pytest.mark.parametrize("src,pattern", [("search.hip", "(?:search_kernel|batch_search_kernel)"),
                                         ("dtw.hip", "dtw_(?:strip|pairs)_kernel")])
def test_task_deals_do_not_split_the_wave(src, pattern, tmp_path):
    found = split_deal_headers(assembly(src, tmp_path), pattern)
    assert len(found) >= 8, sorted(found)
    bad = {k: v for k, v in found.items() if v}
    assert not bad, bad
