"""Compiled-code check of the BOS kernels: no loop that contains a workgroup
barrier may be controlled per lane.

A loop whose continue / exit condition is lowered with lane masks
(`s_andn2_b64 exec, exec, ...` at the loop's own nesting level) lets some
lanes of a wave go round again while others wait outside it; if the loop
body holds `s_barrier`, the waiting lanes never reach the next barrier with
the rest and the workgroup can spin forever on stale shared values. The BOS
kernels keep every such loop on wave-uniform (scalar) values; this test
compiles bos.hip for gfx950 and checks the generated assembly, using the
loop structure that the compiler prints beside it.

(The contraction kernels' tile loops are lane-mask lowered too, but their
bounds are the same in every lane -- tile indices from blockIdx -- so all
lanes leave together; they are not covered here.)
"""
import os
import re
import shutil
import subprocess
from collections import defaultdict

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _functions(text):
    name, lines = None, []
    for ln in text.split("\n"):
        m = re.match(r"^(_Z\w+):", ln)
        if m:
            name, lines = m.group(1), []
        elif name is not None:
            if ln.strip().startswith(".Lfunc_end"):
                yield name, lines
                name = None
            else:
                lines.append(ln)


def lane_controlled_barrier_loops(lines):
    """[(loop header, blocks with lane-mask loop control)] for loops holding s_barrier."""
    own = defaultdict(list)       # loop header -> instructions of blocks at its own level
    children = defaultdict(set)   # loop header -> child loop headers
    cur_loop, cur_label, in_header = None, None, None
    for ln in lines:
        m = re.match(r"^\.L(BB\w+):\s*(.*)$", ln) or re.match(r"^; %bb\.(\d+):\s*(.*)$", ln)
        if m:
            cur_label = m.group(1)
            rest = m.group(2)
            hm = re.search(r"Header=(BB\w+) Depth", rest)
            cur_loop = hm.group(1) if hm else None
            in_header = None
            if "This Loop Header" in rest or "This Inner Loop Header" in rest:
                cur_loop = in_header = cur_label
            continue
        s = ln.strip()
        if s.startswith(";"):
            if in_header:
                cm = re.search(r"Child Loop (BB\w+) Depth", s)
                if cm:
                    children[in_header].add(cm.group(1))
            continue
        if s and cur_loop:
            own[cur_loop].append((cur_label, s))
    bad = []
    for h, ins in own.items():
        body = list(ins)
        for c in children[h]:
            body += own.get(c, [])
        if not any(i.startswith("s_barrier") for _, i in body):
            continue
        lanes = sorted({lab for lab, i in ins if re.match(r"s_andn2_b64\s+exec,\s*exec", i)})
        if lanes:
            bad.append((h, lanes))
    return bad


@pytest.fixture(scope="module")
def bos_asm(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    from paper_2309_03308_amd import build
    out = str(tmp_path_factory.mktemp("isa") / "bos.s")
    cmd = [build.HIPCC, *build.CFLAGS, "--cuda-device-only", "-S",
           os.path.join(build.CSRC, "bos.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def test_bos_kernels_keep_barrier_loops_uniform(bos_asm):
    kernels = [(n, l) for n, l in _functions(bos_asm) if "bos_kernel" in n]
    assert len(kernels) >= 2
    for name, lines in kernels:
        assert sum(ln.strip().startswith("s_barrier") for ln in lines) > 0
        assert lane_controlled_barrier_loops(lines) == [], name


def test_checker_flags_a_lane_controlled_barrier_loop():
    # a hand-made loop whose latch drops lanes by mask and whose body holds a barrier
    lines = """\
.LBB0_1:                                ; =>This Loop Header: Depth=1
	s_barrier
	ds_read_b32 v2, v1
	v_cmp_le_i32_e32 vcc, s4, v2
	s_or_b64 s[0:1], vcc, s[0:1]
	s_andn2_b64 exec, exec, s[0:1]
	s_cbranch_execnz .LBB0_1
; %bb.2:
	s_endpgm""".split("\n")
    assert lane_controlled_barrier_loops(lines) == [("BB0_1", ["BB0_1"])]
    scalar = [ln.replace("s_andn2_b64 exec, exec, s[0:1]", "s_cmp_lt_i32 s4, s5") for ln in lines]
    assert lane_controlled_barrier_loops(scalar) == []
