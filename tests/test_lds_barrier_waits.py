"""Every workgroup barrier in the library's gfx950 code is preceded by a wait
for the LDS stores that may still be in flight when it is reached.

LDS requests of different waves of a workgroup are not kept in order, so a
store to LDS followed by a barrier needs `s_waitcnt lgkmcnt(0)` between
them, or another wave may read or update the word before the store lands.
The compiler places that wait when the store and the barrier are in one
straight run of code, but a store at the end of a loop body that reaches
the barrier at the top of the next iteration only through the loop's back
edge got none (a histogram loop that cleared its counters there lost
counts).  This test compiles each HIP source to gfx950 assembly and checks
both cases: in program order, and across every back edge."""
import os
import re
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2311_02206_amd import build  # noqa: E402

LDS_READS = ("ds_read", "ds_bpermute", "ds_permute", "ds_swizzle")


def lds_store(op):
    return op.startswith("ds_") and not op.startswith(LDS_READS)


def opcode(line):
    t = line.strip()
    return t.split()[0] if t and not t.startswith(";") else ""


def functions(lines):
    heads = [(i, m.group(1)) for i, l in enumerate(lines)
             if (m := re.match(r"^(_Z\S+):", l))]
    heads.append((len(lines), None))
    return [(s, e, name) for (s, name), (e, _) in zip(heads, heads[1:])]


def unwaited_barriers(lines):
    """(function, store line, barrier line) for every barrier that an LDS
    store reaches with no lgkmcnt(0) wait in between, in program order or
    from a loop's back edge to the top of the loop."""
    bad = []
    for s, e, name in functions(lines):
        pending = None
        for i in range(s, e):
            op = opcode(lines[i])
            if "lgkmcnt(0)" in lines[i]:
                pending = None
            elif lds_store(op):
                pending = i
            elif op == "s_barrier" and pending is not None:
                bad.append((name, pending + 1, i + 1))
        labels = {m.group(1): i for i in range(s, e)
                  if (m := re.match(r"^(\.LBB\w+):", lines[i]))}
        for i in range(s, e):
            op = opcode(lines[i])
            if not (op == "s_branch" or op.startswith("s_cbranch")):
                continue
            top = labels.get(lines[i].split()[-1])
            if top is None or top >= i:
                continue  # not a back edge
            store = None
            for k in range(i - 1, s, -1):
                if "lgkmcnt(0)" in lines[k]:
                    break
                if lds_store(opcode(lines[k])):
                    store = k
                    break
            if store is None:
                continue
            for k in range(top, e):
                op = opcode(lines[k])
                if "lgkmcnt(0)" in lines[k] or op == "s_endpgm":
                    break
                if op == "s_barrier":
                    bad.append((name, store + 1, k + 1))
                    break
    return bad


def test_detector_flags_a_store_behind_a_back_edge():
    """The check itself: a loop whose last instruction stores to LDS and
    whose first barrier has no wait is flagged; with the wait it is not."""
    body = ["_Z1kv:", ".LBB0_1:", "\tv_add_u32 v1, v1, v2", "\ts_barrier",
            "\tds_add_u32 v3, v4", "\ts_waitcnt lgkmcnt(0)", "\ts_barrier",
            "\tds_write_b32 v5, v6", "\ts_cbranch_scc1 .LBB0_1", "\ts_endpgm"]
    assert len(unwaited_barriers(body)) == 1
    fixed = body[:3] + ["\ts_waitcnt lgkmcnt(0)"] + body[3:]
    assert unwaited_barriers(fixed) == []
    straight = ["_Z1kv:", "\tds_write_b32 v5, v6", "\ts_barrier", "\ts_endpgm"]
    assert len(unwaited_barriers(straight)) == 1


@pytest.mark.skipif(not shutil.which(build.HIPCC) and not os.path.exists(build.HIPCC),
                    reason="hipcc not available")
def test_every_barrier_waits_for_lds_stores():
    srcs = [p for p in build.sources() if p.endswith(".hip")]
    tmp = tempfile.mkdtemp(prefix="lds_waits_")

    def assemble(src):
        out = os.path.join(tmp, os.path.basename(src) + ".s")
        cmd = [build.HIPCC, *build.FLAGS, "-I", os.path.join(ROOT, "include"),
               "--cuda-device-only", "-S", src, "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return src, out

    try:
        with ThreadPoolExecutor(min(8, len(srcs))) as ex:
            outs = list(ex.map(assemble, srcs))
        bad = []
        for src, out in outs:
            for name, st, bar in unwaited_barriers(open(out).read().split("\n")):
                bad.append(f"{os.path.basename(src)}: {name[:80]} store line {st}, barrier line {bar}")
        assert not bad, "barriers without a wait for LDS stores:\n" + "\n".join(bad[:20])
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
