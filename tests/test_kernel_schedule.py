"""The fused pre-smoothing keeps global loads in flight across its barrier.

k_pre_rr issues the next plane's global loads before each plane's barrier,
so that they overlap the plane's LDS and ALU work; on gfx950 the workgroup
barrier waits only for LDS operations (s_waitcnt lgkmcnt(0)). What undid
that overlap before was the compiler's own waits: loads behind branches
(each predicated on its lane having a task) leave the number of loads issued
after a given one unknown, so a wait for one plane's operands became a wait
for all of them (s_waitcnt vmcnt(0)) ahead of the barrier. This check
compiles k_level.hip for gfx950 to assembly (no GPU needed) and asks, for
each instantiation of the kernel, for a barrier reached with global loads
outstanding: scanning back from the s_barrier, a global load comes before
any wait on the vector-memory counter. (The kernel as it was before its
loads were issued unconditionally and one plane ahead fails it.)
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_bodies(asm, prefix):
    out = {}
    for m in re.finditer(r"^(_Z\S*?" + prefix + r"\S*?):(?:\s|$)", asm, re.M):
        name = m.group(1)
        end = asm.find(".Lfunc_end", m.end())
        out[name] = asm[m.end():end]
    return out


def barrier_with_loads_in_flight(body):
    ins = [l.strip() for l in body.splitlines()]
    ins = [l for l in ins if l and not l.startswith((";", "."))]
    for i, l in enumerate(ins):
        if not l.startswith("s_barrier"):
            continue
        for j in range(i - 1, max(i - 80, -1), -1):
            if ins[j].startswith("s_waitcnt") and "vmcnt" in ins[j]:
                break
            if ins[j].startswith(("global_load", "buffer_load")):
                return True
    return False


def test_fused_presmoothing_barrier_leaves_loads_in_flight():
    from paper_1607_00968_amd import build
    cmd = [build.HIPCC, *build.FLAGS, "--cuda-device-only", "-x", "hip", "-S",
           os.path.join(build.CSRC, "k_level.hip"), "-o", "-"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    bodies = kernel_bodies(r.stdout, "k_pre_rr")
    assert len(bodies) == 3, sorted(bodies)  # <c64,cbf,float>, <c64,c64,float>, <c128,c128,double>
    for name, body in bodies.items():
        assert body.count("s_barrier") >= 2, name
        assert barrier_with_loads_in_flight(body), name
