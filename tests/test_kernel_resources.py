"""No kernel of the library uses per-lane private (scratch) memory.

A kernel with a private segment needs scratch space reserved for every lane
of every wave the queue can hold; with one stream per instance (concurrent
batches), several queues each reserve it, and a kernel with about 22 KB per
lane once made a batched solve fail at dispatch with
HSA_STATUS_ERROR_OUT_OF_RESOURCES. This check compiles every HIP source for
gfx950 with the compiler's kernel-resource-usage remarks (no GPU needed)
and fails on any kernel that reports a non-zero ScratchSize or a dynamic
stack.
"""
import concurrent.futures as cf
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def resource_remarks(src):
    from paper_1607_00968_amd import build
    cmd = [build.HIPCC, *build.FLAGS, "--cuda-device-only", "-x", "hip", "-c", os.path.join(build.CSRC, src),
           "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    kernels, cur = {}, None
    for ln in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", ln)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+(ScratchSize \[bytes/lane\]|Dynamic Stack): (\S+)", ln)
        if m and cur:
            kernels[cur][m.group(1)] = m.group(2)
    return kernels


def test_no_kernel_uses_private_scratch():
    from paper_1607_00968_amd import build
    srcs = [s for s in build.SOURCES if s.endswith(".hip") or s.endswith(".cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(6, len(srcs))) as ex:
        res = dict(zip(srcs, ex.map(resource_remarks, srcs)))
    bad, total = [], 0
    for src, kernels in res.items():
        for name, kv in kernels.items():
            total += 1
            if kv.get("ScratchSize [bytes/lane]", "0") != "0" or kv.get("Dynamic Stack", "False") != "False":
                bad.append((src, name, kv))
    assert total > 50, total  # the remarks were found and parsed
    assert not bad, bad
