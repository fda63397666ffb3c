"""The 3D 128^3 workload (127^3 unknowns, 32 surface sources, FP64) on the
GPU against the oracle's solution at full size.

The oracle's solve of this size takes minutes on the host, so its solution
is stored: tests/golden/layered128_ref.json, written by
tests/golden/make_layered128_ref.py (which calls only oracle/ and synth/),
holds two columns of the oracle's block FGMRES(5) solve to 1e-10 (3-level
V-cycle, banded-LU coarsest), sampled at 1024 seeded random nodes plus the
27 nodes around each source, and each column's full 2-norm.

Checked for every GPU solve at tolerance 1e-8:
  - each of the 32 columns' relative residual, recomputed by the oracle's
    FP64 operator, is at most the tolerance;
  - the sampled values of the two stored columns agree with the oracle's to
    1e-5 relative (2-norm over the sample), and so do the full 2-norms.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "layered128_ref.json")


@pytest.fixture(scope="module")
def problem():
    return synth.layered_3d(n=128, seed=2, nsrc=(8, 4), levels=3)


@pytest.fixture(scope="module")
def reference():
    with open(REF) as fh:
        return json.load(fh)


def check_against_oracle(p, U, tol, ref):
    g = oracle.grid(p.dim, p.n, p.h)
    rr = np.empty(p.nrhs)
    for c0 in range(0, p.nrhs, 8):  # the oracle's operator in slices of 8 columns
        R = p.Q[c0:c0 + 8] - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, U[c0:c0 + 8])
        rr[c0:c0 + 8] = np.linalg.norm(R, axis=1) / np.linalg.norm(p.Q[c0:c0 + 8], axis=1)
    assert rr.max() <= tol * (1 + 1e-6), rr
    errs = []
    for col in ref["columns"]:
        c = col["column"]
        idx = np.asarray(col["nodes"])
        x = np.asarray([float(v) for v in col["re"]]) + 1j * np.asarray([float(v) for v in col["im"]])
        err = np.linalg.norm(U[c, idx] - x) / np.linalg.norm(x)
        nerr = abs(np.linalg.norm(U[c]) - col["norm2"]) / col["norm2"]
        errs.append((err, nerr))
        assert err <= 1e-5 and nerr <= 1e-5, (c, err, nerr)
    print("max relres", rr.max(), "sampled error, norm error", errs)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("block_size,reorth,coarse", [(4, 1, "lu"), (1, 0, "gmres")])
def test_layered128_fp64_matches_oracle(problem, reference, block_size, reorth, coarse):
    p = problem
    kw = dict(coarse="lu") if coarse == "lu" else dict(coarse="gmres", coarse_iters=20)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3, precision="fp64", **kw)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-8, restart=5, max_cycles=3000, block_size=block_size,
                               reorth=reorth)
    assert info["converged_all"], info
    print("cycles", info["cycles"])
    check_against_oracle(p, U.cpu().numpy(), 1e-8, reference)
