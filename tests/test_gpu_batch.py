"""GPU tests of the concurrent batch of independent uneven instances.

Every instance runs the same kernels as its own helm_solve_block, only on a
stream of its own, so results must be bitwise equal to solving the
instances one after another; every instance's residual, recomputed by the
oracle's FP64 operator, must meet the tolerance; per-instance statuses must
be reported.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def small_instances():
    probs = synth.batch_instances(count=8, seed=77, sizes_2d=[64, 96, 128], sizes_3d=[32, 48, 64], ppw=(6.0, 12.0))
    out = []
    for k, p in enumerate(probs):
        nr = 1 + k % 6
        Q = np.ascontiguousarray(p.Q[:nr]) if p.nrhs >= nr else np.ascontiguousarray(
            synth.random_rhs(p.N, nr, 100 + k))
        nc = int(np.prod([c // 2 ** (p.levels - 1) - 1 for c in p.n]))
        kw = dict(coarse="lu") if nc <= 16384 else dict(coarse="gmres", coarse_iters=20)
        hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=p.levels,
                           precision="mixed", **kw)
        out.append((p, hd, torch.from_numpy(Q).cuda()))
    return out


def test_batch_equals_sequential_solves():
    inst = small_instances()
    seq = []
    for p, hd, Q in inst:
        U = torch.zeros_like(Q)
        info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=5, block_size=1, reorth=0, max_cycles=800)
        assert info["converged_all"], p.name
        seq.append((U, info))
    Us = [torch.zeros_like(Q) for _, _, Q in inst]
    infos = pk.helm_solve_batch([hd for _, hd, _ in inst], [Q for _, _, Q in inst], Us, tol=1e-6,
                                restart=5, max_cycles=800, max_threads=4)
    torch.cuda.synchronize()
    for (p, hd, Q), U, info, (Us_, is_) in zip(inst, Us, infos, seq):
        assert info["status"] == 0 and info["converged_all"]
        assert info["cycles"] == is_["cycles"]
        assert torch.equal(U, Us_), p.name
        g = oracle.grid(p.dim, p.n, p.h)
        Qh, Uh = Q.cpu().numpy(), U.cpu().numpy()
        R = Qh - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, Uh)
        rr = np.linalg.norm(R, axis=1) / np.linalg.norm(Qh, axis=1)
        assert rr.max() <= 1e-6 * (1 + 1e-6), (p.name, rr)


def test_batch_reports_per_instance_status():
    inst = small_instances()[:3]
    Us = [torch.zeros_like(Q) for _, _, Q in inst]
    hs = [hd for _, hd, _ in inst]
    infos = pk.helm_solve_batch(hs, [Q for _, _, Q in inst], Us, tol=1e-30, max_cycles=3)
    assert all(i["status"] == pk.HELM_ERR_NOT_CONVERGED and i["cycles"] == 3 for i in infos)
    with pytest.raises(pk.HelmError):
        pk.helm_solve_batch([hs[0], hs[0]], [inst[0][2], inst[0][2]], [Us[0], Us[0]])
