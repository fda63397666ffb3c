"""GPU tests of the HIP-graph execution form of the cycle.

A graph replays exactly the kernels the eager path launches, with the same
arguments and in the same order, so every result must be bitwise equal to
the eager solve. Each case solves once eagerly, then several times from the
graphs (the first solve captures them, later ones replay), with unrelated
eager work and synchronisations between the replays, and compares every
replay with the eager result.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def solve(hd, Q, graph, **kw):
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=kw.pop("restart", 5), block_size=1,
                               max_cycles=kw.pop("max_cycles", 600), reorth=0, graph=graph, **kw)
    torch.cuda.synchronize()
    return U, info


def eager_noise(hd, Q):
    """Unrelated eager work between replays: an operator apply and a residual."""
    Y = torch.empty_like(Q)
    pk.helm_apply(hd, Q, Y)
    pk.helm_residual(hd, Q, Y)
    torch.cuda.synchronize()


def check_replays(hd, Q, replays=3, **kw):
    Ue, ie = solve(hd, Q, False, **dict(kw))
    assert ie["converged_all"]
    for _ in range(replays):
        Ug, ig = solve(hd, Q, True, **dict(kw))
        assert ig["cycles"] == ie["cycles"]
        assert ig["fallback_used"] == ie["fallback_used"]
        assert torch.equal(Ug, Ue)
        eager_noise(hd, Q)
    return ie


def test_graph_2d_mixed_lu():
    p = synth.gradient_2d(levels=3)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="lu")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    check_replays(hd, Q, restart=10)


def test_graph_3d_fp64_gmres_coarsest():
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="fp64", coarse="gmres", coarse_iters=8)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    check_replays(hd, Q)


def test_graph_3d_mixed_w_cycle():
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="lu", cycle="W")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    check_replays(hd, Q)


def trained_blob(p, D, steps=60):
    teach = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                          precision="mixed", coarse="lu")
    net = pk.helm_net_create(D, 8, seed=3)
    pk.helm_net_capture(teach, net, 256)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    pk.helm_solve_block(teach, Q, torch.zeros_like(Q), tol=1e-6, restart=5, block_size=1)
    pk.helm_net_capture(teach, net, 0)
    net.train(steps, 8, lr=2e-3, seed=1)
    return net.save()


def test_graph_learned_coarsest_and_fallback():
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    blob = trained_blob(p, 8)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    hl = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="learned", net=blob, coarse_iters=4)
    info = check_replays(hl, Q)
    assert info["fallback_used"] == 0
    # overflowing weights: each replay's network output is not finite, the
    # cycle is redone eagerly with the GMRES fallback, results stay bitwise equal
    bad = np.frombuffer(blob, dtype=np.uint8).copy()
    prm = bad[16:].view(np.float32)
    prm[: prm.size - 34] = np.where(np.arange(prm.size - 34) % 7 == 0, 1e30, prm[: prm.size - 34])
    hb = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="learned", net=bad.tobytes(), coarse_iters=4)
    info = check_replays(hb, Q, replays=2)
    assert info["fallback_used"] == info["cycles"]


def test_graph_timing_report_small_solve():
    """Not a correctness bound: reports eager vs graph solve time for the 2D
    128^2 workload (every kernel is a few microseconds long)."""
    import time
    p = synth.gradient_2d(levels=3)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="lu")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    solve(hd, Q, True, restart=10)
    t = {}
    for g in (False, True):
        solve(hd, Q, g, restart=10)
        t0 = time.perf_counter()
        for _ in range(3):
            solve(hd, Q, g, restart=10)
        t[g] = (time.perf_counter() - t0) / 3
    print(f"2D 128^2 x 4 RHS mixed: eager {t[False]*1e3:.1f} ms, graph {t[True]*1e3:.1f} ms per solve")
    assert t[True] < 2.0 * t[False]
