"""GPU tests of the persistent cycle: one cooperative launch per cycle that
runs the recorded steps with grid-wide barriers (helm_solve_opts.graph = 2).

In 2D the eager cycle runs the same generic per-point kernels the persistent
kernel calls, so solves must be bitwise equal (same cycles, same U). In 3D
the eager path runs the tiled and fused kernels, whose results differ by
rounding, so the persistent solve must converge to the tolerance in about the
same number of cycles. Each case solves several times to exercise the cached
plan, with unrelated eager work in between.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def solve(hd, Q, form, **kw):
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=kw.pop("restart", 5), block_size=1,
                               max_cycles=kw.pop("max_cycles", 800), reorth=0, graph=form, **kw)
    torch.cuda.synchronize()
    return U, info


@pytest.mark.parametrize("precision,levels", [("mixed", 3), ("fp64", 3), ("fp64", 2), ("mixed", 4)])
def test_persistent_2d_bitwise_equal_to_eager(precision, levels):
    p = synth.gradient_2d(levels=levels)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=levels,
                       precision=precision, coarse="lu")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    # four levels make the coarsest grid too coarse for this wavelength: the
    # comparison then covers 30 unconverged cycles (BF16 -> BF16 transfers)
    cap = 30 if levels == 4 else 800
    Ue, ie = solve(hd, Q, 0, restart=10, max_cycles=cap)
    assert ie["converged_all"] or levels == 4
    for _ in range(3):
        Up, ip = solve(hd, Q, "persistent", restart=10, max_cycles=cap)
        assert ip["cycles"] == ie["cycles"]
        assert torch.equal(Up, Ue)
        Y = torch.empty_like(Q)
        pk.helm_apply(hd, Q, Y)
        torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_persistent_3d_converges_like_eager(precision):
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision=precision, coarse="lu")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    Ue, ie = solve(hd, Q, 0)
    for _ in range(2):
        Up, ip = solve(hd, Q, "persistent")
        assert ip["converged_all"]
        assert pk.helm_residual(hd, Q, Up).max() <= 1e-6
        assert abs(ip["cycles"] - ie["cycles"]) <= max(2, ie["cycles"] // 10)
        rel = float(torch.linalg.norm(Up - Ue) / torch.linalg.norm(Ue))
        assert rel < 1e-4, rel


def test_persistent_rejects_unsupported_cycles():
    p = synth.gradient_2d(levels=3)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    for kw in (dict(coarse="gmres", coarse_iters=8), dict(coarse="lu", cycle="W")):
        hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3, precision="mixed", **kw)
        with pytest.raises(pk.HelmError):
            solve(hd, Q, "persistent")
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3, precision="mixed",
                       coarse="lu")
    with pytest.raises(pk.HelmError):
        pk.helm_solve_batch([hd], [Q], [torch.zeros_like(Q)], graph="persistent")


def test_persistent_timing_report_small_solve():
    """Not a correctness bound: eager, graph and persistent solve times for
    the 2D 128^2 x 4 workload (every kernel is a few microseconds long)."""
    import time
    p = synth.gradient_2d(levels=3)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="lu")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    t = {}
    for form in (0, 1, "persistent"):
        solve(hd, Q, form, restart=10)
        t0 = time.perf_counter()
        for _ in range(3):
            _, info = solve(hd, Q, form, restart=10)
        t[form] = (time.perf_counter() - t0) / 3
    print(f"2D 128^2 x 4 RHS mixed, {info['cycles']} cycles: eager {t[0]*1e3:.1f} ms, graph {t[1]*1e3:.1f} ms, "
          f"persistent {t['persistent']*1e3:.1f} ms per solve")
    assert t["persistent"] < 5.0 * t[0]
