"""helm_residual_noalloc (the residual for callers that cannot allocate)
through the C-ABI against helm_residual, the entry point it is a variant of.

Both run the same kernels; the variant keeps its partial sums in the
library's static device array instead of the handle's buffer, so the
results must be bitwise equal. Two calls in a row, the second on a smaller
input (fewer columns on a smaller grid), check that nothing of the first
call's contents leaks into the second; too many columns is an error.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def case(p, nrhs, seed):
    rng = np.random.default_rng(seed)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=2)
    Q = rng.standard_normal((nrhs, p.N)) + 1j * rng.standard_normal((nrhs, p.N))
    U = 1e-4 * (rng.standard_normal((nrhs, p.N)) + 1j * rng.standard_normal((nrhs, p.N)))
    Q[nrhs // 2] = 0.0  # a zero column reports 0
    return hd, torch.from_numpy(Q).cuda(), torch.from_numpy(U).cuda()


def test_noalloc_residual_equals_helm_residual_on_two_calls():
    big = synth.layered_3d(n=48, nsrc=(2, 2), levels=2, seed=2)   # 47^3 unknowns
    small = synth.gradient_2d(n=40, nsrc=(3,), levels=2)           # 39^2 unknowns
    outs = []
    for p, nrhs, seed in ((big, 40, 1), (small, 5, 2)):
        hd, Q, U = case(p, nrhs, seed)
        a = pk.helm_residual_noalloc(hd, Q, U)
        b = pk.helm_residual(hd, Q, U)
        assert np.all(np.isfinite(a)) and a[nrhs // 2] == 0.0
        assert np.array_equal(a, b), np.abs(a - b).max()
        outs.append(a)
    assert outs[1].shape == (5,)
    with pytest.raises(pk.HelmError) as e:
        hd, Q, U = case(small, 1, 3)
        Qb = torch.zeros((257, small.N), dtype=torch.complex128, device="cuda")
        pk.helm_residual_noalloc(hd, Qb, Qb)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG
