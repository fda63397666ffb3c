"""Multi-frequency batches (frequency continuation needs the same sources at
several frequencies, each with its own hierarchy): helm_setup_batch builds
the hierarchies, helm_solve_batch solves them concurrently.

  - 2D 128^2, 4 sources at the 5 frequencies of the paper's frequency list
    (ratios 2 : 2.5 : 3.5 : 4.5 : 6, the highest at 10 points per
    wavelength), mixed precision: every instance's residual by the oracle's
    operator <= 1e-8 and its error against the oracle's solve at that
    frequency (1e-10) <= 1e-5; the concurrent results are bitwise those of
    the instances solved one after another;
  - 3D 64^3, 16 sources at 3 frequencies: residuals by the oracle's operator;
  - a bad descriptor fails the whole batch set-up and names its instance.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def relres(p, U):
    g = oracle.grid(p.dim, p.n, p.h)
    R = p.Q - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, U)
    return np.linalg.norm(R, axis=1) / np.linalg.norm(p.Q, axis=1)


def test_frequency_sweep_2d_matches_oracle():
    probs = synth.frequency_sweep(synth.gradient_2d())
    hs = pk.helm_setup_batch(probs, precision="mixed")
    Qs = [torch.from_numpy(np.ascontiguousarray(p.Q)).cuda() for p in probs]
    Us = [torch.zeros_like(Q) for Q in Qs]
    infos = pk.helm_solve_batch(hs, Qs, Us, tol=1e-8, restart=5, max_cycles=3000, max_threads=5)
    torch.cuda.synchronize()
    for p, hd, Q, U, info in zip(probs, hs, Qs, Us, infos):
        assert info["status"] == 0 and info["converged_all"], (p.name, info)
        Uh = U.cpu().numpy()
        assert relres(p, Uh).max() <= 1e-8 * (1 + 1e-6)
        ho = oracle.setup_problem(p, levels=3)
        Xo, it, rr, conv = ho.fgmres(p.Q, tol=1e-10, restart=10, maxit=4000)
        assert conv
        err = np.linalg.norm(Uh - Xo, axis=1) / np.linalg.norm(Xo, axis=1)
        print(p.name, "cycles", info["cycles"], "max error", err.max())
        assert err.max() <= 1e-5, (p.name, err)
        U1 = torch.zeros_like(Q)
        i1 = pk.helm_solve_block(hd, Q, U1, tol=1e-8, restart=5, max_cycles=3000, block_size=1, reorth=0)
        assert i1["cycles"] == info["cycles"] and torch.equal(U1, U)


def test_frequency_sweep_3d_residuals():
    probs = synth.frequency_sweep(synth.layered_3d(n=64, nsrc=(4, 4), levels=3, seed=3), freqs=(3.0, 4.5, 6.0))
    hs = pk.helm_setup_batch(probs, precision="mixed", coarse="lu")
    Qs = [torch.from_numpy(np.ascontiguousarray(p.Q)).cuda() for p in probs]
    Us = [torch.zeros_like(Q) for Q in Qs]
    infos = pk.helm_solve_batch(hs, Qs, Us, tol=1e-6, restart=5, max_cycles=3000, max_threads=3)
    torch.cuda.synchronize()
    cyc = []
    for p, U, info in zip(probs, Us, infos):
        assert info["converged_all"]
        assert relres(p, U.cpu().numpy()).max() <= 1e-6 * (1 + 1e-6)
        cyc.append(info["cycles"])
    print("cycles by frequency (low to high)", cyc)


def test_setup_batch_rejects_a_bad_instance():
    probs = synth.frequency_sweep(synth.gradient_2d(n=64, nsrc=(1,), levels=3), freqs=(2.0, 4.0, 6.0))
    probs[2].levels = 9  # more levels than the grid allows
    with pytest.raises(pk.HelmError) as e:
        pk.helm_setup_batch(probs)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG and "instance 2" in str(e.value)
