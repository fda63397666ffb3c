"""The learned coarsest solve as the cycle applies it, and the Adam step,
on the GPU against the oracle (oracle/learned.py, pinned in
tests/test_oracle_learned.py).

  - helm_coarse_solve on a handle with the learned coarsest correction
    (network + restarted GMRES(k) from its guess) against the oracle's
    composition run on the BF16-rounded weights and input the device uses;
    the remaining difference is the BF16 storage of every activation inside
    the network (about 2^-9 per layer; measured 3.2e-3 for the network
    alone), which the GMRES steps then shrink with the residual (measured
    1.7e-4 after two cycles of 8 steps): relative 2-norm <= 1e-2 with k = 0
    and <= 2e-3 with k = 8 (two cycles), in FP64 and in mixed precision
    (FP32 coarsest fields);
  - one helm_net_train_step, then a second, against the oracle's Adam
    (Kingma & Ba, Algorithm 1, FP64) applied to the gradients the device
    computes for the same minibatches (helm_net_loss_grad, deterministic):
    the FP32 master weights agree to FP32 rounding.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import learned as ol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")

RNG = np.random.default_rng(909)


def bf16(a):
    """Round to the nearest BF16 (ties to even), as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def device_view(p):
    """Parameters as the device computes with them: BF16 conv weights, FP32 rest."""
    q = p.astype(np.float64).copy()
    o = 0
    for ci, co in oracle.UNET_LAYERS:
        q[o:o + 27 * ci * co] = bf16(p[o:o + 27 * ci * co])
        o += 27 * ci * co + co
    return q


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("k,restarts", [(0, 1), (8, 2)])
def test_learned_coarse_solve_matches_oracle(precision, k, restarts):
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)  # coarsest 7^3, D = 8
    D = 8
    net = pk.helm_net_create(D, 4, seed=21)
    prm = net.get_params()
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3, precision=precision,
                       coarse="learned", net=net.save(), coarse_iters=k, coarse_restarts=restarts)
    Nc = int(np.prod(pk.helm_level_dims(hd, 2)))
    F = RNG.standard_normal((5, Nc)) + 1j * RNG.standard_normal((5, Nc))
    F[3] = 0.0
    E = torch.empty((5, Nc), dtype=torch.complex128, device="cuda")
    pk.helm_coarse_solve(hd, torch.from_numpy(F).cuda(), E)
    Eg = E.cpu().numpy()
    ho = oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, p.omega, p.shift, 3, coarse="gmres",
                          coarse_iters=max(k, 1))
    dv = device_view(prm)
    Eo, fb = ol.learned_coarse_solve(ho, F, D, lambda x: oracle.unet_forward(dv, bf16(x).astype(np.float64)),
                                     k, restarts)
    assert not fb
    e = rel(Eg, Eo)
    print(precision, k, restarts, "relative difference", e)
    assert e <= (1e-2 if k == 0 else 2e-3), e
    assert np.all(Eg[3] == 0)


def test_train_step_matches_oracle_adam():
    D, B = 8, 2
    net = pk.helm_net_create(D, B, seed=33)
    p0 = net.get_params().astype(np.float64)
    mask = torch.from_numpy((RNG.uniform(size=D ** 3) > 0.2).astype(np.uint8)).cuda()
    g = torch.empty(pk.helm_net_nparams(), dtype=torch.float32, device="cuda")
    grads, params = [], []
    lr = 2e-3
    for step in range(2):
        x = torch.from_numpy(RNG.standard_normal((B, D ** 3, 4)).astype(np.float32)).cuda()
        t = torch.from_numpy(RNG.standard_normal((B, D ** 3, 2)).astype(np.float32)).cuda()
        l0 = net.loss_grad(x, t, mask, g)
        grads.append(g.cpu().numpy().astype(np.float64))
        l1 = net.train_step(x, t, mask, lr=lr)
        assert l1 == l0  # the step's own gradient is the one read above (deterministic)
        params.append(net.get_params().astype(np.float64))
    ref = ol.adam(p0, grads, lr)
    for s in range(2):
        d = np.abs(params[s] - ref[s])
        tol = lr * 2e-5 * (s + 1) + 2e-7 * np.abs(ref[s])
        assert np.all(d <= tol), (s, d.max(), np.argmax(d - tol))
    # the first step moves every parameter with a nonzero gradient by about lr
    moved = np.abs(params[0] - p0)[np.abs(grads[0]) > 1e-4]
    assert np.allclose(moved, lr, rtol=1e-3)


def test_training_resumes_bitwise_from_a_checkpoint():
    """helm_net_get_state / helm_net_set_state: two Adam steps, a checkpoint,
    two more steps; a second network restored from the checkpoint takes the
    same two steps to bitwise the same parameters and moments. Invalid
    states are refused and change nothing."""
    D, B = 8, 2
    rng = np.random.default_rng(11)
    mask = torch.from_numpy((rng.uniform(size=D ** 3) > 0.2).astype(np.uint8)).cuda()
    batches = [(torch.from_numpy(rng.standard_normal((B, D ** 3, 4)).astype(np.float32)).cuda(),
                torch.from_numpy(rng.standard_normal((B, D ** 3, 2)).astype(np.float32)).cuda()) for _ in range(4)]
    a = pk.helm_net_create(D, B, seed=21)
    for x, t in batches[:2]:
        a.train_step(x, t, mask, lr=3e-3)
    state, step = a.get_state()
    n = pk.helm_net_nparams()
    assert step == 2 and state.shape == (3 * n,)
    assert np.array_equal(state[:n], a.get_params())
    assert (state[2 * n:] >= 0).all() and np.abs(state[n:2 * n]).max() > 0
    for x, t in batches[2:]:
        a.train_step(x, t, mask, lr=3e-3)
    b = pk.helm_net_create(D, B, seed=99)
    b.set_state(state, step)
    for x, t in batches[2:]:
        b.train_step(x, t, mask, lr=3e-3)
    sa, ta = a.get_state()
    sb, tb = b.get_state()
    assert ta == tb == 4 and np.array_equal(sa, sb)
    bad = state.copy()
    bad[2 * n + 5] = -1.0
    with pytest.raises(pk.HelmError) as e:
        b.set_state(bad, 2)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG
    bad = state.copy()
    bad[7] = np.nan
    with pytest.raises(pk.HelmError) as e:
        b.set_state(bad, 2)
    assert e.value.status == pk.HELM_ERR_NONFINITE
    with pytest.raises(pk.HelmError):
        b.set_state(state, -1)
    sc, tc = b.get_state()
    assert tc == 4 and np.array_equal(sc, sb)
