"""GPU tests of the learned coarsest-grid correction through the C-ABI.

Parity against the FP64 CPU oracle of the network (oracle/conv_oracle.c):
  - forward: the oracle runs on the BF16-rounded weights and input the
    device holds, so the remaining difference is the BF16 rounding of each
    stored activation (about 2^-9 relative per layer, 10 layers plus pooling
    and upsampling) and FP32 accumulation: relative 2-norm error <= 2e-2;
  - loss and gradient: the backward pass also stores BF16 gradients, and a
    BF16-rounded activation near zero can switch a ReLU mask the FP64 oracle
    does not switch; the error grows towards the input layer (about 6% at
    layer 0 for D = 8). Each layer's block must agree to 0.1 in relative
    2-norm with cosine >= 0.995, the whole gradient to cosine >= 0.999 (an
    indexing mistake gives errors of order 1);
  - captured training pairs: input channels exact up to BF16 storage (4e-3),
    targets against the oracle's banded-LU coarsest solve (FP32 storage: 1e-5).
Solver-level tests: training lowers the loss, a trained network gives a
convergent outer solve, and a non-finite network output falls back to GMRES.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")

RNG = np.random.default_rng(2024)
LAYERS = oracle.UNET_LAYERS


def bf16(a):
    """Round float32 values to the nearest BF16 (ties to even)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def layer_slices():
    out, o = [], 0
    for ci, co in LAYERS:
        nw = 27 * ci * co
        out.append((slice(o, o + nw), slice(o + nw, o + nw + co)))
        o += nw + co
    return out, o


def he_params(scale=1.0):
    sl, o = layer_slices()
    p = np.zeros(o + 34, np.float32)
    for (w, b), (ci, co) in zip(sl, LAYERS):
        p[w] = scale * RNG.standard_normal(w.stop - w.start) * np.sqrt(2.0 / (27 * ci))
        p[b] = 0.1 * RNG.standard_normal(b.stop - b.start)
    p[o:o + 34] = 0.3 * RNG.standard_normal(34)
    return p


def device_view(p):
    """Parameters as the device computes with them: BF16 conv weights, FP32 rest."""
    sl, _ = layer_slices()
    q = p.astype(np.float64).copy()
    for w, _b in sl:
        q[w] = bf16(p[w])
    return q


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cosine(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("D,B", [(8, 2), (12, 1), (16, 3)])
def test_forward_matches_oracle(D, B):
    net = pk.helm_net_create(D, max(B, 2), seed=1)
    p = he_params()
    net.set_params(p)
    x = bf16(RNG.standard_normal((B, D, D, D, 4)).astype(np.float32))
    out = torch.empty((B, D ** 3, 2), dtype=torch.float32, device="cuda")
    net.forward(cuda(x.reshape(B, D ** 3, 4)), out)
    ref = oracle.unet_forward(device_view(p), x.astype(np.float64))
    got = out.cpu().numpy().reshape(ref.shape)
    assert rel(got, ref) <= 2e-2, rel(got, ref)


def test_forward_is_per_sample():
    D = 8
    net = pk.helm_net_create(D, 4, seed=2)
    x = RNG.standard_normal((3, D ** 3, 4)).astype(np.float32)
    out = torch.empty((3, D ** 3, 2), dtype=torch.float32, device="cuda")
    net.forward(cuda(x), out)
    for b in range(3):
        o1 = torch.empty((1, D ** 3, 2), dtype=torch.float32, device="cuda")
        net.forward(cuda(x[b:b + 1]), o1)
        assert torch.equal(o1[0], out[b])  # bitwise: no cross-sample arithmetic


def test_params_roundtrip_and_blob():
    net = pk.helm_net_create(8, 1, seed=3)
    p = he_params()
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    blob = net.save()
    assert blob[:4] == b"HNET" and len(blob) == 16 + 4 * p.size
    assert np.array_equal(np.frombuffer(blob[16:], dtype=np.float32), p)


def test_bad_params_rejected():
    net = pk.helm_net_create(8, 1)
    p = he_params()
    p[5] = np.nan
    with pytest.raises(pk.HelmError):
        net.set_params(p)
    with pytest.raises(pk.HelmError):
        pk.helm_net_create(10, 1)  # edge not a multiple of 4


@pytest.mark.parametrize("D,B", [(8, 2), (12, 2)])
def test_loss_grad_matches_oracle(D, B):
    net = pk.helm_net_create(D, B, seed=4)
    p = he_params()
    net.set_params(p)
    x = bf16(RNG.standard_normal((B, D, D, D, 4)).astype(np.float32))
    t = RNG.standard_normal((B, D, D, D, 2)).astype(np.float32)
    mask = (RNG.uniform(size=(D, D, D)) > 0.25).astype(np.uint8)
    g = torch.empty(pk.helm_net_nparams(), dtype=torch.float32, device="cuda")
    loss = net.loss_grad(cuda(x.reshape(B, -1, 4)), cuda(t.reshape(B, -1, 2)),
                         cuda(mask.ravel(), torch.uint8), g)
    lref, gref = oracle.unet_loss_grad(device_view(p), x.astype(np.float64), t.astype(np.float64),
                                       mask.astype(np.float64))
    assert abs(loss - lref) <= 1e-2 * lref
    gg = g.cpu().numpy().astype(np.float64)
    sl, o = layer_slices()
    prof = []
    for l, (w, b) in enumerate(sl + [(slice(o, o + 34), slice(o + 34, o + 34))]):
        blk = np.r_[w, b]
        prof.append((l, rel(gg[blk], gref[blk]), cosine(gg[blk], gref[blk])))
    print("per-layer (layer, rel err, cosine):", [(l, round(e, 4), round(c, 5)) for l, e, c in prof])
    for l, e, c in prof:
        assert e <= 0.1 and c >= 0.995, (l, e, c)
    assert cosine(gg, gref) >= 0.999


class ConcatForward:
    """HELM_NET_CONCAT=1: the inference passes take the training form of the
    forward pass (skip outputs stored in slices of concatenated buffers, the
    upsampled activations copied beside them)."""

    def __enter__(self):
        os.environ["HELM_NET_CONCAT"] = "1"

    def __exit__(self, *exc):
        os.environ.pop("HELM_NET_CONCAT", None)


@pytest.mark.parametrize("D,B", [(16, 3), (48, 2)])
def test_inference_forward_equals_training_form(D, B):
    """The inference forward feeds the two decoder layers from the skip
    outputs and the coarser activations where they are (no concatenated
    copy, no upsampled copy). Every convolution sees the same values in the
    same channel order, so the output must not change by a bit. D = 48 is
    the network edge at the 192^3 benchmark's coarsest grid."""
    net = pk.helm_net_create(D, B, seed=7)
    net.set_params(he_params())
    x = cuda(RNG.standard_normal((B, D ** 3, 4)).astype(np.float32))
    a = torch.empty((B, D ** 3, 2), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    net.forward(x, a)
    with ConcatForward():
        net.forward(x, b)
    c = torch.empty_like(a)  # the default form again, after the other
    net.forward(x, c)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_learned_coarse_solve_same_in_both_forward_forms():
    """The in-cycle learned coarsest solve (network guess + GMRES) gives
    bitwise the same correction with either form of the forward pass."""
    p, hd = coarse_problem(32, 3)
    nu = pk.helm_level_dims(hd, 2)
    blob = pk.helm_net_create((max(nu) + 3) // 4 * 4, 4, seed=6).save()
    hl = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="learned", net=blob, coarse_iters=4)
    nc = int(np.prod(nu))
    R = cuda(RNG.standard_normal((4, nc)) + 1j * RNG.standard_normal((4, nc)), torch.complex128)
    E1 = torch.empty_like(R)
    E2 = torch.empty_like(R)
    pk.helm_coarse_solve(hl, R, E1)
    with ConcatForward():
        pk.helm_coarse_solve(hl, R, E2)
    torch.cuda.synchronize()
    assert torch.isfinite(E1).all() and torch.equal(E1, E2)


def coarse_problem(n=32, levels=3, precision="fp64", seed_src=(2, 2)):
    p = synth.layered_3d(n=n, nsrc=seed_src, levels=levels, seed=2)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=levels,
                       precision=precision, coarse="lu")
    return p, hd


def test_capture_pairs_match_oracle():
    p, hd = coarse_problem(32, 3)
    nu = pk.helm_level_dims(hd, 2)
    D = (max(nu) + 3) // 4 * 4
    net = pk.helm_net_create(D, 2)
    pk.helm_net_capture(hd, net, 16)
    Nc = int(np.prod(nu))
    F = RNG.standard_normal((3, Nc)) + 1j * RNG.standard_normal((3, Nc))
    F[1] = 0.0  # a zero column is not captured
    E = torch.empty((3, Nc), dtype=torch.complex128, device="cuda")
    pk.helm_coarse_solve(hd, torch.from_numpy(F).cuda(), E)
    assert net.pairs() == 2
    ho = oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, p.omega, p.shift, 3)
    Eref = ho.coarse_solve(F)
    H2 = (p.h[0] * 4) ** 2
    dg = H2 * ho.stencil(2)[:, 13]
    V = D ** 3
    x = torch.empty((V, 4), dtype=torch.float32, device="cuda")
    t = torch.empty((V, 2), dtype=torch.float32, device="cuda")
    for slot, col in ((0, 0), (1, 2)):
        net.pool_read(slot, x, t)
        xv = x.cpu().numpy().reshape(D, D, D, 4)[:nu[2], :nu[1], :nu[0]].reshape(-1, 4)
        tv = t.cpu().numpy().reshape(D, D, D, 2)[:nu[2], :nu[1], :nu[0]].reshape(-1, 2)
        rms = np.sqrt(np.mean(np.abs(F[col]) ** 2))
        assert rel(xv[:, 0] + 1j * xv[:, 1], F[col] / rms) <= 4e-3
        assert rel(xv[:, 2] + 1j * xv[:, 3], dg) <= 4e-3
        assert rel(tv[:, 0] + 1j * tv[:, 1], Eref[col] / (H2 * rms)) <= 1e-5
        # padding is zero
        xa = x.cpu().numpy().reshape(D, D, D, 4)
        assert np.all(xa[nu[2]:] == 0) and np.all(xa[:, nu[1]:] == 0) and np.all(xa[:, :, nu[0]:] == 0)
    pk.helm_net_capture(hd, net, 0)


def train_on(hd, p, net, nrhs=8, pairs=256, steps=150, batch=8, lr=2e-3, seed=0):
    pk.helm_net_capture(hd, net, pairs)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q[:nrhs])).cuda()
    U = torch.zeros_like(Q)
    pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=5, block_size=1)
    pk.helm_net_capture(hd, net, 0)
    return net.train(steps, batch, lr=lr, seed=seed)


def test_capture_pool_spans_problems():
    """max_pairs < 0 keeps the pool: the pairs of two separately seeded
    training models end up in one pool; another coarsest size or a network
    without a pool is refused."""
    hs, ps = [], []
    for j in (0, 1):
        p = synth.training_model(j, n=32, nsrc=(2, 1))
        ps.append(p)
        hs.append(pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                                precision="mixed", coarse="lu"))
    D = (max(pk.helm_level_dims(hs[0], 2)) + 3) // 4 * 4
    net = pk.helm_net_create(D, 2, seed=4)
    with pytest.raises(pk.HelmError):
        pk.helm_net_capture(hs[0], net, -1)  # no pool yet
    counts = []
    for k, (p, hd) in enumerate(zip(ps, hs)):
        pk.helm_net_capture(hd, net, 4096 if k == 0 else -1)
        Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
        info = pk.helm_solve_block(hd, Q, torch.zeros_like(Q), tol=1e-6, restart=5, block_size=1)
        pk.helm_net_capture(hd, net, 0)
        counts.append(net.pairs())
        assert info["converged_all"]
    assert 0 < counts[0] < counts[1] <= 4096, counts
    big = synth.training_model(0, n=64, nsrc=(1, 1))
    hb = pk.helm_setup(big.dim, big.n, big.h, big.m, big.gamma, big.omega, shift=big.shift, levels=3,
                       precision="mixed", coarse="lu")
    with pytest.raises(pk.HelmError):
        pk.helm_net_capture(hb, net, -1)


def test_training_lowers_loss():
    p, hd = coarse_problem(32, 3)
    nu = pk.helm_level_dims(hd, 2)
    D = (max(nu) + 3) // 4 * 4
    net = pk.helm_net_create(D, 8, seed=5)
    hist = train_on(hd, p, net, steps=200)
    assert net.pairs() > 16
    assert np.all(np.isfinite(hist))
    assert hist[-20:].mean() < 0.5 * hist[:20].mean(), (hist[:20].mean(), hist[-20:].mean())


def test_learned_coarse_solve_converges_and_falls_back():
    p, hd = coarse_problem(32, 3)
    nu = pk.helm_level_dims(hd, 2)
    D = (max(nu) + 3) // 4 * 4
    net = pk.helm_net_create(D, 8, seed=6)
    train_on(hd, p, net, steps=100)
    blob = net.save()
    Q = torch.from_numpy(np.ascontiguousarray(p.Q[:4])).cuda()
    for precision in ("fp64", "mixed"):
        # the network's correction refined by 4 coarsest GMRES steps
        hl = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                           precision=precision, coarse="learned", net=blob, coarse_iters=4)
        U = torch.zeros_like(Q)
        info = pk.helm_solve_block(hl, Q, U, tol=1e-6, restart=5, block_size=1, max_cycles=600)
        assert info["converged_all"] and info["fallback_used"] == 0
        assert pk.helm_residual(hl, Q, U).max() <= 1e-6
    # weights that overflow the activations: every coarsest solve falls back
    bad = np.frombuffer(blob, dtype=np.uint8).copy()
    prm = bad[16:].view(np.float32)
    sl, _ = layer_slices()
    for w, _b in sl:
        prm[w] = 1e30
    hb = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       coarse="learned", net=bad.tobytes(), coarse_iters=0)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hb, Q, U, tol=1e-6, restart=5, block_size=1, max_cycles=600)
    assert info["converged_all"] and info["fallback_used"] == info["cycles"]


def test_rate_check_switches_poor_network_to_fallback():
    """The per-cycle rate check (learned_rate): an untrained network used alone
    is a poor coarsest solver. Calibrated with the LU coarsest solver's
    per-cycle factor rho, the check fires at a restart (the solve's own factor
    is above sqrt(rho)), every later coarsest solve is a GMRES fallback, and
    the solve converges; with the check off the network keeps running. The
    graph form gives the same result (the switch turns capture off)."""
    p, hd = coarse_problem(32, 3, precision="mixed")
    Q = torch.from_numpy(np.ascontiguousarray(p.Q[:4])).cuda()
    U = torch.zeros_like(Q)
    ref = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=5, block_size=1, max_cycles=600)
    assert ref["converged_all"] and ref["rate_switch"] == -1
    rho = float(ref["relres"].max()) ** (1.0 / ref["cycles"])
    nu = pk.helm_level_dims(hd, 2)
    D = (max(nu) + 3) // 4 * 4
    blob = pk.helm_net_create(D, 8, seed=11).save()
    hl = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                       precision="mixed", coarse="learned", net=blob, coarse_iters=0)
    Uoff = torch.zeros_like(Q)
    off = pk.helm_solve_block(hl, Q, Uoff, tol=1e-6, restart=5, block_size=1, max_cycles=300)
    assert off["rate_switch"] == -1
    Uon = torch.zeros_like(Q)
    on = pk.helm_solve_block(hl, Q, Uon, tol=1e-6, restart=5, block_size=1, max_cycles=600, learned_rate=rho)
    print("LU cycles", ref["cycles"], "rho", rho, "off", off["cycles"], off["converged_all"],
          "on", on["cycles"], "switch at", on["rate_switch"])
    assert on["converged_all"] and pk.helm_residual(hl, Q, Uon).max() <= 1e-6
    assert on["rate_switch"] > 0
    assert on["fallback_used"] >= on["cycles"] - on["rate_switch"]
    assert (not off["converged_all"]) or on["cycles"] < off["cycles"]
    Ug = torch.zeros_like(Q)
    g = pk.helm_solve_block(hl, Q, Ug, tol=1e-6, restart=5, block_size=1, max_cycles=600, learned_rate=rho,
                            graph=True)
    assert g["cycles"] == on["cycles"] and g["rate_switch"] == on["rate_switch"]
    assert torch.equal(Ug, Uon)
    with pytest.raises(pk.HelmError):
        pk.helm_solve_block(hl, Q, Ug, tol=1e-6, learned_rate=1.5)


def test_learned_guess_beats_gmres_from_zero():
    """The gain test: on a 64^3 layered model (coarsest grid 15^3), k = 4
    GMRES steps started from the trained network's correction need clearly
    fewer outer cycles than 4 steps from zero and than the untrained network;
    GMRES(20) from zero is reported for reference."""
    p = synth.layered_3d(n=64, nsrc=(4, 4), levels=3, seed=3)
    Q = torch.from_numpy(np.ascontiguousarray(p.Q)).cuda()
    teach = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                          precision="mixed", coarse="lu")
    net = pk.helm_net_create(16, 16, seed=0)
    untrained = net.save()
    pk.helm_net_capture(teach, net, 2048)
    pk.helm_solve_block(teach, Q, torch.zeros_like(Q), tol=1e-6, restart=5, block_size=1)
    pk.helm_net_capture(teach, net, 0)
    hist = net.train(600, 16, lr=1e-3, seed=1)
    assert hist[-50:].mean() < 0.15 * hist[:10].mean()
    cyc = {}
    for name, kw in (("learned+4", dict(coarse="learned", net=net.save(), coarse_iters=4)),
                     ("untrained+4", dict(coarse="learned", net=untrained, coarse_iters=4)),
                     ("gmres4", dict(coarse="gmres", coarse_iters=4)),
                     ("gmres20", dict(coarse="gmres", coarse_iters=20)),
                     ("lu", dict(coarse="lu"))):
        hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3,
                           precision="mixed", **kw)
        U = torch.zeros_like(Q)
        info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=5, block_size=1, max_cycles=1500)
        cyc[name] = info["cycles"] if info["converged_all"] else 10 ** 6
    print("outer cycles:", cyc)
    assert cyc["learned+4"] < 0.8 * cyc["gmres4"]
    assert cyc["learned+4"] < 0.8 * cyc["untrained+4"]
    assert cyc["lu"] <= cyc["gmres20"] < 10 ** 6


def test_learned_setup_rejects_bad_blob():
    p = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    with pytest.raises(pk.HelmError):
        pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, coarse="learned", net=b"HNETxxxx")
    with pytest.raises(pk.HelmError):
        pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, coarse="learned", net=None)
