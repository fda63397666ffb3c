"""Pins of the CPU oracle of the learned coarsest-grid correction network.

Forward convolution against scipy.signal.correlate (an independent library
routine), the backward passes by adjointness, pooling/upsampling by their
adjoint pair, and the whole-network gradient by central finite differences.
"""
import numpy as np
import pytest
from scipy.signal import correlate

import oracle

RNG = np.random.default_rng(11)


def rnd(*shape):
    return RNG.standard_normal(shape)


def test_conv3d_forward_matches_scipy_correlate():
    B, D, Cin, Cout = 2, 6, 3, 4
    x = rnd(B, D, D, D, Cin)
    W = rnd(27, Cin, Cout)
    b = rnd(Cout)
    y = oracle.conv3d(x, W, b)
    for s in range(B):
        for co in range(Cout):
            ref = np.full((D, D, D), b[co])
            for ci in range(Cin):
                # numpy array indexed [z][y][x]; W tap t = (dx+1)+3(dy+1)+9(dz+1)
                K = W[:, ci, co].reshape(3, 3, 3)
                ref += correlate(x[s, ..., ci], K, mode="same")
            assert np.allclose(y[s, ..., co], ref, atol=1e-12)


def test_conv3d_relu():
    x = rnd(1, 4, 4, 4, 2)
    W = rnd(27, 2, 3)
    b = rnd(3)
    assert np.allclose(oracle.conv3d(x, W, b, relu=True), np.maximum(oracle.conv3d(x, W, b), 0.0))


def test_conv3d_backward_data_is_adjoint():
    B, D, Cin, Cout = 2, 5, 3, 4
    x = rnd(B, D, D, D, Cin)
    W = rnd(27, Cin, Cout)
    dy = rnd(B, D, D, D, Cout)
    lhs = np.sum(oracle.conv3d(x, W) * dy)
    rhs = np.sum(x * oracle.conv3d_bwd_data(dy, W))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_conv3d_backward_weight_is_adjoint():
    B, D, Cin, Cout = 2, 5, 3, 4
    x = rnd(B, D, D, D, Cin)
    W = rnd(27, Cin, Cout)
    dy = rnd(B, D, D, D, Cout)
    dW, db = oracle.conv3d_bwd_weight(x, dy)
    lhs = np.sum(oracle.conv3d(x, W) * dy)
    assert abs(lhs - np.sum(W * dW)) < 1e-10 * abs(lhs)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2, 3)))


def test_pool_upsample_adjoint_pair():
    x = rnd(2, 8, 8, 8, 3)
    y = rnd(2, 4, 4, 4, 3)
    assert abs(np.sum(oracle.avgpool2(x) * y) - np.sum(x * oracle.upsample2(y)) / 8) < 1e-10
    assert np.allclose(oracle.avgpool2(oracle.upsample2(y)), y)


def test_unet_param_count():
    n = sum(27 * ci * co + co for ci, co in oracle.UNET_LAYERS) + 16 * 2 + 2
    assert oracle.unet_nparams() == n == 354594


def test_unet_gradient_central_differences():
    """Directional derivatives against central differences. The loss of a
    ReLU network is differentiable except on the kinks where a pre-activation
    is zero; a difference quotient whose +-eps step crosses a kink is not the
    derivative (at eps = 1e-6 that happens in most directions here). So each
    direction takes the best of eps = 1e-7, 1e-8, 1e-9: a crossing disappears
    once eps is below the kink's distance, while a wrong gradient (a missing
    factor, a dropped mask) is off by O(1) at every eps. The gradient is of
    order 1e3, so rounding stays near 1e-10 relative even at eps = 1e-9."""
    R = np.random.default_rng(5)
    D, B = 8, 2
    n = oracle.unet_nparams()
    p = 0.1 * R.standard_normal(n)
    x = R.standard_normal((B, D, D, D, 4))
    t = R.standard_normal((B, D, D, D, 2))
    mask = (R.uniform(size=(D, D, D)) > 0.2).astype(float)
    loss, g = oracle.unet_loss_grad(p, x, t, mask)
    for _ in range(4):
        d = R.standard_normal(n)
        errs = []
        for eps in (1e-7, 1e-8, 1e-9):
            lp, _ = oracle.unet_loss_grad(p + eps * d, x, t, mask)
            lm, _ = oracle.unet_loss_grad(p - eps * d, x, t, mask)
            fd = (lp - lm) / (2 * eps)
            errs.append(abs(fd - g @ d) / max(abs(fd), 1e-8))
        assert min(errs) < 1e-5, (errs, g @ d)


def test_unet_forward_consistent_with_loss():
    D, B = 8, 1
    p = 0.1 * rnd(oracle.unet_nparams())
    x = rnd(B, D, D, D, 4)
    out = oracle.unet_forward(p, x)
    loss, _ = oracle.unet_loss_grad(p, x, out)  # target = output -> zero loss
    assert loss < 1e-28


def np_conv3(x, W, b):
    """3x3x3 'same' convolution by its definition, written as 27 shifted
    slices of a zero-padded volume: out[v] = b + sum_t x[v + off(t)] W[t],
    off(t) = (t % 3 - 1, t // 3 % 3 - 1, t // 9 - 1) along (x, y, z); arrays
    are [B][z][y][x][C]. Followed by ReLU (every 3x3x3 layer has one)."""
    D = x.shape[1]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, x.shape[:4] + (W.shape[2],)).copy()
    for t in range(27):
        dx, dy, dz = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
        y += xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + D, 1 + dx:1 + dx + D, :] @ W[t]
    return np.maximum(y, 0.0)


def test_unet_forward_equals_composition():
    """The whole network against its composition from the pinned parts,
    in numpy: encoder 16/16, pool, 32/32, pool, 64/64; decoder upsample,
    concatenate [upsampled, skip] (skip in the trailing channels), 32/32,
    upsample, concatenate, 16/16; linear 1x1x1 head to 2 channels.
    Parameters unpacked in layer order, W[27][Cin][Cout] then b[Cout], the
    head W[16][2] then b[2]. A skip in the wrong channels, a swapped layer or
    a misread packing fails here; none of them would fail the gradient
    check, which differentiates the oracle's own forward pass."""
    D, B = 8, 2
    n = oracle.unet_nparams()
    p = 0.2 * rnd(n)
    x = rnd(B, D, D, D, 4)
    layers, off = [], 0
    for ci, co in oracle.UNET_LAYERS:
        W = p[off:off + 27 * ci * co].reshape(27, ci, co)
        off += 27 * ci * co
        layers.append((W, p[off:off + co]))
        off += co
    Wh, bh = p[off:off + 32].reshape(16, 2), p[off + 32:off + 34]
    assert off + 34 == n

    def pool(a):
        b_, d, c = a.shape[0], a.shape[1] // 2, a.shape[4]
        return a.reshape(b_, d, 2, d, 2, d, 2, c).mean(axis=(2, 4, 6))

    def up(a):
        return a.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)

    L = [lambda a, k=k: np_conv3(a, *layers[k]) for k in range(10)]
    s1 = L[1](L[0](x))
    s2 = L[3](L[2](pool(s1)))
    a5 = L[5](L[4](pool(s2)))
    a7 = L[7](L[6](np.concatenate([up(a5), s2], axis=4)))
    a9 = L[9](L[8](np.concatenate([up(a7), s1], axis=4)))
    ref = a9 @ Wh + bh
    out = oracle.unet_forward(p, x)
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
