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
    D, B = 8, 2
    n = oracle.unet_nparams()
    p = 0.1 * rnd(n)
    x = rnd(B, D, D, D, 4)
    t = rnd(B, D, D, D, 2)
    mask = (RNG.uniform(size=(D, D, D)) > 0.2).astype(float)
    loss, g = oracle.unet_loss_grad(p, x, t, mask)
    for _ in range(4):
        d = rnd(n)
        eps = 1e-6
        lp, _ = oracle.unet_loss_grad(p + eps * d, x, t, mask)
        lm, _ = oracle.unet_loss_grad(p - eps * d, x, t, mask)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g @ d) < 1e-5 * max(abs(fd), 1e-8), (fd, g @ d)


def test_unet_forward_consistent_with_loss():
    D, B = 8, 1
    p = 0.1 * rnd(oracle.unet_nparams())
    x = rnd(B, D, D, D, 4)
    out = oracle.unet_forward(p, x)
    loss, _ = oracle.unet_loss_grad(p, x, out)  # target = output -> zero loss
    assert loss < 1e-28
