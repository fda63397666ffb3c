"""The synthetic inputs follow their stated recipe.

The paper's experiments use the SEG/EAGE model, which is not available; the
workloads are seeded synthetic stand-ins with its velocity range and the
points-per-wavelength rule of the multigrid experiments. These checks pin
each generator to the recipe: velocity range and perturbation size, the
frequency from the points-per-wavelength rule, the absorbing layer (free
top surface), and the sources (first unknown row, outside the layer,
finite-volume amplitude h^-d).
"""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def bench():
    return synth.layered_3d(192, seed=3, nsrc=(8, 8))


def ppw_at_vmin(p):
    v = 1.0 / np.sqrt(p.m)
    return 2 * math.pi * v.min() / (p.omega * p.h[0])


def check_sources(p, count, width):
    n = p.n[0]
    h = p.h[0]
    shape = (n - 1,) * p.dim
    assert p.Q.shape == (count, p.N)
    seen = set()
    for s in range(count):
        nz = np.flatnonzero(p.Q[s])
        assert nz.size == 1 and p.Q[s, nz[0]] == h ** (-p.dim)
        idx = np.unravel_index(nz[0], shape)
        assert idx[0] == 0  # depth index 0: the first unknown row below the free surface
        for lateral in idx[1:]:
            assert width - 1 <= lateral <= n - width - 1  # outside the absorbing layer
        seen.add(idx)
    assert len(seen) == count


def test_benchmark_workload(bench):
    p = bench
    assert p.dim == 3 and p.n == (192, 192, 192) and p.N == 191 ** 3
    v = 1.0 / np.sqrt(p.m)
    assert 1.5 * 0.9 - 1e-12 <= v.min() and v.max() <= 4.5 * 1.1 + 1e-12
    # layers (the same seed without the perturbation: the layer draws come
    # first) are constant in depth rows, at most 8 velocities in 1.5-4.5,
    # increasing with depth; the model is that times (1 + p), max |p| = 0.1
    base = synth.layered_model(3, 192, 3, pert=0.0)
    rows = base[:, 0, 0]
    assert np.all(base == rows[:, None, None])
    assert len(np.unique(rows)) <= 8 and np.all(np.diff(rows) >= 0)
    assert 1.5 <= rows.min() and rows.max() <= 4.5
    assert abs(np.abs(v / base - 1).max() - 0.1) < 1e-12
    assert abs(ppw_at_vmin(p) - 8.0) < 1e-12
    # absorbing layer: 12 cells on the sides and bottom, none at the top
    g = p.gamma
    assert g.shape == (191,) * 3 and g.min() == 0.0
    assert np.all(g[:191 - 12, 12:191 - 12, 12:191 - 12] == 0.0)
    assert g[0, 100, 100] == 0.0 and g[-1, 100, 100] > 0.0 and g[100, 100, 0] > 0.0
    assert abs(g.max() - 0.3) < 0.3 * 0.2
    check_sources(p, 64, 12)


def test_2d_gradient_workload():
    p = synth.gradient_2d()
    assert p.dim == 2 and p.n == (128, 128) and p.restart == 10 and p.levels == 3
    v = 1.0 / np.sqrt(p.m)
    assert np.allclose(v[:, 0], 1.5 + 1.5 * np.arange(1, 128) / 128)
    assert np.all(v == v[:, :1])  # velocity depends on depth only
    assert abs(ppw_at_vmin(p) - 10.0) < 1e-12
    assert np.all(p.gamma[:127 - 16, 16:127 - 16] == 0.0) and p.gamma[-1, 64] > 0.0
    check_sources(p, 4, 16)


def test_training_models_share_the_recipe_not_the_seed(bench):
    t = synth.training_model(0, n=64)
    assert t.levels == 3 and abs(ppw_at_vmin(t) - 8.0) < 1e-12
    check_sources(t, 32, 12)
    v0 = 1.0 / np.sqrt(synth.training_model(0, n=64).m)
    v1 = 1.0 / np.sqrt(synth.training_model(1, n=64).m)
    assert not np.allclose(v0, v1)  # each model has its own seed


def test_batch_instances_rules():
    """First half 2D (n from 64..512 step 32), second half 3D (n from 64,
    96, 128, 160); 8-12 points per wavelength, 3 levels from 8 up (2
    below), 1-32 sources; every instance has its own seed."""
    insts = synth.batch_instances(count=4)
    assert [p.dim for p in insts] == [2, 2, 3, 3]
    for p in insts:
        sizes = range(64, 513, 32) if p.dim == 2 else (64, 96, 128, 160)
        assert p.n[0] in sizes
        w = ppw_at_vmin(p)
        assert 8.0 - 1e-9 <= w <= 12.0 + 1e-9
        assert p.levels == (3 if w >= 8.0 else 2)
        assert 1 <= p.nrhs <= 32
        check_sources(p, p.nrhs, 16 if p.dim == 2 else 12)
    low = synth.batch_instances(count=2, sizes_2d=[64], ppw=(6.0, 7.9))
    assert all(p.levels == 2 for p in low)


def test_frequency_sweep_keeps_model_and_sources():
    import synth
    base = synth.gradient_2d(n=64, nsrc=(2,), levels=3)
    sw = synth.frequency_sweep(base)
    assert len(sw) == 5
    ratios = [p.omega / base.omega for p in sw]
    assert np.allclose(ratios, np.array([2.0, 2.5, 3.5, 4.5, 6.0]) / 6.0)
    for p in sw:
        assert p.m is base.m and p.gamma is base.gamma and p.Q is base.Q and p.levels == base.levels
