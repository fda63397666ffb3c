"""GPU adjoint and transposed solves, sensitivity products (eq:fwisens) and
16-bit field storage, through the C-ABI, against the oracle
(oracle/sens.py, pinned by finite differences and adjoint identities):

  - H^H U = Q (op "HH") against the oracle's adjoint solve, and H^T U = Q
    (op "HT") bitwise equal to the H U = Q solve (H is complex symmetric);
  - J dm and Re sum_s J_s^H w_s for fields from the oracle's solve, the GPU
    solves at 1e-9 against the oracle's at 1e-11: relative error <= 1e-5
    (a 1e-9 residual bounds the error by about kappa * 1e-9);
  - 16-bit storage: the half values and scales equal the oracle's bitwise
    (the same IEEE roundings: FP64 division, FP32, FP16); the products from
    16-bit fields match the oracle's on the unpacked fields.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import sens

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")

RNG = np.random.default_rng(3131)


def dev(a, dtype=np.complex128):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module", params=[(2, 128), (3, 32)])
def case(request):
    dim, n = request.param
    p = synth.gradient_2d(n=n, nsrc=(3,), levels=3) if dim == 2 else synth.layered_3d(n=n, nsrc=(2, 2), levels=3,
                                                                                     seed=2)
    g = oracle.grid(p.dim, p.n, p.h)
    ho = oracle.Hierarchy(g, p.m, p.gamma, p.omega, p.shift, 3)
    U = sens.solve(ho, p.Q, tol=1e-12)
    dm = (0.05 * p.m.max()) * RNG.standard_normal(p.N)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=3)
    return p, ho, hd, U, dm


def test_adjoint_and_transposed_solves(case):
    p, ho, hd, U, dm = case
    W = RNG.standard_normal((p.nrhs, p.N)) + 1j * RNG.standard_normal((p.nrhs, p.N))
    Wd = dev(W)
    Y = torch.zeros_like(Wd)
    info = pk.helm_solve_block(hd, Wd, Y, tol=1e-9, block_size=1, max_cycles=3000, op="HH")
    assert info["converged_all"]
    ref = sens.solve(ho, W, tol=1e-11, op="A")
    assert rel(Y.cpu().numpy(), ref) <= 1e-5
    X1 = torch.zeros_like(Wd)
    X2 = torch.zeros_like(Wd)
    i1 = pk.helm_solve_block(hd, Wd, X1, tol=1e-9, block_size=1, max_cycles=3000, op="H")
    i2 = pk.helm_solve_block(hd, Wd, X2, tol=1e-9, block_size=1, max_cycles=3000, op="HT")
    assert i1["cycles"] == i2["cycles"] and torch.equal(X1, X2)


def test_jvp_and_jtvp_match_oracle(case):
    p, ho, hd, U, dm = case
    Ud = dev(U)
    JV = torch.empty_like(Ud)
    info = pk.helm_jvp(hd, dev(dm, np.float64), JV, U=Ud, tol=1e-9, max_cycles=3000)
    assert info["converged_all"]
    ref = sens.jvp(ho, U, dm, tol=1e-11)
    assert rel(JV.cpu().numpy(), ref) <= 1e-5, rel(JV.cpu().numpy(), ref)
    W = RNG.standard_normal(U.shape) + 1j * RNG.standard_normal(U.shape)
    g = torch.empty(p.N, dtype=torch.float64, device="cuda")
    info = pk.helm_jtvp(hd, dev(W), g, U=Ud, tol=1e-9, max_cycles=3000)
    assert info["converged_all"]
    gref = sens.jtvp(ho, U, W, tol=1e-11)
    assert rel(g.cpu().numpy(), gref) <= 1e-5, rel(g.cpu().numpy(), gref)


def test_fields_16bit_match_oracle(case):
    p, ho, hd, U, dm = case
    Ud = dev(U)
    U16, sc = pk.helm_fields_pack16(hd, Ud)
    href, sref = sens.pack16(U)
    assert np.array_equal(sc.cpu().numpy(), sref)
    assert np.array_equal(U16.cpu().numpy().view(np.uint16), href.view(np.uint16))
    Uu = torch.empty_like(Ud)
    pk.helm_fields_unpack16(hd, U16, sc, Uu)
    Uref = sens.unpack16(href, sref)
    assert np.array_equal(Uu.cpu().numpy(), Uref)
    # products from the 16-bit fields
    JV = torch.empty_like(Ud)
    info = pk.helm_jvp(hd, dev(dm, np.float64), JV, U16=U16, scales=sc, tol=1e-9, max_cycles=3000)
    assert info["converged_all"]
    ref = sens.jvp(ho, Uref, dm, tol=1e-11)
    assert rel(JV.cpu().numpy(), ref) <= 1e-5
    # and the 16-bit fields are within 2^-11 of the full fields (per source scale)
    assert np.max(np.abs(Uref - U) / sref[:, None]) <= 2.0 ** -11
