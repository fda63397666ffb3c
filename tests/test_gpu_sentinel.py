"""Write coverage: no kernel reads device memory that no kernel has written.

With HELM_SENTINEL=1 in the environment every buffer the library allocates
(hierarchy, fields, Krylov and coarsest-solve workspaces, the network's
activations) starts filled with 0xFF bytes, a NaN in FP64, FP32 and BF16.
Caller buffers get the same treatment here: the outputs (U without a warm
start, Z, Y, E, 16-bit fields, J dm, the gradient) and a caller-provided
solve workspace are filled with 0xFF before each call. Every result must then
be finite and bitwise equal to the same call on fresh handles and
zero-filled buffers without the sentinel (the kernels are deterministic and
the finest-level tile is fixed), so a read of unwritten memory anywhere on
these paths would show. Paths: block FGMRES in FP64 and mixed precision
(block sizes 1 and 4; LDS-tiled fused kernels at 16 columns), the K-cycle,
block BiCGSTAB, the learned coarsest correction, the residual, one cycle, the
operator, the coarsest solve, 16-bit fields and the sensitivity products.
"""
import ctypes
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")


def filled(shape, dtype, byte):
    """A CUDA tensor whose every byte is `byte`."""
    t = torch.empty(shape, dtype=dtype, device="cuda")
    t.view(torch.uint8).fill_(byte)
    return t


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


class Sentinel:
    def __enter__(self):
        os.environ["HELM_SENTINEL"] = "1"

    def __exit__(self, *exc):
        os.environ.pop("HELM_SENTINEL", None)


def run_paths(byte):
    """Every covered path on fresh handles, caller buffers filled with
    `byte`; returns a dict of host results."""
    out = {}
    p3 = synth.layered_3d(n=48, nsrc=(4, 4), levels=3, seed=2)  # 16 sources
    Q3 = torch.from_numpy(np.ascontiguousarray(p3.Q)).cuda()
    for prec in ("fp64", "mixed"):
        hd = pk.helm_setup(p3.dim, p3.n, p3.h, p3.m, p3.gamma, p3.omega, shift=p3.shift, levels=3,
                           precision=prec, coarse="gmres", coarse_iters=20)
        pk.helm_set_fine_tile(hd, 16, 16, 16)
        for bs in (1, 4):
            ws = filled(pk.helm_workspace_size(hd, 16, 5), torch.uint8, byte)
            U = filled(Q3.shape, torch.complex128, byte)
            info = pk.helm_solve_block(hd, Q3, U, tol=1e-7, restart=5, block_size=bs, reorth=0, workspace=ws)
            assert info["converged_all"], (prec, bs)
            out[f"solve-{prec}-{bs}"] = host(U)
            out[f"cycles-{prec}-{bs}"] = info["cycles"]
        Z = filled(Q3.shape, torch.complex128, byte)
        out[f"precond-{prec}"] = host(pk.helm_precond(hd, Q3, Z))
        Y = filled(Q3.shape, torch.complex128, byte)
        out[f"apply-{prec}"] = host(pk.helm_apply(hd, Q3, Y))
        out[f"resid-{prec}"] = pk.helm_residual(hd, Q3, torch.from_numpy(out[f"solve-{prec}-1"]).cuda())
        del hd
    # K-cycle, mixed
    hk = pk.helm_setup(p3.dim, p3.n, p3.h, p3.m, p3.gamma, p3.omega, shift=p3.shift, levels=3,
                       precision="mixed", coarse="gmres", coarse_iters=20, cycle="K")
    pk.helm_set_fine_tile(hk, 16, 16, 16)
    U = filled(Q3.shape, torch.complex128, byte)
    assert pk.helm_solve_block(hk, Q3, U, tol=1e-7, restart=5, block_size=1, reorth=0)["converged_all"]
    out["kcycle"] = host(U)
    del hk
    # block BiCGSTAB (2D, FP64, exact coarsest), the coarsest solve, 16-bit
    # fields and the sensitivity products
    p2 = synth.gradient_2d(n=64, nsrc=(4,), levels=3)
    Q2 = torch.from_numpy(np.ascontiguousarray(p2.Q)).cuda()
    h2 = pk.helm_setup(p2.dim, p2.n, p2.h, p2.m, p2.gamma, p2.omega, shift=p2.shift, levels=3)
    U = filled(Q2.shape, torch.complex128, byte)
    assert pk.helm_solve_block(h2, Q2, U, tol=1e-8, block_size=2, method="bicgstab")["converged_all"]
    out["bicgstab"] = host(U)
    nc = int(np.prod(pk.helm_level_dims(h2, 2)))
    R = torch.from_numpy(np.ascontiguousarray(p2.Q[:, :nc])).cuda()
    E = filled(R.shape, torch.complex128, byte)
    out["coarse"] = host(pk.helm_coarse_solve(h2, R, E))
    U16, sc = pk.helm_fields_pack16(h2, U)
    out["pack16"] = host(U16.view(torch.int16)).copy()
    out["scales"] = host(sc)
    U1 = filled(Q2.shape, torch.complex128, byte)
    pk.helm_fields_unpack16(h2, U16, sc, U1)
    out["unpack16"] = host(U1)
    dm = torch.from_numpy(np.linspace(0.0, 1.0, p2.N)).cuda()
    JV = filled(Q2.shape, torch.complex128, byte)
    assert pk.helm_jvp(h2, dm, JV, U=U, tol=1e-9)["converged_all"]
    out["jvp"] = host(JV)
    g = filled((p2.N,), torch.float64, byte)
    assert pk.helm_jtvp(h2, Q2, g, U16=U16, scales=sc, tol=1e-9)["converged_all"]
    out["jtvp"] = host(g)
    del h2
    # learned coarsest correction (an untrained network + 4 GMRES steps)
    p4 = synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)
    Q4 = torch.from_numpy(np.ascontiguousarray(p4.Q)).cuda()
    h4 = pk.helm_setup(p4.dim, p4.n, p4.h, p4.m, p4.gamma, p4.omega, shift=p4.shift, levels=3)
    nu = pk.helm_level_dims(h4, 2)
    net = pk.helm_net_create((max(nu) + 3) // 4 * 4, 4, seed=6)
    blob = net.save()
    net.close()
    del h4
    hl = pk.helm_setup(p4.dim, p4.n, p4.h, p4.m, p4.gamma, p4.omega, shift=p4.shift, levels=3,
                       precision="mixed", coarse="learned", net=blob, coarse_iters=4)
    U = filled(Q4.shape, torch.complex128, byte)
    info = pk.helm_solve_block(hl, Q4, U, tol=1e-6, restart=5, block_size=1, max_cycles=800)
    assert info["converged_all"]
    out["learned"] = host(U)
    del hl
    return out


def test_sentinel_filled_memory_changes_no_result():
    ref = run_paths(0x00)
    with Sentinel():
        # the library reads the variable with the C library's getenv
        libc = ctypes.CDLL(None)
        libc.getenv.restype = ctypes.c_char_p
        assert libc.getenv(b"HELM_SENTINEL") == b"1"
        sen = run_paths(0xFF)
    assert ref.keys() == sen.keys()
    for k in ref:
        a, b = np.asarray(ref[k]), np.asarray(sen[k])
        assert np.isfinite(b.astype(np.float64) if b.dtype.kind in "iu" else b).all(), k
        assert np.array_equal(a, b), k
