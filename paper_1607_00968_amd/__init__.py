"""Python binding of libhelm.so, the MI355X block shifted-Laplacian Helmholtz solver.

The binding only marshals arguments: every step of the solve runs in the
library's HIP kernels. PyTorch provides device memory (complex128 CUDA
tensors) and the current stream. The functions mirror ``include/helm.h``:

    h = helm_setup(dim, n, h, m, gamma, omega, ...)
    info = helm_solve_block(h, Q, U, tol, restart=5, ...)
    relres = helm_residual(h, Q, U)

``Q`` and ``U`` are complex128 tensors on the GPU, shaped ``[nrhs, N]``
(each right-hand side contiguous, grid axis 0 fastest). If the shared library
is missing the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "HelmError", "lib", "LIBPATH", "Handle", "helm_setup", "helm_solve_block",
    "helm_profile_enable", "helm_profile_read", "KERNEL_CLASSES",
    "helm_residual", "helm_residual_noalloc", "helm_apply", "helm_precond", "helm_level_stencil",
    "helm_fields_pack16", "helm_fields_unpack16", "helm_jvp", "helm_jtvp",
    "helm_level_dims", "helm_coarse_solve", "helm_workspace_size", "helm_solve_batch", "ABI_SYMBOLS",
    "Net", "helm_net_nparams", "helm_net_create", "helm_net_capture", "helm_setup_batch",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libhelm.so")
MAX_LEVELS = 8

HELM_OK, HELM_ERR_INVALID_ARG, HELM_ERR_OOM, HELM_ERR_DEVICE = 0, 1, 2, 3
HELM_ERR_NOT_CONVERGED, HELM_ERR_BREAKDOWN, HELM_ERR_NONFINITE, HELM_ERR_UNSUPPORTED = 4, 5, 6, 7
PRECISION = {"fp64": 0, "mixed": 1}
COARSE = {"lu": 0, "learned": 1, "none": 2, "gmres": 3}
CYCLE = {"V": 0, "W": 1, "K": 2}

ABI_SYMBOLS = (
    "helm_setup_desc_default", "helm_setup", "helm_destroy", "helm_workspace_size",
    "helm_solve_block", "helm_solve_batch", "helm_residual", "helm_residual_noalloc", "helm_apply", "helm_precond",
    "helm_level_dims", "helm_level_stencil", "helm_coarse_solve",
    "helm_profile_enable", "helm_profile_read", "helm_fine_tile", "helm_set_fine_tile",
    "helm_status_string", "helm_last_error",
    "helm_net_nparams", "helm_net_create", "helm_net_destroy", "helm_net_set_params",
    "helm_net_get_params", "helm_net_get_state", "helm_net_set_state", "helm_net_save", "helm_net_forward",
    "helm_net_loss_grad",
    "helm_net_capture", "helm_net_pairs", "helm_net_pool_read", "helm_net_train", "helm_net_train_step",
    "helm_fields_pack16", "helm_fields_unpack16", "helm_jvp", "helm_jtvp", "helm_setup_batch",
)
KERNEL_CLASSES = ("fine_sweep", "fine_resid", "outer_apply", "transfer", "coarse_sweep",
                  "coarsest", "gram", "update", "fine_sweep0", "fine_prosweep", "fine_sweep01",
                  "fine_pre_rr")


class HelmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"helm status {status}: {msg}")
        self.status = status


class SetupDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3),
        ("m", C.c_void_p), ("gamma", C.c_void_p), ("omega", C.c_double),
        ("shift", C.c_double), ("levels", C.c_int32),
        ("nu_pre", C.c_int32 * MAX_LEVELS), ("nu_post", C.c_int32 * MAX_LEVELS),
        ("jacobi_weight", C.c_double * MAX_LEVELS), ("precision", C.c_int32),
        ("coarse", C.c_int32), ("cycle", C.c_int32), ("coarse_iters", C.c_int32),
        ("net", C.c_void_p), ("net_bytes", C.c_size_t), ("coarse_restarts", C.c_int32),
    ]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_cycles", C.c_int32), ("block_size", C.c_int32),
                ("warm_start", C.c_int32), ("reorth", C.c_int32), ("graph", C.c_int32),
                ("learned_rate", C.c_double), ("method", C.c_int32), ("op", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("restarts", C.c_int32), ("converged_all", C.c_int32),
                ("fallback_used", C.c_int32), ("t_solve_ms", C.c_double),
                ("relres", C.c_void_p), ("converged", C.c_void_p), ("rate_switch", C.c_int32)]


_lib = None


def lib():
    """The loaded libhelm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "`python -m paper_1607_00968_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIBPATH)
        P, I, D = C.c_void_p, C.c_int32, C.c_double
        L.helm_setup_desc_default.argtypes = [C.POINTER(SetupDesc)]
        L.helm_setup.argtypes = [C.POINTER(SetupDesc), P, C.POINTER(P)]
        L.helm_destroy.argtypes = [P]
        L.helm_workspace_size.argtypes = [P, I, I, C.POINTER(C.c_size_t)]
        L.helm_solve_block.argtypes = [P, I, P, P, D, C.POINTER(SolveOpts), P, C.c_size_t,
                                       C.POINTER(SolveInfo), P]
        L.helm_residual.argtypes = [P, I, P, P, P, P]
        L.helm_residual_noalloc.argtypes = [P, I, P, P, P, P]
        L.helm_fields_pack16.argtypes = [P, I, P, P, P, P]
        L.helm_setup_batch.argtypes = [I, P, P, P]
        L.helm_fields_unpack16.argtypes = [P, I, P, P, P, P]
        L.helm_jvp.argtypes = [P, I, P, P, P, P, P, D, P, P, P]
        L.helm_jtvp.argtypes = [P, I, P, P, P, P, P, D, P, P, P]
        L.helm_solve_batch.argtypes = [I, P, P, P, P, D, C.POINTER(SolveOpts), P, P, I, P]
        L.helm_apply.argtypes = [P, I, I, P, P, P]
        L.helm_precond.argtypes = [P, I, P, P, P]
        L.helm_level_dims.argtypes = [P, I, P]
        L.helm_level_stencil.argtypes = [P, I, P]
        L.helm_coarse_solve.argtypes = [P, I, P, P, P]
        L.helm_profile_enable.argtypes = [P, I]
        L.helm_fine_tile.argtypes = [P, I, P]
        L.helm_set_fine_tile.argtypes = [P, I, P]
        L.helm_profile_read.argtypes = [P, P]
        L.helm_status_string.restype = C.c_char_p
        L.helm_status_string.argtypes = [I]
        L.helm_last_error.restype = C.c_char_p
        L.helm_net_nparams.restype = C.c_int64
        L.helm_net_nparams.argtypes = []
        L.helm_net_create.argtypes = [I, I, C.c_uint64, P, C.POINTER(P)]
        L.helm_net_destroy.argtypes = [P]
        L.helm_net_set_params.argtypes = [P, P]
        L.helm_net_get_params.argtypes = [P, P]
        L.helm_net_get_state.argtypes = [P, P, P]
        L.helm_net_set_state.argtypes = [P, P, C.c_int64]
        L.helm_net_save.argtypes = [P, P, C.POINTER(C.c_size_t)]
        L.helm_net_forward.argtypes = [P, I, P, P, P]
        L.helm_net_loss_grad.argtypes = [P, I, P, P, P, P, C.POINTER(D), P]
        L.helm_net_capture.argtypes = [P, P, I]
        L.helm_net_pairs.restype = C.c_int64
        L.helm_net_pairs.argtypes = [P]
        L.helm_net_pool_read.argtypes = [P, C.c_int64, P, P, P]
        L.helm_net_train.argtypes = [P, I, I, D, C.c_uint64, P, P]
        L.helm_net_train_step.argtypes = [P, I, P, P, P, D, C.POINTER(D), P]
        _lib = L
    return _lib


def _check(st: int, allow=()):
    if st != HELM_OK and st not in allow:
        raise HelmError(st, lib().helm_last_error().decode(errors="replace"))
    return st


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_block(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.dim() == 2
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor [nrhs, N]")
    return C.c_void_p(t.data_ptr())


class Handle:
    """Owns a helm_handle (the device hierarchy)."""

    def __init__(self, ptr, dim, n, levels, precision):
        self.ptr = ptr
        self.dim = dim
        self.n = tuple(n)
        self.levels = levels
        self.precision = precision
        self.N = int(np.prod([c - 1 for c in self.n]))
        self.capture_net = None  # the Net whose pool this handle feeds (kept alive while attached)

    def close(self):
        if self.ptr:
            lib().helm_destroy(self.ptr)
            self.ptr = None
        self.capture_net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _per_level(v, levels, typ):
    if np.isscalar(v):
        v = [v] * levels
    v = list(v) + [v[-1]] * (MAX_LEVELS - len(v))
    return (typ * MAX_LEVELS)(*v[:MAX_LEVELS])


def _setup_desc(dim, n, h, m, gamma, omega, shift=0.2, levels=3, nu_pre=2, nu_post=2,
                jacobi_weight=0.8, precision="fp64", coarse="lu", cycle="V", coarse_iters=20,
                net=None, coarse_restarts=1):
    """(descriptor, host buffers it points at) for helm_setup."""
    d = SetupDesc()
    lib().helm_setup_desc_default(C.byref(d))
    d.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    hh = list(h) + [1.0] * (3 - len(h))
    for a in range(3):
        d.n[a] = int(nn[a])
        d.h[a] = float(hh[a])
    m = np.ascontiguousarray(m, dtype=np.float64).ravel()
    gamma = np.ascontiguousarray(gamma, dtype=np.float64).ravel()
    d.m = m.ctypes.data
    d.gamma = gamma.ctypes.data
    d.omega = float(omega)
    d.shift = float(shift)
    d.levels = int(levels)
    d.nu_pre = _per_level(nu_pre, levels, C.c_int32)
    d.nu_post = _per_level(nu_post, levels, C.c_int32)
    d.jacobi_weight = _per_level(jacobi_weight, levels, C.c_double)
    d.precision = PRECISION[precision]
    d.coarse = COARSE[coarse]
    d.cycle = CYCLE[cycle]
    d.coarse_iters = int(coarse_iters)
    d.coarse_restarts = int(coarse_restarts)
    blob = None
    if net is not None:
        blob = np.ascontiguousarray(np.frombuffer(net, dtype=np.uint8))
        d.net = blob.ctypes.data
        d.net_bytes = blob.nbytes
    return d, (m, gamma, blob, nn)


def helm_setup(dim, n, h, m, gamma, omega, shift=0.2, levels=3, nu_pre=2, nu_post=2,
               jacobi_weight=0.8, precision="fp64", coarse="lu", cycle="V", coarse_iters=20,
               net=None, stream=None, coarse_restarts=1) -> Handle:
    """Build the hierarchy. m, gamma: host float64 arrays of N entries."""
    d, keep = _setup_desc(dim, n, h, m, gamma, omega, shift, levels, nu_pre, nu_post, jacobi_weight, precision,
                          coarse, cycle, coarse_iters, net, coarse_restarts)
    out = C.c_void_p()
    _check(lib().helm_setup(C.byref(d), _stream(stream), C.byref(out)))
    return Handle(out, dim, keep[3][:dim], levels, precision)


def helm_setup_batch(problems, stream=None, **kw) -> list:
    """One hierarchy per problem (objects with dim, n, h, m, gamma, omega,
    shift and levels, e.g. synth.Problem), built by one helm_setup_batch call;
    kw as for helm_setup (shared by all)."""
    k = len(problems)
    descs = (SetupDesc * k)()
    keep = []
    for i, p in enumerate(problems):
        d, kp = _setup_desc(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=p.levels, **kw)
        descs[i] = d
        keep.append(kp)
    out = (C.c_void_p * k)()
    _check(lib().helm_setup_batch(k, descs, _stream(stream), out))
    return [Handle(C.c_void_p(out[i]), p.dim, keep[i][3][:p.dim], p.levels, kw.get("precision", "fp64"))
            for i, p in enumerate(problems)]


def helm_workspace_size(hd: Handle, nrhs: int, restart: int = 5) -> int:
    b = C.c_size_t()
    _check(lib().helm_workspace_size(hd.ptr, nrhs, restart, C.byref(b)))
    return b.value


def _form(graph) -> int:
    """Execution form of the cycle: False/0 eager, True/1 HIP graph,
    "persistent"/2 the cooperative persistent kernel."""
    return 2 if graph == "persistent" else int(graph)


METHOD = {"fgmres": 0, "bicgstab": 1}
OP = {"H": 0, "HT": 1, "HH": 2}


def helm_solve_block(hd: Handle, Q, U, tol=1e-6, restart=5, max_cycles=1000, block_size=0,
                     warm_start=False, reorth=True, workspace=None, stream=None, graph=False,
                     learned_rate=0.0, method="fgmres", op="H") -> dict:
    """Solve H U = Q (U overwritten). Returns a dict with cycles, relres, ...
    reorth: 0 one Gram-Schmidt pass, 1 (True, the default here) always two,
    2 a second pass only where the norm fell below half (the C default when
    no options are passed). graph: False/0 eager, True/1 HIP graphs,
    "persistent"/2 the persistent cycle kernel. learned_rate: the plain
    cycle's calibrated per-cycle reduction factor for the learned coarsest
    correction's rate check (0 = off). method: "fgmres" (block FGMRES(restart))
    or "bicgstab" (block BiCGSTAB, two cycles per iteration). op: "H" (H U = Q),
    "HT" (the transposed system, the same one) or "HH" (the adjoint)."""
    nrhs = Q.shape[0]
    qp, up = _dev_block(Q, "Q"), _dev_block(U, "U")
    if U.shape != Q.shape or Q.shape[1] != hd.N:
        raise ValueError("Q and U must both be [nrhs, N]")
    o = SolveOpts(restart, max_cycles, block_size, int(bool(warm_start)), int(reorth), _form(graph),
                  float(learned_rate), METHOD[method], OP[op])
    rel = np.zeros(nrhs)
    conv = np.zeros(nrhs, np.int32)
    info = SolveInfo()
    info.relres = rel.ctypes.data
    info.converged = conv.ctypes.data
    wp, wb = (None, 0) if workspace is None else (C.c_void_p(workspace.data_ptr()), workspace.numel()
                                                   * workspace.element_size())
    st = _check(lib().helm_solve_block(hd.ptr, nrhs, qp, up, float(tol), C.byref(o), wp, wb,
                                       C.byref(info), _stream(stream)), allow=(HELM_ERR_NOT_CONVERGED,))
    return {"status": st, "cycles": info.cycles, "restarts": info.restarts,
            "converged_all": bool(info.converged_all), "fallback_used": int(info.fallback_used),
            "t_solve_ms": info.t_solve_ms, "relres": rel, "converged": conv.astype(bool),
            "rate_switch": int(info.rate_switch)}


def helm_solve_batch(handles, Qs, Us, tol=1e-6, restart=5, max_cycles=1000, block_size=1, reorth=0,
                     graph=False, max_threads=16, stream=None, learned_rate=0.0, method="fgmres") -> list:
    """Solve independent instances concurrently (one stream and one host
    thread of a pool per instance). Returns one dict per instance, as
    helm_solve_block does, plus "status"."""
    k = len(handles)
    if not (len(Qs) == len(Us) == k) or k == 0:
        raise ValueError("need one Q and one U per handle")
    hs = (C.c_void_p * k)(*[h.ptr for h in handles])
    nr = (C.c_int32 * k)(*[int(q.shape[0]) for q in Qs])
    for h, q, u in zip(handles, Qs, Us):
        _dev_block(q, "Q")
        _dev_block(u, "U")
        if u.shape != q.shape or q.shape[1] != h.N:
            raise ValueError("Q and U must both be [nrhs, N] of their instance")
    qp = (C.c_void_p * k)(*[q.data_ptr() for q in Qs])
    up = (C.c_void_p * k)(*[u.data_ptr() for u in Us])
    o = SolveOpts(restart, max_cycles, block_size, 0, int(reorth), _form(graph), float(learned_rate), METHOD[method])
    infos = (SolveInfo * k)()
    rel = [np.zeros(int(q.shape[0])) for q in Qs]
    conv = [np.zeros(int(q.shape[0]), np.int32) for q in Qs]
    for i in range(k):
        infos[i].relres = rel[i].ctypes.data
        infos[i].converged = conv[i].ctypes.data
    st = (C.c_int32 * k)()
    _check(lib().helm_solve_batch(k, hs, nr, qp, up, float(tol), C.byref(o), infos, st, int(max_threads),
                                  _stream(stream)), allow=(HELM_ERR_NOT_CONVERGED,))
    return [{"status": st[i], "cycles": infos[i].cycles, "restarts": infos[i].restarts,
             "converged_all": bool(infos[i].converged_all), "fallback_used": int(infos[i].fallback_used),
             "t_solve_ms": infos[i].t_solve_ms, "relres": rel[i], "converged": conv[i].astype(bool),
             "rate_switch": int(infos[i].rate_switch)}
            for i in range(k)]


def helm_residual(hd: Handle, Q, U, stream=None) -> np.ndarray:
    nrhs = Q.shape[0]
    rel = np.zeros(nrhs)
    _check(lib().helm_residual(hd.ptr, nrhs, _dev_block(Q, "Q"), _dev_block(U, "U"),
                               rel.ctypes.data, _stream(stream)))
    return rel


def helm_residual_noalloc(hd: Handle, Q, U, stream=None) -> np.ndarray:
    """helm_residual with its partial sums in the library's static device
    array (no device allocation; calls on one device must not overlap)."""
    nrhs = Q.shape[0]
    rel = np.zeros(nrhs)
    _check(lib().helm_residual_noalloc(hd.ptr, nrhs, _dev_block(Q, "Q"), _dev_block(U, "U"),
                                       rel.ctypes.data, _stream(stream)))
    return rel


def _dev_any(t, name, dtype, shape):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def helm_fields_pack16(hd: Handle, U, stream=None):
    """16-bit storage of fields: returns (U16 int16-viewed half pairs [nrhs, N, 2]
    as torch.float16, scales float64 [nrhs]) on the device."""
    import torch
    nrhs = U.shape[0]
    U16 = torch.empty((nrhs, hd.N, 2), dtype=torch.float16, device=U.device)
    sc = torch.empty(nrhs, dtype=torch.float64, device=U.device)
    _check(lib().helm_fields_pack16(hd.ptr, nrhs, _dev_block(U, "U"), C.c_void_p(U16.data_ptr()),
                                    C.c_void_p(sc.data_ptr()), _stream(stream)))
    return U16, sc


def helm_fields_unpack16(hd: Handle, U16, scales, U, stream=None):
    nrhs = U.shape[0]
    _check(lib().helm_fields_unpack16(hd.ptr, nrhs, _dev_any(U16, "U16", U16.dtype, (nrhs, hd.N, 2)),
                                      C.c_void_p(scales.data_ptr()), _dev_block(U, "U"), _stream(stream)))


def _fields_args(hd, U=None, U16=None, scales=None):
    if (U is None) == (U16 is None):
        raise ValueError("give the fields as U or as (U16, scales)")
    if U is not None:
        return U.shape[0], _dev_block(U, "U"), None, None
    return U16.shape[0], None, C.c_void_p(U16.data_ptr()), C.c_void_p(scales.data_ptr())


def helm_jvp(hd: Handle, dm, JV, U=None, U16=None, scales=None, tol=1e-8, stream=None, **solve_kw) -> dict:
    """JV = J dm (eq:fwisens) for every field: dm float64 CUDA [N]."""
    import torch
    nrhs, up, hp, sp = _fields_args(hd, U, U16, scales)
    o = _opts(**solve_kw)
    info, rel, conv = _info(nrhs)
    st = _check(lib().helm_jvp(hd.ptr, nrhs, up, hp, sp, _dev_any(dm, "dm", torch.float64, (hd.N,)),
                               _dev_block(JV, "JV"), float(tol), C.byref(o), C.byref(info), _stream(stream)),
                allow=(HELM_ERR_NOT_CONVERGED,))
    return _info_dict(st, info, rel, conv)


def helm_jtvp(hd: Handle, W, g, U=None, U16=None, scales=None, tol=1e-8, stream=None, **solve_kw) -> dict:
    """g = Re sum_s J_s^H w_s: W complex128 CUDA [nrhs, N], g float64 CUDA [N]."""
    import torch
    nrhs, up, hp, sp = _fields_args(hd, U, U16, scales)
    o = _opts(**solve_kw)
    info, rel, conv = _info(nrhs)
    st = _check(lib().helm_jtvp(hd.ptr, nrhs, up, hp, sp, _dev_block(W, "W"),
                                _dev_any(g, "g", torch.float64, (hd.N,)), float(tol), C.byref(o),
                                C.byref(info), _stream(stream)), allow=(HELM_ERR_NOT_CONVERGED,))
    return _info_dict(st, info, rel, conv)


def _opts(restart=5, max_cycles=1000, block_size=1, reorth=0, graph=False, learned_rate=0.0, method="fgmres"):
    return SolveOpts(restart, max_cycles, block_size, 0, int(reorth), _form(graph), float(learned_rate),
                     METHOD[method], 0)


def _info(nrhs):
    rel = np.zeros(nrhs)
    conv = np.zeros(nrhs, np.int32)
    info = SolveInfo()
    info.relres = rel.ctypes.data
    info.converged = conv.ctypes.data
    return info, rel, conv


def _info_dict(st, info, rel, conv):
    return {"status": st, "cycles": info.cycles, "restarts": info.restarts,
            "converged_all": bool(info.converged_all), "fallback_used": int(info.fallback_used),
            "t_solve_ms": info.t_solve_ms, "relres": rel, "converged": conv.astype(bool),
            "rate_switch": int(info.rate_switch)}


def helm_apply(hd: Handle, X, Y, shifted=False, stream=None):
    _check(lib().helm_apply(hd.ptr, 1 if shifted else 0, X.shape[0], _dev_block(X, "X"),
                            _dev_block(Y, "Y"), _stream(stream)))
    return Y


def helm_precond(hd: Handle, R, Z, stream=None):
    _check(lib().helm_precond(hd.ptr, R.shape[0], _dev_block(R, "R"), _dev_block(Z, "Z"),
                              _stream(stream)))
    return Z


def helm_coarse_solve(hd: Handle, R, E, stream=None):
    _check(lib().helm_coarse_solve(hd.ptr, R.shape[0], _dev_block(R, "R"), _dev_block(E, "E"),
                                   _stream(stream)))
    return E


def helm_level_dims(hd: Handle, level: int):
    nu = (C.c_int32 * 3)()
    _check(lib().helm_level_dims(hd.ptr, level, nu))
    return tuple(nu[a] for a in range(3))


def helm_level_stencil(hd: Handle, level: int) -> np.ndarray:
    """Stencil of level >= 1 as complex128 [N_l, 3^dim]."""
    nu = helm_level_dims(hd, level)
    ns = 27 if hd.dim == 3 else 9
    st = np.zeros((int(np.prod(nu)), ns), np.complex128)
    _check(lib().helm_level_stencil(hd.ptr, level, st.ctypes.data))
    return st


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int32), ("total_ms", C.c_double)]


def helm_profile_enable(hd: Handle, enable: bool = True):
    """Start (counters reset) or stop per-class kernel timing with HIP events."""
    _check(lib().helm_profile_enable(hd.ptr, 1 if enable else 0))


def helm_profile_read(hd: Handle) -> dict:
    """{class: (launches, total_ms)} for every kernel class."""
    arr = (KernelStat * len(KERNEL_CLASSES))()
    _check(lib().helm_profile_read(hd.ptr, C.cast(arr, C.c_void_p)))
    return {name: (arr[i].launches, arr[i].total_ms) for i, name in enumerate(KERNEL_CLASSES)}


def helm_fine_tile(hd: Handle, nrhs: int):
    """(rows per lane, planes per z-chunk) used for nrhs columns (autotuned on first use)."""
    t = (C.c_int32 * 2)()
    _check(lib().helm_fine_tile(hd.ptr, nrhs, t))
    return int(t[0]), int(t[1])


def helm_set_fine_tile(hd: Handle, nrhs: int, ry: int, zc: int):
    """Force the tile of the finest-level stencil kernels for nrhs columns."""
    t = (C.c_int32 * 2)(ry, zc)
    _check(lib().helm_set_fine_tile(hd.ptr, nrhs, t))


# ---- learned coarsest-grid correction ---------------------------------------
def helm_net_nparams() -> int:
    return int(lib().helm_net_nparams())


def _dev_f32(t, name, shape=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


class Net:
    """Owns a helm_net: the coarsest-grid correction network on D^3 volumes."""

    def __init__(self, ptr, D, max_batch):
        self.ptr = ptr
        self.D = D
        self.max_batch = max_batch

    def close(self):
        if self.ptr:
            lib().helm_net_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != helm_net_nparams():
            raise ValueError("wrong parameter count")
        _check(lib().helm_net_set_params(self.ptr, C.c_void_p(p.ctypes.data)))

    def get_params(self) -> np.ndarray:
        p = np.empty(helm_net_nparams(), dtype=np.float32)
        _check(lib().helm_net_get_params(self.ptr, C.c_void_p(p.ctypes.data)))
        return p

    def get_state(self):
        """Training checkpoint: (float32 [3 * nparams] = parameters, Adam's
        first and second moments; the Adam step count)."""
        st = np.empty(3 * helm_net_nparams(), dtype=np.float32)
        t = C.c_int64(0)
        _check(lib().helm_net_get_state(self.ptr, C.c_void_p(st.ctypes.data), C.byref(t)))
        return st, t.value

    def set_state(self, state, step: int):
        """Restore a checkpoint from get_state."""
        st = np.ascontiguousarray(state, dtype=np.float32)
        if st.size != 3 * helm_net_nparams():
            raise ValueError("wrong state size")
        _check(lib().helm_net_set_state(self.ptr, C.c_void_p(st.ctypes.data), int(step)))

    def save(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().helm_net_save(self.ptr, None, C.byref(n)))
        buf = (C.c_uint8 * n.value)()
        _check(lib().helm_net_save(self.ptr, C.cast(buf, C.c_void_p), C.byref(n)))
        return bytes(buf)

    def forward(self, x, out, stream=None):
        """x: float32 CUDA [B, D^3, 4] -> out: float32 CUDA [B, D^3, 2]."""
        B = x.shape[0]
        V = self.D ** 3
        _check(lib().helm_net_forward(self.ptr, B, _dev_f32(x, "x", (B, V, 4)),
                                      _dev_f32(out, "out", (B, V, 2)), _stream(stream)))

    def loss_grad(self, x, target, mask, grad, stream=None) -> float:
        """Loss and its gradient (into grad, float32 CUDA [nparams])."""
        import torch
        B = x.shape[0]
        V = self.D ** 3
        if not (mask.is_cuda and mask.dtype == torch.uint8 and mask.numel() == V and mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 CUDA tensor of D^3 entries")
        loss = C.c_double(0.0)
        _check(lib().helm_net_loss_grad(self.ptr, B, _dev_f32(x, "x", (B, V, 4)),
                                        _dev_f32(target, "target", (B, V, 2)), C.c_void_p(mask.data_ptr()),
                                        _dev_f32(grad, "grad", (helm_net_nparams(),)), C.byref(loss),
                                        _stream(stream)))
        return loss.value

    def pairs(self) -> int:
        return int(lib().helm_net_pairs(self.ptr))

    def pool_read(self, i, x, target, stream=None):
        """Pool entry i into x float32 CUDA [D^3, 4] and target [D^3, 2]."""
        V = self.D ** 3
        _check(lib().helm_net_pool_read(self.ptr, int(i), _dev_f32(x, "x", (V, 4)),
                                        _dev_f32(target, "target", (V, 2)), _stream(stream)))

    def train_step(self, x, target, mask, lr=1e-3, stream=None) -> float:
        """One Adam step on the given minibatch (x [B, D^3, 4], target
        [B, D^3, 2] float32 CUDA, mask uint8 CUDA [D^3]); returns the loss."""
        import torch
        B = x.shape[0]
        V = self.D ** 3
        if not (mask.is_cuda and mask.dtype == torch.uint8 and mask.numel() == V and mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 CUDA tensor of D^3 entries")
        loss = C.c_double(0.0)
        _check(lib().helm_net_train_step(self.ptr, B, _dev_f32(x, "x", (B, V, 4)),
                                         _dev_f32(target, "target", (B, V, 2)), C.c_void_p(mask.data_ptr()),
                                         float(lr), C.byref(loss), _stream(stream)))
        return loss.value

    def train(self, steps, batch, lr=1e-3, seed=0, stream=None) -> np.ndarray:
        hist = np.zeros(steps, dtype=np.float64)
        _check(lib().helm_net_train(self.ptr, int(steps), int(batch), float(lr), int(seed),
                                    C.c_void_p(hist.ctypes.data), _stream(stream)))
        return hist


def helm_net_create(D: int, max_batch: int, seed: int = 0, stream=None) -> Net:
    out = C.c_void_p()
    _check(lib().helm_net_create(int(D), int(max_batch), int(seed), _stream(stream), C.byref(out)))
    return Net(out, D, max_batch)


def helm_net_capture(hd: Handle, net: Net, max_pairs: int):
    """Store (input, exact target) pairs of hd's coarsest solves in net's pool
    (max_pairs == 0 detaches). While attached, the handle holds a reference
    to the network, so the pool outlives every solve that writes to it."""
    _check(lib().helm_net_capture(hd.ptr, net.ptr, int(max_pairs)))
    if int(max_pairs) == 0:
        if hd.capture_net is net:
            hd.capture_net = None
    else:
        hd.capture_net = net
