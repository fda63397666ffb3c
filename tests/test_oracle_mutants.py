"""Planted mistakes in the CPU oracle: do the pins catch them?

Each case copies the oracle's C sources to a temporary directory, plants one
plausible slip in the copy (a sign, a weight, a dropped term or conjugate, a
transposed operand, a mirrored tap), compiles it to a library of its own,
points the oracle package at that library and runs the pins named beside the
mistake: at least one of them must fail. The oracle's own sources and library
are never changed, and the package is pointed back at them afterwards.

Every planted slip keeps all memory accesses in bounds (offsets stay inside
the same 3^d neighbourhood, loops keep their ranges), so a mutant can give
wrong numbers but cannot fault.
"""
import contextlib
import os
import subprocess

import pytest

import oracle
import test_oracle_cnn as cnn
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__))


def kron(dim, n, beta):
    return lambda: pins.test_apply_fine_matches_kronecker_assembly(dim, n, beta)


# (name, file, text in the oracle, replacement, which occurrence, pins)
MUTANTS = [
    # operator (eq:helm, eq:LinearSystem)
    ("damping sign", "helm_oracle.c", "(1.0 - I * (gam + beta))", "(1.0 + I * (gam + beta))", 0,
     [kron(3, 6, 0.2)]),
    ("shift dropped", "helm_oracle.c", "(1.0 - I * (gam + beta))", "(1.0 - I * gam)", 0, [kron(2, 8, 0.2)]),
    ("off-diagonal sign", "helm_oracle.c", "acc -= w * us[gidx(g, d[0], d[1], d[2])]",
     "acc += w * us[gidx(g, d[0], d[1], d[2])]", 0, [kron(2, 8, 0.0)]),
    ("one spacing for every axis", "helm_oracle.c", "lap += 2.0 / (g->h[a] * g->h[a]);",
     "lap += 2.0 / (g->h[0] * g->h[0]);", 0, [kron(3, 6, 0.0)]),
    # transfers
    ("interpolation weight", "helm_oracle.c", "(dx ? 0.5 : 1.0)", "(dx ? 0.25 : 1.0)", 0,
     [lambda: pins.test_prolong_restrict_match_kron(2, 8)]),
    ("restriction scale", "helm_oracle.c", "1.0 / (double)(1 << g->dim)", "1.0 / (double)(1 << (g->dim - 1))", 0,
     [lambda: pins.test_prolong_restrict_match_kron(3, 8)]),
    ("restriction ignores the z offset", "helm_oracle.c", "int fz = g->dim == 3 ? 2 * Z + 1 + dz : 0;",
     "int fz = g->dim == 3 ? 2 * Z + 1 : 0;", 1, [lambda: pins.test_prolong_restrict_match_kron(3, 8)]),
    # Galerkin coarse operators
    ("coarse stencil mirrored", "helm_oracle.c", "if (col) stc[cj * 27 + sidx(ox, oy, oz)] = y[cj];",
     "if (col) stc[cj * 27 + sidx(-ox, -oy, -oz)] = y[cj];", 0,
     [lambda: pins.test_galerkin_matches_triple_product(2, 16)]),
    # smoothing
    ("Jacobi without its damping weight", "helm_oracle.c", "u[j] += w * (f[j] - r[j]) / st[i * 27 + sidx(0, 0, 0)];",
     "u[j] += (f[j] - r[j]) / st[i * 27 + sidx(0, 0, 0)];", 0, [pins.test_jacobi_sine_mode_amplification]),
    ("cycle smoother residual sign", "helm_oracle.c", "u[j] += H->w[l] * (f[j] - r[j])", "u[j] += H->w[l] * (r[j] - f[j])",
     0, [lambda: pins.test_vcycle_equals_dense_composition(2, 16, 3)]),
    ("cycle smooths with the unshifted operator", "helm_oracle.c",
     "orc_apply_fine(&H->g[0], H->m, H->gamma, H->omega, H->beta, nrhs, u, out);",
     "orc_apply_fine(&H->g[0], H->m, H->gamma, H->omega, 0.0, nrhs, u, out);", 0,
     [lambda: pins.test_vcycle_equals_dense_composition(3, 8, 2)]),
    # the cycle
    ("cycle residual sign", "helm_oracle.c", "for (int64_t j = 0; j < N * nrhs; ++j) r[j] = f[j] - r[j];",
     "for (int64_t j = 0; j < N * nrhs; ++j) r[j] = r[j] - f[j];", 0,
     [lambda: pins.test_vcycle_equals_dense_composition(2, 16, 3)]),
    ("coarse correction subtracted", "helm_oracle.c", "for (int64_t j = 0; j < N * nrhs; ++j) u[j] += r[j];",
     "for (int64_t j = 0; j < N * nrhs; ++j) u[j] -= r[j];", 0,
     [lambda: pins.test_vcycle_equals_dense_composition(2, 16, 3)]),
    ("W-cycle second correction subtracted", "helm_oracle.c", "for (int64_t j = 0; j < n2; ++j) ec[j] += d2[j];",
     "for (int64_t j = 0; j < n2; ++j) ec[j] -= d2[j];", 0,
     [lambda: pins.test_wcycle_equals_dense_composition(2, 32, 4)]),
    # coarsest solves
    ("LU back substitution sign", "helm_oracle.c", "for (int64_t j = k + 1; j <= cend; ++j) acc -= BAND(b, k, j) * v[j];",
     "for (int64_t j = k + 1; j <= cend; ++j) acc += BAND(b, k, j) * v[j];", 0,
     [lambda: pins.test_coarsest_band_lu_equals_dense_solve(2, 16, 2)]),
    ("coarse GMRES without the conjugate", "helm_oracle.c", "for (int64_t t = 0; t < n; ++t) d += conj(vi[t]) * w[t];",
     "for (int64_t t = 0; t < n; ++t) d += vi[t] * w[t];", 0,
     [lambda: pins.test_vcycle_with_gmres_coarsest_equals_dense(3)]),
    ("coarse GMRES restart replaces the iterate", "helm_oracle.c", "for (int64_t t = 0; t < n; ++t) us[t] += d[t];",
     "for (int64_t t = 0; t < n; ++t) us[t] = d[t];", 0, [pins.test_coarse_gmres_restarts_equal_krylov_minimisers]),
    ("relaxation-only coarsest with half the sweeps", "helm_oracle.c", "int sweeps = H->nu_pre[l] + H->nu_post[l];",
     "int sweeps = H->nu_pre[l];", 0, [lambda: pins.test_vcycle_with_relaxed_coarsest_equals_dense(2, 16, 3)]),
    # dense helpers
    ("reflector without its factor 2", "helm_oracle.c", "y[i] -= 2.0 * v[i] * d;", "y[i] -= v[i] * d;", 0,
     [pins.test_householder_qr]),
    ("back substitution transposed", "helm_oracle.c", "acc -= a[(int64_t)j * mr + i] * Y[(int64_t)c * nc + j];",
     "acc -= a[(int64_t)i * mr + j] * Y[(int64_t)c * nc + j];", 0, [pins.test_lstsq_matches_numpy]),
    # block FGMRES
    ("warm start ignored", "helm_oracle.c", "if (!warm) memset(X, 0, sizeof(ozc) * blk);",
     "memset(X, 0, sizeof(ozc) * blk);", 0, [pins.test_fgmres_warm_start_is_a_shifted_cold_solve]),
    ("block Gram without the conjugate", "helm_oracle.c", "acc += conj(va[n]) * wb[n];", "acc += va[n] * wb[n];", 0,
     [pins.test_fgmres_identity_prec_equals_scipy_gmres]),
    ("solution updated from V, not Z (not flexible)", "helm_oracle.c", "acc += Z[(int64_t)jj * blk",
     "acc += V[(int64_t)jj * blk", 0, [pins.test_residual_estimates_track_true_residual]),
    ("block least-squares right-hand side transposed", "helm_oracle.c", "B[(int64_t)b * r + a] = S[b * p + a];",
     "B[(int64_t)b * r + a] = S[a * p + b];", 0, [pins.test_block_fgmres_saturates_to_exact_in_one_cycle]),
    ("restart residual of the shifted operator", "helm_oracle.c",
     "orc_apply_fine(&Hh->g[0], Hh->m, Hh->gamma, Hh->omega, 0.0, p, X, V);",
     "orc_apply_fine(&Hh->g[0], Hh->m, Hh->gamma, Hh->omega, Hh->beta, p, X, V);", 0,
     [lambda: pins.test_fgmres_manufactured_solution(1)]),
    # deflation of dependent directions (rank-revealing QR)
    ("rank-revealing QR keeps the pivoted column order in R", "helm_oracle.c",
     "R[(int64_t)perm[j] * p + i] = (i < r && i <= j)", "R[(int64_t)j * p + i] = (i < r && i <= j)", 0,
     [pins.test_householder_qr_rank_revealing, lambda: pins.test_fgmres_duplicate_and_dependent_sources(5)]),
    ("least squares divides by a dropped direction's zero diagonal", "helm_oracle.c",
     "a[(int64_t)i * mr + i] != 0 ? acc / a[(int64_t)i * mr + i] : 0",
     "acc / a[(int64_t)i * mr + i]", 0, [lambda: pins.test_fgmres_duplicate_and_dependent_sources(5)]),
    ("rank-revealing QR without pivoting", "helm_oracle.c", "if (nj > best) {", "if (j == k) {", 0,
     [pins.test_householder_qr_rank_revealing]),
    # the network oracle
    ("convolution taps mirrored", "conv_oracle.c",
     "const int xx = X + t % 3 - 1, yy = Y + (t / 3) % 3 - 1, zz = Z + t / 9 - 1;",
     "const int xx = X - (t % 3 - 1), yy = Y - ((t / 3) % 3 - 1), zz = Z - (t / 9 - 1);", 0,
     [cnn.test_conv3d_forward_matches_scipy_correlate]),
    ("backward data taps not mirrored", "conv_oracle.c",
     "const int xx = X - (t % 3 - 1), yy = Y - ((t / 3) % 3 - 1), zz = Z - (t / 9 - 1);",
     "const int xx = X + t % 3 - 1, yy = Y + (t / 3) % 3 - 1, zz = Z + t / 9 - 1;", 0,
     [cnn.test_conv3d_backward_data_is_adjoint]),
    ("backward weight taps mirrored", "conv_oracle.c",
     "const int xx = X + t % 3 - 1, yy = Y + (t / 3) % 3 - 1, zz = Z + t / 9 - 1;",
     "const int xx = X - (t % 3 - 1), yy = Y - ((t / 3) % 3 - 1), zz = Z - (t / 9 - 1);", 1,
     [cnn.test_conv3d_backward_weight_is_adjoint]),
    ("pooling weight 1/4 instead of 1/8", "conv_oracle.c", "0.125 * s", "0.25 * s", 0,
     [cnn.test_pool_upsample_adjoint_pair]),
    ("skip connection in the wrong channels", "conv_oracle.c", "put_slice(V, 16, s1, 48, 32, A->c1);",
     "put_slice(V, 16, s1, 48, 16, A->c1);", 0, [cnn.test_unet_forward_equals_composition]),
    ("ReLU mask of the last layer dropped in the gradient", "conv_oracle.c", "relu_mask(V * 16, A.a9, g9);", ";", 0,
     [cnn.test_unet_gradient_central_differences]),
    ("loss gradient without its factor 2", "conv_oracle.c", "g_out[i * 2 + c] = 2.0 * (A.out", "g_out[i * 2 + c] = (A.out",
     0, [cnn.test_unet_gradient_central_differences]),
    # K-cycle coarse correction
    ("K-cycle combines the basis instead of the preconditioned vectors", "helm_oracle.c",
     "for (int64_t t = 0; t < n; ++t) es[t] += z[(int64_t)c * n + t] * y[c];",
     "for (int64_t t = 0; t < n; ++t) es[t] += v[(int64_t)c * n + t] * y[c];", 0,
     [lambda: pins.test_kcycle_equals_dense_minimal_residual(2, 32, 3)]),
    ("K-cycle second direction not normalised", "helm_oracle.c",
     "for (int64_t t = 0; t < n; ++t) v[n + t] = w[t] / hn;",
     "for (int64_t t = 0; t < n; ++t) v[n + t] = w[t];", 0,
     [lambda: pins.test_kcycle_equals_dense_minimal_residual(2, 32, 3)]),
]


def plant(text, old, new, occ):
    at = -1
    for _ in range(occ + 1):
        at = text.find(old, at + 1)
        assert at >= 0, f"the oracle no longer contains {old!r} (occurrence {occ})"
    return text[:at] + new + text[at + len(old):]


@contextlib.contextmanager
def oracle_library(path):
    saved = (oracle._LIBPATH, oracle._lib)
    oracle._LIBPATH, oracle._lib = path, None
    try:
        yield
    finally:
        oracle._LIBPATH, oracle._lib = saved


@pytest.mark.parametrize("name,fname,old,new,occ,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, fname, old, new, occ, checks):
    for f in ("helm_oracle.c", "helm_oracle.h", "conv_oracle.c"):
        with open(os.path.join(SRC, f)) as fh:
            text = fh.read()
        if f == fname:
            changed = plant(text, old, new, occ)
            assert changed != text
            text = changed
        (tmp_path / f).write_text(text)
    lib = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-w",
                           str(tmp_path / "helm_oracle.c"), str(tmp_path / "conv_oracle.c"), "-o", lib, "-lm"])
    caught = []
    with oracle_library(lib):
        for check in checks:
            try:
                check()
            except AssertionError as e:
                caught.append(str(e)[:80])
    assert caught, f"no pin caught the planted mistake: {name}"


def test_unmutated_copy_passes_the_same_pins(tmp_path):
    """The harness itself: the copied, recompiled oracle without a planted
    mistake passes every pin used above (so a caught mutant is caught for
    its mistake, not for the build)."""
    for f in ("helm_oracle.c", "helm_oracle.h", "conv_oracle.c"):
        with open(os.path.join(SRC, f)) as fh:
            (tmp_path / f).write_text(fh.read())
    lib = str(tmp_path / "libcopy.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-w",
                           str(tmp_path / "helm_oracle.c"), str(tmp_path / "conv_oracle.c"), "-o", lib, "-lm"])
    with oracle_library(lib):
        for m in MUTANTS:
            for check in m[5]:
                check()


# Planted mistakes in the oracle's learned coarsest solve and Adam update
# (oracle/learned.py, numpy): each mutant is the module's source with one
# slip, loaded as a module of its own and run through the pins named beside it.
import importlib.util  # noqa: E402
import sys  # noqa: E402

import test_oracle_learned as lpins  # noqa: E402

_P32 = []


def _p32():
    """The pins' 32^3 layered problem (built once)."""
    if not _P32:
        _P32.append(lpins.synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2))
    return _P32[0]


LEARNED_MUTANTS = [
    ("rms over the whole volume", "axis=1) / Nc)", "axis=1) / D ** 3)",
     [lambda: lpins.test_constant_network_closed_form(_p32())]),
    ("output scaled by H instead of H^2", "E[b] = (H2 * rms[b])", "E[b] = (np.sqrt(H2) * rms[b])",
     [lambda: lpins.test_probe_networks_see_the_stated_channels(_p32())]),
    ("diagonal channels without H^2", "centre = (H2 * st[:, 13])", "centre = (st[:, 13])",
     [lambda: lpins.test_probe_networks_see_the_stated_channels(_p32())]),
    ("GMRES restarts ignore the network's guess", "E = E + hier_gmres.coarse_solve(R)",
     "E = hier_gmres.coarse_solve(R)", [lambda: lpins.test_perfect_network_gives_the_exact_solve(_p32(), 8, 2)]),
    ("fallback only on non-finite output", "np.abs(out).max(initial=0.0) <= 1e4", "True",
     [lambda: lpins.test_fallback_on_nonfinite_or_huge_output(_p32())]),
    ("Adam without bias correction", "mhat = m / (1.0 - b1 ** t)", "mhat = m",
     [lpins.test_adam_two_steps_worked_by_hand]),
    ("Adam second moment of |g|", "v = b2 * v + (1.0 - b2) * g * g", "v = b2 * v + (1.0 - b2) * np.abs(g)",
     [lpins.test_adam_two_steps_worked_by_hand]),
]


@pytest.mark.parametrize("name,old,new,checks", LEARNED_MUTANTS, ids=[m[0] for m in LEARNED_MUTANTS])
def test_learned_pins_catch_planted_mistake(tmp_path, name, old, new, checks):
    """Also run unmutated by test_learned_unmutated_copy_passes below."""
    with open(os.path.join(SRC, "learned.py")) as fh:
        text = fh.read()
    changed = plant(text, old, new, 0)
    assert changed != text
    path = tmp_path / "learned_mutant.py"
    path.write_text(changed)
    spec = importlib.util.spec_from_file_location("oracle.learned_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    sys.modules["oracle.learned_mutant"] = mod
    spec.loader.exec_module(mod)
    saved = lpins.ol
    lpins.ol = mod
    caught = []
    try:
        for check in checks:
            try:
                check()
            except AssertionError as e:
                caught.append(str(e)[:80])
    finally:
        lpins.ol = saved
        sys.modules.pop("oracle.learned_mutant", None)
    assert caught, f"no pin caught the planted mistake: {name}"


def test_learned_unmutated_copy_passes(tmp_path):
    """The harness for the learned oracle: a copy of the module loaded the
    same way, without a planted mistake, passes every pin used above."""
    with open(os.path.join(SRC, "learned.py")) as fh:
        text = fh.read()
    path = tmp_path / "learned_copy.py"
    path.write_text(text)
    spec = importlib.util.spec_from_file_location("oracle.learned_copy", str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    sys.modules["oracle.learned_copy"] = mod
    spec.loader.exec_module(mod)
    saved = lpins.ol
    lpins.ol = mod
    try:
        for m in LEARNED_MUTANTS:
            for check in m[3]:
                check()
    finally:
        lpins.ol = saved
        sys.modules.pop("oracle.learned_copy", None)


# Planted mistakes in the oracle's block BiCGSTAB (oracle/bicgstab.py).
import test_oracle_bicgstab as bpins  # noqa: E402

BICG_MUTANTS = [
    ("beta with the wrong sign", "beta = -np.linalg.solve(A, Rt.conj() @ T.T)", "beta = np.linalg.solve(A, Rt.conj() @ T.T)",
     [lambda: bpins.test_single_rhs_unpreconditioned_matches_scipy(0.1, (4, 8, 12), 1e-10)]),
    ("update without omega", "X = X + alpha.T @ Phat + omega * Shat", "X = X + alpha.T @ Phat + Shat",
     [lambda: bpins.test_single_rhs_unpreconditioned_matches_scipy(0.1, (4, 8, 12), 1e-10)]),
    ("shadow inner product without conjugate", "A = Rt.conj() @ V.T", "A = Rt @ V.T",
     [lambda: bpins.test_single_rhs_unpreconditioned_matches_scipy(0.1, (4, 8, 12), 1e-10)]),
    ("direction update keeps V", "P = R + beta.T @ (P - omega * V)", "P = R + beta.T @ P",
     [lambda: bpins.test_single_rhs_unpreconditioned_matches_scipy(0.1, (4, 8, 12), 1e-10)]),
]


def _load_module_copy(tmp_path, fname, text, modname):
    path = tmp_path / (modname + ".py")
    path.write_text(text)
    spec = importlib.util.spec_from_file_location("oracle." + modname, str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    sys.modules["oracle." + modname] = mod
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name,old,new,checks", BICG_MUTANTS, ids=[m[0] for m in BICG_MUTANTS])
def test_bicgstab_pins_catch_planted_mistake(tmp_path, name, old, new, checks):
    with open(os.path.join(SRC, "bicgstab.py")) as fh:
        text = fh.read()
    changed = plant(text, old, new, 0)
    assert changed != text
    mod = _load_module_copy(tmp_path, "bicgstab.py", changed, "bicgstab_mutant")
    saved = bpins.ob
    bpins.ob = mod
    caught = []
    try:
        for check in checks:
            try:
                check()
            except AssertionError as e:
                caught.append(str(e)[:80])
    finally:
        bpins.ob = saved
        sys.modules.pop("oracle.bicgstab_mutant", None)
    assert caught, f"no pin caught the planted mistake: {name}"


def test_bicgstab_unmutated_copy_passes(tmp_path):
    with open(os.path.join(SRC, "bicgstab.py")) as fh:
        mod = _load_module_copy(tmp_path, "bicgstab.py", fh.read(), "bicgstab_copy")
    saved = bpins.ob
    bpins.ob = mod
    try:
        for m in BICG_MUTANTS:
            for check in m[3]:
                check()
    finally:
        bpins.ob = saved
        sys.modules.pop("oracle.bicgstab_copy", None)


# Planted mistakes in the oracle's sensitivity products and 16-bit storage
# (oracle/sens.py).
import test_oracle_sens as spins  # noqa: E402

SENS_MUTANTS = [
    ("damping factor with the wrong sign", "(1.0 - 1j * hier._gamma)", "(1.0 + 1j * hier._gamma)",
     [lambda: spins.test_jvp_equals_central_difference(spins.setup_problem())]),
    ("adjoint products without the field's conjugate", "np.conj(dH_dm_factor(hier)[None, :] * U) * Y",
     "dH_dm_factor(hier)[None, :] * U * Y", [lambda: spins.test_adjoint_identities(spins.setup_problem())]),
    ("adjoint solve without the conjugations", 'return np.conj(solve(hier, np.conj(B), tol, "H"))',
     'return solve(hier, B, tol, "H")', [lambda: spins.test_adjoint_identities(spins.setup_problem())]),
    ("16-bit scale from the modulus", "np.max(np.maximum(np.abs(U.real), np.abs(U.imag)), axis=1)",
     "np.max(np.abs(U), axis=1)", [spins.test_pack16_bounds]),
]


@pytest.mark.parametrize("name,old,new,checks", SENS_MUTANTS, ids=[m[0] for m in SENS_MUTANTS])
def test_sens_pins_catch_planted_mistake(tmp_path, name, old, new, checks):
    with open(os.path.join(SRC, "sens.py")) as fh:
        text = fh.read()
    changed = plant(text, old, new, 0)
    assert changed != text
    mod = _load_module_copy(tmp_path, "sens.py", changed, "sens_mutant")
    saved = spins.sens
    spins.sens = mod
    caught = []
    try:
        for check in checks:
            try:
                check()
            except AssertionError as e:
                caught.append(str(e)[:80])
    finally:
        spins.sens = saved
        sys.modules.pop("oracle.sens_mutant", None)
    assert caught, f"no pin caught the planted mistake: {name}"


def test_sens_unmutated_copy_passes(tmp_path):
    with open(os.path.join(SRC, "sens.py")) as fh:
        mod = _load_module_copy(tmp_path, "sens.py", fh.read(), "sens_copy")
    saved = spins.sens
    spins.sens = mod
    try:
        for m in SENS_MUTANTS:
            for check in m[3]:
                check()
    finally:
        spins.sens = saved
        sys.modules.pop("oracle.sens_copy", None)
