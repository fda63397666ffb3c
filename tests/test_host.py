"""Host-side checks that need no GPU: the ctypes mirrors of the ABI structs
follow include/helm.h field by field, every documented precondition of
helm_setup is validated before any device call, the network's training models are not the benchmark's model,
and the bench finds the committed traffic figure of the tile it ran with."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helm.h")


def header_struct_fields(name):
    """Field names, in order, of `typedef struct { ... } name;` in helm.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ident = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*(?:\[[^\]]*\])?\s*$", decl)
        fields.append(ident[0])
    return fields


@pytest.mark.parametrize("cname,pyname", [("helm_setup_desc", "SetupDesc"), ("helm_solve_opts", "SolveOpts"),
                                          ("helm_solve_info", "SolveInfo")])
def test_ctypes_structs_follow_the_header(cname, pyname):
    import paper_1607_00968_amd as pk
    py = [f[0] for f in getattr(pk, pyname)._fields_]
    assert py == header_struct_fields(cname)


def test_new_options_are_validated_without_device():
    import paper_1607_00968_amd as pk
    m = np.ones(7 * 7)
    g = np.zeros(7 * 7)
    for bad in (-1, 17):
        with pytest.raises(pk.HelmError) as e:
            pk.helm_setup(2, (8, 8), (1 / 8, 1 / 8), m, g, omega=1.0, levels=2, coarse="gmres", coarse_restarts=bad,
                          stream=0)
        assert e.value.status == pk.HELM_ERR_INVALID_ARG


def test_training_models_are_not_the_benchmark_model():
    import synth
    bench_m = synth.layered_3d(n=32, seed=3, nsrc=(8, 8)).m
    ms = [synth.training_model(j, n=32).m for j in range(4)]
    for j, mj in enumerate(ms):
        assert mj.shape == bench_m.shape
        assert not np.allclose(mj, bench_m), j
        for k in range(j):
            assert not np.allclose(mj, ms[k]), (j, k)
    t = synth.training_model(0, n=32)
    assert t.levels == 3 and t.Q.shape[0] == 32


def test_bench_reads_the_traffic_of_each_committed_tile():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    text = open(os.path.join(ROOT, "profiles", "fine_kernels_mixed_192x64_traffic.md")).read()
    lines = re.findall(r"^traffic: .*kernel=(\w+) .*tile=(\d+)x(\d+) bytes_per_launch=(\d+) algorithmic=(\d+)",
                       text, flags=re.M)
    assert lines
    kb = bench.fine_kernel_bytes("mixed", 191 ** 3, 95 ** 3, 64)
    for kernel, ry, zc, byts, alg in lines:
        # each line's algorithmic bytes are the bench's own count for that class
        assert int(alg) == kb[kernel], kernel
        v = bench.committed_traffic("mixed", 192, 64, (int(ry), int(zc)), kernel)
        assert v == int(byts) and kb[kernel] < v < 2 * kb[kernel], kernel
    assert bench.committed_traffic("mixed", 192, 64, (4, 7)) is None
    assert bench.committed_traffic("fp64", 192, 64, (int(lines[0][1]), int(lines[0][2]))) is None


def _setup_case(**over):
    """A valid small 2D set-up (8^2 cells, 2 levels) with `over` applied;
    m and gamma follow the grid unless given."""
    kw = dict(dim=2, n=(8, 8), h=(1 / 8, 1 / 8), omega=1.0, levels=2, coarse="lu")
    kw.update(over)
    N = int(np.prod([c - 1 for c in kw["n"]]))
    m = kw.pop("m", np.ones(N))
    g = kw.pop("gamma", np.zeros(N))
    dim, n, h, omega = kw.pop("dim"), kw.pop("n"), kw.pop("h"), kw.pop("omega")
    return dim, n, h, m, g, omega, kw


def _bad(x, i, v):
    x = np.array(x, dtype=float)
    x[i] = v
    return x


BAD_SETUPS = [
    ("one level", dict(levels=1), "INVALID_ARG"),
    ("more levels than the maximum", dict(levels=9, n=(512, 512)), "INVALID_ARG"),
    ("n not a multiple of 2^(levels-1)", dict(levels=3, n=(10, 8)), "INVALID_ARG"),
    ("no coarsest unknown", dict(levels=3, n=(4, 4)), "INVALID_ARG"),
    ("zero spacing", dict(h=(0.0, 1 / 8)), "INVALID_ARG"),
    ("omega zero", dict(omega=0.0), "INVALID_ARG"),
    ("omega NaN", dict(omega=float("nan")), "INVALID_ARG"),
    ("negative shift", dict(shift=-0.1), "INVALID_ARG"),
    ("m zero", dict(m=_bad(np.ones(49), 5, 0.0)), "INVALID_ARG"),
    ("m NaN", dict(m=_bad(np.ones(49), 5, np.nan)), "NONFINITE"),
    ("gamma negative", dict(gamma=_bad(np.zeros(49), 3, -1e-3)), "INVALID_ARG"),
    ("gamma infinite", dict(gamma=_bad(np.zeros(49), 3, np.inf)), "NONFINITE"),
    ("negative sweep count", dict(nu_pre=-1), "INVALID_ARG"),
    ("NaN Jacobi weight", dict(jacobi_weight=float("nan")), "INVALID_ARG"),
    ("GMRES coarsest with 0 steps", dict(coarse="gmres", coarse_iters=0), "INVALID_ARG"),
    ("GMRES coarsest with 33 steps (beyond the basis list)", dict(coarse="gmres", coarse_iters=33), "INVALID_ARG"),
    ("learned coarsest with 33 steps", dict(coarse="learned", coarse_iters=33), "INVALID_ARG"),
]


@pytest.mark.parametrize("name,over,status", BAD_SETUPS, ids=[b[0] for b in BAD_SETUPS])
def test_setup_rejects_bad_input_before_any_device_call(name, over, status):
    """Every documented precondition of helm_setup is checked on the host
    before the first HIP call: here, without a GPU, each bad descriptor gets
    its own status (a check that came after a device call would report a
    device error instead)."""
    import paper_1607_00968_amd as pk
    dim, n, h, m, g, omega, kw = _setup_case(**over)
    with pytest.raises(pk.HelmError) as e:
        pk.helm_setup(dim, n, h, m, g, omega, stream=0, **kw)
    assert e.value.status == getattr(pk, "HELM_ERR_" + status), str(e.value)


@pytest.mark.parametrize("D,max_batch", [(6, 4), (0, 4), (260, 4), (8, 0), (8, 1025)])
def test_net_create_rejects_bad_shape_before_any_device_call(D, max_batch):
    """The network's edge must be a multiple of 4 in 4..256 and the batch
    1..1024; both are checked before the first device allocation."""
    import paper_1607_00968_amd as pk
    with pytest.raises(pk.HelmError) as e:
        pk.helm_net_create(D, max_batch, seed=0, stream=0)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG, str(e.value)


def test_bench_algorithmic_bytes_of_the_fine_sweep():
    """The roofline's numerator: a damped-Jacobi sweep from a nonzero guess
    reads u and f and writes u (3 x 8 B per point and RHS in mixed, 3 x 16 B
    in FP64) and reads one coefficient per point (w/D: 8 B in mixed, 16 B
    in FP64): 10.76 GB per launch at 191^3 unknowns x 64 RHS in mixed."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    N = 191 ** 3
    assert bench.fine_sweep_bytes("mixed", N, 64) == N * (3 * 8 * 64 + 8) == 10758392824
    assert bench.fine_sweep_bytes("fp64", N, 64) == N * (3 * 16 * 64 + 16)


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; --gpus N > 1 exits with a message before
    any device is touched."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_kernel_classes_follow_the_header():
    """The binding's kernel-class names cover the header's HELM_K_* enum, in order."""
    import paper_1607_00968_amd as pk
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"enum\s*\{\s*(HELM_K_FINE_SWEEP\s*=\s*0[^}]*)\}", text)
    assert m
    names = [t.strip().split("=")[0].strip() for t in m.group(1).split(",") if t.strip()]
    assert names[-1] == "HELM_K_NCLASS"
    assert [n[len("HELM_K_"):].lower() for n in names[:-1]] == list(pk.KERNEL_CLASSES)


def test_pre_rr_alu_figure():
    """The fused pre-smoothing's ALU figure: 83.75 flops per fine point and
    column (6 + 36 + 28 + 110/8), against 157.3 TFLOP/s published and 39.3 T
    lane operations per second."""
    import bench
    assert bench.PRE_RR_FLOPS == 83.75
    a = bench.pre_rr_alu("mixed", 1000, 64, 1e-3)
    assert a["flops_per_launch"] == 1000 * 64 * 83.75
    assert abs(a["achieved"] - 1000 * 64 * 83.75 / 1e-3 / 1e12) < 0.01
    assert a["peak_published"] == 157.3 and a["peak_lane_ops"] == 39.3
    assert bench.pre_rr_alu("fp64", 1000, 64, 1e-3)["peak_published"] == 78.6
