"""The C-ABI library loads and exports every symbol include/helm.h declares.

No compute call is made: this runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_paper_boundary():
    syms = declared_symbols()
    for name in ("helm_setup", "helm_solve_block", "helm_residual"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import paper_1607_00968_amd as pk
    if not os.path.exists(pk.LIBPATH):
        from paper_1607_00968_amd import build
        build.build()
    lib = ctypes.CDLL(pk.LIBPATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(pk.ABI_SYMBOLS) <= set(declared_symbols())


def test_status_strings_without_device():
    import paper_1607_00968_amd as pk
    L = pk.lib()
    for st in range(8):
        assert L.helm_status_string(st)


def test_setup_rejects_bad_arguments_without_device():
    """Argument validation happens before any device call."""
    import numpy as np
    import paper_1607_00968_amd as pk
    m = np.ones(7 * 7)
    g = np.zeros(7 * 7)
    with pytest.raises(pk.HelmError) as e:
        pk.helm_setup(2, (8, 8), (1 / 8, 1 / 8), m, g, omega=-1.0, stream=0)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG
    with pytest.raises(pk.HelmError) as e:  # 8 cells cannot be coarsened 3 times
        pk.helm_setup(2, (8, 8), (1 / 8, 1 / 8), m, g, omega=1.0, levels=4, stream=0)
    assert e.value.status == pk.HELM_ERR_INVALID_ARG
    bad = m.copy()
    bad[3] = np.nan
    with pytest.raises(pk.HelmError) as e:
        pk.helm_setup(2, (8, 8), (1 / 8, 1 / 8), bad, g, omega=1.0, levels=2, stream=0)
    assert e.value.status == pk.HELM_ERR_NONFINITE
