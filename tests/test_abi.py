"""C-ABI library: loads on the CPU, exports every declared symbol, rejects bad
arguments before touching the device, and builds the collision tensor on the host
so that the host logic can be checked against the oracle without a GPU."""
import ctypes

import numpy as np
import pytest

from paper_2607_13740_amd import gracedg as G


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = G.declared_symbols()
    assert "gd_init_tensor" in names and "gd_rk_step" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_invalid_arguments_are_rejected():
    L = G.lib()
    k = G._Kernel(0, 1.0)
    lv = np.array([0.5])
    f = G._Frag(0, -11 / 6, 1, lv.ctypes.data_as(G._DP))
    g = G._Grid(1.0, 0.5, 0, 0)              # x_max < x_min
    h = G._VP()
    assert L.gd_init_tensor(ctypes.byref(k), ctypes.byref(f), 8, 1, ctypes.byref(g), ctypes.byref(h)) == G.GD_EINVAL
    assert b"x_min" in L.gd_last_error()
    g = G._Grid(1e-3, 1e3, 0, 0)
    assert L.gd_init_tensor(ctypes.byref(k), ctypes.byref(f), 8, 5, ctypes.byref(g), ctypes.byref(h)) == G.GD_EINVAL
    assert L.gd_init_tensor(ctypes.byref(k), ctypes.byref(f), 100, 3, ctypes.byref(g), ctypes.byref(h)) == G.GD_EINVAL
    k2 = G._Kernel(9, 1.0)
    assert L.gd_init_tensor(ctypes.byref(k2), ctypes.byref(f), 8, 1, ctypes.byref(g), ctypes.byref(h)) == G.GD_EINVAL
    with pytest.raises(G.GDError):
        G.Tensor(8, 1, 1e-3, 1e3, frag="powerlaw", levels=(0.6, 0.5))   # levels must ascend
    with pytest.raises(G.GDError, match="Maxwellian"):
        G.Tensor(8, 1, 1e-3, 1e3, kernel="maxwell", v0=0.0, frag="general", levels=(1.0,))
    with pytest.raises(G.GDError, match="Maxwellian"):
        G.Tensor(8, 1, 1e-3, 1e3, kernel="maxwell", v0=0.5, v_bounce=-0.1, frag="general", levels=(1.0,))
    with pytest.raises(G.GDError, match="alpha"):
        G.Tensor(8, 1, 1e-3, 1e3, frag="general", alpha=-2.0, levels=(1.0,))
    assert L.gd_rk_advance(None, None, None, None, 1.0, 0.1, 1.0, 0.0, 1, None, None) == G.GD_EINVAL
    f9 = G._Frag(9, -11 / 6, 1, lv.ctypes.data_as(G._DP))
    assert L.gd_init_tensor(ctypes.byref(k), ctypes.byref(f9), 8, 1, ctypes.byref(g), ctypes.byref(h)) == G.GD_EINVAL


def test_tensor_info_counts():
    t = G.Tensor(6, 2, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    inf = t.info()
    assert inf["P"] == 18 and inf["n_out"] == 5 + 6 * 2
    assert 0 < inf["nnz_folded"] <= inf["n_out"] * 18 * 19 // 2
    assert inf["flops_per_eval"] == 2.0 * inf["nnz_folded"]
    t2 = G.Tensor(6, 2, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=False)
    assert t2.info()["n_out"] == 6 + 6 * 2


def test_checked_build_exports_every_declared_symbol():
    """The checked build (device checks on, -DGD_CHECKS) has the same C ABI; built here
    when a checkout has none."""
    import os
    from paper_2607_13740_amd import build as B
    if not os.path.exists(B.LIB_CHECKS):
        B.build(checks=True)
    L = ctypes.CDLL(B.LIB_CHECKS)
    for n in G.declared_symbols():
        assert hasattr(L, n), n
    f = ctypes.c_uint(5)
    assert L.gd_plan_checks(None, ctypes.byref(f)) == G.GD_EINVAL
