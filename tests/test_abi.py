"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol include/rt.h declares, computes Eq. 20 on the host like the oracle, and rejects
bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1001_3301_amd import rt, synth as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = rt.lib()
    hdr = open(os.path.join(ROOT, "include", "rt.h")).read()
    declared = set(re.findall(r"^\s*(?:rt_status|void|const char \*|long|int)\s*\**(rt_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(rt.EXPORTS), declared ^ set(rt.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n_nu", [1, 32, 61, 64])
def test_star_bin_flux_matches_oracle(n_nu):
    nu = sy.frequencies(n_nu)
    a = rt.star_bin_flux(sy.T_STAR, nu)
    b = oracle.star_bins(sy.T_STAR, nu)
    assert np.max(np.abs(a / b - 1)) < 1e-12
    assert abs(a.sum() / (sy.SIGMA_SB * sy.T_STAR ** 4) - 1) < 1e-13


def test_star_bin_flux_rejects_bad_input():
    with pytest.raises(rt.RtError):
        rt.star_bin_flux(-1.0, [1e12, 2e12])
    with pytest.raises(rt.RtError):
        rt.star_bin_flux(5800.0, [2e12, 1e12])


def test_create_rejects_bad_grids_before_device_use():
    L = rt.lib()
    rf = np.geomspace(1, 10, 9)
    tf = np.linspace(0, np.pi, 5)
    pf = np.linspace(0, 2 * np.pi, 3)
    h = C.c_void_p()
    bad = [(rf[::-1].copy(), tf, pf, 8), (rf, tf, pf, 65), (rf, tf, pf, 0),
           (rf, np.linspace(0, 4.0, 5), pf, 8),
           (np.array([1.0, 2.0]), tf, pf, 8),           # one radial cell (the colouring needs two)
           (np.geomspace(1, 10, 4001), tf, pf, 8)]      # a column too long for the ray trace's LDS
    for r_, t_, p_, nnu in bad:
        g = rt.Grid(len(r_) - 1, len(t_) - 1, len(p_) - 1, r_.ctypes.data_as(rt.dp),
                    t_.ctypes.data_as(rt.dp), p_.ctypes.data_as(rt.dp))
        assert L.rt_create(C.byref(h), C.byref(g), nnu, None) == rt.RT_EINVAL
        assert len(L.rt_last_error(None)) > 0
    assert L.rt_create(None, None, 8, None) == rt.RT_EINVAL


def test_null_context_is_rejected():
    L = rt.lib()
    assert L.rt_raytrace(None, None, None, None, None, None, None, None, None) == rt.RT_EINVAL
    assert L.rt_fld_solve(None, None, None, None) == rt.RT_EINVAL
