"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol of include/osv.h, validates arguments, and its cluster selection
matches the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2106_06149_amd import _lib as L, api, synth
from oracle import osv_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    lib = L.load()
    hdr = open(os.path.join(ROOT, "include", "osv.h")).read()
    declared = set(re.findall(r"\b(osv_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def test_status_strings():
    lib = L.load()
    for st in range(0, -8, -1):
        assert lib.osv_status_string(st).decode()
    assert lib.osv_status_string(5).decode() == "unknown status"


@pytest.mark.parametrize("k", [1, 3])
def test_plan_matches_oracle(k):
    cen, r = synth.workload(k, geometry_only=True)
    spec = synth.WORKLOADS[k]
    counts, lmos, coef = api.plan_clusters(cen, api.Selection(0, spec["cut2"], spec["cut3"]))
    cl, c, order = O.select_clusters(cen, spec["sel_mode"], spec["cut2"], spec["cut3"])
    assert counts["n_clusters"] == len(cl)
    ours = [tuple(int(x) for x in row if x >= 0) for row in lmos]
    assert ours == [tuple(X) for X in cl]
    assert np.array_equal(coef, c)
    assert counts["n_pair_blocks"] == sum(len(X) * (len(X) + 1) // 2 for X in cl)


def test_plan_large_lattice_counts():
    cen, r = synth.workload(4, geometry_only=True)
    counts, _, coef = api.plan_clusters(cen, api.Selection(0, 15.0, 7.0))
    assert (counts["n1b"], counts["n2b"], counts["n3b"]) == (400, 56012, 113438)
    assert counts["n_pair_blocks"] == 849064


def test_plan_full_mode():
    cen = np.zeros((5, 3))
    counts, lmos, coef = api.plan_clusters(cen, api.Selection(L.OSV_SEL_FULL))
    assert counts["n_clusters"] == 1 and counts["n_pair_blocks"] == 15 and coef[0] == 1.0
    # every ordered pair (p,q) couples to (p,m) and (m,q): 10 domains (q>p) + 5 diagonal
    assert counts["n_domains"] == 15


def test_argument_validation_without_gpu():
    lib = L.load()
    h = ctypes.c_void_p()
    sel = L.OsvSelect(0, 15.0, 8.0, 1e-2, 0.2, 1e-8)
    # NULL system
    assert lib.osv_build_pairs(None, ctypes.byref(sel), 0, None, ctypes.byref(h)) == L.OSV_E_ARG
    assert h.value is None
    r = np.array([3, 0], dtype=np.int32)
    sysc = L.OsvSystem(2, 10, 5, r.ctypes.data_as(ctypes.c_void_p), 1, 1, 0, 1, 1, None)
    assert lib.osv_build_pairs(ctypes.byref(sysc), ctypes.byref(sel), 0, None, ctypes.byref(h)) == L.OSV_E_ARG
    assert b"centroid" in lib.osv_last_error(None) or b"r[" in lib.osv_last_error(None)
    # unknown precision / mixed without FP32 C
    r = np.array([3, 3], dtype=np.int32)
    cen = np.zeros((2, 3))
    sysc = L.OsvSystem(2, 10, 5, r.ctypes.data_as(ctypes.c_void_p), 1, 1, 0, 1, 1,
                       cen.ctypes.data_as(ctypes.c_void_p))
    assert lib.osv_build_pairs(ctypes.byref(sysc), ctypes.byref(sel), 7, None, ctypes.byref(h)) == L.OSV_E_ARG
    assert lib.osv_build_pairs(ctypes.byref(sysc), ctypes.byref(sel), 1, None, ctypes.byref(h)) == L.OSV_E_ARG
    bad = L.OsvSelect(9, 15.0, 8.0, 1e-2, 0.2, 1e-8)
    assert lib.osv_build_pairs(ctypes.byref(sysc), ctypes.byref(bad), 0, None, ctypes.byref(h)) == L.OSV_E_ARG
    # domain too large
    r = np.array([60, 60], dtype=np.int32)
    sysc = L.OsvSystem(2, 100, 5, r.ctypes.data_as(ctypes.c_void_p), 1, 1, 0, 1, 1,
                       cen.ctypes.data_as(ctypes.c_void_p))
    # r_i > nvir is caught before any device work
    r2 = np.array([3, 200], dtype=np.int32)
    sysc2 = L.OsvSystem(2, 100, 5, r2.ctypes.data_as(ctypes.c_void_p), 1, 1, 0, 1, 1,
                        cen.ctypes.data_as(ctypes.c_void_p))
    assert lib.osv_build_pairs(ctypes.byref(sysc2), ctypes.byref(sel), 0, None, ctypes.byref(h)) == L.OSV_E_ARG
    # NULL context calls
    assert lib.osv_solve_clusters(None, 1e-10, 10, None, None) == L.OSV_E_ARG
    E = ctypes.c_double()
    assert lib.osv_energy(None, None, ctypes.byref(E), None, None) == L.OSV_E_ARG
    assert lib.osv_densities(None, None, None, None, None, None) == L.OSV_E_ARG
    assert lib.osv_query(None, None) == L.OSV_E_ARG
    lib.osv_destroy(None)
