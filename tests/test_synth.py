"""Generator checks: shapes, OSV orthonormality, symmetry, reproducibility, and
the cluster counts of the five workloads."""
import numpy as np
import pytest

from paper_2106_06149_amd import synth
from oracle import osv_oracle as O


def test_small_system_invariants():
    s = synth.make_system(5, 30, 20, (3, 7), seed=3)
    assert s.Q.shape == (30, s.nosv) and s.Q.flags.f_contiguous
    assert s.C.shape == (s.nosv, 20) and s.C.flags.c_contiguous
    for i in range(5):
        assert np.allclose(s.Qi(i).T @ s.Qi(i), np.eye(s.r[i]), atol=1e-13)
        assert np.allclose(s.Ci(i), s.Qi(i).T @ s.B[i], atol=1e-14)
    assert np.allclose(s.F_occ, s.F_occ.T)
    assert np.all(s.r >= 3) and np.all(s.r <= 7)


def test_reproducible():
    a = synth.make_system(4, 20, 10, 3, seed=5, geometry="lattice", spacing=2.5, c_direct=True,
                          c_dtype=np.float32)
    b = synth.make_system(4, 20, 10, 3, seed=5, geometry="lattice", spacing=2.5, c_direct=True,
                          c_dtype=np.float32)
    assert np.array_equal(a.Q, b.Q) and np.array_equal(a.C, b.C) and a.C.dtype == np.float32
    cen, r = synth.make_system(4, 20, 10, 3, seed=5, geometry="lattice", spacing=2.5,
                               geometry_only=True)
    assert np.array_equal(cen, a.centroid) and np.array_equal(r, a.r)


def test_workload0_recipe():
    s = synth.workload(0)
    assert (s.nocc, s.nvir, s.naux) == (6, 60, 150) and np.all(s.r == 8)
    assert np.allclose(s.centroid[:, 0], 2.0 * np.arange(6))
    off = s.F_occ - np.diag(np.diag(s.F_occ))
    assert np.isclose(off[0, 1], 0.02 * np.exp(-2.0 / 3.0))
    assert np.all(np.diag(s.F_occ) >= -1.2) and np.all(np.diag(s.F_occ) <= -0.4)
    assert np.all(s.eps_vir >= 0.3) and np.all(s.eps_vir <= 4.0)


@pytest.mark.parametrize("k,counts", [(1, (32, 196, 172)), (3, (64, 420, 364)),
                                      (2, (128, 7902, 48926))])
def test_workload_cluster_counts(k, counts):
    cen, r = synth.workload(k, geometry_only=True)
    spec = synth.WORKLOADS[k]
    cl, coef, order = O.select_clusters(cen, spec["sel_mode"], spec["cut2"], spec["cut3"])
    assert tuple(int((order == n).sum()) for n in (1, 2, 3)) == counts
