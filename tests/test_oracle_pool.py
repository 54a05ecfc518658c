"""The cluster-parallel oracle driver gives the oracle's own results: the same
energies per cluster and, summed in a different grouping, the same densities."""
import numpy as np

from paper_2106_06149_amd import synth
from oracle import osv_oracle as O, pool


def test_pool_matches_serial_oracle():
    s = synth.make_system(6, 30, 24, (3, 6), seed=11, cut2=4.5, cut3=4.5)
    a = O.solve(s, dvir=True)
    b = pool.solve(s, nproc=3, dvir=True)
    assert b["workers"] == 3
    assert np.array_equal(a["E_cluster"], b["E_cluster"])
    assert abs(a["E"] - b["E"]) <= 1e-14 * abs(a["E"])
    assert np.allclose(a["E_orders"], b["E_orders"], rtol=1e-13, atol=0)
    for k in ("dE_dC", "dE_dF", "dE_deps", "Dvir"):
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-14 * np.abs(a[k]).max()), k
