"""GPU parity with the cross-projected pair-domain integrals of eq:aijkl built from
B (osv_build_pairs_exact) against the oracle with the same integrals: energies,
MBE orders, cluster energies and the one-electron densities element by element."""
import numpy as np
import pytest

from paper_2106_06149_amd import _lib as L, synth
from paper_2106_06149_amd.api import OSVContext
from oracle import osv_oracle as O, pool as OP

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def run(s, dvir=False):
    oc = OSVContext.from_system(s, device="cuda:0", k_exact=True)
    oc.solve(tau_R=1e-10)
    E, orders, Ecl = oc.energy(per_cluster=True)
    with pytest.raises(L.OSVError) as e:
        oc.densities(dC=True)
    assert e.value.status == L.OSV_E_ARG
    _, dF, de, Dv = oc.densities(dC=False, dvir=dvir)
    out = dict(E=E, orders=orders, Ecl=Ecl.cpu().numpy(), dF=dF.cpu().numpy(), de=de.cpu().numpy(),
               Dv=None if Dv is None else Dv.cpu().numpy())
    oc.close()
    return out


def compare(g, ref, tol=1e-8):
    assert abs(g["E"] - ref["E"]) <= 1e-8, (g["E"], ref["E"])
    assert np.abs(g["Ecl"] - ref["E_cluster"]).max() <= 1e-8
    if not np.isnan(ref["E_orders"][0]):
        assert np.abs(g["orders"] - ref["E_orders"]).max() <= 1e-8
    for a, b in ((g["dF"], ref["dE_dF"]), (g["de"], ref["dE_deps"])):
        assert np.abs(a - b).max() <= tol * np.abs(b).max()
    if g["Dv"] is not None:
        assert np.abs(g["Dv"] - ref["Dvir"]).max() <= tol * np.abs(ref["Dvir"]).max()


def test_exact_integrals_small_ragged():
    s = synth.make_system(5, 90, 70, [17, 35, 9, 33, 21], seed=12, cut2=4.5, cut3=4.5)
    say("case cross-projected integrals nocc=5 r=[17,35,9,33,21]")
    g = run(s, dvir=True)
    ref = O.solve(s, k_exact=True, dvir=True)
    compare(g, ref)
    r1 = O.solve(s, densities=False)["E"]
    assert abs(g["E"] - r1) > 1e-6 * abs(r1)      # the two readings differ here


def test_exact_integrals_full_osv_mp2_workload0():
    s = synth.workload(0)
    say("case cross-projected integrals, workload 0 (full OSV-MP2)")
    compare(run(s), O.solve(s, k_exact=True))


def test_exact_integrals_workload1():
    s = synth.workload(1)
    say(f"case cross-projected integrals, workload 1 (nocc=32), oracle on {OP.default_workers()} workers")
    compare(run(s), OP.solve(s, k_exact=True))
