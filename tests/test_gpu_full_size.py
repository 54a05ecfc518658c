"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (same selection, precision and solve threshold):

* per-cluster energies E^X of a seeded sample of clusters against the FP64
  oracle computing those clusters one by one (clusters are independent);
* identities that hold at any size for the whole MBE energy and its densities
  (E is homogeneous of degree 4 in C and of degree -1 in (eps_vir, F_occ));
* mixed precision against the FP64 GPU path on the same input;
* central finite differences through the torch.autograd.Function on the
  nocc = 64 gradient workload (FP64);
* every density element against the oracle on the whole nocc = 64 gradient
  workload, and on 27-LMO lattice systems drawn by the nocc = 128 and nocc = 400
  recipes (their full nvir, naux and r ranges and cutoffs), FP64 and mixed;
  the oracle runs its independent clusters in worker processes.
"""
import numpy as np
import pytest
import torch

from paper_2106_06149_amd import synth
from paper_2106_06149_amd.api import OSVContext, Selection, plan_clusters
from paper_2106_06149_amd.autograd import OSVEnergy
from oracle import osv_oracle as O, pool as OP

pytestmark = pytest.mark.gpu

TAU_R = 1e-10
E_CLUSTER_TOL = 1e-8     # Eh, per cluster (FP64 bar; the mixed K error is far below it)
MIXED_TOL = 1e-6         # Eh, whole MBE energy, mixed vs FP64


def say(msg):
    print(msg, flush=True)


def sample_clusters(s, n1, n2, n3, seed):
    sel = Selection(s.sel_mode, s.cut2, s.cut3)
    counts, lmos, coef = plan_clusters(s.centroid, sel)
    size = (lmos >= 0).sum(axis=1)
    rng = np.random.default_rng(seed)
    idx = []
    for k, n in ((1, n1), (2, n2), (3, n3)):
        cand = np.flatnonzero(size == k)
        idx += list(rng.choice(cand, size=min(n, len(cand)), replace=False))
    return sorted(int(i) for i in idx), lmos


def oracle_cluster_energies(s, idx, lmos):
    pb = O.PairBlocks(s)
    out = []
    for n in idx:
        X = [int(x) for x in lmos[n] if x >= 0]
        cl = O.Cluster(pb, X)
        cl.solve(TAU_R, 100)
        out.append(cl.energy())
    return np.array(out)


def run(s, precision):
    oc = OSVContext.from_system(s, device="cuda:0", precision=precision)
    info = oc.solve(tau_R=TAU_R)
    E, orders, Ecl = oc.energy(per_cluster=True)
    dC, dF, de, _ = oc.densities()
    C = oc.C.double()
    euler_C = float(torch.sum(C * dC))
    euler_F = float(torch.dot(oc.eps, de) + torch.sum(oc.F * dF))
    out = dict(E=E, orders=orders, Ecl=Ecl.cpu().numpy(), info=info, euler_C=euler_C,
               euler_F=euler_F, counts=oc.counts)
    oc.close()
    del C, dC, dF, de
    torch.cuda.empty_cache()
    return out


def check_euler(g, rel=1e-8):
    E = g["E"]
    assert abs(g["euler_C"] - 4.0 * E) <= rel * abs(E), (g["euler_C"], 4 * E)
    assert abs(g["euler_F"] + E) <= rel * abs(E), (g["euler_F"], -E)


@pytest.mark.parametrize("k", [2, 4])
def test_full_size_sampled_clusters_and_identities(k):
    spec = synth.WORKLOADS[k]
    say(f"case workload {k} ({spec['name']}): generating")
    s = synth.workload(k)
    say(f"case workload {k}: mixed GPU run")
    gm = run(s, 1)
    assert gm["info"]["converged"]
    say(f"case workload {k}: FP64 GPU run")
    gd = run(s, 0)
    say(f"case workload {k}: E mixed {gm['E']:.10f} fp64 {gd['E']:.10f}")
    assert abs(gm["E"] - gd["E"]) <= MIXED_TOL
    assert np.all(np.abs(gm["orders"] - gd["orders"]) <= MIXED_TOL)
    assert abs(sum(gd["orders"]) - gd["E"]) <= 1e-9 * abs(gd["E"])
    check_euler(gm)
    check_euler(gd)
    idx, lmos = sample_clusters(s, 3, 6, 9, seed=100 + k)
    say(f"case workload {k}: oracle on clusters {idx}")
    ref = oracle_cluster_energies(s, idx, lmos)
    np.testing.assert_allclose(gd["Ecl"][idx], ref, rtol=0, atol=E_CLUSTER_TOL)
    np.testing.assert_allclose(gm["Ecl"][idx], ref, rtol=0, atol=E_CLUSTER_TOL)


def test_gradient_workload_finite_differences():
    """Workload 3 (nocc = 64, FP64): dE/dC, dE/dF_occ and dE/deps_vir from the
    autograd backward against central differences, h = 1e-4, 20 seeded entries
    (10 of C, 5 symmetric f_uv, 5 of eps_vir)."""
    s = synth.workload(3)
    dev = torch.device("cuda:0")
    Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T)).to(dev)
    C = torch.from_numpy(s.C).to(dev).requires_grad_(True)
    F = torch.from_numpy(s.F_occ).to(dev).requires_grad_(True)
    eps = torch.from_numpy(s.eps_vir).to(dev).requires_grad_(True)
    sel = Selection(s.sel_mode, s.cut2, s.cut3)
    say("case workload 3: autograd forward/backward")
    E = OSVEnergy.apply(C, F, eps, Qt, s.r, s.centroid, sel, 0)
    gC, gF, ge = torch.autograd.grad(E, (C, F, eps))
    gC, gF, ge = gC.cpu().numpy(), gF.cpu().numpy(), ge.cpu().numpy()

    def energy(Cx, Fx, ex):
        with torch.no_grad():
            return float(OSVEnergy.apply(Cx, Fx, ex, Qt, s.r, s.centroid, sel, 0))

    h = 1e-4
    rng = np.random.default_rng(2106)
    C0, F0, e0 = C.detach(), F.detach(), eps.detach()
    checked = []
    # C entries: rows chosen at random, the column with the largest |dE/dC| in that row
    # half of the time so that the check is not dominated by near-zero derivatives
    for t in range(10):
        a = int(rng.integers(0, s.nosv))
        b = int(np.argmax(np.abs(gC[a]))) if t % 2 == 0 else int(rng.integers(0, s.naux))
        Cp = C0.clone(); Cp[a, b] += h
        Cm = C0.clone(); Cm[a, b] -= h
        fd = (energy(Cp, F0, e0) - energy(Cm, F0, e0)) / (2 * h)
        checked.append(("C", a, b, fd, gC[a, b]))
    for t in range(5):
        u = int(rng.integers(0, s.nocc - 1))
        v = u + (t % 2)           # neighbours and diagonal entries
        Fp = F0.clone(); Fp[u, v] += h; Fp[v, u] = Fp[u, v]
        Fm = F0.clone(); Fm[u, v] -= h; Fm[v, u] = Fm[u, v]
        fd = (energy(C0, Fp, e0) - energy(C0, Fm, e0)) / (2 * h)
        an = gF[u, v] + (gF[v, u] if u != v else 0.0)
        checked.append(("F", u, v, fd, an))
    for t in range(5):
        a = int(rng.integers(0, s.nvir))
        ep = e0.clone(); ep[a] += h
        em = e0.clone(); em[a] -= h
        fd = (energy(C0, F0, ep) - energy(C0, F0, em)) / (2 * h)
        checked.append(("eps", a, -1, fd, ge[a]))
    for name, a, b, fd, an in checked:
        say(f"  FD {name}[{a},{b}] fd={fd:.10e} analytic={an:.10e}")
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (name, a, b, fd, an)
    assert max(abs(c[4]) for c in checked) > 1e-3   # the check is not vacuous


DENS_TOL = 1e-8          # densities: max |GPU - oracle| over the largest entry (FP64 path)
DENS_TOL_MIXED = 1e-7    # mixed path: K from the exact FP32 digits, truncated below 2^-43


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(1e-300, np.max(np.abs(b))))


def run_dens(s, precision, dvir=False):
    oc = OSVContext.from_system(s, device="cuda:0", precision=precision)
    info = oc.solve(tau_R=TAU_R)
    E, orders, Ecl = oc.energy(per_cluster=True)
    dC, dF, de, Dv = oc.densities(dvir=dvir)
    out = dict(E=E, orders=orders, Ecl=Ecl.cpu().numpy(), dC=dC.cpu().numpy(), dF=dF.cpu().numpy(),
               de=de.cpu().numpy(), Dv=None if Dv is None else Dv.cpu().numpy(), info=info)
    oc.close()
    return out


def compare_dens(g, ref, tol, etol=E_CLUSTER_TOL):
    assert abs(g["E"] - ref["E"]) <= etol, (g["E"], ref["E"])
    assert np.max(np.abs(g["Ecl"] - ref["E_cluster"])) <= etol
    assert np.max(np.abs(g["orders"] - ref["E_orders"])) <= etol
    for gk, rk in (("dC", "dE_dC"), ("dF", "dE_dF"), ("de", "dE_deps")):
        e = rel_err(g[gk], ref[rk])
        say(f"  {gk}: max |gpu - oracle| / max |oracle| = {e:.2e}")
        assert e <= tol, (gk, e)
    if g["Dv"] is not None and "Dvir" in ref:
        e = rel_err(g["Dv"], ref["Dvir"])
        say(f"  Dvir: {e:.2e}")
        assert e <= tol, ("Dvir", e)


def test_gradient_workload_densities_elementwise():
    """Workload 3 (nocc = 64, 848 clusters, FP64): every element of dE/dC,
    dE/dF_occ and dE/deps_vir, the MBE orders and each cluster energy against the
    oracle solving all clusters."""
    s = synth.workload(3)
    say("case workload 3: GPU FP64 run")
    g = run_dens(s, 0)
    say(f"case workload 3: oracle over all clusters ({OP.default_workers()} workers)")
    ref = OP.solve(s, tau_R=TAU_R)
    compare_dens(g, ref, DENS_TOL)


@pytest.mark.parametrize("k", [2, 4])
def test_lattice_27_lmo_densities_elementwise(k):
    """27 LMOs on the jittered lattice drawn by the recipe of workload k (its nvir,
    naux, r range, FP32 C and cutoffs): energies and every density element against
    the oracle, in FP64 (1e-8 of the largest entry) and mixed precision (1e-7)."""
    s = synth.workload(k, nocc=27)
    say(f"case 27-LMO lattice by the workload {k} recipe: nvir={s.nvir} naux={s.naux} "
        f"sum r={s.nosv}: GPU runs")
    gd = run_dens(s, 0)
    gm = run_dens(s, 1)
    say(f"case 27-LMO lattice workload {k}: oracle over all clusters ({OP.default_workers()} workers)")
    ref = OP.solve(s, tau_R=TAU_R)
    say(f"  {len(ref['clusters'])} clusters, E = {ref['E']:.10f}")
    compare_dens(gd, ref, DENS_TOL)
    compare_dens(gm, ref, DENS_TOL_MIXED)
