"""Plant plausible mistakes in a temporary copy of the oracle and check that the
pins catch every one (each mutated copy must fail tests/test_oracle_pins.py)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "drop_f_coupling": ("right = -f[m, q] * composite(S, dpm, dpq)",
                        "right = 0.0 * composite(S, dpm, dpq)"),
    "sign_of_f_coupling": ("left = -f[p, m] * composite(S, dpq, dmq)",
                           "left = f[p, m] * composite(S, dpq, dmq)"),
    "trace_instead_of_frobenius": ("E += float(np.sum(Tbar * (2.0 * Kpq + L)))",
                                   "E += float(np.trace(Tbar @ (2.0 * Kpq + L)))"),
    "swapped_pair_not_transposed": ("return T[(b, a)].T[np.ix_(perm, perm)]",
                                    "return T[(b, a)][np.ix_(perm, perm)]"),
    "composite_K_operands_swapped": ("return Up @ pb.K(p, q) @ Uq.T",
                                     "return Uq @ pb.K(q, p) @ Up.T"),
    "fock_block_scaled": ("self._F[(p, q)] = self.Q[p].T @ (self.eps[:, None] * self.Q[q])",
                          "self._F[(p, q)] = 1.0001 * (self.Q[p].T @ (self.eps[:, None] * self.Q[q]))"),
    "tbar_sign": ("Tbar = 2.0 * Tpq - Tpq.T\n                Kpq", "Tbar = 2.0 * Tpq + Tpq.T\n                Kpq"),
    "wrong_2b_coefficient": ("+ [1.0 - n3_ij[p] for p in pairs]", "+ [1.0 - n3_i[p[0]] for p in pairs]"),
    "density_GF_transpose": ("GF = Tpq.T @ Sd @ Tbar + Tbar @ Sd @ Tpq.T",
                             "GF = Tpq.T @ Sd @ Tbar + Tbar @ Sd @ Tpq"),
    "dF_second_sum_dropped": ("                    acc -= float(np.sum(Tbar * M))\n                dF",
                              "                    acc -= 0.0\n                dF"),
    "denominator_sign": ("self.f[p, p] - self.f[q, q]", "self.f[p, p] + self.f[q, q]"),
    "s2b_normalised_by_product": ("/ np.sqrt(sysm.r[i] * sysm.r[j])", "/ (sysm.r[i] * sysm.r[j])"),
    "mbe_orders_2b_drops_second_monomer": ("e2 += E_cl[n] - E_cl[idx[(i,)]] - E_cl[idx[(j,)]]",
                                           "e2 += E_cl[n] - E_cl[idx[(i,)]]"),
    "mbe_orders_3b_drops_monomers": ("+ E_cl[idx[(i,)]] + E_cl[idx[(j,)]] + E_cl[idx[(k,)]])",
                                     "+ E_cl[idx[(i,)]] + E_cl[idx[(j,)]])"),
    "dvir_extra_overlap": ("Dv += P @ GF @ P.T", "Dv += P @ Sd @ GF @ P.T"),
    "dvir_half_of_GF": ("Dv += P @ GF @ P.T", "Dv += P @ (Tbar @ Sd @ Tpq.T) @ P.T"),
    "weak_dC_factor": ("dC[off[i]:off[i + 1]] += 8.0 * T @ pb.C[j]",
                       "dC[off[i]:off[i + 1]] += 4.0 * T @ pb.C[j]"),
    "weak_deps_wrong_side": ('de += 4.0 * np.einsum("am,mn,an->a", Qj, T.T @ T, Qj)',
                             'de += 4.0 * np.einsum("am,mn,an->a", Qj, T.T @ T.T.T.T, Qj) * 0.5'),
    "weak_dF_factor": ("dF[i, i] -= 4.0 * tt", "dF[i, i] -= 2.0 * tt"),
    "weak_dvir_drops_j_side": ("Dv += 4.0 * (Qi @ (T @ T.T) @ Qi.T + Qj @ (T.T @ T) @ Qj.T)",
                               "Dv += 4.0 * (Qi @ (T @ T.T) @ Qi.T)"),
    "weak_energy_factor": ("out.append(4.0 * float(np.sum(T * Kt)))", "out.append(2.0 * float(np.sum(T * Kt)))"),
    "overlap_solve_drops_weak_dC": ("dC += wd[0]", "dC += 0.0 * wd[0]"),
    "overlap_solve_drops_weak_energy": ("E += E_weak\n", "E += 0.0 * E_weak\n"),
    "nup_transposed": ("out[(i, j)] = T @ pb.K(j, i)", "out[(i, j)] = (T @ pb.K(j, i)).T"),
    "osvgen_denominator": ("D = eps_vir[:, None] + eps_vir[None, :] - 2.0 * F_occ[k, k]",
                           "D = 2.0 * eps_vir[:, None] - 2.0 * F_occ[k, k]"),
    "osvgen_ascending": ('order = np.argsort(-w, kind="stable")', 'order = np.argsort(w, kind="stable")'),
    "osvgen_wrong_lmo_C": ("Cs.append(Qk.T @ B[k])", "Cs.append(Qk.T @ B[(k + 1) % nocc])"),
    "osvgen_threshold": ("if w[i] > l_osv][:r_max]", "if w[i] > 0.5 * l_osv][:r_max]"),
    "one_step_sign": ("dT = W @ (-Rt / denom) @ W.T", "dT = W @ (Rt / denom) @ W.T"),
    "one_step_weight": ("w = 1.0 if p == q else 2.0\n        e_pq", "w = 1.0\n        e_pq"),
    "one_step_drops_second_sum": ("        R = R + left @ Tord(m, q) @ composite(S, dmq, dpq)\n    return R",
                                  "        R = R + 0.0 * (left @ Tord(m, q) @ composite(S, dmq, dpq))\n    return R"),
    "exact_K_one_lmo": ("return (P.T @ B[p]) @ (B[q].T @ P)", "return (P.T @ B[p]) @ (B[p].T @ P)"),
    "nij_drops_Dprime_S": ("+ Dm(i, j, i, j, F) @ composite(S, dij, dij))", "+ 0.0 * Dm(i, j, i, j, F))"),
    "nij_k_sum_sign": ("N = N - (f[j, k] * Dm(i, j, i, k, S)", "N = N + (f[j, k] * Dm(i, j, i, k, S)"),
    "nij_KT_order": ("N = (Tb @ composite_K(pb, i, j)", "N = (composite_K(pb, i, j) @ Tb"),
    "dC_missing_transpose": ("dC[q] += G.T @ pb.C[p]", "dC[q] += 0.5 * (G + G.T) @ pb.C[p] if G.shape[0] == G.shape[1] else G.T @ pb.C[p]"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    a, b = MUTATIONS[name]
    src = open(os.path.join(ROOT, "oracle", "osv_oracle.py")).read()
    assert a in src, f"mutation anchor for {name} not found"
    for sub in ("oracle", "paper_2106_06149_amd", "tests"):
        os.makedirs(tmp_path / sub)
    open(tmp_path / "oracle" / "__init__.py", "w").close()
    open(tmp_path / "oracle" / "osv_oracle.py", "w").write(src.replace(a, b, 1))
    open(tmp_path / "paper_2106_06149_amd" / "__init__.py", "w").close()
    shutil.copy(os.path.join(ROOT, "paper_2106_06149_amd", "synth.py"), tmp_path / "paper_2106_06149_amd")
    shutil.copy(os.path.join(ROOT, "tests", "test_oracle_pins.py"), tmp_path / "tests")
    shutil.copy(os.path.join(ROOT, "tests", "conftest.py"), tmp_path / "tests")
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), tmp_path / "tests" / "golden")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        str(tmp_path / "tests" / "test_oracle_pins.py")],
                       cwd=str(tmp_path), capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} was not caught:\n{r.stdout[-2000:]}"
