"""FP64 CPU oracle for the MBE(3)-OSV-MP2 per-cluster hot path.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product path never does.  It is a
plain, slow, obviously-correct restatement of the method in NumPy float64 and
shares no code with the HIP library.

Paper: Liang & Yang, "Third-order many-body expansion of OSV-MP2 wavefunction
for low-order scaling analytical gradient computation" (arXiv 2106.06149).

What is computed, in the paper's notation:
  * orbital-pair blocks S_(i,j) = Q_i^T Q_j, F_(i,j) = Q_i^T diag(eps) Q_j and
    K_ij = C_i C_j^T (Algorithm 1, pair tasks; eq:aijkl);
  * composite pair-domain matrices A_(ij,kl) assembled from those blocks with
    A_(ij,kl)^T = A_(kl,ij) (eq:aijkl, eq:aadjoint);
  * per cluster X (1, 2 or 3 LMOs, or all LMOs), the residual equations
    eq:rij restricted to k in X, solved by preconditioned Jacobi;
  * the Hylleraas cluster energy eq:ec;
  * the MBE inclusion-exclusion of cluster energies (eq:mbe1, with the cluster
    expansions eq:tmbediag/eq:tmbeoff giving the same coefficients);
  * exact densities dE/dC_i, dE/df_ij, dE/deps_a at fixed Q via Hylleraas
    stationarity (the amplitudes make no contribution; cf. eq:dv, eq:do,
    eq:ec2eY and the OSV density matrices D_(ij,kl)), MBE-summed per cluster
    (eq:mbe2).

Readings taken where the paper is silent (each is listed in the design notes):
  R1 K_(pq,pq) = U_p K_pq U_q^T with U_p = P_pq^T Q_p: fitted integrals are
     represented in their own LMO's OSV span (B_p ~ Q_p C_p).
  R2 <A B> is the Frobenius inner product sum(A * B).
  R3 pairs are ordered; E = sum_p e_pp + 2 sum_{p<q} e_pq.
  R4 the diagonal-pair domain is Q_p alone.
  R5 Jacobi sweeps from T = 0, preconditioned in the pseudo-canonical basis of
     each pair domain; a cluster stops when max_pairs ||W^T R W||_F < tau_R and
     returns the amplitudes at which that residual was evaluated.
  R7 eigenvalues of S_(pq,pq) at or below tau_S are dropped.
  R9 clusters: 2b pairs with centroid distance <= cut2, 3b triples with all
     three distances <= cut3 and all three sub-pairs selected (downward closed).
  R10 densities are the exact derivative of the MBE energy.
  R15 weak pairs (correlation scheme for weak 2b clusters; eq:2bscreen): pairs
     i < j with 1e-7 <= s2b_ij <= l_2b (not strong, not discarded) keep only the
     dispersion block T_(i,j) (i -> OSVs of i, j -> OSVs of j) in the
     pseudo-canonical bases of the diagonal domains (R4); with the other blocks
     projected out the one-block residual K~ + (e~_a + e~_b - f_ii - f_jj) T
     vanishes in one step, and the pair contributes <Tbar, K> over both
     orderings, 4 <T, K~> (the exchange block is not represented); its
     densities follow from the stationarity of the one-block Hylleraas
     functional (weak_pair_densities).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

SEL_DISTANCE = 0
SEL_OVERLAP = 1
SEL_FULL = 2


# ---------------------------------------------------------------------------
# Cluster selection and MBE coefficients (MBE(3) partitioning section;
# eq:2bscreen, eq:3bscreen; inclusion-exclusion of eq:mbe1)
# ---------------------------------------------------------------------------

def select_clusters(centroid: np.ndarray, mode: int, cut2: float = 15.0, cut3: float = 8.0,
                    s2b: np.ndarray = None, l2b: float = 1e-2, l3b: float = 0.2):
    """Return (clusters, coef, order) in canonical order: all 1b (ascending),
    then 2b (lexicographic), then 3b (lexicographic); FULL gives one cluster."""
    nocc = centroid.shape[0]
    if mode == SEL_FULL:
        return [tuple(range(nocc))], np.array([1.0]), np.array([0])
    if mode == SEL_DISTANCE:
        d = np.sqrt(((centroid[:, None, :] - centroid[None, :, :]) ** 2).sum(-1))
        keep2 = lambda i, j: d[i, j] <= cut2
        keep3 = lambda i, j, k: d[i, j] <= cut3 and d[i, k] <= cut3 and d[j, k] <= cut3
    elif mode == SEL_OVERLAP:
        keep2 = lambda i, j: s2b[i, j] > l2b
        keep3 = lambda i, j, k: (s2b[i, j] + s2b[i, k] + s2b[j, k]) / 3.0 > l3b
    else:
        raise ValueError(mode)
    pairs = [(i, j) for i in range(nocc) for j in range(i + 1, nocc) if keep2(i, j)]
    pset = set(pairs)
    triples = [(i, j, k) for (i, j, k) in itertools.combinations(range(nocc), 3)
               if (i, j) in pset and (i, k) in pset and (j, k) in pset and keep3(i, j, k)]
    n2 = np.zeros(nocc)
    n3_i = np.zeros(nocc)
    n3_ij: Dict[Tuple[int, int], int] = {p: 0 for p in pairs}
    for (i, j) in pairs:
        n2[i] += 1
        n2[j] += 1
    for (i, j, k) in triples:
        for a in (i, j, k):
            n3_i[a] += 1
        for p in ((i, j), (i, k), (j, k)):
            n3_ij[p] += 1
    clusters = [(i,) for i in range(nocc)] + pairs + triples
    coef = ([1.0 - n2[i] + n3_i[i] for i in range(nocc)]
            + [1.0 - n3_ij[p] for p in pairs] + [1.0] * len(triples))
    order = [1] * nocc + [2] * len(pairs) + [3] * len(triples)
    return clusters, np.array(coef), np.array(order)


def s2b_metric(sysm) -> np.ndarray:
    """Pairwise OSV overlap metric eq:2bscreen: sum (Q_i^T Q_j)^2 / sqrt(n_i n_j)."""
    n = sysm.nocc
    s = np.eye(n)
    for i in range(n):
        for j in range(i + 1, n):
            o = sysm.Qi(i).T @ sysm.Qi(j)
            s[i, j] = s[j, i] = float((o * o).sum()) / np.sqrt(sysm.r[i] * sysm.r[j])
    return s


# ---------------------------------------------------------------------------
# Orbital-pair blocks and composite pair-domain matrices (eq:aijkl)
# ---------------------------------------------------------------------------

class PairBlocks:
    """Lazily computed orbital-pair blocks S_(p,q), F_(p,q), K_pq (float64).  With
    k_exact the pair-domain integrals are the cross-projected ones of eq:aijkl,
    K_(pq,pq) = P_pq^T B_p B_q^T P_pq (the system's B), instead of reading R1."""

    def __init__(self, sysm, k_exact: bool = False):
        self.sys = sysm
        self.k_exact = k_exact
        if k_exact and getattr(sysm, "B", None) is None:
            raise ValueError("cross-projected integrals need the fitted integrals B")
        self.Q = [np.asarray(sysm.Qi(i), dtype=np.float64) for i in range(sysm.nocc)]
        self.C = [np.asarray(sysm.Ci(i), dtype=np.float64) for i in range(sysm.nocc)]
        self.eps = np.asarray(sysm.eps_vir, dtype=np.float64)
        # a full symmetric virtual Fock matrix, when the system carries one (used
        # to differentiate with respect to its off-diagonal entries); otherwise
        # the canonical diag(eps)
        fv = getattr(sysm, "F_vir", None)
        self.Fvir = None if fv is None else np.asarray(fv, dtype=np.float64)
        self.f = np.asarray(sysm.F_occ, dtype=np.float64)
        self._S: Dict = {}
        self._F: Dict = {}
        self._K: Dict = {}

    def S(self, p, q):
        if p == q:
            return np.eye(self.Q[p].shape[1])      # OSV orthonormality, S_(p,p) = 1
        if (p, q) not in self._S:
            self._S[(p, q)] = self.Q[p].T @ self.Q[q]
            self._S[(q, p)] = self._S[(p, q)].T
        return self._S[(p, q)]

    def F(self, p, q):
        if (p, q) not in self._F:
            if self.Fvir is None:
                self._F[(p, q)] = self.Q[p].T @ (self.eps[:, None] * self.Q[q])
            else:
                self._F[(p, q)] = self.Q[p].T @ self.Fvir @ self.Q[q]
            self._F[(q, p)] = self._F[(p, q)].T
        return self._F[(p, q)]

    def K(self, p, q):
        if (p, q) not in self._K:
            self._K[(p, q)] = self.C[p] @ self.C[q].T
            self._K[(q, p)] = self._K[(p, q)].T
        return self._K[(p, q)]


def dom(a: int, b: int) -> Tuple[int, ...]:
    """Orbital list of the domain of the ordered pair (a, b): [Q_a Q_b], or Q_a (R4)."""
    return (a,) if a == b else (a, b)


def composite(blockfn, rows: Sequence[int], cols: Sequence[int]) -> np.ndarray:
    """A_(rows, cols) = [Q_rows]^T A [Q_cols] assembled from orbital blocks."""
    return np.block([[blockfn(a, b) for b in cols] for a in rows])


def composite_K(pb: PairBlocks, p: int, q: int) -> np.ndarray:
    """K_(pq,pq) = U_p K_pq U_q^T, U_p = P_pq^T Q_p (reading R1); with pb.k_exact the
    four blocks (p mu|q nu) of eq:aijkl from B: P_pq^T B_p B_q^T P_pq."""
    d = dom(p, q)
    if pb.k_exact:
        P = np.hstack([pb.Q[o] for o in d])
        B = pb.sys.B
        return (P.T @ B[p]) @ (B[q].T @ P)
    Up = composite(pb.S, d, (p,))
    Uq = composite(pb.S, d, (q,))
    return Up @ pb.K(p, q) @ Uq.T


# ---------------------------------------------------------------------------
# One cluster: residual eq:rij, Jacobi solve, Hylleraas energy eq:ec
# ---------------------------------------------------------------------------

class Cluster:
    def __init__(self, pb: PairBlocks, X: Sequence[int], tau_S: float = 1e-8):
        self.pb = pb
        self.X = tuple(X)
        self.f = pb.f
        self.pairs = [(p, q) for p in self.X for q in self.X if p <= q]
        self.Kc = {}
        self.W = {}
        self.denom = {}
        for (p, q) in self.pairs:
            d = dom(p, q)
            self.Kc[(p, q)] = composite_K(pb, p, q)
            S = composite(pb.S, d, d)
            F = composite(pb.F, d, d)
            # canonical orthogonalisation, then pseudo-canonicalisation (R5, R7)
            s, U = np.linalg.eigh(S)
            keep = s > tau_S
            Xo = U[:, keep] / np.sqrt(s[keep])[None, :]
            e, V = np.linalg.eigh(Xo.T @ F @ Xo)
            self.W[(p, q)] = Xo @ V
            self.denom[(p, q)] = e[:, None] + e[None, :] - self.f[p, p] - self.f[q, q]

    # amplitudes -----------------------------------------------------------
    @staticmethod
    def swap_perm(ra: int, rb: int) -> np.ndarray:
        """Index map from basis (a, b) to basis (b, a) of the same two OSV sets."""
        return np.concatenate([np.arange(rb, rb + ra), np.arange(0, rb)])

    def T_ordered(self, T: Dict, a: int, b: int) -> np.ndarray:
        """T_ab in basis dom(a, b); for a > b, T_ab = Pi^T T_ba^T Pi (T^{ab} = T^{ba,T})."""
        if a <= b:
            return T[(a, b)]
        ra, rb = self.pb.Q[a].shape[1], self.pb.Q[b].shape[1]
        perm = self.swap_perm(ra, rb)
        return T[(b, a)].T[np.ix_(perm, perm)]

    def residual(self, T: Dict, p: int, q: int, with_K: bool = True) -> np.ndarray:
        """eq:rij for the ordered pair (p, q), k restricted to the cluster."""
        S, F, f = self.pb.S, self.pb.F, self.f
        dpq = dom(p, q)
        R = composite_K(self.pb, p, q) if with_K else 0.0
        for m in self.X:
            dpm = dom(p, m)
            dmq = dom(m, q)
            right = -f[m, q] * composite(S, dpm, dpq)
            if m == q:
                right = right + composite(F, dpm, dpq)
            R = R + composite(S, dpq, dpm) @ self.T_ordered(T, p, m) @ right
            left = -f[p, m] * composite(S, dpq, dmq)
            if p == m:
                left = left + composite(F, dpq, dmq)
            R = R + left @ self.T_ordered(T, m, q) @ composite(S, dmq, dpq)
        return R

    def solve(self, tau_R: float = 1e-10, max_sweeps: int = 100):
        T = {pq: np.zeros_like(self.Kc[pq]) for pq in self.pairs}
        sweeps = 0
        while True:
            R = {pq: self.residual(T, *pq) for pq in self.pairs}
            Rt = {pq: self.W[pq].T @ R[pq] @ self.W[pq] for pq in self.pairs}
            nrm = max(np.linalg.norm(Rt[pq]) for pq in self.pairs)
            if nrm < tau_R or sweeps >= max_sweeps:
                break
            for pq in self.pairs:
                W = self.W[pq]
                T[pq] = T[pq] + W @ (-Rt[pq] / self.denom[pq]) @ W.T
            sweeps += 1
        self.T = T
        self.sweeps = sweeps
        self.max_residual = nrm
        self.converged = nrm < tau_R
        return T

    def energy(self, T: Dict = None) -> float:
        """Hylleraas E = sum over ordered pairs <Tbar_pq, 2 K_(pq,pq) + L_pq[T]>, L = R - K."""
        T = self.T if T is None else T
        E = 0.0
        for p in self.X:
            for q in self.X:
                Tpq = self.T_ordered(T, p, q)
                Tbar = 2.0 * Tpq - Tpq.T
                Kpq = composite_K(self.pb, p, q)
                L = self.residual(T, p, q, with_K=False)
                E += float(np.sum(Tbar * (2.0 * Kpq + L)))
        return E

    def energy_KT(self, T: Dict = None) -> float:
        """sum over ordered pairs <K_(pq,pq), Tbar_pq> (equals eq:ec when R = 0)."""
        T = self.T if T is None else T
        E = 0.0
        for p in self.X:
            for q in self.X:
                Tpq = self.T_ordered(T, p, q)
                E += float(np.sum(composite_K(self.pb, p, q) * (2.0 * Tpq - Tpq.T)))
        return E

    # densities --------------------------------------------------------------
    def densities(self, T: Dict = None, dvir: bool = False):
        """Exact partial derivatives of the Hylleraas energy at the converged T:
        dE/dC_p (list), dE/df (nocc x nocc), dE/deps (nvir); with dvir also the
        full virtual density D^v = sum over ordered pairs P_pq G^F_pq P_pq^T
        (first term of eq:dv), the derivative with respect to every entry of a
        virtual Fock matrix taken as independent, whose diagonal is dE/deps."""
        T = self.T if T is None else T
        pb = self.pb
        S = pb.S
        nocc = pb.f.shape[0]
        nvir = pb.eps.shape[0]
        dC = {p: np.zeros_like(pb.C[p]) for p in self.X}
        dF = np.zeros((nocc, nocc))
        de = np.zeros(nvir)
        Dv = np.zeros((nvir, nvir)) if dvir else None
        for p in self.X:
            for q in self.X:
                d = dom(p, q)
                Tpq = self.T_ordered(T, p, q)
                Tbar = 2.0 * Tpq - Tpq.T
                Up = composite(S, d, (p,))
                Uq = composite(S, d, (q,))
                # dE/dK_pq = U_p^T (2 Tbar) U_q ; K_pq = C_p C_q^T
                G = Up.T @ (2.0 * Tbar) @ Uq
                dC[p] += G @ pb.C[q]
                dC[q] += G.T @ pb.C[p]
                # dE/dF_(pq,pq) and the virtual projector P_pq = [Q_p Q_q]
                Sd = composite(S, d, d)
                GF = Tpq.T @ Sd @ Tbar + Tbar @ Sd @ Tpq.T
                P = np.hstack([pb.Q[o] for o in d])
                # diagonal of P GF P^T: de_a = sum_xy P_ax GF_xy P_ay
                de += np.sum((P @ GF) * P, axis=1)
                if dvir:
                    Dv += P @ GF @ P.T
        # dE/df_uv from the f-weighted overlap terms of eq:rij
        for u in self.X:
            for v in self.X:
                acc = 0.0
                for p in self.X:
                    Tbar = 2.0 * self.T_ordered(T, p, v) - self.T_ordered(T, p, v).T
                    M = composite(S, dom(p, v), dom(p, u)) @ self.T_ordered(T, p, u) \
                        @ composite(S, dom(p, u), dom(p, v))
                    acc -= float(np.sum(Tbar * M))
                for q in self.X:
                    Tbar = 2.0 * self.T_ordered(T, u, q) - self.T_ordered(T, u, q).T
                    M = composite(S, dom(u, q), dom(v, q)) @ self.T_ordered(T, v, q) \
                        @ composite(S, dom(v, q), dom(u, q))
                    acc -= float(np.sum(Tbar * M))
                dF[u, v] += acc
        if dvir:
            return dC, dF, de, Dv
        return dC, dF, de


# ---------------------------------------------------------------------------
# Whole problem: MBE energies and densities
# ---------------------------------------------------------------------------

def solve(sysm, mode: int = None, cut2: float = None, cut3: float = None,
          tau_R: float = 1e-10, tau_S: float = 1e-8, max_sweeps: int = 100,
          densities: bool = True, clusters=None, coef=None, order=None,
          l2b: float = 1e-2, l3b: float = 0.2, dvir: bool = False, weak: bool = True,
          k_exact: bool = False):
    """Solve every selected cluster and combine by MBE.  Returns a dict with E,
    E_orders (E_1b, dE_2b, dE_3b), E_cluster, sweeps, and (optionally) dE_dC
    [sum r, naux], dE_dF [nocc, nocc], dE_deps [nvir] and, with dvir, the full
    virtual density Dvir [nvir, nvir].  With the overlap selection (and weak) the
    weak 2b clusters' one-block energies (R15) are added to E and to dE_2b, and
    their densities to the densities; E_weak holds their sum."""
    mode = sysm.sel_mode if mode is None else mode
    cut2 = sysm.cut2 if cut2 is None else cut2
    cut3 = sysm.cut3 if cut3 is None else cut3
    s2b = None
    if clusters is None:
        s2b = s2b_metric(sysm) if mode == SEL_OVERLAP else None
        clusters, coef, order = select_clusters(sysm.centroid, mode, cut2, cut3, s2b, l2b, l3b)
    pb = PairBlocks(sysm, k_exact=k_exact)
    E_cl = np.zeros(len(clusters))
    sweeps = np.zeros(len(clusters), dtype=np.int64)
    maxres = 0.0
    converged = True
    off = sysm.off
    dC = np.zeros((sysm.nosv, sysm.naux))
    dF = np.zeros((sysm.nocc, sysm.nocc))
    de = np.zeros(sysm.nvir)
    Dv = np.zeros((sysm.nvir, sysm.nvir)) if (densities and dvir) else None
    T_all = []
    for n, X in enumerate(clusters):
        cl = Cluster(pb, X, tau_S)
        cl.solve(tau_R, max_sweeps)
        E_cl[n] = cl.energy()
        sweeps[n] = cl.sweeps
        maxres = max(maxres, cl.max_residual)
        converged = converged and cl.converged
        T_all.append(cl.T)
        if densities and coef[n] != 0.0:
            dens = cl.densities(dvir=dvir)
            c_dC, c_dF, c_de = dens[:3]
            if not k_exact:   # with cross-projected integrals E does not depend on C
                for p, g in c_dC.items():
                    dC[off[p]:off[p + 1]] += coef[n] * g
            dF += coef[n] * c_dF
            de += coef[n] * c_de
            if dvir:
                Dv += coef[n] * dens[3]
    E = float(np.dot(coef, E_cl))
    E_orders = mbe_orders(clusters, order, E_cl)
    E_weak = 0.0
    if mode == SEL_OVERLAP and weak:
        s2b = s2b_metric(sysm) if s2b is None else s2b
        E_weak = float(np.sum(weak_pairs(sysm, l2b, s2b=s2b)[1]))
        E += E_weak
        E_orders = E_orders + np.array([0.0, E_weak, 0.0])
        if densities:
            wd = weak_pair_densities(sysm, l2b, s2b=s2b, dvir=dvir)
            dC += wd[0]
            dF += wd[1]
            de += wd[2]
            if dvir:
                Dv += wd[3]
    out = dict(E=E, E_orders=E_orders, E_cluster=E_cl, clusters=clusters, coef=coef,
               order=order, sweeps=sweeps, max_residual=maxres, converged=converged,
               T=T_all, pair_blocks=sum(len(X) * (len(X) + 1) // 2 for X in clusters),
               E_weak=E_weak)
    if densities:
        out.update(dE_dC=None if k_exact else dC, dE_dF=dF, dE_deps=de)
        if dvir:
            out["Dvir"] = Dv
    return out


def mbe_orders(clusters, order, E_cl):
    """E_1b = sum E^I, dE_2b = sum (E^IJ - E^I - E^J), dE_3b = sum of 3-body increments."""
    if order[0] == 0:   # one full cluster: no MBE orders
        return np.array([np.nan, np.nan, np.nan])
    idx = {X: n for n, X in enumerate(clusters)}
    e1 = sum(E_cl[n] for n, X in enumerate(clusters) if len(X) == 1)
    e2 = 0.0
    e3 = 0.0
    for n, X in enumerate(clusters):
        if len(X) == 2:
            i, j = X
            e2 += E_cl[n] - E_cl[idx[(i,)]] - E_cl[idx[(j,)]]
        elif len(X) == 3:
            i, j, k = X
            e3 += (E_cl[n] - E_cl[idx[(i, j)]] - E_cl[idx[(i, k)]] - E_cl[idx[(j, k)]]
                   + E_cl[idx[(i,)]] + E_cl[idx[(j,)]] + E_cl[idx[(k,)]])
    return np.array([e1, e2, e3])


def amplitude_mbe_energy(sysm, res) -> float:
    """Energy from collective amplitudes T_(pq) = sum_{X containing p,q} c_X T^X_pq
    (eq:tmbediag, eq:tmbeoff), evaluated as sum over ordered pairs <K_(pq,pq), Tbar>."""
    pb = PairBlocks(sysm)
    coll: Dict[Tuple[int, int], np.ndarray] = {}
    for X, c, T in zip(res["clusters"], res["coef"], res["T"]):
        for pq, t in T.items():
            coll[pq] = coll.get(pq, 0.0) + c * t
    E = 0.0
    for (p, q), t in coll.items():
        tb = 2.0 * t - t.T
        e = float(np.sum(composite_K(pb, p, q) * tb))
        E += e if p == q else 2.0 * e
    return E


# ---------------------------------------------------------------------------
# Independent checkers
# ---------------------------------------------------------------------------

def mp2_canonical(B: np.ndarray, eps_vir: np.ndarray, F_occ: np.ndarray):
    """Closed-shell DF-MP2 in the full virtual space.  The occupied Fock matrix is
    diagonalised and the fitted integrals rotated; then
    E = -sum_{ijab} (ia|jb)[2(ia|jb) - (ib|ja)] / (e_a + e_b - e_i - e_j).
    Returns (E, dE/deps_vir) with dE/deps_c = sum_ij [(T Tbar^T)_cc + (T^T Tbar)_cc]."""
    e_occ, U = np.linalg.eigh(F_occ)
    Bt = np.einsum("ji,jaP->iaP", U, B)
    n = B.shape[0]
    E = 0.0
    de = np.zeros(eps_vir.shape[0])
    for i in range(n):
        for j in range(n):
            Kij = Bt[i] @ Bt[j].T
            D = eps_vir[:, None] + eps_vir[None, :] - e_occ[i] - e_occ[j]
            T = -Kij / D
            Tbar = 2.0 * T - T.T
            E += float(np.sum(Kij * Tbar))
            de += np.einsum("ab,ab->a", T, Tbar) + np.einsum("ab,ab->b", T, Tbar)
    return E, de


def dense_solve_energy(pb: PairBlocks, X: Sequence[int], rcond: float = 1e-12) -> float:
    """Solve the cluster's linear residual equations R(T) = 0 directly: build the
    matrix of T -> R(T) - K column by column and solve it with lstsq; return the
    Hylleraas energy at that solution."""
    cl = Cluster(pb, X)
    shapes = {pq: cl.Kc[pq].shape for pq in cl.pairs}
    sizes = [int(np.prod(shapes[pq])) for pq in cl.pairs]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    N = int(offs[-1])

    def unpack(v):
        return {pq: v[offs[n]:offs[n + 1]].reshape(shapes[pq]) for n, pq in enumerate(cl.pairs)}

    A = np.zeros((N, N))
    for col in range(N):
        v = np.zeros(N)
        v[col] = 1.0
        Tu = unpack(v)
        A[:, col] = np.concatenate([cl.residual(Tu, *pq, with_K=False).ravel() for pq in cl.pairs])
    b = -np.concatenate([cl.Kc[pq].ravel() for pq in cl.pairs])
    x = np.linalg.lstsq(A, b, rcond=rcond)[0]
    return cl.energy(unpack(x))


# ---------------------------------------------------------------------------
# Weak 2b clusters: one-block dispersion scheme (R15)
# ---------------------------------------------------------------------------

WEAK_MIN = 1e-7   # pairs below this s2b are discarded (weak 2b section)


def weak_pairs(sysm, l2b: float, s2b: np.ndarray = None):
    """Weak pairs (i, j), i < j, with WEAK_MIN <= s2b_ij <= l2b, and for each its
    one-block energy 4 <T, K~> with T = -K~ / (e~_i[a] + e~_j[b] - f_ii - f_jj),
    K~ = V_i^T K_ij V_j and (e~_p, V_p) the eigenpairs of F_(p,p) (the diagonal
    domain's pseudo-canonical basis; S_(p,p) = 1).  Returns (pairs, energies)."""
    if s2b is None:
        s2b = s2b_metric(sysm)
    pb = PairBlocks(sysm)
    n = sysm.nocc
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if WEAK_MIN <= s2b[i, j] <= l2b]
    eig = {}
    for p in sorted({x for pq in pairs for x in pq}):
        eig[p] = np.linalg.eigh(pb.F(p, p))
    out = []
    for (i, j) in pairs:
        (ei, Vi), (ej, Vj) = eig[i], eig[j]
        Kt = Vi.T @ pb.K(i, j) @ Vj
        D = ei[:, None] + ej[None, :] - pb.f[i, i] - pb.f[j, j]
        T = -Kt / D
        out.append(4.0 * float(np.sum(T * Kt)))
    return pairs, np.array(out)


def weak_pair_nup(sysm, l2b: float, s2b: np.ndarray = None):
    """The upper block of the weak pairs' OSV-response intermediate in the one-block
    approximation of eq:nij2b, N^up_ij = T_(i,j) K_(j,i) (r_i x r_i, OSV basis of
    LMO i; the lower block is taken as zero).  Since K_ij = Q_i^T B_i B_j^T Q_j and
    the one-block energy is stationary in T with dE/dK_ij = 8 T, an OSV rotation
    Q_i -> Q_i (1 + h A) at fixed F_(i,i) moves the energy by 8 h <A, (N^up)^T>.
    Returns {(i, j): N^up} in pair order."""
    if s2b is None:
        s2b = s2b_metric(sysm)
    pb = PairBlocks(sysm)
    n = sysm.nocc
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if WEAK_MIN <= s2b[i, j] <= l2b]
    eig = {p: np.linalg.eigh(pb.F(p, p)) for p in sorted({x for pq in pairs for x in pq})}
    out = {}
    for (i, j) in pairs:
        (ei, Vi), (ej, Vj) = eig[i], eig[j]
        Kt = Vi.T @ pb.K(i, j) @ Vj
        T = Vi @ (-Kt / (ei[:, None] + ej[None, :] - pb.f[i, i] - pb.f[j, j])) @ Vj.T
        out[(i, j)] = T @ pb.K(j, i)
    return out


def weak_pair_densities(sysm, l2b: float, s2b: np.ndarray = None, dvir: bool = False):
    """Exact derivatives of the summed weak-pair energies (R15) at fixed Q.  The
    one-block energy is the stationary value of
        E_H(T) = 8 <T, K_ij> + 4 <T, F_(i,i) T + T F_(j,j) - (f_ii + f_jj) T>
    (OSV basis, S_(i,i) = 1), whose stationarity is the one-block residual, so
    at the solution T (OSV basis, V_i T~ V_j^T):
        dE/dK_ij = 8 T  ->  dE/dC_i += 8 T C_j,  dE/dC_j += 8 T^T C_i;
        dE/dF_(i,i) = 4 T T^T, dE/dF_(j,j) = 4 T^T T  ->  dE/deps through Q;
        dE/df_ii = dE/df_jj = -4 <T, T>.
    Returns (dE/dC [sum r x naux], dE/dF_occ [nocc x nocc], dE/deps [nvir]) and,
    with dvir, the full virtual density Q_i 4TT^T Q_i^T + Q_j 4T^T T Q_j^T summed
    over the pairs (the derivative with respect to a full virtual Fock matrix)."""
    if s2b is None:
        s2b = s2b_metric(sysm)
    pb = PairBlocks(sysm)
    n = sysm.nocc
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if WEAK_MIN <= s2b[i, j] <= l2b]
    off = np.concatenate([[0], np.cumsum(sysm.r)]).astype(int)
    dC = np.zeros((off[-1], pb.C[0].shape[1]))
    dF = np.zeros((n, n))
    de = np.zeros(pb.eps.shape[0])
    Dv = np.zeros((pb.eps.shape[0], pb.eps.shape[0])) if dvir else None
    eig = {p: np.linalg.eigh(pb.F(p, p)) for p in sorted({x for pq in pairs for x in pq})}
    for (i, j) in pairs:
        (ei, Vi), (ej, Vj) = eig[i], eig[j]
        Kt = Vi.T @ pb.K(i, j) @ Vj
        Tt = -Kt / (ei[:, None] + ej[None, :] - pb.f[i, i] - pb.f[j, j])
        T = Vi @ Tt @ Vj.T
        dC[off[i]:off[i + 1]] += 8.0 * T @ pb.C[j]
        dC[off[j]:off[j + 1]] += 8.0 * T.T @ pb.C[i]
        Qi, Qj = pb.Q[i], pb.Q[j]
        de += 4.0 * np.einsum("am,mn,an->a", Qi, T @ T.T, Qi)
        de += 4.0 * np.einsum("am,mn,an->a", Qj, T.T @ T, Qj)
        if dvir:
            Dv += 4.0 * (Qi @ (T @ T.T) @ Qi.T + Qj @ (T.T @ T) @ Qj.T)
        tt = float(np.sum(T * T))
        dF[i, i] -= 4.0 * tt
        dF[j, j] -= 4.0 * tt
    if dvir:
        return dC, dF, de, Dv
    return dC, dF, de


# ---------------------------------------------------------------------------
# OSV generation from the fitted integrals (eq:svd, eq:osv)
# ---------------------------------------------------------------------------

def diagonal_pair_amplitudes(B: np.ndarray, eps_vir: np.ndarray, F_occ: np.ndarray, k: int) -> np.ndarray:
    """[T_kk]_ab = (ka|kb) / (f_aa + f_bb - 2 f_kk) with (ka|kb) = sum_P B_k[a,P] B_k[b,P]
    (the text's sign: positive, so T_kk is positive semidefinite as the elementwise
    product of two positive semidefinite matrices)."""
    K = B[k] @ B[k].T
    D = eps_vir[:, None] + eps_vir[None, :] - 2.0 * F_occ[k, k]
    return K / D


def generate_osvs(B: np.ndarray, eps_vir: np.ndarray, F_occ: np.ndarray, l_osv: float = 1e-4,
                  r_max: int = None):
    """OSVs of every LMO k (eq:svd): the orthonormal eigenvectors of T_kk whose
    eigenvalues omega exceed l_osv, largest first, at most r_max of them; each
    eigenvector's entry of largest magnitude (first one on ties) is made positive.
    Returns (r [nocc], Q [nvir, sum r] column blocks per LMO, C [sum r, naux] with
    C_k = Q_k^T B_k (eq:osv applied to the fitted integrals), omega list)."""
    nocc, nvir, naux = B.shape
    r_max = nvir if r_max is None else r_max
    rs, Qs, Cs, oms = [], [], [], []
    for k in range(nocc):
        w, V = np.linalg.eigh(diagonal_pair_amplitudes(B, eps_vir, F_occ, k))
        order = np.argsort(-w, kind="stable")
        keep = [i for i in order if w[i] > l_osv][:r_max]
        Qk = V[:, keep].copy()
        for c in range(Qk.shape[1]):
            m = int(np.argmax(np.abs(Qk[:, c])))
            if Qk[m, c] < 0.0:
                Qk[:, c] = -Qk[:, c]
        rs.append(len(keep))
        Qs.append(Qk)
        Cs.append(Qk.T @ B[k])
        oms.append(w[keep])
    return (np.array(rs, dtype=np.int32), np.asfortranarray(np.hstack(Qs)),
            np.ascontiguousarray(np.vstack(Cs)), oms)


# ---------------------------------------------------------------------------
# One-step high-order correction (section on the high-order MBE(n) contribution)
# ---------------------------------------------------------------------------

def collective_amplitudes(res) -> Dict[Tuple[int, int], np.ndarray]:
    """T_(pq) = sum over clusters X holding p and q of c_X T^X_pq: the MBE(3)
    expansions eq:tmbediag / eq:tmbeoff written with the inclusion-exclusion
    coefficients (composite OSV basis of domain [pq])."""
    coll: Dict[Tuple[int, int], np.ndarray] = {}
    for c, T in zip(res["coef"], res["T"]):
        for pq, t in T.items():
            coll[pq] = coll.get(pq, 0.0) + c * t
    return coll


def k_range(res, p: int, q: int):
    """The LMOs m that pair (p, q) correlates with in the selected clusters: every
    LMO of a cluster holding both p and q (sorted)."""
    out = set()
    for X in res["clusters"]:
        if p in X and q in X:
            out.update(X)
    return sorted(out)


def residual_over(pb: PairBlocks, T: Dict, p: int, q: int, ms) -> np.ndarray:
    """eq:rij for the ordered pair (p, q), p <= q, with the sums over k running over
    the LMOs ms, amplitudes T[(a, b)] (a <= b) in the composite bases; the swapped
    pair's amplitudes are T^{ba} = (T^{ab})^T in the swapped basis."""
    S, F, f = pb.S, pb.F, pb.f

    def Tord(a, b):
        if a <= b:
            return T[(a, b)]
        ra, rb = pb.Q[a].shape[1], pb.Q[b].shape[1]
        perm = np.concatenate([np.arange(rb, rb + ra), np.arange(0, rb)])
        return T[(b, a)].T[np.ix_(perm, perm)]

    dpq = dom(p, q)
    R = composite_K(pb, p, q)
    for m in ms:
        dpm, dmq = dom(p, m), dom(m, q)
        right = -f[m, q] * composite(S, dpm, dpq)
        if m == q:
            right = right + composite(F, dpm, dpq)
        R = R + composite(S, dpq, dpm) @ Tord(p, m) @ right
        left = -f[p, m] * composite(S, dpq, dmq)
        if p == m:
            left = left + composite(F, dpq, dmq)
        R = R + left @ Tord(m, q) @ composite(S, dmq, dpq)
    return R


def one_step_correction(sysm, res, tau_S: float = 1e-8):
    """The posterior correction of the converged MBE(3) amplitudes: the residual
    eq:rij of every selected pair (p, q) at the collective amplitudes, with k over
    the LMOs that share a cluster with p and q, then one preconditioned Jacobi step
    in the pair domain's pseudo-canonical basis W (W^T S W = 1, W^T F W = diag e~):
        dT = W [-(W^T dR W) / (e~_a + e~_b - f_pp - f_qq)] W^T,
    and the change of the energy sum_pairs w <K_(pq,pq), 2T - T^T> (w = 1 for
    p = q, 2 otherwise) that the step makes.  Returns dict(dE, E_coll, max_dR,
    dR, dT) with max_dR the largest ||W^T dR W||_F."""
    pb = PairBlocks(sysm)
    coll = collective_amplitudes(res)
    dE = 0.0
    E_coll = 0.0
    max_dR = 0.0
    dR_all, dT_all, per_pair = {}, {}, {}
    for (p, q) in sorted(coll):
        d = dom(p, q)
        S = composite(pb.S, d, d)
        F = composite(pb.F, d, d)
        s, U = np.linalg.eigh(S)
        keep = s > tau_S
        Xo = U[:, keep] / np.sqrt(s[keep])[None, :]
        e, V = np.linalg.eigh(Xo.T @ F @ Xo)
        W = Xo @ V
        denom = e[:, None] + e[None, :] - pb.f[p, p] - pb.f[q, q]
        dR = residual_over(pb, coll, p, q, k_range(res, p, q))
        Rt = W.T @ dR @ W
        max_dR = max(max_dR, float(np.linalg.norm(Rt)))
        dT = W @ (-Rt / denom) @ W.T
        K = composite_K(pb, p, q)
        w = 1.0 if p == q else 2.0
        e_pq = w * float(np.sum(K * (2.0 * dT - dT.T)))
        c_pq = w * float(np.sum(K * (2.0 * coll[(p, q)] - coll[(p, q)].T)))
        dE += e_pq
        E_coll += c_pq
        dR_all[(p, q)] = dR
        dT_all[(p, q)] = dT
        per_pair[(p, q)] = (e_pq, c_pq, float(np.linalg.norm(Rt)))
    return dict(dE=dE, E_coll=E_coll, max_dR=max_dR, dR=dR_all, dT=dT_all, pairs=per_pair)


# ---------------------------------------------------------------------------
# OSV response intermediate N_ij (eq:nij) and its MBE (eq:nmbeii, eq:nmbeij)
# ---------------------------------------------------------------------------

def osv_response(sysm, res, k_exact: bool = False):
    """N_ij of eq:nij for every ordered pair (i, j) of every cluster X, at the
    cluster's converged amplitudes and with k over X, in the composite OSV basis of
    (i, j):
        N_ij = Tbar K_(ij,ij) + D_(ij,ij) F_(ij,ij) + D'_(ij,ij) S_(ij,ij)
               - sum_k [f_jk D_(ij,ik) S_(ik,ij) + f_ik D_(ij,kj) S_(kj,ij)],
        D_(ij,kl)  = 1/2 [Tbar_ij S_(ij,kl) T_kl + Tbar_ij^T S_(ij,kl) T_kl^T],
        D'_(ij,kl) = the same with F_(ij,kl),
    combined over clusters with the MBE coefficients (eq:nmbeii / eq:nmbeij written
    with the inclusion-exclusion coefficients).  Returns {(i, j): N_ij}, ordered
    pairs, both orientations."""
    pb = PairBlocks(sysm, k_exact=k_exact)
    S, F, f = pb.S, pb.F, pb.f
    out: Dict[Tuple[int, int], np.ndarray] = {}
    for X, c, T in zip(res["clusters"], res["coef"], res["T"]):
        if c == 0.0:
            continue
        cl = Cluster.__new__(Cluster)
        cl.pb, cl.X, cl.f = pb, tuple(X), f

        def Tord(a, b):
            return cl.T_ordered(T, a, b)

        def Dm(i, j, k, l, M):
            Tb = 2.0 * Tord(i, j) - Tord(i, j).T
            A = composite(M, dom(i, j), dom(k, l))
            return 0.5 * (Tb @ A @ Tord(k, l) + Tb.T @ A @ Tord(k, l).T)

        for i in X:
            for j in X:
                dij = dom(i, j)
                Tb = 2.0 * Tord(i, j) - Tord(i, j).T
                N = (Tb @ composite_K(pb, i, j) + Dm(i, j, i, j, S) @ composite(F, dij, dij)
                     + Dm(i, j, i, j, F) @ composite(S, dij, dij))
                for k in X:
                    N = N - (f[j, k] * Dm(i, j, i, k, S) @ composite(S, dom(i, k), dij)
                             + f[i, k] * Dm(i, j, k, j, S) @ composite(S, dom(k, j), dij))
                out[(i, j)] = out.get((i, j), 0.0) + c * N
    return out
