// Host side of libosvmbe: argument checks, cluster selection and MBE
// coefficients, the pair/domain/coupling/term structure that drives the
// kernels, device memory, stage orchestration and the C ABI of osv.h.
#include "osv.h"
#include "osv_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <dlfcn.h>

using namespace osv;

namespace {

thread_local std::string g_last_error = "";

struct Selection {
  std::vector<int> lmo_ptr, lmo;  // LMOs of each cluster (ascending)
  std::vector<double> coef;       // c_X
  std::vector<int> order;         // 1, 2, 3 (0 for the single full cluster)
  std::vector<int> n2, n3i;       // per LMO: selected pairs / triples holding it
  std::vector<int> n3ij;          // per selected pair (in 2b order): triples holding it
  int64_t n1 = 0, n2b = 0, n3b = 0;
};

// MBE(3) selection (downward closed) and inclusion-exclusion coefficients:
// c = 1 (3b), 1 - n3(IJ) (2b), 1 - n2(I) + n3(I) (1b).  keep2/keep3 decide;
// near3(i, j) must hold for every pair of a kept triple (a pre-filter: the
// triples are searched over the selected pairs that pass it).
template <class K2, class K3, class N3>
void select_mbe(int nocc, K2 keep2, K3 keep3, N3 near3, Selection &s) {
  std::vector<std::pair<int, int>> pairs;
  std::vector<std::vector<int>> nbr(nocc);
  // near[i * nocc + j], i < j: the pair is selected and passes near3
  std::vector<char> near((size_t)nocc * nocc, 0);
  for (int i = 0; i < nocc; i++)
    for (int j = i + 1; j < nocc; j++)
      if (keep2(i, j)) {
        pairs.push_back({i, j});
        if (near3(i, j)) {
          nbr[i].push_back(j);
          near[(size_t)i * nocc + j] = 1;
        }
      }
  std::vector<std::array<int, 3>> triples;
  for (int i = 0; i < nocc; i++)
    for (int j : nbr[i])
      for (int k : nbr[j])
        if (near[(size_t)i * nocc + k] && keep3(i, j, k)) triples.push_back({i, j, k});
  // nbr lists are ascending, so triples come out lexicographic
  s.n2.assign(nocc, 0);
  s.n3i.assign(nocc, 0);
  // pair index of (i, j), i < j: a dense table beside near (which is nocc^2
  // bytes) while it stays small, else a hash map
  const bool dense = (long long)nocc * nocc <= (1LL << 26);
  std::vector<int> pdense(dense ? (size_t)nocc * nocc : 0, -1);
  std::unordered_map<long long, int> pidx;
  for (size_t t = 0; t < pairs.size(); t++) {
    s.n2[pairs[t].first]++;
    s.n2[pairs[t].second]++;
    const long long key = (long long)pairs[t].first * nocc + pairs[t].second;
    if (dense) pdense[(size_t)key] = (int)t;
    else pidx[key] = (int)t;
  }
  auto pair_index = [&](int i, int j) {
    const long long key = (long long)i * nocc + j;
    return dense ? pdense[(size_t)key] : pidx[key];
  };
  s.n3ij.assign(pairs.size(), 0);
  for (auto &t : triples) {
    for (int a = 0; a < 3; a++) s.n3i[t[a]]++;
    s.n3ij[pair_index(t[0], t[1])]++;
    s.n3ij[pair_index(t[0], t[2])]++;
    s.n3ij[pair_index(t[1], t[2])]++;
  }
  s.lmo_ptr.assign(1, 0);
  s.lmo.clear();
  s.coef.clear();
  s.order.clear();
  const size_t ncl = (size_t)nocc + pairs.size() + triples.size();
  s.lmo_ptr.reserve(ncl + 1);
  s.lmo.reserve((size_t)nocc + 2 * pairs.size() + 3 * triples.size());
  s.coef.reserve(ncl);
  s.order.reserve(ncl);
  for (int i = 0; i < nocc; i++) {
    s.lmo.push_back(i);
    s.lmo_ptr.push_back((int)s.lmo.size());
    s.coef.push_back(1.0 - s.n2[i] + s.n3i[i]);
    s.order.push_back(1);
  }
  for (size_t t = 0; t < pairs.size(); t++) {
    s.lmo.push_back(pairs[t].first);
    s.lmo.push_back(pairs[t].second);
    s.lmo_ptr.push_back((int)s.lmo.size());
    s.coef.push_back(1.0 - s.n3ij[t]);
    s.order.push_back(2);
  }
  for (auto &t : triples) {
    for (int a = 0; a < 3; a++) s.lmo.push_back(t[a]);
    s.lmo_ptr.push_back((int)s.lmo.size());
    s.coef.push_back(1.0);
    s.order.push_back(3);
  }
  s.n1 = nocc;
  s.n2b = (int64_t)pairs.size();
  s.n3b = (int64_t)triples.size();
}

void select_full(int nocc, Selection &s) {
  s.lmo_ptr = {0, nocc};
  s.lmo.resize(nocc);
  std::iota(s.lmo.begin(), s.lmo.end(), 0);
  s.coef = {1.0};
  s.order = {0};
  s.n1 = s.n2b = s.n3b = 0;
}

double dist(const double *c, int i, int j) {
  double dx = c[3 * i] - c[3 * j], dy = c[3 * i + 1] - c[3 * j + 1], dz = c[3 * i + 2] - c[3 * j + 2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

void select_distance(int nocc, const double *cen, double cut2, double cut3, Selection &s) {
  select_mbe(
      nocc, [&](int i, int j) { return dist(cen, i, j) <= cut2; },
      [&](int i, int j, int k) {
        return dist(cen, i, j) <= cut3 && dist(cen, i, k) <= cut3 && dist(cen, j, k) <= cut3;
      },
      [&](int i, int j) { return dist(cen, i, j) <= cut3; }, s);
}

// Structure derived from a selection: domains, couplings, cluster pairs, terms.
struct Plan {
  std::vector<Domain> doms;
  std::vector<int> dom_of;  // nocc*nocc -> domain id (p <= q) or -1
  std::vector<Coupling> cpls;
  std::vector<CPair> cps;
  std::vector<Term> terms;
  std::vector<Cluster> cls;
  std::vector<int> queue;
  long long n_slot = 0;   // sum n^2 over domains
  long long n_vec = 0;    // sum (np^2 + np) over domains: K~^T and e~ slots
  long long n_T = 0;      // amplitude doubles
  long long n_M = 0;      // coupling doubles
  long long rs_stride = 0;
  long long n_pl = 0;     // dE/dF inner-product doubles
  int64_t n_pair_blocks = 0;
  int n_big = 0;          // leading queue entries too large for the LDS tables
  int n_first = 0;        // end of the queue's first LDS launch (clusters of <= 2 LMOs)
};

// Builds the pair domains of the plan (all the S/F/K blocks and the domain
// preparation need).  r/off may be null (counts only, domain sizes unknown).
int build_domains(int nocc, const Selection &s, const int *r, const int *off, Plan &P,
                  std::string &err) {
  P.dom_of.assign((size_t)nocc * nocc, -1);
  const int ncl = (int)s.coef.size();
  auto rr = [&](int i) { return r ? r[i] : 1; };
  // domains in (p, q) lexicographic order
  std::vector<char> need((size_t)nocc * nocc, 0);
  for (int X = 0; X < ncl; X++)
    for (int a = s.lmo_ptr[X]; a < s.lmo_ptr[X + 1]; a++)
      for (int b = a; b < s.lmo_ptr[X + 1]; b++) need[(size_t)s.lmo[a] * nocc + s.lmo[b]] = 1;
  for (int p = 0; p < nocc; p++)
    for (int q = p; q < nocc; q++)
      if (need[(size_t)p * nocc + q]) {
        Domain D{};
        D.p = p;
        D.q = q;
        D.rp = rr(p);
        D.rq = (p == q) ? 0 : rr(q);
        D.n = D.rp + D.rq;
        D.np = (D.n + 15) / 16 * 16;
        D.offp = off ? off[p] : 0;
        D.offq = off ? off[q] : 0;
        if (r && D.n > DMAX) {
          err = "pair domain (" + std::to_string(p) + "," + std::to_string(q) + ") has dimension " +
                std::to_string(D.n) + " > OSV_MAX_DOMAIN";
          return OSV_E_ARG;
        }
        D.moff = P.n_slot;
        D.voff = P.n_vec;
        P.n_slot += (long long)D.n * D.n;
        P.n_vec += (long long)D.np * D.np + D.np;
        P.dom_of[(size_t)p * nocc + q] = (int)P.doms.size();
        P.doms.push_back(D);
      }
  return OSV_OK;
}

// Runs f(i) for i in [0, n) on up to 16 host threads (at most one per `grain`
// items), in contiguous ranges.
template <class F>
void parallel_for(long long n, F f, long long grain = 2048) {
  const unsigned hc = std::thread::hardware_concurrency();
  const int nt = (int)std::max<long long>(1, std::min<long long>({16, hc ? (long long)hc : 1, (n + grain - 1) / grain}));
  if (nt == 1) {
    for (long long i = 0; i < n; i++) f(i);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int k = 0; k < nt; k++)
    th.emplace_back([&, k]() {
      const long long lo = n * k / nt, hi = n * (k + 1) / nt;
      for (long long i = lo; i < hi; i++) f(i);
    });
  for (auto &t : th) t.join();
}

// Builds the clusters' pairs, terms and couplings and the work queue (after
// build_domains; runs on the host while the device forms S, F, K and the domains).
// The pairs and terms are laid out from per-cluster counts and filled on several
// threads; the couplings are numbered in order of first use over the terms, in one
// pass over their keys, so the tables do not depend on the thread count.
void build_clusters(int nocc, const Selection &s, Plan &P) {
  const int ncl = (int)s.coef.size();
  auto dom_id = [&](int a, int b) {
    return a <= b ? P.dom_of[(size_t)a * nocc + b] : P.dom_of[(size_t)b * nocc + a];
  };
  const long long ND = (long long)P.doms.size();
  // 1. per-cluster counts, then offsets: pairs, terms, amplitude doubles, dE/dF doubles
  std::vector<long long> cpo(ncl + 1, 0), tmo(ncl + 1, 0), tof(ncl + 1, 0), plo(ncl + 1, 0);
  parallel_for(ncl, [&](long long X) {
    const int l0 = s.lmo_ptr[X], nl = s.lmo_ptr[X + 1] - l0;
    cpo[X + 1] = (long long)nl * (nl + 1) / 2;
    tmo[X + 1] = cpo[X + 1] * 2 * (nl - 1);
    plo[X + 1] = (long long)nl * nl;
    long long nT = 0;
    for (int a = 0; a < nl; a++)
      for (int b = a; b < nl; b++) {
        const long long np = P.doms[dom_id(s.lmo[l0 + a], s.lmo[l0 + b])].np;
        nT += 2 * np * np;
      }
    tof[X + 1] = nT;
  });
  for (int X = 0; X < ncl; X++) {
    cpo[X + 1] += cpo[X];
    tmo[X + 1] += tmo[X];
    tof[X + 1] += tof[X];
    plo[X + 1] += plo[X];
  }
  P.cps.assign(cpo[ncl], CPair{});
  P.terms.assign(tmo[ncl], Term{});
  P.cls.assign(ncl, Cluster{});
  std::vector<long long> keys(tmo[ncl]);   // coupling key A * ND + B of each term
  std::vector<long long> rs_max(ncl, 0);
  // 2. clusters, pairs and terms of eq:rij
  parallel_for(ncl, [&](long long X) {
    Cluster &C = P.cls[X];
    const int l0 = s.lmo_ptr[X], nl = s.lmo_ptr[X + 1] - l0;
    C.cp0 = (int)cpo[X];
    C.ncp = (int)(cpo[X + 1] - cpo[X]);
    C.nlmo = nl;
    C.lmo0 = l0;
    C.toff0 = P.n_T + tof[X];
    C.poff = P.n_pl + plo[X];
    C.term0 = (int)tmo[X];
    C.term1 = (int)tmo[X + 1];
    // local pair index table (nl <= nocc; the pairs (a, b), a <= b, in row order)
    auto lpair = [&](int a, int b) {
      if (a > b) std::swap(a, b);
      return C.cp0 + a * nl - a * (a - 1) / 2 + (b - a);
    };
    long long toff = C.toff0;
    for (int a = 0; a < nl; a++)
      for (int b = a; b < nl; b++) {
        CPair &cp = P.cps[lpair(a, b)];
        cp.dom = dom_id(s.lmo[l0 + a], s.lmo[l0 + b]);
        cp.la = a;
        cp.lb = b;
        cp.w = (a == b) ? 1 : 2;
        cp.toff = toff;
        cp.init = -1;
        const long long np = P.doms[cp.dom].np;
        toff += 2 * np * np;
      }
    int ti = C.term0;
    long long rs = 0;
    for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
      CPair &cp = P.cps[c];
      cp.term0 = ti;
      const int a = cp.la, b = cp.lb;
      const int p = s.lmo[l0 + a], q = s.lmo[l0 + b];
      auto add = [&](int src, int flags, int fa, int fb, int la, int lb) {
        Term &t = P.terms[ti];
        t.src = src;
        const int tgt = cp.dom, sd = P.cps[src].dom;
        const int A = std::min(tgt, sd), B = std::max(tgt, sd);
        keys[ti] = (long long)A * ND + B;
        t.flags = flags | (tgt != A ? 1 : 0);
        t.fa = fa;
        t.fb = fb;
        t.la = la;
        t.lb = lb;
        ti++;
      };
      // first sum: m != q, source ordered (p, m), coefficient f_mq
      for (int mm = 0; mm < nl; mm++) {
        if (mm == b) continue;
        const int m = s.lmo[l0 + mm];
        add(lpair(a, mm), (p > m) ? 2 : 0, m, q, mm, b);
      }
      // second sum: m != p, source ordered (m, q), coefficient f_pm
      for (int mm = 0; mm < nl; mm++) {
        if (mm == a) continue;
        const int m = s.lmo[l0 + mm];
        add(lpair(mm, b), (m > q) ? 2 : 0, p, m, a, mm);
      }
      cp.nterm = ti - cp.term0;
      // the solve's P pass keeps one np x np product per term of the pair in scratch
      const long long npt = P.doms[cp.dom].np;
      rs = std::max(rs, (long long)cp.nterm * npt * npt);
    }
    rs_max[X] = rs;
  });
  P.n_T += tof[ncl];
  P.n_pl += plo[ncl];
  P.n_pair_blocks += cpo[ncl];
  for (int X = 0; X < ncl; X++) P.rs_stride = std::max(P.rs_stride, rs_max[X]);
  // 3. couplings keyed by (A, B), A < B, numbered in order of first use: open
  // addressing with linear probing, key and id in one slot, each probe prefetched
  // a few terms ahead
  struct Slot {
    long long key;
    long long id;
  };
  size_t cap = 1024;
  while ((long long)cap < 16 * ND) cap <<= 1;   // grown below at half load
  std::vector<Slot> tab(cap, Slot{-1, -1});
  auto hsh = [&](long long key) {
    return (size_t)((unsigned long long)key * 0x9E3779B97F4A7C15ull >> 17) & (cap - 1);
  };
  const long long nterm = (long long)keys.size();
  constexpr int PF = 16;
  for (long long t = 0; t < nterm; t++) {
    if (t + PF < nterm) __builtin_prefetch(&tab[hsh(keys[t + PF])]);
    const long long key = keys[t];
    size_t h = hsh(key);
    while (tab[h].key != -1 && tab[h].key != key) h = (h + 1) & (cap - 1);
    if (tab[h].key == -1) {
      if (2 * (P.cpls.size() + 1) > cap) {   // rehash at half load
        std::vector<Slot> old;
        old.swap(tab);
        cap <<= 1;
        tab.assign(cap, Slot{-1, -1});
        for (const Slot &e : old)
          if (e.key != -1) {
            size_t g = hsh(e.key);
            while (tab[g].key != -1) g = (g + 1) & (cap - 1);
            tab[g] = e;
          }
        h = hsh(key);
        while (tab[h].key != -1) h = (h + 1) & (cap - 1);
      }
      Coupling c{};
      c.A = (int)(key / ND);
      c.B = (int)(key - (long long)c.A * ND);
      const long long sz = (long long)P.doms[c.A].np * P.doms[c.B].np;
      c.offAB = P.n_M;
      c.offBA = P.n_M + sz;
      P.n_M += 2 * sz;
      tab[h].key = key;
      tab[h].id = (long long)P.cpls.size();
      P.cpls.push_back(c);
    }
    P.terms[t].cpl = (int)tab[h].id;
  }
  // Work-queue order: the canonical cluster order, in which neighbouring clusters
  // share LMOs, so workgroups running at the same time touch the same couplings
  // (allocated above in order of first use) and nearby amplitude slots.  Cluster
  // costs vary by less than 2^3 in MBE(3) runs, so there is no long tail to
  // schedule first.
  P.queue.resize(ncl);
  std::iota(P.queue.begin(), P.queue.end(), 0);
  // clusters too large for the solve's LDS descriptor tables go first
  auto big = [&](int x) {
    return P.cls[x].ncp > SOLVE_MAXT || P.cls[x].term1 - P.cls[x].term0 > SOLVE_MAXTERM;
  };
  auto mid = std::stable_partition(P.queue.begin(), P.queue.end(), big);
  P.n_big = (int)(mid - P.queue.begin());
  // Warm start of the 3-LMO clusters: they run after the 1- and 2-LMO clusters
  // (a second launch), and each of their pairs starts from the final amplitudes of
  // the same pair in a 2-LMO cluster of the same LMOs (p < q: the cluster {p, q};
  // p = q: the cluster of p with the next LMO of the triple), which live in the
  // same pair-domain basis.  The fixed point, and so the converged result, does
  // not depend on the start.
  {
    std::unordered_map<long long, int> two;   // (p, q), p < q -> 2-LMO cluster
    for (int X = 0; X < ncl; X++)
      if (P.cls[X].nlmo == 2) {
        const int p = s.lmo[P.cls[X].lmo0], q = s.lmo[P.cls[X].lmo0 + 1];
        two[(long long)std::min(p, q) * nocc + std::max(p, q)] = X;
      }
    // slot of pair (p, q) in the 2-LMO cluster {u, v} (-1 if that cluster is absent)
    auto slot = [&](int u, int v, int p, int q) -> long long {
      auto it = two.find((long long)std::min(u, v) * nocc + std::max(u, v));
      if (it == two.end()) return -1;
      const Cluster &C = P.cls[it->second];
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
        const int a = s.lmo[C.lmo0 + P.cps[c].la], b = s.lmo[C.lmo0 + P.cps[c].lb];
        if ((a == p && b == q) || (a == q && b == p)) return P.cps[c].toff;
      }
      return -1;
    };
    parallel_for(ncl, [&](long long X) {
      const Cluster &C = P.cls[X];
      if (C.nlmo != 3 || C.ncp > SOLVE_MAXT || C.term1 - C.term0 > SOLVE_MAXTERM) return;
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
        CPair &cp = P.cps[c];
        const int p = s.lmo[C.lmo0 + cp.la], q = s.lmo[C.lmo0 + cp.lb];
        if (p != q) {
          cp.init = slot(p, q, p, q);
        } else {
          const int o1 = s.lmo[C.lmo0 + (cp.la + 1) % 3], o2 = s.lmo[C.lmo0 + (cp.la + 2) % 3];
          cp.init = slot(p, o1, p, p);
          if (cp.init < 0) cp.init = slot(p, o2, p, p);
        }
      }
    });
    auto first = [&](int x) { return P.cls[x].nlmo <= 2; };
    auto mid2 = std::stable_partition(P.queue.begin() + P.n_big, P.queue.end(), first);
    P.n_first = (int)(mid2 - P.queue.begin());
  }
}

int build_plan(int nocc, const Selection &s, const int *r, const int *off, Plan &P,
               std::string &err) {
  const int rc = build_domains(nocc, s, r, off, P, err);
  if (rc) return rc;
  build_clusters(nocc, s, P);
  return OSV_OK;
}

}  // namespace

// host-side index lists of the densities (built once per context)
struct DensHost {
  bool ready = false;
  std::vector<long long> ptr, toff, bptr, pptr, pidx;
  std::vector<double> cf;
  std::vector<int2> blocks;
  std::vector<int> bdom, bpart;
  std::vector<int> adj_order;   // domains by adjoint cost (entries x np^3), largest first
};

struct osv_ctx {
  int nocc = 0, nvir = 0, naux = 0, nosv = 0, precision = 0, c_dtype = 0, mode = 0;
  std::vector<int> r, off;
  const double *Q = nullptr, *eps = nullptr, *F = nullptr;
  const void *C = nullptr;
  double tau_S = 1e-8;
  Selection sel;
  Plan plan;
  osv_counts counts{};
  std::vector<int2> tiles;
  // device memory
  std::vector<void *> allocs;
  double *dS = nullptr, *dF = nullptr, *dK = nullptr, *dW = nullptr, *dY = nullptr, *dKt = nullptr;
  double *dEpst = nullptr, *dMinev = nullptr, *dM = nullptr, *dT = nullptr, *dRs = nullptr;
  double *dT2 = nullptr;  // second amplitude buffer of the solve (Jacobi ping-pong)
  double *dC64 = nullptr; // FP64 copy of an FP32 C (made when an FP64 product needs it)
  std::vector<int2> tiles128;
  int2 *dTiles128 = nullptr;
  double *dEcl = nullptr, *dPl = nullptr, *dMaxres = nullptr, *dWts = nullptr, *dEout = nullptr;
  int *dRank = nullptr, *dSweeps = nullptr, *dCounter = nullptr, *dQueue = nullptr, *dFlag = nullptr;
  int *dOff = nullptr, *dR = nullptr, *dPrepIds = nullptr, *dCplIds = nullptr;
  std::vector<int> cpl_ids;   // couplings by size class (host copy of dCplIds)
  std::vector<int2> weak;     // weak 2b clusters (i < j), overlap selection only
  std::vector<int2> weak_dd;  // their diagonal domains ((i, i), (j, j))
  int2 *dWeak = nullptr;      // their diagonal domains
  double *dWeakE = nullptr;   // their one-block energies
  // the weak pairs inside the MBE energy and densities (overlap selection): per
  // pair its amplitudes in the OSV bases (slot at weak_toff), energy and <T, T>;
  // per LMO the weak pairs holding it (CSR, pair order)
  std::vector<long long> weak_toff, weak_lptr;
  std::vector<int> weak_lidx;
  long long weak_nT = 0;
  int2 *dWeakDom = nullptr, *dWeakLmo = nullptr;
  long long *dWeakToff = nullptr, *dWeakLptr = nullptr;
  int *dWeakLidx = nullptr;
  double *dWeakT = nullptr, *dWeakEa = nullptr, *dWeakTT = nullptr, *dWeakSum = nullptr;
  long long *dDiagMoff = nullptr;  // per LMO p: W slot of domain (p, p), or -1
  Domain *dDom = nullptr;
  Coupling *dCpl = nullptr;
  CPair *dCp = nullptr;
  Term *dTerms = nullptr;
  TermFlat *dTflat = nullptr;
  Cluster *dCl = nullptr;
  int2 *dTiles = nullptr;
  void *dDig = nullptr;
  int *dExps = nullptr;
  // mixed dE/dC: C^T (FP32), its digit planes and exponents, those of G^K
  float *dCt = nullptr;
  unsigned char *dDigCt = nullptr, *dDigG = nullptr;
  int *dExpCt = nullptr, *dExpG = nullptr;
  // mixed S and F: digit planes of the rows of Q^T and of Q^T diag(eps)
  unsigned char *dDigQr = nullptr, *dDigQe = nullptr;
  int *dExpQr = nullptr, *dExpQe = nullptr;
  double *dQe = nullptr;
  // mixed G^F Q^T: Q (nvir x sum r, FP64) and its digit planes and exponents
  double *dQn = nullptr;
  unsigned char *dDigQ = nullptr;
  int *dExpQ = nullptr;
  int2 *dDigTiles = nullptr;
  int ndig_tiles = 0;
  int nwg = 1;
  // densities (allocated on first use)
  bool dens_ready = false;
  DensHost dh;
  double *dGK = nullptr, *dGF = nullptr, *dGd = nullptr, *dZt = nullptr, *dDcoef = nullptr;
  double *dColPart = nullptr;  // partial column sums of dE/deps
  double *dClcoef = nullptr;
  int *dAdjOrder = nullptr;
  long long *dDptr = nullptr, *dDtoff = nullptr, *dBptr = nullptr, *dPptr = nullptr, *dPidx = nullptr;
  int *dBdom = nullptr, *dBpart = nullptr;
  int2 *dBlocks = nullptr;
  int nblocks = 0;
  // cross-projected pair-domain integrals from B (osv_build_pairs_exact)
  bool k_exact = false;
  double *dCx = nullptr;   // C_p = Q_p^T B_p computed from B
  // one-step high-order correction (built on first use)
  bool hc_ready = false;
  double hc_bytes = 0.0, hc_flops = 0.0;   // collective sums: bytes; residual step: flops
  double hc_ms[2] = {0.0, 0.0};            // device times of the last call
  int hc_nwg = 1;
  int *dHcQueue = nullptr, *dHcCounter = nullptr;
  double *dHcScr = nullptr;
  double *dTc = nullptr, *dHcOut = nullptr;
  long long *dCoff = nullptr, *dCtptr = nullptr;
  CTerm *dCterms = nullptr;
  // OSV response N_ij (built on first use)
  bool nij_ready = false;
  std::vector<NijTarget> nij_tg;   // in queue (cost) order
  long long nij_out = 0;           // output doubles
  double nij_flops = 0.0;          // MFMA flops of one evaluation (kept ranks)
  int nij_nwg = 1;
  NijTarget *dNijTg = nullptr;
  int *dNijEntCp = nullptr, *dNijCounter = nullptr, *dNijMate = nullptr;
  double *dNijEntC = nullptr, *dNijScr = nullptr;
  int2 *dNijLmo = nullptr, *dNijBcol = nullptr;
  long long *dWeakNoff = nullptr;  // weak pairs' N^up offsets (built on first use)
  // state
  bool solved = false;
  std::string err;
  double stage_ms[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double stage_flops[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<double> flops_sweep;  // per cluster: residual-term flops of one sweep
  double flops_warm0 = 0.0;         // sum of flops_sweep over warm-started clusters
  std::vector<int> rank_host;
  ~osv_ctx() {
    // work still queued on the caller's stream may use these blocks: finish it
    // before they go back to the cache and a later context reuses them
    if (!allocs.empty()) (void)hipDeviceSynchronize();
    for (void *p : allocs) pool_free(p);
  }
};

namespace {

int fail(osv_ctx *ctx, int code, const std::string &msg) {
  g_last_error = msg;
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return fail(ctx, _e == hipErrorOutOfMemory ? OSV_E_NOMEM : OSV_E_HIP,                \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                      \
  } while (0)

template <class T>
int dalloc(osv_ctx *ctx, T **p, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void *q = nullptr;
  hipError_t e = pool_alloc(&q, bytes);
  if (e != hipSuccess)
    return fail(ctx, e == hipErrorOutOfMemory ? OSV_E_NOMEM : OSV_E_HIP,
                "device allocation of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  ctx->allocs.push_back(q);
  *p = (T *)q;
  return OSV_OK;
}

template <class T>
int upload(osv_ctx *ctx, T **p, const std::vector<T> &v, hipStream_t s) {
  int rc = dalloc(ctx, p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIPCHK(ctx, hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return OSV_OK;
}

// Pinned host staging for the large table uploads: one buffer per device, kept
// for the process and grown when a batch needs more.  A batch copies its tables
// into it on the host and the device reads them by DMA in stream order; an event
// recorded after the copies guards the next reuse (the next batch waits for it
// before writing).  Pageable sources would be staged by the runtime in small
// pieces after the preceding kernels, with the host copying in between.
struct PinnedStage {
  std::mutex mu;
  char *p = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
};
std::mutex g_stage_mu;
std::map<int, PinnedStage> g_stage;

struct Up {
  void **dst;
  const void *src;
  size_t bytes;
};
template <class T>
void add_up(std::vector<Up> &ups, T **dst, const std::vector<T> &v) {
  ups.push_back(Up{reinterpret_cast<void **>(dst), v.data(), v.size() * sizeof(T)});
}

// device buffers for every table of the batch (from the block cache) and their
// contents, copied through the pinned staging buffer on stream s
int upload_batch(osv_ctx *ctx, const std::vector<Up> &ups, hipStream_t s) {
  size_t total = 0;
  for (const Up &u : ups) total += (u.bytes + 255) & ~(size_t)255;
  for (const Up &u : ups) {
    char *d = nullptr;
    int rc = dalloc(ctx, &d, u.bytes);
    if (rc) return rc;
    *u.dst = d;
  }
  int dev = 0;
  HIPCHK(ctx, hipGetDevice(&dev));
  PinnedStage *st;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    st = &g_stage[dev];
  }
  std::lock_guard<std::mutex> lk(st->mu);
  if (st->done) HIPCHK(ctx, hipEventSynchronize(st->done));   // the last batch has been read
  else HIPCHK(ctx, hipEventCreateWithFlags(&st->done, hipEventDisableTiming));
  if (total > st->cap) {
    if (st->p) HIPCHK(ctx, hipHostFree(st->p));
    st->p = nullptr;
    st->cap = 0;
    const size_t want = std::max(total, (size_t)1 << 20);
    HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void **>(&st->p), want, hipHostMallocDefault));
    st->cap = want;
  }
  size_t o = 0;
  for (const Up &u : ups) {
    if (u.bytes) {
      // into pinned memory in 4 MB pieces on the host threads (about 150 MB of
      // plan tables at nocc = 400), then the table's copy to the device
      constexpr size_t PIECE = (size_t)4 << 20;
      const size_t np = (u.bytes + PIECE - 1) / PIECE;
      char *dst = st->p + o;
      const char *src = static_cast<const char *>(u.src);
      parallel_for(
          (long long)np,
          [&](long long k) {
            const size_t b = (size_t)k * PIECE, e = std::min(u.bytes, b + PIECE);
            std::memcpy(dst + b, src + b, e - b);
          },
          1);
      HIPCHK(ctx, hipMemcpyAsync(*u.dst, st->p + o, u.bytes, hipMemcpyHostToDevice, s));
    }
    o += (u.bytes + 255) & ~(size_t)255;
  }
  HIPCHK(ctx, hipEventRecord(st->done, s));
  return OSV_OK;
}

// the FP64 copy of an FP32 C, made once per context
int c64(osv_ctx *ctx, hipStream_t s) {
  if (ctx->dC64) return OSV_OK;
  const long long n = (long long)ctx->nosv * ctx->naux;
  int rc = dalloc(ctx, &ctx->dC64, (size_t)n);
  if (rc) return rc;
  HIPCHK(ctx, launch_f32_to_f64((const float *)ctx->C, ctx->dC64, n, s));
  return OSV_OK;
}

struct StageTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit StageTimer(hipStream_t st) : s(st) {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, s);
  }
  // records the end of the stage; the value is read after the stream is synchronised
  void stop() { (void)hipEventRecord(b, s); }
  double ms() {
    float t = 0.f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.0;
    return t;
  }
  ~StageTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// tiles (ti <= tj, tsz x tsz) of the sum(r) x sum(r) index space that hold a domain block
// tiles of tsz x tsz covering the orbital-pair blocks of every domain (and the
// (i, j) blocks of the weak pairs, whose K the one-block scheme reads)
std::vector<int2> make_tiles(const Plan &P, int nosv, bool all, int tsz,
                             const std::vector<int2> *weak = nullptr, const int *off = nullptr,
                             const int *r = nullptr) {
  const int nt = (nosv + tsz - 1) / tsz;
  std::vector<char> mark((size_t)nt * nt, all ? 1 : 0);
  auto block = [&](int po, int pr, int qo, int qr) {
    const int a0 = po / tsz, a1 = (po + pr - 1) / tsz, b0 = qo / tsz, b1 = (qo + qr - 1) / tsz;
    for (int a = a0; a <= a1; a++)
      for (int b = b0; b <= b1; b++) mark[(size_t)std::min(a, b) * nt + std::max(a, b)] = 1;
  };
  if (!all) {
    for (const Domain &D : P.doms) {
      const int qo = (D.p == D.q) ? D.offp : D.offq, qr = (D.p == D.q) ? D.rp : D.rq;
      block(D.offp, D.rp, qo, qr);
    }
    if (weak)
      for (const int2 &w : *weak) block(off[w.x], r[w.x], off[w.y], r[w.y]);
  }
  std::vector<int2> t;
  for (int a = 0; a < nt; a++)
    for (int b = a; b < nt; b++)
      if (mark[(size_t)a * nt + b]) t.push_back(make_int2(a, b));
  return t;
}

}  // namespace

static int build_impl(osv_ctx *ctx, const osv_system *sys, const osv_select *sel, int32_t precision,
                      hipStream_t stream) {
  long long nosv = 0;
  for (int i = 0; i < sys->nocc; i++) nosv += sys->r[i];
  ctx->nocc = sys->nocc;
  ctx->nvir = sys->nvir;
  ctx->naux = sys->naux;
  ctx->nosv = (int)nosv;
  ctx->precision = precision;
  ctx->c_dtype = sys->C_dtype;
  ctx->mode = sel->mode;
  ctx->Q = sys->Q;
  ctx->C = sys->C;
  ctx->eps = sys->eps_vir;
  ctx->F = sys->F_occ;
  ctx->tau_S = sel->tau_S;
  ctx->r.assign(sys->r, sys->r + sys->nocc);
  ctx->off.assign(sys->nocc + 1, 0);
  for (int i = 0; i < sys->nocc; i++) ctx->off[i + 1] = ctx->off[i] + ctx->r[i];
  hipStream_t s = stream;
  const int nocc = ctx->nocc, N = ctx->nosv;
  const long long ld = N;
  int rc;

  // input checks on the device (NaN / Inf); the flag is read once the host has
  // selected the clusters
  if ((rc = dalloc(ctx, &ctx->dFlag, 4))) return rc;
  HIPCHK(ctx, launch_fill_i32(ctx->dFlag, 0, 4, s));
  HIPCHK(ctx, launch_check_finite(ctx->Q, (long long)ctx->nvir * N, ctx->dFlag, s));
  if (ctx->c_dtype == OSV_DT_F32)
    HIPCHK(ctx, launch_check_finite_f32((const float *)ctx->C, (long long)N * ctx->naux, ctx->dFlag, s));
  else
    HIPCHK(ctx, launch_check_finite((const double *)ctx->C, (long long)N * ctx->naux, ctx->dFlag, s));
  HIPCHK(ctx, launch_check_finite(ctx->eps, ctx->nvir, ctx->dFlag, s));
  HIPCHK(ctx, launch_check_finite(ctx->F, (long long)nocc * nocc, ctx->dFlag, s));

  if ((rc = dalloc(ctx, &ctx->dS, (size_t)ld * ld))) return rc;
  if ((rc = dalloc(ctx, &ctx->dF, (size_t)ld * ld))) return rc;
  if ((rc = dalloc(ctx, &ctx->dK, (size_t)ld * ld))) return rc;
  if ((rc = upload(ctx, &ctx->dOff, ctx->off, s))) return rc;
  if ((rc = upload(ctx, &ctx->dR, ctx->r, s))) return rc;
  // mixed precision: the digit splits of the rows of Q^T, Q^T diag(eps) and C do
  // not depend on the selection and run while the host selects
  const bool digits = precision == OSV_MIXED && ctx->naux <= digit_max_k();
  const bool sf_digits = precision == OSV_MIXED && ctx->nvir <= digit_max_k();
  if (digits) {
    if ((rc = dalloc(ctx, (unsigned char **)&ctx->dDig, digit_bytes(N, ctx->naux)))) return rc;
    if ((rc = dalloc(ctx, &ctx->dExps, N))) return rc;
  }
  if (sf_digits) {
    if ((rc = dalloc(ctx, &ctx->dDigQr, digit_bytes(N, ctx->nvir)))) return rc;
    if ((rc = dalloc(ctx, &ctx->dDigQe, digit_bytes(N, ctx->nvir)))) return rc;
    if ((rc = dalloc(ctx, &ctx->dExpQr, N))) return rc;
    if ((rc = dalloc(ctx, &ctx->dExpQe, N))) return rc;
    if ((rc = dalloc(ctx, &ctx->dQe, (size_t)N * ctx->nvir))) return rc;
  }
  StageTimer t_sf_split(s);
  if (sf_digits) {
    HIPCHK(ctx, launch_scale_cols(ctx->Q, ctx->eps, N, ctx->nvir, ctx->dQe, s));
    HIPCHK(ctx, launch_split_digits_f64(ctx->Q, ctx->nvir, N, ctx->nvir, ctx->dExpQr, ctx->dDigQr, s));
    HIPCHK(ctx, launch_split_digits_f64(ctx->dQe, ctx->nvir, N, ctx->nvir, ctx->dExpQe, ctx->dDigQe, s));
  }
  t_sf_split.stop();
  StageTimer t_k_split(s);
  if (digits) HIPCHK(ctx, launch_split_digits((const float *)ctx->C, N, ctx->naux, ctx->dExps, ctx->dDig, s));
  t_k_split.stop();

  const auto h0 = std::chrono::steady_clock::now();
  // cluster selection
  if (sel->mode == OSV_SEL_DISTANCE) {
    select_distance(nocc, sys->centroid, sel->cut2, sel->cut3, ctx->sel);
  } else if (sel->mode == OSV_SEL_FULL) {
    select_full(nocc, ctx->sel);
  } else {
    // overlap metric eq:2bscreen needs every S block: full S first
    std::vector<int2> all = make_tiles(ctx->plan, N, true, 64), all128 = make_tiles(ctx->plan, N, true, 128);
    int2 *dAll = nullptr, *dAll128 = nullptr;
    if ((rc = upload(ctx, &dAll, all, s))) return rc;
    if ((rc = upload(ctx, &dAll128, all128, s))) return rc;
    HIPCHK(ctx, launch_syrk_f64(ctx->Q, 0, ctx->nvir, N, ctx->nvir, nullptr, ctx->dS, nullptr, ld, dAll,
                                (int)all.size(), dAll128, (int)all128.size(), s));
    double *dSq = nullptr;
    if ((rc = dalloc(ctx, &dSq, (size_t)nocc * nocc))) return rc;
    HIPCHK(ctx, launch_block_sumsq(ctx->dS, ld, ctx->dOff, ctx->dR, nocc, dSq, s));
    std::vector<double> sq((size_t)nocc * nocc);
    HIPCHK(ctx, hipMemcpyAsync(sq.data(), dSq, sq.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    auto s2b = [&](int i, int j) { return sq[(size_t)i * nocc + j] / std::sqrt((double)ctx->r[i] * ctx->r[j]); };
    select_mbe(
        nocc, [&](int i, int j) { return s2b(i, j) > sel->l2b; },
        [&](int i, int j, int k) { return (s2b(i, j) + s2b(i, k) + s2b(j, k)) / 3.0 > sel->l3b; },
        [](int, int) { return true; }, ctx->sel);
    // weak 2b clusters: neither strong nor discarded (one-block scheme)
    for (int i = 0; i < nocc; i++)
      for (int j = i + 1; j < nocc; j++) {
        const double v = s2b(i, j);
        if (v >= OSV_WEAK_MIN && !(v > sel->l2b)) ctx->weak.push_back(make_int2(i, j));
      }
  }
  {
    int flag = 0;
    HIPCHK(ctx, hipMemcpyAsync(&flag, ctx->dFlag, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (flag) return fail(ctx, OSV_E_NONFINITE, "NaN or Inf in Q, C, eps_vir or F_occ");
  }
  {
    std::string err;
    rc = build_domains(nocc, ctx->sel, ctx->r.data(), ctx->off.data(), ctx->plan, err);
    if (rc) return fail(ctx, rc, err);
  }
  Plan &P = ctx->plan;
  const Selection &S = ctx->sel;
  ctx->weak_dd.resize(ctx->weak.size());
  for (size_t w = 0; w < ctx->weak.size(); w++)
    ctx->weak_dd[w] = make_int2(P.dom_of[(size_t)ctx->weak[w].x * nocc + ctx->weak[w].x],
                                P.dom_of[(size_t)ctx->weak[w].y * nocc + ctx->weak[w].y]);
  if (!ctx->weak.empty()) {
    const size_t nw = ctx->weak.size();
    ctx->weak_toff.resize(nw);
    ctx->weak_nT = 0;
    ctx->weak_lptr.assign(nocc + 1, 0);
    for (size_t w = 0; w < nw; w++) {
      ctx->weak_toff[w] = ctx->weak_nT;
      ctx->weak_nT += (long long)ctx->r[ctx->weak[w].x] * ctx->r[ctx->weak[w].y];
      ctx->weak_lptr[ctx->weak[w].x + 1]++;
      ctx->weak_lptr[ctx->weak[w].y + 1]++;
    }
    for (int i = 0; i < nocc; i++) ctx->weak_lptr[i + 1] += ctx->weak_lptr[i];
    ctx->weak_lidx.assign(ctx->weak_lptr[nocc], 0);
    std::vector<long long> fill(ctx->weak_lptr.begin(), ctx->weak_lptr.end() - 1);
    for (size_t w = 0; w < nw; w++) {
      ctx->weak_lidx[fill[ctx->weak[w].x]++] = (int)w;
      ctx->weak_lidx[fill[ctx->weak[w].y]++] = (int)w;
    }
  }
  ctx->tiles = make_tiles(P, N, false, 64, &ctx->weak, ctx->off.data(), ctx->r.data());
  ctx->tiles128 = make_tiles(P, N, false, 128, &ctx->weak, ctx->off.data(), ctx->r.data());
  const int ndom = (int)P.doms.size();
  // everything the device stages before the couplings need is allocated and
  // uploaded first: uploads from pageable host memory wait for the stream
  if ((rc = upload(ctx, &ctx->dTiles, ctx->tiles, s))) return rc;
  if ((rc = upload(ctx, &ctx->dTiles128, ctx->tiles128, s))) return rc;
  if ((rc = upload(ctx, &ctx->dDom, P.doms, s))) return rc;
  if ((rc = dalloc(ctx, &ctx->dW, P.n_slot))) return rc;
  if ((rc = dalloc(ctx, &ctx->dY, P.n_slot))) return rc;
  if ((rc = dalloc(ctx, &ctx->dKt, P.n_vec))) return rc;
  if ((rc = dalloc(ctx, &ctx->dMinev, ndom))) return rc;
  if ((rc = dalloc(ctx, &ctx->dRank, ndom))) return rc;
  // prep order: diagonal domains (p, p), then the others, each by LDS size class
  // (n <= 32, <= 64, <= PREP_N3, <= DMAX); a domain (p, q) whose approximate Fock
  // eigenbasis is not taken starts its eigensolve from the eigenvectors of (p, p)
  // and (q, q)
  int prep_cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    // one stable counting sort by (group g, class, DMAX - n): within a class the
    // largest domains come first (the cost grows as n^3)
    constexpr int NKEY = 8 * (DMAX + 1);
    std::vector<int> cnt(NKEY + 1, 0), key((size_t)ndom), ids((size_t)ndom);
    std::vector<long long> dmoff((size_t)nocc, -1);
    for (int d = 0; d < ndom; d++) {
      const Domain &D = P.doms[d];
      const int n = D.n, cls = n <= 32 ? 0 : (n <= 64 ? 1 : (n <= PREP_N3 ? 2 : 3));
      const int g = D.p == D.q ? 0 : 1;
      key[d] = (4 * g + cls) * (DMAX + 1) + (DMAX - n);
      cnt[key[d] + 1]++;
      prep_cnt[4 * g + cls]++;
      if (g == 0) dmoff[D.p] = D.moff;
    }
    for (int k = 0; k < NKEY; k++) cnt[k + 1] += cnt[k];
    for (int d = 0; d < ndom; d++) ids[cnt[key[d]]++] = d;
    if ((rc = upload(ctx, &ctx->dPrepIds, ids, s))) return rc;
    if ((rc = upload(ctx, &ctx->dDiagMoff, dmoff, s))) return rc;
  }
  if (digits || sf_digits) {
    // 128 x 64 tiles of the digit products: pairs of 64-row tiles of the tile list
    const int nt = (N + 63) / 64;
    std::vector<char> mark((size_t)((nt + 1) / 2) * nt, 0);
    std::vector<int2> dt;
    for (const int2 &t : ctx->tiles) {
      const size_t k = (size_t)(t.x / 2) * nt + t.y;
      if (!mark[k]) {
        mark[k] = 1;
        dt.push_back(make_int2(t.x / 2, t.y));
      }
    }
    ctx->ndig_tiles = (int)dt.size();
    if ((rc = upload(ctx, &ctx->dDigTiles, dt, s))) return rc;
  }
  double host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();

  // S and F blocks: one pass over Q^T (rows = OSVs, k = virtuals)
  StageTimer t_sf(s);
  if (sf_digits) {
    // mixed precision: S = Q Q^T and F = Q diag(eps) Q^T from the six-digit splits of
    // the rows of Q^T and of Q^T diag(eps) made above, as K (below 2^-42 of each
    // row's scale left out)
    HIPCHK(ctx, launch_syrk_digits(ctx->dDigQr, N, ctx->nvir, ctx->dExpQr, ctx->dS, ld, ctx->dDigTiles,
                                   ctx->ndig_tiles, s));
    HIPCHK(ctx, launch_syr2_digits(ctx->dDigQr, ctx->dDigQe, N, ctx->nvir, ctx->dExpQr, ctx->dExpQe, ctx->dF,
                                   ld, ctx->dDigTiles, ctx->ndig_tiles, s));
  } else {
    HIPCHK(ctx, launch_syrk_f64(ctx->Q, 0, ctx->nvir, N, ctx->nvir, ctx->eps, ctx->dS, ctx->dF, ld,
                                ctx->dTiles, (int)ctx->tiles.size(), ctx->dTiles128,
                                (int)ctx->tiles128.size(), s));
  }
  t_sf.stop();
  StageTimer t_k(s);
  if (digits) {
    HIPCHK(ctx, launch_syrk_digits(ctx->dDig, N, ctx->naux, ctx->dExps, ctx->dK, ld, ctx->dDigTiles,
                                   ctx->ndig_tiles, s));
  } else {
    const void *Cd = ctx->C;
    if (ctx->c_dtype == OSV_DT_F32) {
      // FP64 copy of the FP32 input for the FP64 tile kernel (also used by dE/dC)
      if ((rc = c64(ctx, s))) return rc;
      Cd = ctx->dC64;
    }
    HIPCHK(ctx, launch_syrk_f64(Cd, 0, ctx->naux, N, ctx->naux, nullptr, ctx->dK, nullptr, ld,
                                ctx->dTiles, (int)ctx->tiles.size(), ctx->dTiles128,
                                (int)ctx->tiles128.size(), s));
  }
  t_k.stop();
  // pair-domain preparation
  StageTimer t_prep(s);
  HIPCHK(ctx, launch_domain_prep(ctx->dDom, ctx->dPrepIds, prep_cnt, ctx->dS, ctx->dF, ctx->dK, ld,
                                 ctx->tau_S, nullptr, ctx->dW, ctx->dY, ctx->dKt, ctx->dRank,
                                 ctx->dMinev, s));
  HIPCHK(ctx, launch_domain_prep(ctx->dDom,
                                 ctx->dPrepIds + (prep_cnt[0] + prep_cnt[1] + prep_cnt[2] + prep_cnt[3]),
                                 prep_cnt + 4, ctx->dS, ctx->dF, ctx->dK, ld, ctx->tau_S,
                                 ctx->dDiagMoff, ctx->dW, ctx->dY, ctx->dKt, ctx->dRank,
                                 ctx->dMinev, s));
  t_prep.stop();

  // clusters, terms and couplings on the host while the device works
  const auto h1 = std::chrono::steady_clock::now();
  build_clusters(nocc, ctx->sel, P);
  host_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h1).count();
  ctx->counts.n1b = S.n1;
  ctx->counts.n2b = S.n2b;
  ctx->counts.n3b = S.n3b;
  ctx->counts.n_clusters = (int64_t)S.coef.size();
  ctx->counts.n_pair_blocks = P.n_pair_blocks;
  ctx->counts.n_domains = (int64_t)P.doms.size();
  ctx->counts.n_couplings = (int64_t)P.cpls.size();
  const int ncl = (int)P.cls.size();
  // couplings by size class: both domains with n <= 64, then the others
  int n64 = 0;
  {
    std::vector<int> &ids = ctx->cpl_ids;
    ids.clear();
    ids.reserve(P.cpls.size());
    for (int pass = 0; pass < 2; pass++) {
      for (int c = 0; c < (int)P.cpls.size(); c++) {
        const bool small = std::max(P.doms[P.cpls[c].A].n, P.doms[P.cpls[c].B].n) <= tuning().cpl_split;
        if (small == (pass == 0)) ids.push_back(c);
      }
      if (pass == 0) n64 = (int)ids.size();
    }
  }
  // the plan tables (about 150 MB at nocc = 400) go up on the caller's stream
  // behind the preparation kernels, through the pinned staging buffer
  {
    std::vector<Up> ups;
    add_up(ups, &ctx->dCpl, P.cpls);
    add_up(ups, &ctx->dCp, P.cps);
    add_up(ups, &ctx->dTerms, P.terms);
    add_up(ups, &ctx->dCl, P.cls);
    add_up(ups, &ctx->dQueue, P.queue);
    add_up(ups, &ctx->dCplIds, ctx->cpl_ids);
    if ((rc = upload_batch(ctx, ups, s))) return rc;
  }
  ctx->stage_ms[8] = host_ms;
  StageTimer t_cpl(s);
  if ((rc = dalloc(ctx, &ctx->dM, P.n_M))) return rc;
  HIPCHK(ctx, launch_couplings(ctx->dCpl, ctx->dCplIds, n64, (int)P.cpls.size() - n64, ctx->dDom,
                               ctx->dRank, ctx->dS, ld, ctx->dW,
                               ctx->dM, s));
  t_cpl.stop();
  // solve-time buffers
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  ctx->nwg = std::max(1, std::min(ncl, ncu));   // one persistent workgroup per CU (LDS-bound)
  if ((rc = dalloc(ctx, &ctx->dTflat, P.terms.size()))) return rc;
  HIPCHK(ctx, launch_term_flat(ctx->dTerms, (long long)P.terms.size(), ctx->dCp, ctx->dCpl, ctx->dDom,
                               ctx->dRank, ctx->F, nocc, ctx->dTflat, s));
  if ((rc = dalloc(ctx, &ctx->dT, P.n_T))) return rc;
  if ((rc = dalloc(ctx, &ctx->dT2, P.n_T))) return rc;
  if ((rc = dalloc(ctx, &ctx->dRs, (size_t)ctx->nwg * P.rs_stride))) return rc;
  if ((rc = dalloc(ctx, &ctx->dEcl, ncl))) return rc;
  if ((rc = dalloc(ctx, &ctx->dPl, P.n_pl))) return rc;
  if ((rc = dalloc(ctx, &ctx->dMaxres, ncl))) return rc;
  if ((rc = dalloc(ctx, &ctx->dSweeps, ncl))) return rc;
  if ((rc = dalloc(ctx, &ctx->dCounter, 3))) return rc;
  // MBE weights: E, E_1b, dE_2b, dE_3b
  {
    std::vector<double> w((size_t)4 * ncl, 0.0);
    int p2 = 0;
    for (int X = 0; X < ncl; X++) {
      w[X] = S.coef[X];
      if (S.order[X] == 1) {
        int i = S.lmo[S.lmo_ptr[X]];
        w[(size_t)ncl + X] = 1.0;
        w[(size_t)2 * ncl + X] = -S.n2[i];
        w[(size_t)3 * ncl + X] = S.n3i[i];
      } else if (S.order[X] == 2) {
        w[(size_t)2 * ncl + X] = 1.0;
        w[(size_t)3 * ncl + X] = -S.n3ij[p2++];
      } else if (S.order[X] == 3) {
        w[(size_t)3 * ncl + X] = 1.0;
      }
    }
    if ((rc = upload(ctx, &ctx->dWts, w, s))) return rc;
    if ((rc = dalloc(ctx, &ctx->dEout, 4))) return rc;
  }
  // the ranks (and the stage times) once the couplings and the term table are done;
  // the host work above ran while they did
  ctx->rank_host.resize(ndom);
  HIPCHK(ctx, hipMemcpyAsync(ctx->rank_host.data(), ctx->dRank, ndom * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  for (int d = 0; d < ndom; d++)
    if (ctx->rank_host[d] < 1) {
      return fail(ctx, OSV_E_DOMAIN, "pair domain (" + std::to_string(P.doms[d].p) + "," +
                                         std::to_string(P.doms[d].q) + ") has rank 0 after the tau_S cut");
    }
  ctx->stage_ms[0] = t_sf_split.ms() + t_sf.ms();
  ctx->stage_ms[1] = t_k_split.ms() + t_k.ms();
  ctx->stage_ms[2] = t_prep.ms();
  ctx->stage_ms[3] = t_cpl.ms();
  return OSV_OK;
}


// ---- allocation-free weak-pair entry point -----------------------------------
// Device memory for osv_weak_pairs_noalloc: per weak pair its two diagonal
// domains (int2) and its energy (double), then the fixed-order sum.  One copy per
// device, held while the process runs; every call on a device shares it.
constexpr long long NOALLOC_MAX_WEAK = 1LL << 20;
constexpr size_t NOALLOC_BYTES = (size_t)NOALLOC_MAX_WEAK * (sizeof(int2) + sizeof(double)) + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// out = sum of x[0..n) in a fixed order: thread t sums x[t], x[t + 256], ...,
// then the 256 partial sums are added pairwise in a fixed tree
__global__ __launch_bounds__(256) void k_sum_fixed(const double *x, long long n, double *out) {
  __shared__ double red[256];
  double v = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) v += x[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// the device address of this device's scratch, looked up once per device
static int scratch_ptr(osv_ctx *ctx, unsigned char **out) {
  static std::mutex mu;
  static std::map<int, unsigned char *> addr;
  int dev = 0;
  HIPCHK(ctx, hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *p = nullptr;
    HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ctx, OSV_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    it = addr.emplace(dev, (unsigned char *)p).first;
  }
  *out = it->second;
  return OSV_OK;
}


// Device buffers of one osv_generate_osvs call, returned to the block cache on exit.
struct GenBuffers {
  std::vector<void *> blocks;
  template <class T>
  hipError_t get(T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = pool_alloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) blocks.push_back(q);
    *p = (T *)q;
    return e;
  }
  ~GenBuffers() {
    if (!blocks.empty()) (void)hipDeviceSynchronize();
    for (void *q : blocks) pool_free(q);
  }
};

// ---- tuning table ------------------------------------------------------------
namespace osv {
namespace {
std::once_flag g_tuning_once;
Tuning g_tuning;
std::mutex g_tuning_mu;

// allowed values per key; returns false for an unknown key or value
bool tuning_set(const std::string &k, int v) {
  auto in = [&](std::initializer_list<int> a) { return std::find(a.begin(), a.end(), v) != a.end(); };
  if (k == "gemm_ks" && in({8, 16, 32})) g_tuning.gemm_ks = v;
  else if (k == "prep_nt_small" && in({128, 256})) g_tuning.prep_nt[0] = v;
  else if (k == "prep_nt_mid" && in({256, 512, 1024})) g_tuning.prep_nt[1] = v;
  else if (k == "prep_nt_big" && in({512, 1024})) g_tuning.prep_nt[2] = v;
  else if (k == "cpl_split" && in({0, 64})) g_tuning.cpl_split = v;
  else if (k == "solve_split" && in({0, 1})) g_tuning.solve_split = v;
  else return false;
  return true;
}

bool tuning_get(const std::string &k, int *v) {
  if (k == "gemm_ks") *v = g_tuning.gemm_ks;
  else if (k == "prep_nt_small") *v = g_tuning.prep_nt[0];
  else if (k == "prep_nt_mid") *v = g_tuning.prep_nt[1];
  else if (k == "prep_nt_big") *v = g_tuning.prep_nt[2];
  else if (k == "cpl_split") *v = g_tuning.cpl_split;
  else if (k == "solve_split") *v = g_tuning.solve_split;
  else return false;
  return true;
}

// "key value" lines; '#' starts a comment; returns the number of entries applied,
// or -1 if the file cannot be read, -2 on a bad line
int tuning_read(const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) return -1;
  char line[256];
  int n = 0, bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    char *h = std::strchr(line, '#');
    if (h) *h = 0;
    char key[64];
    int v = 0;
    const int got = std::sscanf(line, "%63s %d", key, &v);
    if (got <= 0) continue;
    if (got != 2 || !tuning_set(key, v)) bad = 1;
    else n++;
  }
  std::fclose(f);
  return bad ? -2 : n;
}

std::string library_dir() {
  Dl_info info;
  if (dladdr((const void *)&library_dir, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t s = p.find_last_of('/');
    return s == std::string::npos ? std::string(".") : p.substr(0, s);
  }
  return ".";
}

void tuning_init() {
  const char *env = std::getenv("OSV_TUNING_FILE");
  std::string path = env ? std::string(env) : library_dir() + "/osv_tuning.txt";
  if (!path.empty()) (void)tuning_read(path.c_str());
}
}  // namespace

Tuning &tuning() {
  std::call_once(g_tuning_once, tuning_init);
  return g_tuning;
}
}  // namespace osv

extern "C" {

const char *osv_status_string(int st) {
  switch (st) {
    case OSV_OK: return "ok";
    case OSV_E_ARG: return "invalid argument";
    case OSV_E_HIP: return "HIP runtime error";
    case OSV_E_NOMEM: return "out of memory";
    case OSV_E_NOT_CONVERGED: return "residual iteration did not converge";
    case OSV_E_NONFINITE: return "non-finite value in input or residual";
    case OSV_E_STATE: return "called before a converged solve";
    case OSV_E_DOMAIN: return "pair domain of rank 0";
    default: return "unknown status";
  }
}

const char *osv_last_error(const osv_ctx *ctx) {
  if (ctx) return ctx->err.c_str();
  return g_last_error.c_str();
}

int osv_plan_clusters(int32_t nocc, const double *centroid, const osv_select *sel,
                      osv_counts *counts, int32_t *lmos, double *coef, int64_t cap) {
  if (nocc < 1 || !sel || !counts) return fail(nullptr, OSV_E_ARG, "osv_plan_clusters: bad arguments");
  Selection s;
  if (sel->mode == OSV_SEL_DISTANCE) {
    if (!centroid) return fail(nullptr, OSV_E_ARG, "DISTANCE selection needs centroids");
    if (!(sel->cut2 >= 0) || !(sel->cut3 >= 0)) return fail(nullptr, OSV_E_ARG, "negative cutoff");
    select_distance(nocc, centroid, sel->cut2, sel->cut3, s);
  } else if (sel->mode == OSV_SEL_FULL) {
    select_full(nocc, s);
  } else {
    return fail(nullptr, OSV_E_ARG, "osv_plan_clusters supports DISTANCE and FULL selection");
  }
  Plan P;
  std::string err;
  int rc = build_plan(nocc, s, nullptr, nullptr, P, err);
  if (rc) return fail(nullptr, rc, err);
  counts->n1b = s.n1;
  counts->n2b = s.n2b;
  counts->n3b = s.n3b;
  counts->n_clusters = (int64_t)s.coef.size();
  counts->n_pair_blocks = P.n_pair_blocks;
  counts->n_domains = (int64_t)P.doms.size();
  counts->n_couplings = (int64_t)P.cpls.size();
  const int64_t ncl = (int64_t)s.coef.size();
  if ((lmos || coef) && cap < ncl) return fail(nullptr, OSV_E_ARG, "capacity below the cluster count");
  if (lmos && sel->mode != OSV_SEL_FULL)
    for (int64_t X = 0; X < ncl; X++)
      for (int a = 0; a < 3; a++) {
        int i = s.lmo_ptr[X] + a;
        lmos[3 * X + a] = (i < s.lmo_ptr[X + 1]) ? s.lmo[i] : -1;
      }
  if (coef)
    for (int64_t X = 0; X < ncl; X++) coef[X] = s.coef[X];
  return OSV_OK;
}

int osv_build_pairs(const osv_system *sys, const osv_select *sel, int32_t precision,
                    hipStream_t stream, osv_ctx **out) {
  if (!out) return fail(nullptr, OSV_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sys || !sel) return fail(nullptr, OSV_E_ARG, "sys or sel is NULL");
  if (sys->nocc < 1 || sys->nvir < 1 || sys->naux < 1)
    return fail(nullptr, OSV_E_ARG, "nocc, nvir and naux must be >= 1");
  if (!sys->r || !sys->Q || !sys->C || !sys->eps_vir || !sys->F_occ)
    return fail(nullptr, OSV_E_ARG, "NULL array in osv_system");
  if (sys->C_dtype != OSV_DT_F64 && sys->C_dtype != OSV_DT_F32)
    return fail(nullptr, OSV_E_ARG, "unknown C_dtype");
  if (precision != OSV_FP64 && precision != OSV_MIXED)
    return fail(nullptr, OSV_E_ARG, "unknown precision");
  if (precision == OSV_MIXED && sys->C_dtype != OSV_DT_F32)
    return fail(nullptr, OSV_E_ARG, "OSV_MIXED needs C in FP32");
  if (sel->mode != OSV_SEL_DISTANCE && sel->mode != OSV_SEL_OVERLAP && sel->mode != OSV_SEL_FULL)
    return fail(nullptr, OSV_E_ARG, "unknown selection mode");
  if (sel->mode == OSV_SEL_DISTANCE && (!sys->centroid || !(sel->cut2 >= 0) || !(sel->cut3 >= 0)))
    return fail(nullptr, OSV_E_ARG, "DISTANCE selection needs centroids and cutoffs >= 0");
  if (!(sel->tau_S >= 0.0)) return fail(nullptr, OSV_E_ARG, "tau_S must be >= 0");
  long long nosv = 0;
  for (int i = 0; i < sys->nocc; i++) {
    if (sys->r[i] < 1 || sys->r[i] > sys->nvir || sys->r[i] > OSV_MAX_DOMAIN)
      return fail(nullptr, OSV_E_ARG, "r[" + std::to_string(i) + "] out of range");
    nosv += sys->r[i];
  }
  if (nosv > (1LL << 30)) return fail(nullptr, OSV_E_ARG, "sum(r) too large");

  osv_ctx *ctx = new (std::nothrow) osv_ctx();
  if (!ctx) return fail(nullptr, OSV_E_NOMEM, "host allocation");
  int rc = build_impl(ctx, sys, sel, precision, stream);
  if (rc != OSV_OK) {
    g_last_error = ctx->err;
    delete ctx;
    return rc;
  }
  *out = ctx;
  return OSV_OK;
}

int osv_build_pairs_exact(const osv_system *sys, const double *B, const osv_select *sel, int32_t precision,
                          hipStream_t stream, osv_ctx **out) {
  if (!out) return fail(nullptr, OSV_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sys || !sel || !B) return fail(nullptr, OSV_E_ARG, "sys, sel or B is NULL");
  if (precision != OSV_FP64)
    return fail(nullptr, OSV_E_ARG, "cross-projected integrals are built in FP64 only (precision OSV_FP64)");
  if (sys->nocc < 1 || sys->nvir < 1 || sys->naux < 1 || !sys->r || !sys->Q || !sys->eps_vir || !sys->F_occ)
    return fail(nullptr, OSV_E_ARG, "bad sizes or NULL array in osv_system");
  long long nosv = 0;
  for (int i = 0; i < sys->nocc; i++) {
    if (sys->r[i] < 1 || sys->r[i] > sys->nvir || sys->r[i] > OSV_MAX_DOMAIN)
      return fail(nullptr, OSV_E_ARG, "r[" + std::to_string(i) + "] out of range");
    nosv += sys->r[i];
  }
  if (nosv > (1LL << 30)) return fail(nullptr, OSV_E_ARG, "sum(r) too large");
  osv_ctx *ctx = new (std::nothrow) osv_ctx();
  if (!ctx) return fail(nullptr, OSV_E_NOMEM, "host allocation");
  auto bail = [&](int rc) {
    g_last_error = ctx->err;
    delete ctx;
    return rc;
  };
  hipStream_t s = stream;
  const int nvir = sys->nvir, naux = sys->naux, nocc = sys->nocc;
  int rc;
  // B must be finite; then C_p = Q_p^T B_p (rows of Q^T times B_p)
  int *flag = nullptr;
  if ((rc = dalloc(ctx, &flag, 1))) return bail(rc);
  {
    hipError_t e = launch_fill_i32(flag, 0, 1, s);
    if (e == hipSuccess) e = launch_check_finite(B, (long long)nocc * nvir * naux, flag, s);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(fail(ctx, OSV_E_HIP, std::string("B check: ") + hipGetErrorString(e)));
    if (h) return bail(fail(ctx, OSV_E_NONFINITE, "NaN or Inf in B"));
  }
  if ((rc = dalloc(ctx, &ctx->dCx, (size_t)nosv * naux))) return bail(rc);
  {
    long long o = 0;
    for (int p = 0; p < nocc; p++) {
      const hipError_t e = launch_gemm_nn_f64(sys->Q + o * nvir, nvir, B + (long long)p * nvir * naux, 0, naux,
                                              ctx->dCx + o * naux, naux, sys->r[p], naux, nvir, 1.0, s);
      if (e != hipSuccess) return bail(fail(ctx, OSV_E_HIP, std::string("C from B: ") + hipGetErrorString(e)));
      o += sys->r[p];
    }
  }
  osv_system sx = *sys;
  sx.C = ctx->dCx;
  sx.C_dtype = OSV_DT_F64;
  if ((rc = build_impl(ctx, &sx, sel, OSV_FP64, s))) return bail(rc);
  // the off-diagonal domains' K~ from the cross-projected integrals
  Plan &P = ctx->plan;
  double *Pt = nullptr, *Vt = nullptr, *Gp = nullptr, *Gq = nullptr;
  if ((rc = dalloc(ctx, &Pt, (size_t)DMAX * nvir))) return bail(rc);
  if ((rc = dalloc(ctx, &Vt, (size_t)DMAX * nvir))) return bail(rc);
  if ((rc = dalloc(ctx, &Gp, (size_t)DMAX * naux))) return bail(rc);
  if ((rc = dalloc(ctx, &Gq, (size_t)DMAX * naux))) return bail(rc);
  for (size_t d = 0; d < P.doms.size(); d++) {
    const Domain &D = P.doms[d];
    if (D.p == D.q) continue;
    const int n = D.n, dt = ctx->rank_host[d];
    hipError_t e = hipMemcpyAsync(Pt, sys->Q + (long long)D.offp * nvir, (size_t)D.rp * nvir * 8,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(Pt + (long long)D.rp * nvir, sys->Q + (long long)D.offq * nvir, (size_t)D.rq * nvir * 8,
                         hipMemcpyDeviceToDevice, s);
    // V^T = W^T P^T (dt x nvir), then Gp = V^T B_p, Gq = V^T B_q
    if (e == hipSuccess) e = launch_gemm_tn_f64(ctx->dW + D.moff, n, Pt, nvir, Vt, nvir, dt, nvir, n, 1.0, s);
    if (e == hipSuccess)
      e = launch_gemm_nn_f64(Vt, nvir, B + (long long)D.p * nvir * naux, 0, naux, Gp, naux, dt, naux, nvir, 1.0, s);
    if (e == hipSuccess)
      e = launch_gemm_nn_f64(Vt, nvir, B + (long long)D.q * nvir * naux, 0, naux, Gq, naux, dt, naux, nvir, 1.0, s);
    if (e == hipSuccess) e = launch_exact_ktilde(Gp, Gq, dt, naux, ctx->dKt + D.voff, D.np, s);
    if (e != hipSuccess) return bail(fail(ctx, OSV_E_HIP, std::string("cross-projected K: ") + hipGetErrorString(e)));
  }
  {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(fail(ctx, OSV_E_HIP, std::string("cross-projected K: ") + hipGetErrorString(e)));
  }
  ctx->k_exact = true;
  *out = ctx;
  return OSV_OK;
}

int osv_query(const osv_ctx *ctx, osv_counts *out) {
  if (!ctx || !out) return fail(nullptr, OSV_E_ARG, "osv_query: NULL argument");
  *out = ctx->counts;
  return OSV_OK;
}

// algorithmic flops of the build stages and of one sweep per cluster (host; the
// solve runs it while its kernel occupies the GPU)
static void count_flops(osv_ctx *ctx) {
  if (!ctx->flops_sweep.empty() || ctx->plan.cls.empty()) return;
  Plan &P = ctx->plan;
    const std::vector<int> &rk = ctx->rank_host;
    double fsf = 0, fk = 0, fc = 0;
    for (const Domain &D : P.doms) {
      double rp = D.rp, rq = (D.p == D.q) ? D.rp : D.rq;
      fsf += (D.p == D.q ? 2.0 : 4.0) * rp * rq * ctx->nvir;
      fk += 2.0 * rp * rq * ctx->naux;
    }
    for (const Coupling &c : P.cpls) {
      double nA = P.doms[c.A].n, nB = P.doms[c.B].n, dA = rk[c.A], dB = rk[c.B];
      fc += 2.0 * (nA * dB * nB + dA * dB * nA);
    }
    // domain preparation, algorithmic: the products around the eigensolvers at the
    // kept rank dt, and 9 m^3 per symmetric eigendecomposition with vectors of order m
    // (the count of a tridiagonal-reduction solver; the cyclic Jacobi method used
    // here does several times more)
    double fp = 0.0;
    for (size_t d = 0; d < P.doms.size(); d++) {
      const Domain &D = P.doms[d];
      const double n = D.n, dt = rk[d], rp = D.rp;
      if (D.p == D.q) {
        fp += 9.0 * n * n * n + 2.0 * dt * rp * rp + 2.0 * dt * dt * rp;
      } else {
        const double rq = D.rq;
        fp += 2.0 * rq * rq * rp + 2.0 * rq * rq * rq / 3.0   // Gram matrix, Cholesky and L^-1
              + 2.0 * rp * rq * rq                             // -B Z
              + 2.0 * n * n * n                                // warm start X diag(V_p, V_q)
              + 2.0 * n * n * dt + 2.0 * n * dt * dt           // X^T F X
              + 9.0 * dt * dt * dt                             // Fock eigensolve
              + 2.0 * n * dt * dt + 2.0 * dt * n * n           // W = X V, Y = W^T S
              + 2.0 * dt * rp * rq + 2.0 * dt * dt * rq;       // K~
      }
    }
    ctx->stage_flops[0] = fsf;
    ctx->stage_flops[1] = fk;
    ctx->stage_flops[2] = fp;
    ctx->stage_flops[3] = fc;
    ctx->flops_sweep.assign(P.cls.size(), 0.0);
    for (size_t X = 0; X < P.cls.size(); X++) {
      const Cluster &C = P.cls[X];
      double f = 0;
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
        double nt = rk[P.cps[c].dom];
        for (int t = P.cps[c].term0; t < P.cps[c].term0 + P.cps[c].nterm; t++) {
          double ns = rk[P.cps[P.terms[t].src].dom];
          f += 2.0 * (nt * ns * ns + nt * nt * ns);
        }
      }
      ctx->flops_sweep[X] = f;
      // a cluster that starts from amplitudes of an earlier launch also takes the
      // terms in its sweep 0
      bool warm = false;
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) warm = warm || P.cps[c].init >= 0;
      if (warm) ctx->flops_warm0 += f;
    }
  }

static void densities_host(osv_ctx *ctx);
static int upload_density_tables(osv_ctx *ctx, hipStream_t s);

int osv_solve_clusters(osv_ctx *ctx, double tau_R, int32_t max_sweeps, hipStream_t s,
                       osv_solve_info *info) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!(tau_R > 0.0) || max_sweeps < 1) return fail(ctx, OSV_E_ARG, "tau_R must be > 0 and max_sweeps >= 1");
  ctx->solved = false;
  Plan &P = ctx->plan;
  const int ncl = (int)P.cls.size();
  SolveArgs a{};
  a.cl = ctx->dCl;
  a.cp = ctx->dCp;
  a.terms = ctx->dTerms;
  a.tflat = ctx->dTflat;
  a.dom = ctx->dDom;
  a.dom_rank = ctx->dRank;
  a.cpl = ctx->dCpl;
  a.M = ctx->dM;
  a.Kep = ctx->dKt;
  a.F_occ = ctx->F;
  a.nocc = ctx->nocc;
  a.T = ctx->dT;
  a.T2 = ctx->dT2;
  a.Rs = ctx->dRs;
  a.rs_stride = P.rs_stride;
  a.Ecl = ctx->dEcl;
  a.Pl = ctx->dPl;
  a.sweeps = ctx->dSweeps;
  a.maxres = ctx->dMaxres;
  a.queue = ctx->dQueue;
  a.counter = ctx->dCounter;
  a.n_clusters = ncl;
  a.tau_R = tau_R;
  a.max_sweeps = max_sweeps;
  a.split = tuning().solve_split;
  StageTimer t(s);
  HIPCHK(ctx, launch_fill_i32(ctx->dCounter, 0, 3, s));
  HIPCHK(ctx, launch_solve(a, P.n_big, P.n_first, ctx->nwg, s));
  // the weak pairs' one-block amplitudes (one step each, in the OSV bases)
  const int nweak = (int)ctx->weak.size();
  if (nweak > 0) {
    int rc;
    if (!ctx->dWeakT) {
      if ((rc = upload(ctx, &ctx->dWeakDom, ctx->weak_dd, s))) return rc;
      if ((rc = upload(ctx, &ctx->dWeakLmo, ctx->weak, s))) return rc;
      if ((rc = upload(ctx, &ctx->dWeakToff, ctx->weak_toff, s))) return rc;
      if ((rc = upload(ctx, &ctx->dWeakLptr, ctx->weak_lptr, s))) return rc;
      if ((rc = upload(ctx, &ctx->dWeakLidx, ctx->weak_lidx, s))) return rc;
      if ((rc = dalloc(ctx, &ctx->dWeakT, (size_t)ctx->weak_nT))) return rc;
      if ((rc = dalloc(ctx, &ctx->dWeakEa, nweak))) return rc;
      if ((rc = dalloc(ctx, &ctx->dWeakTT, nweak))) return rc;
      if ((rc = dalloc(ctx, &ctx->dWeakSum, 1))) return rc;
    }
    HIPCHK(ctx, launch_weak_amplitudes(ctx->dWeakDom, nweak, ctx->dDom, ctx->dRank, ctx->dK,
                                       (long long)ctx->nosv, ctx->dW, ctx->dKt, ctx->F, ctx->nocc,
                                       ctx->dWeakToff, ctx->dWeakT, ctx->dWeakEa, ctx->dWeakTT, s));
  }
  t.stop();
  // host bookkeeping while the kernel runs (the density tables are uploaded by
  // the first osv_densities call)
  count_flops(ctx);
  densities_host(ctx);
  std::vector<int> sw(ncl);
  std::vector<double> mr(ncl);
  HIPCHK(ctx, hipMemcpyAsync(sw.data(), ctx->dSweeps, ncl * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(mr.data(), ctx->dMaxres, ncl * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  ctx->stage_ms[4] = t.ms();
  osv_solve_info inf{};
  inf.converged = 1;
  bool nonfinite = false;
  // a cluster that stops at sweep s has taken the terms in sweeps 1..s, and also
  // in sweep 0 when it started from amplitudes of an earlier launch
  double fs = ctx->flops_warm0;
  for (int X = 0; X < ncl; X++) fs += ctx->flops_sweep[X] * sw[X];
  ctx->stage_flops[4] = fs;
  for (int X = 0; X < ncl; X++) {
    inf.sweeps = std::max(inf.sweeps, sw[X]);
    if (!std::isfinite(mr[X])) nonfinite = true;
    else inf.max_residual = std::max(inf.max_residual, mr[X]);
    if (!(mr[X] < tau_R)) {
      inf.converged = 0;
      inf.n_not_converged++;
    }
  }
  if (info) *info = inf;
  if (nonfinite) return fail(ctx, OSV_E_NONFINITE, "residual is not finite");
  if (!inf.converged)
    return fail(ctx, OSV_E_NOT_CONVERGED, std::to_string(inf.n_not_converged) + " clusters did not converge");
  ctx->solved = true;
  return OSV_OK;
}

int osv_energy(osv_ctx *ctx, hipStream_t s, double *E, double *E_orders, double *E_cluster) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!E) return fail(ctx, OSV_E_ARG, "E is NULL");
  if (!ctx->solved) return fail(ctx, OSV_E_STATE, "osv_energy before a converged solve");
  const int ncl = (int)ctx->plan.cls.size();
  StageTimer t(s);
  HIPCHK(ctx, launch_wdot(ctx->dEcl, ctx->dWts, ncl, 4, ctx->dEout, s));
  const long long nweak = (long long)ctx->weak.size();
  if (nweak > 0) {
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, (const double *)ctx->dWeakEa, nweak,
                       ctx->dWeakSum);
    HIPCHK(ctx, hipGetLastError());
  }
  t.stop();
  double h[4], ew = 0.0;
  HIPCHK(ctx, hipMemcpyAsync(h, ctx->dEout, sizeof(h), hipMemcpyDeviceToHost, s));
  if (nweak > 0) HIPCHK(ctx, hipMemcpyAsync(&ew, ctx->dWeakSum, sizeof(double), hipMemcpyDeviceToHost, s));
  if (E_cluster)
    HIPCHK(ctx, hipMemcpyAsync(E_cluster, ctx->dEcl, ncl * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  ctx->stage_ms[5] = t.ms();
  // the weak pairs are 2-body increments: E and dE_2b include them
  *E = h[0] + ew;
  if (E_orders) {
    if (ctx->mode == OSV_SEL_FULL) {
      E_orders[0] = E_orders[1] = E_orders[2] = std::nan("");
    } else {
      E_orders[0] = h[1];
      E_orders[1] = h[2] + ew;
      E_orders[2] = h[3];
    }
  }
  return OSV_OK;
}

// Host part of the densities' bookkeeping (it depends on the plan only, so the
// solve runs it while its kernel occupies the GPU).
static void densities_host(osv_ctx *ctx) {
  DensHost &H = ctx->dh;
  if (H.ready) return;
  Plan &P = ctx->plan;
  const Selection &S = ctx->sel;
  const int ndom = (int)P.doms.size(), ncl = (int)P.cls.size(), nocc = ctx->nocc;
  // per domain: (amplitude offset, c_X) over the clusters holding it, cluster order
  // (counting sort by domain)
  H.ptr.assign(ndom + 1, 0);
  for (int X = 0; X < ncl; X++) {
    if (S.coef[X] == 0.0) continue;
    const Cluster &C = P.cls[X];
    for (int c = C.cp0; c < C.cp0 + C.ncp; c++) H.ptr[P.cps[c].dom + 1]++;
  }
  for (int d = 0; d < ndom; d++) H.ptr[d + 1] += H.ptr[d];
  // launch order of the adjoint: a diagonal domain is held by hundreds of clusters
  // and costs up to 100 times the mean, so the costly ones go first and the many
  // short ones fill the CUs around them
  {
    std::vector<double> cost(ndom);
    for (int d = 0; d < ndom; d++) {
      const double np = P.doms[d].np;
      cost[d] = (double)(H.ptr[d + 1] - H.ptr[d]) * np * np * np;
    }
    H.adj_order.resize(ndom);
    std::iota(H.adj_order.begin(), H.adj_order.end(), 0);
    std::stable_sort(H.adj_order.begin(), H.adj_order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
  }
  H.toff.assign(H.ptr[ndom], 0);
  H.cf.assign(H.ptr[ndom], 0.0);
  {
    std::vector<long long> fill(H.ptr.begin(), H.ptr.end() - 1);
    for (int X = 0; X < ncl; X++) {
      if (S.coef[X] == 0.0) continue;
      const Cluster &C = P.cls[X];
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
        const long long k = fill[P.cps[c].dom]++;
        H.toff[k] = P.cps[c].toff;
        H.cf[k] = S.coef[X];
      }
    }
  }
  // G^F orbital blocks
  H.blocks.clear();
  H.bptr.assign(1, 0);
  H.bdom.clear();
  H.bpart.clear();
  std::vector<std::vector<std::pair<int, int>>> diag_src(nocc);
  for (int d = 0; d < ndom; d++) {
    const Domain &D = P.doms[d];
    diag_src[D.p].push_back({d, 0});
    if (D.q != D.p) diag_src[D.q].push_back({d, 1});
  }
  for (int d = 0; d < ndom; d++) {
    const Domain &D = P.doms[d];
    H.blocks.push_back(make_int2(D.p, D.q));
    if (D.p == D.q) {
      for (auto &e : diag_src[D.p]) {
        H.bdom.push_back(e.first);
        H.bpart.push_back(e.second);
      }
    } else {
      H.bdom.push_back(d);
      H.bpart.push_back(0);
    }
    H.bptr.push_back((long long)H.bdom.size());
  }
  // dE/dF: per entry (u, v) the (cluster, inner-product index) list, cluster order
  // (counting sort by entry)
  const size_t ne = (size_t)nocc * nocc;
  H.pptr.assign(ne + 1, 0);
  for (int X = 0; X < ncl; X++) {
    if (S.coef[X] == 0.0) continue;
    const Cluster &C = P.cls[X];
    for (int a = 0; a < C.nlmo; a++)
      for (int b = 0; b < C.nlmo; b++)
        H.pptr[(size_t)S.lmo[C.lmo0 + a] * nocc + S.lmo[C.lmo0 + b] + 1]++;
  }
  for (size_t e = 0; e < ne; e++) H.pptr[e + 1] += H.pptr[e];
  H.pidx.assign(2 * H.pptr[ne], 0);
  {
    std::vector<long long> fill(H.pptr.begin(), H.pptr.end() - 1);
    for (int X = 0; X < ncl; X++) {
      if (S.coef[X] == 0.0) continue;
      const Cluster &C = P.cls[X];
      for (int a = 0; a < C.nlmo; a++)
        for (int b = 0; b < C.nlmo; b++) {
          const size_t e = (size_t)S.lmo[C.lmo0 + a] * nocc + S.lmo[C.lmo0 + b];
          const long long k = fill[e]++;
          H.pidx[2 * k] = X;
          H.pidx[2 * k + 1] = C.poff + (long long)a * C.nlmo + b;
        }
    }
  }
  H.ready = true;
}

// The per-domain tables of the densities (host side built by densities_host) to
// the device on stream s.
static int upload_density_tables(osv_ctx *ctx, hipStream_t s) {
  DensHost &H = ctx->dh;
  const Selection &S = ctx->sel;
  ctx->nblocks = (int)H.blocks.size();
  std::vector<Up> ups;
  add_up(ups, &ctx->dDptr, H.ptr);
  add_up(ups, &ctx->dAdjOrder, H.adj_order);
  add_up(ups, &ctx->dDtoff, H.toff);
  add_up(ups, &ctx->dDcoef, H.cf);
  add_up(ups, &ctx->dBlocks, H.blocks);
  add_up(ups, &ctx->dBptr, H.bptr);
  add_up(ups, &ctx->dBdom, H.bdom);
  add_up(ups, &ctx->dBpart, H.bpart);
  add_up(ups, &ctx->dPptr, H.pptr);
  add_up(ups, &ctx->dPidx, H.pidx);
  add_up(ups, &ctx->dClcoef, S.coef);
  return upload_batch(ctx, ups, s);
}

static int prepare_densities(osv_ctx *ctx, hipStream_t s) {
  if (ctx->dens_ready) return OSV_OK;
  densities_host(ctx);
  Plan &P = ctx->plan;
  const int N = ctx->nosv;
  int rc;
  if (!ctx->dDptr && (rc = upload_density_tables(ctx, s))) return rc;
  const long long ld = N;
  if ((rc = dalloc(ctx, &ctx->dGK, (size_t)ld * ld))) return rc;
  if ((rc = dalloc(ctx, &ctx->dGF, (size_t)ld * ld))) return rc;
  if ((rc = dalloc(ctx, &ctx->dGd, P.n_slot))) return rc;
  if ((rc = dalloc(ctx, &ctx->dZt, (size_t)N * ctx->nvir))) return rc;
  if ((rc = dalloc(ctx, &ctx->dColPart,
                   (size_t)((N + COLDOT_ROWS - 1) / COLDOT_ROWS) * ctx->nvir)))
    return rc;
  HIPCHK(ctx, launch_fill_f64(ctx->dGK, 0.0, ld * ld, s));
  HIPCHK(ctx, launch_fill_f64(ctx->dGF, 0.0, ld * ld, s));
  ctx->dens_ready = true;
  return OSV_OK;
}

int osv_weak_pairs(osv_ctx *ctx, hipStream_t s, double *E_weak, int64_t *n_weak, double *E_pairs,
                   int32_t *pairs) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!E_weak) return fail(ctx, OSV_E_ARG, "E_weak is NULL");
  const int nw = (int)ctx->weak.size();
  if (n_weak) *n_weak = nw;
  *E_weak = 0.0;
  if (pairs)
    for (int w = 0; w < nw; w++) {
      pairs[2 * w] = ctx->weak[w].x;
      pairs[2 * w + 1] = ctx->weak[w].y;
    }
  if (nw == 0) return OSV_OK;
  const int nocc = ctx->nocc;
  int rc;
  if (!ctx->dWeak) {
    if ((rc = upload(ctx, &ctx->dWeak, ctx->weak_dd, s))) return rc;
    if ((rc = dalloc(ctx, &ctx->dWeakE, nw))) return rc;
  }
  HIPCHK(ctx, launch_weak(ctx->dWeak, nw, ctx->dDom, ctx->dRank, ctx->dK, (long long)ctx->nosv,
                          ctx->dW, ctx->dKt, ctx->F, nocc, ctx->dWeakE, s));
  std::vector<double> e(nw);
  HIPCHK(ctx, hipMemcpyAsync(e.data(), ctx->dWeakE, nw * sizeof(double), hipMemcpyDeviceToHost, s));
  if (E_pairs)
    HIPCHK(ctx, hipMemcpyAsync(E_pairs, ctx->dWeakE, nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  double t = 0.0;
  for (int w = 0; w < nw; w++) t += e[w];
  *E_weak = t;
  return OSV_OK;
}

int osv_weak_pairs_noalloc(osv_ctx *ctx, hipStream_t s, double *E_weak, int64_t *n_weak,
                           double *E_pairs, int32_t *pairs) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!E_weak) return fail(ctx, OSV_E_ARG, "E_weak is NULL");
  const long long nw = (long long)ctx->weak.size();
  if (n_weak) *n_weak = nw;
  *E_weak = 0.0;
  if (nw > NOALLOC_MAX_WEAK)
    return fail(ctx, OSV_E_ARG, std::to_string(nw) + " weak pairs exceed the allocation-free limit of " +
                                    std::to_string(NOALLOC_MAX_WEAK));
  if (pairs)
    for (long long w = 0; w < nw; w++) {
      pairs[2 * w] = ctx->weak[w].x;
      pairs[2 * w + 1] = ctx->weak[w].y;
    }
  if (nw == 0) return OSV_OK;
  unsigned char *base = nullptr;
  int rc = scratch_ptr(ctx, &base);
  if (rc) return rc;
  // layout: energies (nw doubles), the sum (one double), the domain table (nw int2)
  double *dE = (double *)base;
  double *dSum = dE + nw;
  int2 *dDD = (int2 *)(dSum + 1);
  HIPCHK(ctx, hipMemcpyAsync(dDD, ctx->weak_dd.data(), nw * sizeof(int2), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, launch_weak(dDD, (int)nw, ctx->dDom, ctx->dRank, ctx->dK, (long long)ctx->nosv, ctx->dW,
                          ctx->dKt, ctx->F, ctx->nocc, dE, s));
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, (const double *)dE, nw, dSum);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipMemcpyAsync(E_weak, dSum, sizeof(double), hipMemcpyDeviceToHost, s));
  if (E_pairs)
    HIPCHK(ctx, hipMemcpyAsync(E_pairs, dE, nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return OSV_OK;
}

// device times and algorithmic flops of the last osv_generate_osvs call of this thread
thread_local double g_gen_stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};

int osv_generation_stats(double *out8) {
  if (!out8) return fail(nullptr, OSV_E_ARG, "osv_generation_stats: out is NULL");
  for (int i = 0; i < 8; i++) out8[i] = g_gen_stats[i];
  return OSV_OK;
}

int osv_generate_osvs(int32_t nocc, int32_t nvir, int32_t naux, const double *B, const double *eps_vir,
                      const double *F_occ, double l_osv, int32_t r_max, hipStream_t s, int32_t *r,
                      double *omega, double *Q, double *C) {
  if (nocc < 1 || nvir < 1 || naux < 1 || !B || !eps_vir || !F_occ || !r || !Q)
    return fail(nullptr, OSV_E_ARG, "osv_generate_osvs: bad sizes or NULL pointer");
  if (nvir > OSV_GEN_MAX_NVIR)
    return fail(nullptr, OSV_E_ARG, "osv_generate_osvs: nvir above " + std::to_string(OSV_GEN_MAX_NVIR));
  if (r_max < 1 || r_max > nvir || r_max > OSV_MAX_DOMAIN)
    return fail(nullptr, OSV_E_ARG, "osv_generate_osvs: r_max must lie in [1, min(nvir, OSV_MAX_DOMAIN)]");
  if (!(l_osv == l_osv)) return fail(nullptr, OSV_E_ARG, "osv_generate_osvs: l_osv is NaN");
  const long long n2 = (long long)nvir * nvir;
  GenBuffers gb;
  int *flag = nullptr;
  double *T = nullptr, *d = nullptr, *e = nullptr, *tau = nullptr, *om = nullptr, *Z = nullptr;
  int *rk = nullptr, *doff = nullptr;
  int2 *tiles = nullptr, *tiles128 = nullptr;
  hipError_t he;
#define GENCHK(expr)                                                                           \
  do {                                                                                         \
    he = (expr);                                                                               \
    if (he != hipSuccess)                                                                      \
      return fail(nullptr, he == hipErrorOutOfMemory ? OSV_E_NOMEM : OSV_E_HIP,                \
                  std::string("osv_generate_osvs: ") + #expr + ": " + hipGetErrorString(he)); \
  } while (0)
  GENCHK(gb.get(&flag, 4));
  GENCHK(launch_fill_i32(flag, 0, 4, s));
  GENCHK(launch_check_finite(B, (long long)nocc * nvir * naux, flag, s));
  GENCHK(launch_check_finite(eps_vir, nvir, flag, s));
  GENCHK(launch_check_finite(F_occ, (long long)nocc * nocc, flag, s));
  int hflag = 0;
  GENCHK(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  GENCHK(hipStreamSynchronize(s));
  if (hflag) return fail(nullptr, OSV_E_NONFINITE, "osv_generate_osvs: NaN or Inf in B, eps_vir or F_occ");
  GENCHK(gb.get(&T, (size_t)nocc * n2));
  GENCHK(gb.get(&d, (size_t)nocc * nvir));
  GENCHK(gb.get(&e, (size_t)nocc * nvir));
  GENCHK(gb.get(&tau, (size_t)nocc * nvir));
  GENCHK(gb.get(&om, (size_t)nocc * r_max));
  GENCHK(gb.get(&Z, (size_t)nocc * nvir * r_max));
  GENCHK(gb.get(&rk, nocc));
  GENCHK(gb.get(&doff, nocc));
  // (ka|kb) = B_k B_k^T for every k on all tiles of the nvir x nvir matrix
  std::vector<int2> t64, t128;
  for (int a = 0; a < (nvir + 63) / 64; a++)
    for (int b = a; b < (nvir + 63) / 64; b++) t64.push_back(make_int2(a, b));
  for (int a = 0; a < (nvir + 127) / 128; a++)
    for (int b = a; b < (nvir + 127) / 128; b++) t128.push_back(make_int2(a, b));
  GENCHK(gb.get(&tiles, t64.size()));
  GENCHK(gb.get(&tiles128, t128.size()));
  GENCHK(hipMemcpyAsync(tiles, t64.data(), t64.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  GENCHK(hipMemcpyAsync(tiles128, t128.data(), t128.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  StageTimer t_prod(s);
  for (int k = 0; k < nocc; k++)
    GENCHK(launch_syrk_f64(B + (long long)k * nvir * naux, 0, naux, nvir, naux, nullptr, T + (long long)k * n2,
                           nullptr, nvir, tiles, (int)t64.size(), tiles128, (int)t128.size(), s));
  t_prod.stop();
  StageTimer t_tri(s);
  GENCHK(launch_osv_denom(T, nvir, eps_vir, F_occ, nocc, s));
  GENCHK(launch_osv_tridiag(T, nocc, nvir, l_osv, r_max, d, e, tau, rk, om, s));
  t_tri.stop();
  std::vector<int> hr(nocc), hoff(nocc);
  GENCHK(hipMemcpyAsync(hr.data(), rk, nocc * sizeof(int), hipMemcpyDeviceToHost, s));
  GENCHK(hipStreamSynchronize(s));
  int tot = 0;
  for (int k = 0; k < nocc; k++) {
    hoff[k] = tot;
    tot += hr[k];
    r[k] = hr[k];
  }
  GENCHK(hipMemcpyAsync(doff, hoff.data(), nocc * sizeof(int), hipMemcpyHostToDevice, s));
  if (omega) GENCHK(launch_fill_f64(omega, 0.0, (long long)nocc * r_max, s));
  double *om_out = omega;
  if (!om_out) GENCHK(gb.get(&om_out, (size_t)nocc * r_max));
  StageTimer t_vec(s);
  GENCHK(launch_osv_vectors(T, nocc, nvir, r_max, d, e, tau, rk, om, doff, Z, Q, om_out, s));
  t_vec.stop();
  // C_k = Q_k^T B_k: rows off_k .. of C
  StageTimer t_c(s);
  if (C)
    for (int k = 0; k < nocc; k++)
      if (hr[k] > 0)
        GENCHK(launch_gemm_nn_f64(Q + (long long)hoff[k] * nvir, nvir, B + (long long)k * nvir * naux, 0,
                                  naux, C + (long long)hoff[k] * naux, naux, hr[k], naux, nvir, 1.0, s));
  t_c.stop();
  GENCHK(hipStreamSynchronize(s));
  // algorithmic flops: the symmetric products (ka|kb) nvir^2 naux per LMO, the
  // Householder reduction 4/3 nvir^3 per LMO, the reflectors applied to the kept
  // vectors 4 nvir^2 r_k, C = Q^T B 2 r_k nvir naux
  {
    const double nv = nvir, na = naux;
    g_gen_stats[0] = t_prod.ms();
    g_gen_stats[1] = nocc * nv * nv * na;
    g_gen_stats[2] = t_tri.ms();
    g_gen_stats[3] = nocc * 4.0 / 3.0 * nv * nv * nv;
    g_gen_stats[4] = t_vec.ms();
    g_gen_stats[5] = 4.0 * nv * nv * tot;
    g_gen_stats[6] = t_c.ms();
    g_gen_stats[7] = C ? 2.0 * tot * nv * na : 0.0;
  }
#undef GENCHK
  return OSV_OK;
}

// Host tables of the one-step correction: collective slots per domain and, per
// target domain (p, q), the terms of eq:rij with k over the LMOs that share a
// cluster with p and q.
static int build_correction(osv_ctx *ctx, hipStream_t s) {
  Plan &P = ctx->plan;
  const Selection &S = ctx->sel;
  const int nocc = ctx->nocc, ndom = (int)P.doms.size();
  auto dom_id = [&](int a, int b) {
    return a <= b ? P.dom_of[(size_t)a * nocc + b] : P.dom_of[(size_t)b * nocc + a];
  };
  // k ranges: every LMO of every cluster that holds the pair
  std::vector<std::vector<int>> range(ndom);
  for (size_t X = 0; X < P.cls.size(); X++) {
    const Cluster &C = P.cls[X];
    for (int a = 0; a < C.nlmo; a++)
      for (int b = a; b < C.nlmo; b++) {
        auto &rg = range[dom_id(S.lmo[C.lmo0 + a], S.lmo[C.lmo0 + b])];
        for (int c = 0; c < C.nlmo; c++) rg.push_back(S.lmo[C.lmo0 + c]);
      }
  }
  std::unordered_map<long long, int> cmap;
  cmap.reserve(P.cpls.size() * 2);
  for (size_t c = 0; c < P.cpls.size(); c++)
    cmap[(long long)P.cpls[c].A * ndom + P.cpls[c].B] = (int)c;
  std::vector<long long> coff(ndom), tptr(ndom + 1, 0);
  long long nTc = 0;
  for (int d = 0; d < ndom; d++) {
    coff[d] = nTc;
    nTc += 2LL * P.doms[d].np * P.doms[d].np;
  }
  std::vector<CTerm> terms;
  for (int d = 0; d < ndom; d++) {
    auto &rg = range[d];
    std::sort(rg.begin(), rg.end());
    rg.erase(std::unique(rg.begin(), rg.end()), rg.end());
    const int p = P.doms[d].p, q = P.doms[d].q;
    auto add = [&](int a, int b, int fa, int fb) -> bool {
      const int sd = dom_id(a, b);
      if (sd < 0) return false;
      CTerm t{};
      t.src = sd;
      t.fa = fa;
      t.fb = fb;
      t.ldT = P.doms[sd].np;
      t.tsrc = coff[sd] + ((a > b) ? (long long)P.doms[sd].np * P.doms[sd].np : 0LL);
      const int A = std::min(d, sd), B = std::max(d, sd);
      auto it = cmap.find((long long)A * ndom + B);
      if (it == cmap.end()) return false;
      const Coupling &c = P.cpls[it->second];
      t.moff = (d == c.B) ? c.offAB : c.offBA;    // M(src, tgt)
      terms.push_back(t);
      return true;
    };
    for (int m : rg) {
      if (m != q && !add(p, m, m, q)) return fail(ctx, OSV_E_HIP, "one-step correction: missing coupling");
      if (m != p && !add(m, q, p, m)) return fail(ctx, OSV_E_HIP, "one-step correction: missing coupling");
    }
    tptr[d + 1] = (long long)terms.size();
  }
  // algorithmic work: the collective sums read every cluster slot of a domain and
  // write the domain's two slots; the residual step takes 2 (dt ns^2 + dt^2 ns)
  // flops per term at the kept ranks
  {
    densities_host(ctx);
    const DensHost &H = ctx->dh;
    double by = 0.0, fl = 0.0;
    for (int d = 0; d < ndom; d++) {
      const double np2 = 2.0 * P.doms[d].np * P.doms[d].np;
      by += 8.0 * np2 * (double)(H.ptr[d + 1] - H.ptr[d] + 1);
      const double dt = ctx->rank_host[d];
      for (long long t = tptr[d]; t < tptr[d + 1]; t++) {
        const double ns = ctx->rank_host[terms[t].src];
        fl += 2.0 * (dt * ns * ns + dt * dt * ns);
      }
    }
    ctx->hc_bytes = by;
    ctx->hc_flops = fl;
  }
  int rc;
  if ((rc = upload(ctx, &ctx->dCoff, coff, s))) return rc;
  if ((rc = upload(ctx, &ctx->dCtptr, tptr, s))) return rc;
  if ((rc = upload(ctx, &ctx->dCterms, terms, s))) return rc;
  if ((rc = dalloc(ctx, &ctx->dTc, (size_t)nTc))) return rc;
  if ((rc = dalloc(ctx, &ctx->dHcOut, (size_t)3 * ndom))) return rc;
  // the residual step's queue: domains with the most terms first
  {
    std::vector<int> q(ndom);
    std::iota(q.begin(), q.end(), 0);
    std::stable_sort(q.begin(), q.end(),
                     [&](int x, int y) { return tptr[x + 1] - tptr[x] > tptr[y + 1] - tptr[y]; });
    if ((rc = upload(ctx, &ctx->dHcQueue, q, s))) return rc;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    ctx->hc_nwg = std::max(1, std::min(ndom, ncu));
    if ((rc = dalloc(ctx, &ctx->dHcCounter, 1))) return rc;
    if ((rc = dalloc(ctx, &ctx->dHcScr, (size_t)collective_step_scratch(ctx->hc_nwg)))) return rc;
  }
  ctx->hc_ready = true;
  return OSV_OK;
}

// Host tables of the OSV response N_ij: per stored pair domain (a target) the
// clusters holding it with c_X != 0 (cluster order), the LMOs that its k-sums
// reach with their accumulator columns and, per residual term of those clusters,
// the columns of the source's LMO blocks; the output layout (domain order, N_pq
// then N_qp) and the targets in decreasing order of cost for the work queue.
static void nij_host(osv_ctx *ctx, const std::vector<double> &Fh, std::vector<NijTarget> &tg,
                     std::vector<int> &ent_cp, std::vector<double> &ent_c, std::vector<int2> &lmo_tab,
                     std::vector<int2> &bcol, std::vector<int> &tmate, int &lb_max) {
  Plan &P = ctx->plan;
  const Selection &S = ctx->sel;
  const int ndom = (int)P.doms.size(), ncl = (int)P.cls.size();
  std::vector<long long> eptr(ndom + 1, 0);
  for (int X = 0; X < ncl; X++) {
    if (S.coef[X] == 0.0) continue;
    const Cluster &C = P.cls[X];
    for (int c = C.cp0; c < C.cp0 + C.ncp; c++) eptr[P.cps[c].dom + 1]++;
  }
  for (int d = 0; d < ndom; d++) eptr[d + 1] += eptr[d];
  ent_cp.assign(eptr[ndom], 0);
  ent_c.assign(eptr[ndom], 0.0);
  {
    std::vector<long long> fill(eptr.begin(), eptr.end() - 1);
    for (int X = 0; X < ncl; X++) {
      if (S.coef[X] == 0.0) continue;
      const Cluster &C = P.cls[X];
      for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
        const long long k = fill[P.cps[c].dom]++;
        ent_cp[k] = c;
        ent_c[k] = S.coef[X];
      }
    }
  }
  tg.assign(ndom, NijTarget{});
  lmo_tab.clear();
  bcol.assign(P.terms.size(), make_int2(-1, -1));
  // diagonal targets (p, p): the sum-1 term of source (p, m) and the sum-2 term of
  // (m, p) share the source slots; with f_mp == f_pm they are taken as one
  tmate.assign(P.terms.size(), -1);
  const int nocc = ctx->nocc;
  for (int X = 0; X < ncl; X++) {
    if (S.coef[X] == 0.0) continue;
    const Cluster &C = P.cls[X];
    for (int c = C.cp0; c < C.cp0 + C.ncp; c++) {
      const CPair &cp = P.cps[c];
      if (cp.la != cp.lb || cp.nterm != 2 * (C.nlmo - 1)) continue;
      const int h = C.nlmo - 1;
      for (int j = 0; j < h; j++) {
        const int t1 = cp.term0 + j, t2 = cp.term0 + h + j;
        const Term &a1 = P.terms[t1], &a2 = P.terms[t2];
        if (a1.src != a2.src) continue;
        if (Fh[(size_t)a1.fa * nocc + a1.fb] != Fh[(size_t)a2.fa * nocc + a2.fb]) continue;
        tmate[t1] = t2;
        tmate[t2] = -2;
      }
    }
  }
  lb_max = 0;
  ctx->nij_out = 0;
  ctx->nij_flops = 0.0;
  std::vector<double> cost(ndom, 0.0);
  std::vector<int> lm;
  for (int d = 0; d < ndom; d++) {
    const Domain &D = P.doms[d];
    lm.clear();
    for (long long en = eptr[d]; en < eptr[d + 1]; en++) {
      const CPair &cp = P.cps[ent_cp[en]];
      for (int t = cp.term0; t < cp.term0 + cp.nterm; t++) {
        const Domain &E = P.doms[P.cps[P.terms[t].src].dom];
        lm.push_back(E.p);
        lm.push_back(E.q);
      }
    }
    std::sort(lm.begin(), lm.end());
    lm.erase(std::unique(lm.begin(), lm.end()), lm.end());
    NijTarget T{};
    T.dom = d;
    T.nlmo = (int)lm.size();
    T.lmo0 = (long long)lmo_tab.size();
    T.ent0 = eptr[d];
    T.ent1 = eptr[d + 1];
    std::vector<int> col(lm.size());
    int lb = 0;
    for (size_t l = 0; l < lm.size(); l++) {
      col[l] = lb;
      lmo_tab.push_back(make_int2(lm[l], lb));
      lb += ctx->r[lm[l]];
    }
    T.lb = lb;
    lb_max = std::max(lb_max, lb);
    auto column = [&](int x) {
      return col[std::lower_bound(lm.begin(), lm.end(), x) - lm.begin()];
    };
    // flops of the tile products at the kept ranks
    const double n = D.n, dt = ctx->rank_host[d];
    const double rp = D.rp, rq = (D.p == D.q) ? D.rp : D.rq;
    double fl = 0.0;
    for (long long en = eptr[d]; en < eptr[d + 1]; en++) {
      const CPair &cp = P.cps[ent_cp[en]];
      fl += 8.0 * dt * dt * dt;
      for (int t = cp.term0; t < cp.term0 + cp.nterm; t++) {
        const int e = P.cps[P.terms[t].src].dom;
        const Domain &E = P.doms[e];
        bcol[t] = make_int2(column(E.p), E.p == E.q ? -1 : column(E.q));
        const double ns = ctx->rank_host[e], ne = E.n;
        if (tmate[t] == -1) fl += 4.0 * dt * ns * ns + 4.0 * dt * dt * ns + 2.0 * dt * ne * ns;
        else if (tmate[t] >= 0) fl += 2.0 * dt * ns * ns + 2.0 * dt * dt * ns + 2.0 * dt * ne * ns;
      }
    }
    const bool diag = D.p == D.q;
    fl += 2.0 * dt * n * dt + 2.0 * dt * rp * dt + 2.0 * dt * rq * rp + 2.0 * dt * n * (dt + n) +
          2.0 * dt * n * lb + 2.0 * dt * n * rq + 2.0 * n * n * dt;
    if (!diag) fl += 2.0 * dt * rq * dt + 2.0 * dt * rp * rq + 2.0 * dt * n * rp + 2.0 * n * n * dt;
    ctx->nij_flops += fl;
    cost[d] = fl;
    T.outF = ctx->nij_out;
    ctx->nij_out += (long long)D.n * D.n;
    if (diag) {
      T.outR = -1;
    } else {
      T.outR = ctx->nij_out;
      ctx->nij_out += (long long)D.n * D.n;
    }
    tg[d] = T;
  }
  std::stable_sort(tg.begin(), tg.end(),
                   [&](const NijTarget &x, const NijTarget &y) { return cost[x.dom] > cost[y.dom]; });
}

static int build_nij(osv_ctx *ctx, hipStream_t s) {
  std::vector<int> ent_cp;
  std::vector<double> ent_c;
  std::vector<int2> lmo_tab, bcol;
  std::vector<int> tmate;
  std::vector<double> Fh((size_t)ctx->nocc * ctx->nocc);
  HIPCHK(ctx, hipMemcpyAsync(Fh.data(), ctx->F, Fh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  int lb_max = 0;
  nij_host(ctx, Fh, ctx->nij_tg, ent_cp, ent_c, lmo_tab, bcol, tmate, lb_max);
  int rc;
  if ((rc = upload(ctx, &ctx->dNijTg, ctx->nij_tg, s))) return rc;
  if ((rc = upload(ctx, &ctx->dNijEntCp, ent_cp, s))) return rc;
  if ((rc = upload(ctx, &ctx->dNijEntC, ent_c, s))) return rc;
  if ((rc = upload(ctx, &ctx->dNijLmo, lmo_tab, s))) return rc;
  if ((rc = upload(ctx, &ctx->dNijBcol, bcol, s))) return rc;
  if ((rc = upload(ctx, &ctx->dNijMate, tmate, s))) return rc;
  if ((rc = dalloc(ctx, &ctx->dNijCounter, 1))) return rc;
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int ntg = (int)ctx->nij_tg.size();
  ctx->nij_nwg = std::max(1, std::min(ntg, ncu));   // one 8-wave workgroup per CU (registers)
  const long long stride = nij_scratch_doubles(lb_max);
  if ((rc = dalloc(ctx, &ctx->dNijScr, (size_t)(stride * ctx->nij_nwg)))) return rc;
  ctx->nij_ready = true;
  return OSV_OK;
}

int osv_response_layout(const osv_ctx *ctx, int64_t *n_pairs, int64_t *n_doubles, int32_t *pairs,
                        int64_t *offsets) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  const Plan &P = ctx->plan;
  long long np = 0, nd = 0;
  for (const Domain &D : P.doms) {
    const long long n2 = (long long)D.n * D.n;
    for (int o = 0; o < (D.p == D.q ? 1 : 2); o++) {
      if (pairs) {
        pairs[2 * np] = o ? D.q : D.p;
        pairs[2 * np + 1] = o ? D.p : D.q;
      }
      if (offsets) offsets[np] = nd;
      np++;
      nd += n2;
    }
  }
  if (n_pairs) *n_pairs = np;
  if (n_doubles) *n_doubles = nd;
  return OSV_OK;
}

int osv_response(osv_ctx *ctx, hipStream_t s, double *N, double *ms_flops) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!N) return fail(ctx, OSV_E_ARG, "osv_response: N is NULL");
  if (!ctx->solved) return fail(ctx, OSV_E_STATE, "osv_response before a converged solve");
  if (ctx->k_exact)
    return fail(ctx, OSV_E_ARG, "osv_response: the pair-domain integrals must be those of osv_build_pairs");
  int rc;
  if (!ctx->nij_ready && (rc = build_nij(ctx, s))) return rc;
  NijArgs a{};
  a.tg = ctx->dNijTg;
  a.ntg = (int)ctx->nij_tg.size();
  a.ent_cp = ctx->dNijEntCp;
  a.ent_c = ctx->dNijEntC;
  a.lmo_tab = ctx->dNijLmo;
  a.bcol = ctx->dNijBcol;
  a.tmate = ctx->dNijMate;
  a.cp = ctx->dCp;
  a.terms = ctx->dTerms;
  a.tflat = ctx->dTflat;
  a.dom = ctx->dDom;
  a.rank = ctx->dRank;
  a.W = ctx->dW;
  a.Y = ctx->dY;
  a.Kep = ctx->dKt;
  a.M = ctx->dM;
  a.T = ctx->dT;
  a.S = ctx->dS;
  a.F = ctx->dF;
  a.K = ctx->dK;
  a.ld = ctx->nosv;
  a.F_occ = ctx->F;
  a.nocc = ctx->nocc;
  a.off = ctx->dOff;
  a.r = ctx->dR;
  a.scr = ctx->dNijScr;
  a.counter = ctx->dNijCounter;
  a.N = N;
  int lb_max = 0;
  for (const NijTarget &t : ctx->nij_tg) lb_max = std::max(lb_max, t.lb);
  a.scr_stride = nij_scratch_doubles(lb_max);
  StageTimer t_n(s);
  HIPCHK(ctx, launch_nij(a, ctx->nij_nwg, s));
  t_n.stop();
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (ms_flops) {
    ms_flops[0] = t_n.ms();
    ms_flops[1] = ctx->nij_flops;
  }
  return OSV_OK;
}

int osv_weak_response(osv_ctx *ctx, hipStream_t s, int64_t *n_doubles, double *N_up) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  const int nweak = (int)ctx->weak.size();
  std::vector<long long> noff(nweak + 1, 0);
  for (int w = 0; w < nweak; w++) {
    const long long ri = ctx->r[ctx->weak[w].x];
    noff[w + 1] = noff[w] + ri * ri;
  }
  if (n_doubles) *n_doubles = noff[nweak];
  if (!N_up) return OSV_OK;
  if (!ctx->solved) return fail(ctx, OSV_E_STATE, "osv_weak_response before a converged solve");
  if (nweak == 0) return OSV_OK;
  int rc;
  if (!ctx->dWeakNoff && (rc = upload(ctx, &ctx->dWeakNoff, noff, s))) return rc;
  HIPCHK(ctx, launch_weak_nup(ctx->dWeakLmo, nweak, ctx->dOff, ctx->dR, ctx->dWeakToff, ctx->dWeakT, ctx->dK,
                              (long long)ctx->nosv, ctx->dWeakNoff, N_up, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  return OSV_OK;
}

int osv_high_order_correction(osv_ctx *ctx, hipStream_t s, double *dE, double *E_coll, double *max_dR,
                              double *per_domain) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!dE) return fail(ctx, OSV_E_ARG, "dE is NULL");
  if (!ctx->solved) return fail(ctx, OSV_E_STATE, "osv_high_order_correction before a converged solve");
  int rc;
  densities_host(ctx);
  if (!ctx->dDptr && (rc = upload_density_tables(ctx, s))) return rc;
  if (!ctx->hc_ready && (rc = build_correction(ctx, s))) return rc;
  Plan &P = ctx->plan;
  const int ndom = (int)P.doms.size();
  StageTimer t_col(s);
  HIPCHK(ctx, launch_collective(ctx->dDom, ndom, ctx->dAdjOrder, ctx->dDptr, ctx->dDtoff, ctx->dDcoef, ctx->dT, ctx->dCoff,
                                ctx->dTc, s));
  t_col.stop();
  StageTimer t_step(s);
  HIPCHK(ctx, launch_collective_step(ctx->dDom, ndom, ctx->dRank, ctx->dCtptr, ctx->dCterms, ctx->dTc,
                                     ctx->dCoff, ctx->dM, ctx->dKt, ctx->F, ctx->nocc, ctx->dHcQueue,
                                     ctx->dHcCounter, ctx->dHcScr, ctx->hc_nwg, ctx->dHcOut, s));
  t_step.stop();
  std::vector<double> h((size_t)3 * ndom);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), ctx->dHcOut, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  ctx->hc_ms[0] = t_col.ms();
  ctx->hc_ms[1] = t_step.ms();
  double a = 0.0, b = 0.0, m = 0.0;
  for (int d = 0; d < ndom; d++) {
    a += h[3 * d];
    b += h[3 * d + 1];
    m = std::max(m, std::sqrt(h[3 * d + 2]));
  }
  *dE = a;
  if (E_coll) *E_coll = b;
  if (max_dR) *max_dR = m;
  if (per_domain)
    for (int d = 0; d < ndom; d++) {
      per_domain[3 * d] = h[3 * d];
      per_domain[3 * d + 1] = h[3 * d + 1];
      per_domain[3 * d + 2] = std::sqrt(h[3 * d + 2]);
    }
  return OSV_OK;
}

int osv_correction_stats(const osv_ctx *ctx, double *out4) {
  if (!ctx || !out4) return fail(nullptr, OSV_E_ARG, "osv_correction_stats: NULL argument");
  out4[0] = ctx->hc_ms[0];
  out4[1] = ctx->hc_bytes;
  out4[2] = ctx->hc_ms[1];
  out4[3] = ctx->hc_flops;
  return OSV_OK;
}

int osv_densities(osv_ctx *ctx, hipStream_t s, double *dE_dC, double *dE_dFocc, double *dE_deps,
                  double *Dvir_full) {
  if (!ctx) return fail(nullptr, OSV_E_ARG, "ctx is NULL");
  if (!ctx->solved) return fail(ctx, OSV_E_STATE, "osv_densities before a converged solve");
  if (dE_dC && ctx->k_exact)
    return fail(ctx, OSV_E_ARG, "osv_densities: no dE/dC with cross-projected integrals (E depends on B)");
  int rc = prepare_densities(ctx, s);
  if (rc) return rc;
  Plan &P = ctx->plan;
  const int ndom = (int)P.doms.size(), N = ctx->nosv;
  const long long ld = N;
  StageTimer t_adj(s);
  HIPCHK(ctx, launch_adjoint(ctx->dDom, ndom, ctx->dAdjOrder, ctx->dRank, ctx->dW, ctx->dY, ctx->dT, ctx->dDptr, ctx->dDtoff,
                             ctx->dDcoef, ctx->dGK, ld, ctx->dGd, s));
  HIPCHK(ctx, launch_assemble_gf(ctx->dDom, ctx->dBptr, ctx->dBdom, ctx->dBpart, ctx->dBlocks, ctx->nblocks,
                                 ctx->dOff, ctx->dR, ctx->dGd, ctx->dGF, ld, s));
  const int nweak = (int)ctx->weak.size();
  // the weak pairs' G^K (i, j) blocks and G^F diagonal blocks
  HIPCHK(ctx, launch_weak_densities(nweak, ctx->nocc, ctx->dWeakLmo, ctx->dOff, ctx->dR, ctx->dWeakToff,
                                    ctx->dWeakT, ctx->dWeakTT, ctx->dWeakLptr, ctx->dWeakLidx, ctx->dGK,
                                    ctx->dGF, ld, nullptr, s));
  t_adj.stop();
  StageTimer t_bt(s);
  if (dE_dC) {
    if (ctx->precision == OSV_MIXED && ctx->c_dtype == OSV_DT_F32 && N <= digit_max_k()) {
      // mixed precision: dE/dC = 2 G^K C from exact int8 digits, as K: the rows of
      // G^K and of C^T (one per auxiliary function) each split into six 7-bit
      // digits with their own power-of-two scale, products summed in int32 per
      // digit level; what is left out is below 2^-42 of each row's scale
      const int naux = ctx->naux;
      if (!ctx->dCt) {
        if ((rc = dalloc(ctx, &ctx->dCt, (size_t)naux * N))) return rc;
        if ((rc = dalloc(ctx, &ctx->dDigCt, digit_bytes(naux, N)))) return rc;
        if ((rc = dalloc(ctx, &ctx->dExpCt, naux))) return rc;
        if (!ctx->dDigG && (rc = dalloc(ctx, &ctx->dDigG, digit_bytes(N, N)))) return rc;
        if (!ctx->dExpG && (rc = dalloc(ctx, &ctx->dExpG, N))) return rc;
      }
      HIPCHK(ctx, launch_transpose_f32((const float *)ctx->C, N, naux, ctx->dCt, s));
      HIPCHK(ctx, launch_split_digits(ctx->dCt, naux, N, ctx->dExpCt, ctx->dDigCt, s));
      HIPCHK(ctx, launch_split_digits_f64(ctx->dGK, ld, N, N, ctx->dExpG, ctx->dDigG, s));
      HIPCHK(ctx, launch_gemm_digits(ctx->dDigG, N, ctx->dDigCt, naux, N, ctx->dExpG, ctx->dExpCt, 1,
                                     dE_dC, naux, s));
    } else {
      const double *Cd = (const double *)ctx->C;
      if (ctx->c_dtype == OSV_DT_F32) {
        if ((rc = c64(ctx, s))) return rc;
        Cd = ctx->dC64;
      }
      HIPCHK(ctx, launch_gemm_nn_f64(ctx->dGK, ld, Cd, 0, ctx->naux, dE_dC, ctx->naux, N, ctx->naux, N, 2.0, s));
    }
  }
  if (dE_deps || Dvir_full) {
    // Z^T = G^F Q^T  (Q^T is row-major sum(r) x nvir)
    if (ctx->precision == OSV_MIXED && N <= digit_max_k()) {
      // mixed precision: from six-digit splits of the rows of G^F and of Q (one per
      // virtual), as dE/dC; below 2^-42 of each row's scale is left out
      const int nvir = ctx->nvir;
      if (!ctx->dQn) {
        if ((rc = dalloc(ctx, &ctx->dQn, (size_t)nvir * N))) return rc;
        if ((rc = dalloc(ctx, &ctx->dDigQ, digit_bytes(nvir, N)))) return rc;
        if ((rc = dalloc(ctx, &ctx->dExpQ, nvir))) return rc;
        if (!ctx->dDigG && (rc = dalloc(ctx, &ctx->dDigG, digit_bytes(N, N)))) return rc;
        if (!ctx->dExpG && (rc = dalloc(ctx, &ctx->dExpG, N))) return rc;
      }
      HIPCHK(ctx, launch_transpose_f64(ctx->Q, N, nvir, ctx->dQn, s));
      HIPCHK(ctx, launch_split_digits_f64(ctx->dQn, N, nvir, N, ctx->dExpQ, ctx->dDigQ, s));
      HIPCHK(ctx, launch_split_digits_f64(ctx->dGF, ld, N, N, ctx->dExpG, ctx->dDigG, s));
      HIPCHK(ctx, launch_gemm_digits(ctx->dDigG, N, ctx->dDigQ, nvir, N, ctx->dExpG, ctx->dExpQ, 0,
                                     ctx->dZt, nvir, s));
    } else {
      HIPCHK(ctx, launch_gemm_nn_f64(ctx->dGF, ld, ctx->Q, 0, ctx->nvir, ctx->dZt, ctx->nvir, N, ctx->nvir, N,
                                     1.0, s));
    }
    if (dE_deps) HIPCHK(ctx, launch_coldot(ctx->Q, ctx->dZt, N, ctx->nvir, ctx->dColPart, dE_deps, s));
    if (Dvir_full)
      HIPCHK(ctx, launch_gemm_tn_f64(ctx->Q, ctx->nvir, ctx->dZt, ctx->nvir, Dvir_full, ctx->nvir, ctx->nvir,
                                     ctx->nvir, N, 1.0, s));
  }
  if (dE_dFocc) {
    HIPCHK(ctx, launch_pocc(ctx->dPptr, ctx->dPidx, ctx->dClcoef, ctx->dPl, ctx->nocc, dE_dFocc, s));
    HIPCHK(ctx, launch_weak_densities(nweak, ctx->nocc, ctx->dWeakLmo, ctx->dOff, ctx->dR, ctx->dWeakToff,
                                      ctx->dWeakT, ctx->dWeakTT, ctx->dWeakLptr, ctx->dWeakLidx, nullptr,
                                      nullptr, ld, dE_dFocc, s));
  }
  t_bt.stop();
  HIPCHK(ctx, hipStreamSynchronize(s));
  ctx->stage_ms[6] = t_adj.ms();
  ctx->stage_ms[7] = t_bt.ms();
  {
    double fa = 0, fb = 0;
    const Selection &S = ctx->sel;
    std::vector<int> nent(ndom, 0);
    for (size_t X = 0; X < P.cls.size(); X++) {
      if (S.coef[X] == 0.0) continue;
      for (int c = P.cls[X].cp0; c < P.cls[X].cp0 + P.cls[X].ncp; c++) nent[P.cps[c].dom]++;
    }
    for (int d = 0; d < ndom; d++) {
      const Domain &D = P.doms[d];
      double dt = ctx->rank_host[d], n = D.n, rp = D.rp, rq = (D.p == D.q) ? D.rp : D.rq;
      fa += nent[d] * 4.0 * dt * dt * dt + 2.0 * n * dt * dt + 2.0 * n * n * dt + 2.0 * dt * dt * rq +
            2.0 * rp * dt * rq;
      double mult = (D.p == D.q) ? 1.0 : 2.0;
      if (dE_dC) fb += mult * 2.0 * rp * rq * ctx->naux;
      if (dE_deps || Dvir_full) fb += mult * 2.0 * rp * rq * ctx->nvir;
    }
    if (dE_deps) fb += 2.0 * N * ctx->nvir;
    if (Dvir_full) fb += 2.0 * (double)ctx->nvir * ctx->nvir * N;
    ctx->stage_flops[6] = fa;
    ctx->stage_flops[7] = fb;
  }
  return OSV_OK;
}

int osv_stage_times(const osv_ctx *ctx, double *ms9) {
  if (!ctx || !ms9) return fail(nullptr, OSV_E_ARG, "osv_stage_times: NULL argument");
  for (int i = 0; i < 9; i++) ms9[i] = ctx->stage_ms[i];
  return OSV_OK;
}

int osv_stage_flops(const osv_ctx *ctx, double *f9) {
  if (!ctx || !f9) return fail(nullptr, OSV_E_ARG, "osv_stage_flops: NULL argument");
  count_flops(const_cast<osv_ctx *>(ctx));   // build-stage counts if no solve has run yet
  for (int i = 0; i < 9; i++) f9[i] = ctx->stage_flops[i];
  return OSV_OK;
}

void osv_destroy(osv_ctx *ctx) { delete ctx; }

int osv_release_cached_memory(int32_t device) {
  if (device < -1) return fail(nullptr, OSV_E_ARG, "device must be >= -1");
  pool_release(device);
  return OSV_OK;
}

int64_t osv_cached_bytes(int32_t device) { return (int64_t)pool_cached_bytes(device); }

int osv_set_tuning(const char *key, int32_t value) {
  if (!key) return fail(nullptr, OSV_E_ARG, "osv_set_tuning: key is NULL");
  (void)tuning();
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  if (!tuning_set(key, value))
    return fail(nullptr, OSV_E_ARG, std::string("osv_set_tuning: unknown key or value ") + key + " " +
                                        std::to_string(value));
  return OSV_OK;
}

int osv_get_tuning(const char *key, int32_t *value) {
  if (!key || !value) return fail(nullptr, OSV_E_ARG, "osv_get_tuning: NULL argument");
  (void)tuning();
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  int v = 0;
  if (!tuning_get(key, &v)) return fail(nullptr, OSV_E_ARG, std::string("osv_get_tuning: unknown key ") + key);
  *value = v;
  return OSV_OK;
}

int osv_load_tuning(const char *path) {
  if (!path) return fail(nullptr, OSV_E_ARG, "osv_load_tuning: path is NULL");
  (void)tuning();
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  const int n = tuning_read(path);
  if (n == -1) return fail(nullptr, OSV_E_ARG, std::string("osv_load_tuning: cannot read ") + path);
  if (n == -2) return fail(nullptr, OSV_E_ARG, std::string("osv_load_tuning: bad entry in ") + path);
  return OSV_OK;
}

}  // extern "C"
