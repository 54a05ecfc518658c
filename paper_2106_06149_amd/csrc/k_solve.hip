// Cluster residual solve: eq:rij for every pair of every cluster, Jacobi
// sweeps in each pair domain's pseudo-canonical basis, Hylleraas energy eq:ec.
//
// In the basis W of domain [pq] (W^T S W = 1, W^T F W = diag(e~)) the residual of
// the unordered pair p <= q of cluster X reads
//   R~_pq = K~_pq + (e~_a + e~_b - f_pp - f_qq) T~_pq
//         + sum_terms (-f_ab) M op(T~_src) M^T,     M = W_pq^T S_(pq,src) W_src,
// with one term per LMO m of X in each of the two k-sums of eq:rij, except the
// m = q (first sum) and m = p (second sum) terms, which are the diagonal factor.
// op is a transpose when the source pair is ordered (a, b) with a > b, because
// the canonical amplitudes satisfy T^{ba} = (T^{ab})^T.
//
// One workgroup (4 wave64, one per SIMD) owns one cluster at a time: it pops
// clusters from a cost-sorted queue, zeroes the cluster's amplitudes, and iterates
//   R~ from the current T~ for every pair; stop if max ||R~||_F < tau_R;
//   otherwise T~ <- T~ - R~ / (e~_a + e~_b - f_pp - f_qq)
// to convergence inside the kernel.  At the stopping sweep it records
//   E^X = sum_pairs w <2 T~ - T~^T, K~ + R~>       (eq:ec; w = 1 for p = q, 2 for p < q)
// and, in one more pass over the terms at the same amplitudes, the inner
// products <Tbar~_tgt, M op(T~_src) M^T> that make up dE/df_ab.
//
// A term Y = M op(T) M^T runs on FP64 MFMA 16x16x4 tiles.  Wave w owns the
// 16-wide target blocks i = w and i = w + 4: for each it forms the column block
// X'(:, i) of X' = op(T)^T M^T in registers, then Y^T(:, i) = M X'(:, i).  The f64
// MFMA accumulator layout (lane l, register v -> row 4v + (l >> 4), column l & 15)
// equals the B-operand layout of the k-rows 4v..4v+3, so X' (scaled by the term's
// coefficient) feeds the second product straight from registers, accumulating
// into R~ of the target, which stays in MFMA accumulators across its terms.
// M and op(T) stream through LDS in 16-wide chunks, double-buffered, with the
// next chunk's global loads issued into registers before the current chunk is
// multiplied.  Tbar~ of the target sits in LDS.
// Every reduction has a fixed order, so results are bitwise reproducible.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SNT = 256;        // threads per workgroup (4 wave64, one per SIMD)
constexpr int NW = SNT / 64;    // waves
constexpr int NS = 2;           // 16-wide target blocks per wave (blocks w, w + NW)
constexpr int MT = 7;           // 16-tiles per dimension covering DMAX = 100
constexpr int TLD = 16 * MT;    // 112: padded dimension
constexpr int KC = 16;          // chunk width (k or m)
constexpr int TPC = KC / 16;    // MFMA tiles per chunk
constexpr int MLD = KC + 1;     // LDS stride of M chunks (conflict-free column reads)

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// fixed-order block sums of NV values (red: NW * NV doubles)
template <int NV>
__device__ __forceinline__ void block_sums(double *v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; c++) {
    double x = wsum(v[c]);
    if (lane == 0) red[c * NW + wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; c++) {
    double t = 0.0;
    for (int w = 0; w < NW; w++) t += red[c * NW + w];
    v[c] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One LDS chunk of a term: pass 1 chunk c (c < nc1 = ceil(ns/KC)) holds
// op(T)(KC c .. KC c + KC-1, :) in Ts (row = m - KC c) and M(:, KC c ..) in Mc
// (col = m - KC c); pass 2 chunk c (nc1 <= c) holds M(:, KC(c-nc1) ..) in Mc.
// Each thread moves PF values of each part: it loads them from global memory
// into registers (prefetch) and later stores them into the LDS buffer (commit),
// so the next chunk's loads are in flight while the current one is multiplied.
// Thread-to-element maps use shifts only and keep KC- or 128-wide runs of
// threads on consecutive addresses for either storage order.
constexpr int PF = KC * 128 / SNT;  // values per thread and part

struct TermDesc {
  const double *T, *M;
  double coef;
  int ldT, ldM, trT, trM, ns, nkb, nc1;
};

__device__ __forceinline__ TermDesc term_desc(const SolveArgs &a, int t) {
  const TermFlat f = a.tflat[t];
  TermDesc d;
  d.T = a.T + f.tsrc;
  d.M = a.M + f.moff;
  d.coef = f.coef;
  d.ldT = f.ldT;
  d.ldM = f.ldM;
  d.trM = f.flags & 1;
  d.trT = (f.flags >> 1) & 1;
  d.ns = f.ns;
  d.nkb = (d.ns + 15) >> 4;
  d.nc1 = (d.ns + KC - 1) / KC;
  return d;
}

// element (row, col) of slot s in a KC x 128 (Ts part: chunk row, column) or
// 128 x KC (Mc part: matrix row, chunk column) tile; "wide" = 128 consecutive
// threads along the 128 side, otherwise KC consecutive threads along the KC side
__device__ __forceinline__ void slot_rc(int tid, int s, bool wide, bool ts_part, int &r, int &c) {
  constexpr int WS = SNT / 128, NSs = SNT / KC;  // slot strides of the two maps
  if (ts_part) {
    if (wide) { c = tid & 127; r = (tid >> 7) + WS * s; }
    else { r = tid % KC; c = tid / KC + NSs * s; }
  } else {
    if (wide) { r = tid & 127; c = (tid >> 7) + WS * s; }
    else { c = tid % KC; r = tid / KC + NSs * s; }
  }
}

__device__ __forceinline__ void prefetch(const TermDesc &d, int c, int nt, double *pt, double *pm) {
  const int tid = threadIdx.x;
  const bool p1 = c < d.nc1;
  const int col0 = KC * (p1 ? c : c - d.nc1);
  if (p1) {
    // op(T)(col0 + r, k): trT = 0 -> T[(col0 + r) ldT + k] (wide along k);
    //                     trT = 1 -> T[k ldT + col0 + r]  (32 along r)
#pragma unroll
    for (int s = 0; s < PF; s++) {
      int r, k;
      slot_rc(tid, s, !d.trT, true, r, k);
      const int m = col0 + r;
      double v = 0.0;
      if (m < d.ns && k < d.ns) v = d.trT ? d.T[k * d.ldT + m] : d.T[m * d.ldT + k];
      pt[s] = v;
    }
  }
  // M(i, col0 + cc): trM = 0 -> M[i ldM + col0 + cc] (32 along cc);
  //                  trM = 1 -> M[(col0 + cc) ldM + i] (wide along i)
#pragma unroll
  for (int s = 0; s < PF; s++) {
    int i, cc;
    slot_rc(tid, s, d.trM, false, i, cc);
    const int m = col0 + cc;
    double v = 0.0;
    if (i < nt && m < d.ns) v = d.trM ? d.M[m * d.ldM + i] : d.M[i * d.ldM + m];
    pm[s] = v;
  }
}

__device__ __forceinline__ void commit(const TermDesc &d, int c, double *Ts, double *Mc,
                                       const double *pt, const double *pm) {
  const int tid = threadIdx.x;
  if (c < d.nc1) {
#pragma unroll
    for (int s = 0; s < PF; s++) {
      int r, k;
      slot_rc(tid, s, !d.trT, true, r, k);
      if (k < TLD) Ts[r * TLD + k] = pt[s];
    }
  }
#pragma unroll
  for (int s = 0; s < PF; s++) {
    int i, cc;
    slot_rc(tid, s, d.trM, false, i, cc);
    if (i < TLD) Mc[i * MLD + cc] = pm[s];
  }
}

__global__ void k_term_flat(const Term *terms, long long nterms, const CPair *cp,
                            const Coupling *cpl, const Domain *dom, const int *rank,
                            const double *F_occ, int nocc, TermFlat *out) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nterms) return;
  const Term tm = terms[t];
  const CPair ps = cp[tm.src];
  const Coupling c = cpl[tm.cpl];
  TermFlat f;
  f.tsrc = ps.toff;
  f.moff = c.off;
  f.coef = -F_occ[tm.fa * nocc + tm.fb];
  f.ldT = dom[ps.dom].n;
  f.ldM = dom[c.B].n;
  f.ns = rank[ps.dom];
  f.flags = tm.flags;
  out[t] = f;
}

hipError_t launch_term_flat(const Term *terms, long long nterms, const CPair *cp,
                            const Coupling *cpl, const Domain *dom, const int *rank,
                            const double *F_occ, int nocc, TermFlat *out, hipStream_t s) {
  if (nterms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_term_flat, dim3((unsigned)((nterms + 255) / 256)), dim3(256), 0, s, terms,
                     nterms, cp, cpl, dom, rank, F_occ, nocc, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(SNT) void k_solve(SolveArgs a) {
  __shared__ double Ts[2][KC * TLD];
  __shared__ double Mc[2][TLD * MLD];
  __shared__ double Tb[TLD * TLD];  // Tbar~^T(j, i) = 2 T~(i,j) - T~(j,i) of the current target
  __shared__ double red[3 * NW];
  __shared__ int s_cur;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  double *Rs = a.Rs + (long long)blockIdx.x * a.rs_stride;
  for (;;) {
    if (tid == 0) s_cur = atomicAdd(a.counter, 1);
    __syncthreads();
    const int qi = s_cur;
    __syncthreads();
    if (qi >= a.n_clusters) break;
    const int X = a.queue[qi];
    const Cluster cl = a.cl[X];
    const int nl = cl.nlmo;
    double *Pl = a.Pl + cl.poff;
    for (int c = 0; c < cl.ncp; c++) {
      const CPair P = a.cp[cl.cp0 + c];
      const int n = a.dom[P.dom].n;
      double *T = a.T + P.toff;
      for (int e = tid; e < n * n; e += SNT) T[e] = 0.0;
    }
    __syncthreads();
    int sweep = 0, buf = 0;
    double maxn = 0.0, E = 0.0;
    bool pmode = false;  // after convergence: one pass for the dE/df inner products
    for (;;) {
      if (!pmode) {
        maxn = 0.0;
        E = 0.0;
        if (tid == 0)
          for (int e = 0; e < nl * nl; e++) Pl[e] = 0.0;
      }
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const Domain D = a.dom[P.dom];
        const int n = D.n, nt = a.dom_rank[P.dom];
        const double *T = a.T + P.toff;
        const double *Kt = a.Kt + D.moff;
        const double *ep = a.epst + D.voff;
        double *R = Rs + (P.toff - cl.toff0);
        const double fd = a.F_occ[D.p * a.nocc + D.p] + a.F_occ[D.q * a.nocc + D.q];
        const int njb = (nt + 15) >> 4;
        const int ipad = njb * 16;
        // Tbar~^T of the target into LDS (zero in the padding)
        for (int e = tid; e < ipad * ipad; e += SNT) {
          const int j = e / ipad, i = e - j * ipad;
          Tb[j * TLD + i] = (i < nt && j < nt) ? 2.0 * T[i * n + j] - T[j * n + i] : 0.0;
        }
        // coupling-term accumulators of R~^T(j, i): slot s holds target block
        // ib = wave + NW s, tile jb covers rows j = 16 jb + lhi + 4v, lane column
        // i = 16 ib + l15; K~ + Delta T~ is added when R~ is stored
        d4 Racc[NS][MT];
#pragma unroll
        for (int s = 0; s < NS; s++)
#pragma unroll
          for (int jb = 0; jb < MT; jb++) Racc[s][jb] = (d4){0, 0, 0, 0};
        __syncthreads();
        if ((sweep > 0 || pmode) && P.nterm > 0) {
          double pt[PF], pm[PF];
          TermDesc d = term_desc(a, P.term0);
          prefetch(d, 0, nt, pt, pm);
          for (int t = P.term0; t < P.term0 + P.nterm; t++) {
            // in the P pass each term is accumulated alone with unit weight
            const double coef = pmode ? 1.0 : d.coef;
            const bool has_next = (t + 1 < P.term0 + P.nterm);
            const TermDesc dn = has_next ? term_desc(a, t + 1) : d;
            const int nkb = d.nkb;
            if (pmode) {
#pragma unroll
              for (int s = 0; s < NS; s++)
#pragma unroll
                for (int jb = 0; jb < MT; jb++) Racc[s][jb] = (d4){0, 0, 0, 0};
            }
            // pass 1: X'(:, i-blocks) = op(T)^T M^T over m-chunks of KC
            d4 Xp[NS][MT];
#pragma unroll
            for (int s = 0; s < NS; s++)
#pragma unroll
              for (int kb = 0; kb < MT; kb++) Xp[s][kb] = (d4){0, 0, 0, 0};
            const int nc1 = d.nc1, nc2 = (nkb + TPC - 1) / TPC;
            for (int c = 0; c < nc1; c++) {
              commit(d, c, Ts[buf], Mc[buf], pt, pm);
              __syncthreads();
              prefetch(d, c + 1, nt, pt, pm);   // next pass-1 chunk or the first pass-2 chunk
              const double *ts = Ts[buf], *mc = Mc[buf];
              double bv[NS][KC / 4];
#pragma unroll
              for (int s = 0; s < NS; s++)
#pragma unroll
                for (int kk = 0; kk < KC / 4; kk++)
                  bv[s][kk] = mc[((wave + NW * s) * 16 + l15) * MLD + 4 * kk + lhi];
#pragma unroll
              for (int kb = 0; kb < MT; kb++) {
                if (kb < nkb) {
                  double av[KC / 4];
#pragma unroll
                  for (int kk = 0; kk < KC / 4; kk++) av[kk] = ts[(4 * kk + lhi) * TLD + kb * 16 + l15];
#pragma unroll
                  for (int s = 0; s < NS; s++)
                    if (wave + NW * s < njb)
#pragma unroll
                      for (int kk = 0; kk < KC / 4; kk++) Xp[s][kb] = mfma(av[kk], bv[s][kk], Xp[s][kb]);
                }
              }
              buf ^= 1;
            }
            // pass 2: R~^T(:, i-blocks) += coef M X'(:, i-blocks), TPC X' tiles per chunk;
            // the loop consumes Xp[.][0 .. TPC-1] and shifts the register arrays down
            for (int kc = 0; kc < nc2; kc++) {
              commit(d, nc1 + kc, Ts[buf], Mc[buf], pt, pm);
              __syncthreads();
              if (kc + 1 < nc2) prefetch(d, nc1 + kc + 1, nt, pt, pm);
              else if (has_next) prefetch(dn, 0, nt, pt, pm);
              const double *mc = Mc[buf];
              double bx[NS][KC / 4];
#pragma unroll
              for (int s = 0; s < NS; s++)
#pragma unroll
                for (int kk = 0; kk < KC / 4; kk++) bx[s][kk] = coef * Xp[s][kk >> 2][kk & 3];
#pragma unroll
              for (int jb = 0; jb < MT; jb++) {
                if (jb < njb) {
                  double av[KC / 4];
#pragma unroll
                  for (int kk = 0; kk < KC / 4; kk++) av[kk] = mc[(jb * 16 + l15) * MLD + 4 * kk + lhi];
#pragma unroll
                  for (int s = 0; s < NS; s++)
                    if (wave + NW * s < njb) {
#pragma unroll
                      for (int tt = 0; tt < TPC; tt++)
                        if (TPC * kc + tt < nkb)
#pragma unroll
                          for (int kk = 4 * tt; kk < 4 * tt + 4; kk++)
                            Racc[s][jb] = mfma(av[kk], bx[s][kk], Racc[s][jb]);
                    }
                }
              }
#pragma unroll
              for (int s = 0; s < NS; s++)
#pragma unroll
                for (int q = 0; q < MT - TPC; q++) Xp[s][q] = Xp[s][q + TPC];
              buf ^= 1;
            }
            if (pmode) {
              // <Tbar~_tgt, Y> (padded entries of Y and Tb are zero)
              double vs[1] = {0.0};
#pragma unroll
              for (int s = 0; s < NS; s++) {
                const int i = (wave + NW * s) * 16 + l15;
#pragma unroll
                for (int jb = 0; jb < MT; jb++) {
                  if (jb < njb) {
#pragma unroll
                    for (int v = 0; v < 4; v++) vs[0] += Tb[(jb * 16 + lhi + 4 * v) * TLD + i] * Racc[s][jb][v];
                  }
                }
              }
              block_sums<1>(vs, red);
              if (tid == 0) {
                const Term tm = a.terms[t];
                Pl[tm.la * nl + tm.lb] -= vs[0];
                if (P.la != P.lb) Pl[tm.lb * nl + tm.la] -= vs[0];
              }
            }
            d = dn;
          }
        }
        if (pmode) continue;
        // store R~ (transposed: R[j*n + i] = R~(i, j)); norm, energy, same-pair dE/df
        double sv[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < NS; s++) {
          const int i = (wave + NW * s) * 16 + l15;
#pragma unroll
          for (int jb = 0; jb < MT; jb++) {
            if (jb < njb) {
#pragma unroll
              for (int v = 0; v < 4; v++) {
                const int j = jb * 16 + lhi + 4 * v;
                if (i < nt && j < nt) {
                  const double kij = Kt[i * n + j];
                  const double tij = T[i * n + j];
                  const double r = Racc[s][jb][v] + kij + (ep[i] + ep[j] - fd) * tij;
                  const double tb = Tb[j * TLD + i];
                  R[j * n + i] = r;
                  sv[0] += r * r;
                  sv[1] += tb * (kij + r);
                  sv[2] += tb * tij;
                }
              }
            }
          }
        }
        block_sums<3>(sv, red);
        const double nrm = sqrt(sv[0]);
        maxn = (nrm > maxn || nrm != nrm) ? nrm : maxn;
        E += P.w * sv[1];
        if (tid == 0) {
          Pl[P.la * nl + P.la] -= 2.0 * sv[2];
          if (P.la != P.lb) Pl[P.lb * nl + P.lb] -= 2.0 * sv[2];
        }
      }
      if (pmode) break;
      if (maxn < a.tau_R || maxn != maxn || sweep >= a.max_sweeps) {
        pmode = true;  // amplitudes final: inner products of the terms at this T
        continue;
      }
      // Jacobi update of every pair of the cluster (R holds R~ transposed)
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const Domain D = a.dom[P.dom];
        const int n = D.n, nt = a.dom_rank[P.dom];
        double *T = a.T + P.toff;
        const double *ep = a.epst + D.voff;
        const double *R = Rs + (P.toff - cl.toff0);
        const double fd = a.F_occ[D.p * a.nocc + D.p] + a.F_occ[D.q * a.nocc + D.q];
        for (int e = tid; e < nt * nt; e += SNT) {
          const int j = e / nt, ii = e - j * nt;
          T[ii * n + j] -= R[j * n + ii] / (ep[ii] + ep[j] - fd);
        }
      }
      __syncthreads();
      sweep++;
    }
    if (tid == 0) {
      a.Ecl[X] = E;
      a.sweeps[X] = sweep;
      a.maxres[X] = maxn;
    }
    __syncthreads();
  }
}

hipError_t launch_solve(const SolveArgs &a, int nwg, hipStream_t s) {
  if (a.n_clusters <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve, dim3(nwg), dim3(SNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace osv
