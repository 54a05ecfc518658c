// OSV response intermediate N_ij (eq:nij) and its MBE (eq:nmbeii / eq:nmbeij
// written with the inclusion-exclusion coefficients), for every ordered pair of
// the strong clusters, in the composite OSV basis of the pair.
//
// In the pseudo-canonical basis W of a pair domain d = [pq] (W^T S_dd W = 1,
// W^T F_dd W = diag(e~)) the cluster amplitudes are T = W t W^T, Tbar = W tb W^T
// with tb = 2t - t^T, and every term of eq:nij takes the form W (.) R with a
// right factor R that does not depend on the cluster:
//   Tbar K_d                     = W tb (W^T K_d)
//   D_(d,d) F_dd                 = W 1/2 (tb t + tb^T t^T) (W^T F_dd)
//   D'_(d,d) S_dd                = W 1/2 (tb e~ t + tb^T e~ t^T) Y,      Y = W^T S_dd
//   f D_(d,e) S_(e,d)            = W 1/2 (tb P + tb^T P') W_e^T S_(e,d)
// with P = M(d,e) op(t_e), P' = M(d,e) op(t_e)^T, M(d,e) = W^T S_(d,e) W_e the
// coupling of the residual, op the orientation of the source pair.  The k-sum
// terms are the residual's own terms (the same sources and coefficients -f);
// the two with e = d (k = q in the first sum, k = p in the second) join the
// D' term as the factor (e~ - f_pp - f_qq).  Summed over the clusters X holding
// the pair with their coefficients c_X, the cluster-dependent left factors
// accumulate in dt x dt matrices (G_K, G_F, G_Y) and, for the k-sums, in one
// dt x r_x block per LMO x that the sums reach (W_e^T S_(e,d) is the stack of
// the source's LMO rows); the right factors are applied once per pair:
//   N_pq = W [ G_K Y_p K_pq S_(q,d) + G_F W^T F_dd + G_Y Y + sum_x B_x S_(x,d) ].
// The reversed pair (q, p) has Tbar^T in place of Tbar and the same D terms, so
// in the basis [pq] it differs only in its integral term, G_K^T Y_q K_qp S_(p,d);
// its result is written in the basis [qp].
//
// For a diagonal target (p, p) the sum-1 term of source (p, m) and the sum-2 term
// of (m, p) have the same source slots and (when f_mp == f_pm, which the host
// checks) the same coefficient; together they are (tb + tb^T) M (t_e + t_e^T),
// one product instead of two.
//
// One persistent eight-wave workgroup per CU takes target domains from a work
// queue (largest cost first).  The per-cluster products run on the LDS-staged
// FP64 MFMA tile product (gemm_lds); their operands are the amplitude, coupling
// and W slots and per-workgroup scratch (the cluster's [tb | tb^T] and
// [t, (e~ - f) t ; t^T, (e~ - f) t^T], the products P, P', Z, the accumulators).
// The final per-domain products use register-fed tiles (mma_tiles).
#include "osv_internal.h"
#include "tiles.h"

namespace osv {

constexpr int NNT = 512;       // threads per workgroup (8 waves)
constexpr int NLD = 112;       // row stride of the dt-row work matrices (np <= 112)
constexpr int NLD2 = 2 * NLD;  // row stride of [P | P']

long long nij_scratch_doubles(int lb_max) {
  return 10LL * NLD * NLD + 2LL * NLD * NLD2 + (long long)NLD2 * NLD2 + (long long)NLD * lb_max;
}

__global__ __launch_bounds__(NNT) void k_nij(NijArgs a) {
  __shared__ int s_next;
  __shared__ __align__(16) double lds[gemm_lds_doubles()];
  const int tid = threadIdx.x;
  double *GK = a.scr + (long long)blockIdx.x * a.scr_stride;
  double *GF = GK + NLD * NLD, *GY = GF + NLD * NLD, *Z = GY + NLD * NLD, *A = Z + NLD * NLD;
  double *AR = A + NLD * NLD, *H1 = AR + NLD * NLD, *X1 = H1 + NLD * NLD, *X2 = X1 + NLD * NLD;
  double *TS = X2 + NLD * NLD, *PP = TS + NLD * NLD, *TB = PP + NLD * NLD2, *BFY = TB + NLD * NLD2;
  double *B = BFY + NLD2 * NLD2;
  for (;;) {
    if (tid == 0) s_next = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = s_next;
    __syncthreads();
    if (it >= a.ntg) break;
    const NijTarget tg = a.tg[it];
    const Domain D = a.dom[tg.dom];
    const int n = D.n, dt = a.rank[tg.dom], np = D.np, rp = D.rp;
    const bool diag = D.p == D.q;
    const int rq = diag ? rp : D.rq;          // columns of K_pq (K_pp for p == q)
    const int offq = diag ? D.offp : D.offq;
    const int lb = tg.lb;
    const long long ld = a.ld;
    const double *W = a.W + D.moff, *Y = a.Y + D.moff;
    const double *ev = a.Kep + D.voff + (long long)np * np;
    const double fs = a.F_occ[(long long)D.p * a.nocc + D.p] + a.F_occ[(long long)D.q * a.nocc + D.q];
    // S_(x,d)(k, j): rows of LMO x (global OSV offset ox), columns of the domain
    auto sxd = [&](int x, int ox, int k, int j) -> double {
      const bool inp = j < rp;
      const int y = inp ? D.p : D.q, jj = inp ? j : j - rp, oy = inp ? D.offp : D.offq;
      if (y == x) return k == jj ? 1.0 : 0.0;
      return a.S[(long long)(ox + k) * ld + oy + jj];
    };
    for (int e = tid; e < dt * NLD; e += NNT) {
      GK[e] = 0.0;
      GF[e] = 0.0;
      GY[e] = 0.0;
    }
    for (long long e = tid; e < (long long)dt * lb; e += NNT) B[e] = 0.0;
    __syncthreads();
    for (long long en = tg.ent0; en < tg.ent1; en++) {
      const CPair cp = a.cp[a.ent_cp[en]];
      const double c = a.ent_c[en];
      const double *t = a.T + cp.toff, *tT = t + (long long)np * np;
      // TB = [tb | tb^T] (dt x 2dt); BFY = [t, (e~ - f) t ; t^T, (e~ - f) t^T] (2dt x 2dt)
      for (int e = tid; e < dt * dt; e += NNT) {
        const int i = e / dt, k = e - i * dt;
        const double x = t[i * np + k], xT = tT[i * np + k];
        const double tb = 2.0 * x - xT, w = ev[i] - fs;
        GK[i * NLD + k] += c * tb;
        TS[i * NLD + k] = x + xT;   // tb + tb^T
        TB[i * NLD2 + k] = tb;
        TB[i * NLD2 + dt + k] = 2.0 * xT - x;
        BFY[i * NLD2 + k] = x;
        BFY[i * NLD2 + dt + k] = w * x;
        BFY[(dt + i) * NLD2 + k] = xT;
        BFY[(dt + i) * NLD2 + dt + k] = w * xT;
      }
      __syncthreads();
      // G_F += c/2 TB [t ; t^T],  G_Y += c/2 TB [(e~ - f) t ; (e~ - f) t^T]
      const Mat tbm{TB, NLD2, 0};
      gemm_lds<NNT>(dt, dt, 2 * dt, tbm, Mat{BFY, NLD2, 0}, lds,
                    [&](int i, int j, double v) { GF[i * NLD + j] += 0.5 * c * v; });
      gemm_lds<NNT>(dt, dt, 2 * dt, tbm, Mat{BFY + dt, NLD2, 0}, lds,
                    [&](int i, int j, double v) { GY[i * NLD + j] += 0.5 * c * v; });
      for (int tt = cp.term0; tt < cp.term0 + cp.nterm; tt++) {
        const int mate = a.tmate[tt];
        if (mate < -1) continue;   // taken with its sum-1 partner
        const TermFlat f = a.tflat[tt];
        const int flags = a.terms[tt].flags;
        const Domain E = a.dom[a.cp[a.terms[tt].src].dom];
        const int2 bc = a.bcol[tt];
        const int ns = f.ns, ldT = f.ldT, ldM = f.ldM;
        const double *op = a.T + f.tsrc;
        const double *opT = (flags & 2) ? op - (long long)ldT * ldT : op + (long long)ldT * ldT;
        const Mat mt{a.M + f.moff, ldM, 1};   // M(tgt, src) (M(src, tgt) is stored)
        if (mate >= 0) {
          // diagonal target: the terms of source (p, m) and (m, p) with equal
          // coefficients add up to (tb + tb^T) M(tgt, src) (t_e + t_e^T)
          gemm_lds<NNT>(dt, ns, ns, mt, Mat{op, ldT, 0, opT}, lds,
                        [&](int i, int j, double v) { PP[i * NLD + j] = v; });
          __syncthreads();
          gemm_lds<NNT>(dt, ns, dt, Mat{TS, NLD, 0}, Mat{PP, NLD, 0}, lds,
                        [&](int i, int j, double v) { Z[i * NLD + j] = v; });
        } else {
          // [P ; P'] = [M(tgt, src) op(t_e) ; M(tgt, src) op(t_e)^T]
          gemm_lds<NNT>(dt, ns, ns, mt, Mat{op, ldT, 0}, lds,
                        [&](int i, int j, double v) { PP[i * NLD + j] = v; });
          gemm_lds<NNT>(dt, ns, ns, mt, Mat{opT, ldT, 0}, lds,
                        [&](int i, int j, double v) { PP[(dt + i) * NLD + j] = v; });
          __syncthreads();
          // Z = tb P + tb^T P'
          gemm_lds<NNT>(dt, ns, 2 * dt, tbm, Mat{PP, NLD, 0}, lds,
                        [&](int i, int j, double v) { Z[i * NLD + j] = v; });
        }
        __syncthreads();
        // the source's LMO blocks of B += (c (-f) / 2) Z W_e^T
        const double sc = 0.5 * c * f.coef;
        const int rpe = E.rp;
        gemm_lds<NNT>(dt, E.n, ns, Mat{Z, NLD, 0}, Mat{a.W + E.moff, E.n, 1}, lds,
                      [&](int i, int j, double v) {
                        const int col = j < rpe ? bc.x + j : bc.y + j - rpe;
                        B[(long long)i * lb + col] += sc * v;
                      });
      }
    }
    __syncthreads();
    // H1 = G_F W^T, X1 = G_K Y_p, X2 = G_K^T Y_q
    mma_tiles<NNT>(dt, n, dt, [&](int i, int k) { return GF[i * NLD + k]; },
                   [&](int k, int j) { return W[j * n + k]; },
                   [&](int i, int j, double v) { H1[i * NLD + j] = v; });
    mma_tiles<NNT>(dt, rp, dt, [&](int i, int k) { return GK[i * NLD + k]; },
                   [&](int k, int j) { return Y[k * n + j]; },
                   [&](int i, int j, double v) { X1[i * NLD + j] = v; });
    if (!diag)
      mma_tiles<NNT>(dt, rq, dt, [&](int i, int k) { return GK[k * NLD + i]; },
                     [&](int k, int j) { return Y[k * n + rp + j]; },
                     [&](int i, int j, double v) { X2[i * NLD + j] = v; });
    __syncthreads();
    // KF = X1 K_pq (dt x rq) and KR = X2 K_qp (dt x rp), side by side in PP
    mma_tiles<NNT>(dt, rq, rp, [&](int i, int k) { return X1[i * NLD + k]; },
                   [&](int k, int j) { return a.K[(long long)(D.offp + k) * ld + offq + j]; },
                   [&](int i, int j, double v) { PP[i * NLD2 + j] = v; });
    if (!diag)
      mma_tiles<NNT>(dt, rp, rq, [&](int i, int k) { return X2[i * NLD + k]; },
                     [&](int k, int j) { return a.K[(long long)(D.offp + j) * ld + offq + k]; },
                     [&](int i, int j, double v) { PP[i * NLD2 + NLD + j] = v; });
    __syncthreads();
    // A = G_Y Y + H1 F_dd + sum_x B_x S_(x,d)   (every call tiles dt x n alike, so
    // each element of A stays with one lane and needs no barrier between calls)
    mma_tiles<NNT>(dt, n, dt + n, [&](int i, int k) { return k < dt ? GY[i * NLD + k] : H1[i * NLD + k - dt]; },
                   [&](int k, int j) {
                     return k < dt ? Y[k * n + j] : comp_elem(a.F, ld, D, D, k - dt, j, false);
                   },
                   [&](int i, int j, double v) { A[i * NLD + j] = v; });
    for (int l = 0; l < tg.nlmo; l++) {
      const int2 xb = a.lmo_tab[tg.lmo0 + l];
      const int x = xb.x, bo = xb.y, rx = a.r[x], ox = a.off[x];
      mma_tiles<NNT>(dt, n, rx, [&](int i, int k) { return B[(long long)i * lb + bo + k]; },
                     [&](int k, int j) { return sxd(x, ox, k, j); },
                     [&](int i, int j, double v) { A[i * NLD + j] += v; });
    }
    // A_R = A + KR S_(p,d);  A_F = A + KF S_(q,d)
    if (!diag)
      mma_tiles<NNT>(dt, n, rp, [&](int i, int k) { return PP[i * NLD2 + NLD + k]; },
                     [&](int k, int j) { return sxd(D.p, D.offp, k, j); },
                     [&](int i, int j, double v) { AR[i * NLD + j] = A[i * NLD + j] + v; });
    mma_tiles<NNT>(dt, n, rq, [&](int i, int k) { return PP[i * NLD2 + k]; },
                   [&](int k, int j) { return sxd(diag ? D.p : D.q, offq, k, j); },
                   [&](int i, int j, double v) { A[i * NLD + j] += v; });
    __syncthreads();
    // N_pq = W A_F;  N_qp = W A_R with rows and columns in the order [Q_q Q_p]
    double *NF = a.N + tg.outF;
    mma_tiles<NNT>(n, n, dt, [&](int i, int k) { return W[i * n + k]; },
                   [&](int k, int j) { return A[k * NLD + j]; },
                   [&](int i, int j, double v) { NF[i * n + j] = v; });
    if (!diag) {
      double *NR = a.N + tg.outR;
      const int rqq = D.rq;
      mma_tiles<NNT>(n, n, dt, [&](int i, int k) { return W[i * n + k]; },
                     [&](int k, int j) { return AR[k * NLD + j]; },
                     [&](int i, int j, double v) {
                       const int u = i < rp ? i + rqq : i - rp, w = j < rp ? j + rqq : j - rp;
                       NR[u * n + w] = v;
                     });
    }
    __syncthreads();
  }
}

// Weak pairs (one-block scheme): N^up_ij = T_(i,j) K_(j,i) (r_i x r_i), one
// workgroup per pair; T is the pair's one-block amplitude in the OSV bases
// (r_i x r_j row-major at toff[w]); K_(j,i) is read as the transpose of the
// K_(i,j) block.
__global__ __launch_bounds__(256) void k_weak_nup(const int2 *__restrict__ lmo, const int *__restrict__ off,
                                                  const int *__restrict__ r, const long long *__restrict__ toff,
                                                  const double *__restrict__ T, const double *__restrict__ K,
                                                  long long ld, const long long *__restrict__ noff, double *N) {
  const int w = blockIdx.x;
  const int i = lmo[w].x, j = lmo[w].y;
  const int ri = r[i], rj = r[j], oi = off[i], oj = off[j];
  const double *Tw = T + toff[w];
  double *out = N + noff[w];
  mma_tiles<256>(ri, ri, rj, [&](int a, int k) { return Tw[a * rj + k]; },
                 [&](int k, int b) { return K[(long long)(oi + b) * ld + oj + k]; },
                 [&](int a, int b, double v) { out[a * ri + b] = v; });
}

hipError_t launch_weak_nup(const int2 *lmo, int nweak, const int *off, const int *r, const long long *toff,
                           const double *T, const double *K, long long ld, const long long *noff, double *N,
                           hipStream_t s) {
  if (nweak <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weak_nup, dim3(nweak), dim3(256), 0, s, lmo, off, r, toff, T, K, ld, noff, N);
  return hipGetLastError();
}

hipError_t launch_nij(const NijArgs &a, int nwg, hipStream_t s) {
  if (a.ntg <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(a.counter, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nij, dim3(nwg), dim3(NNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace osv
