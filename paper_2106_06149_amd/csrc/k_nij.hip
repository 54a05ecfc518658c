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
// One persistent workgroup per target domain at a time (work queue in cost
// order); the products run on FP64 MFMA 16x16x4 tiles whose operands are read
// from the amplitude, coupling and W slots and from per-workgroup scratch.
#include "osv_internal.h"
#include "tiles.h"

namespace osv {

constexpr int NNT = 256;       // threads per workgroup
constexpr int NLD = 112;       // row stride of the dt-row work matrices (np <= 112)
constexpr int NLD2 = 2 * NLD;  // row stride of [P | P']

long long nij_scratch_doubles(int lb_max) {
  return 9LL * NLD * NLD + (long long)NLD * NLD2 + (long long)NLD * lb_max;
}

__global__ __launch_bounds__(NNT) void k_nij(NijArgs a) {
  __shared__ int s_next;
  const int tid = threadIdx.x;
  double *GK = a.scr + (long long)blockIdx.x * a.scr_stride;
  double *GF = GK + NLD * NLD, *GY = GF + NLD * NLD, *Z = GY + NLD * NLD, *A = Z + NLD * NLD;
  double *AR = A + NLD * NLD, *H1 = AR + NLD * NLD, *X1 = H1 + NLD * NLD, *X2 = X1 + NLD * NLD;
  double *PP = X2 + NLD * NLD, *B = PP + NLD * NLD2;
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
      // [tb | tb^T](i, k)
      auto tbb = [&](int i, int k) -> double {
        return k < dt ? 2.0 * t[i * np + k] - tT[i * np + k]
                      : 2.0 * tT[i * np + k - dt] - t[i * np + k - dt];
      };
      for (int e = tid; e < dt * dt; e += NNT) {
        const int i = e / dt, k = e - i * dt;
        GK[i * NLD + k] += c * (2.0 * t[i * np + k] - tT[i * np + k]);
      }
      // [G_F | G_Y] += c/2 [tb | tb^T] [t, (e~ - f) t ; t^T, (e~ - f) t^T]
      mma_tiles<NNT>(dt, 2 * dt, 2 * dt, tbb,
                     [&](int k, int j) -> double {
                       const int kk = k < dt ? k : k - dt;
                       const double *src = k < dt ? t : tT;
                       return j < dt ? src[kk * np + j] : (ev[kk] - fs) * src[kk * np + j - dt];
                     },
                     [&](int i, int j, double v) {
                       if (j < dt) GF[i * NLD + j] += 0.5 * c * v;
                       else GY[i * NLD + j - dt] += 0.5 * c * v;
                     });
      for (int tt = cp.term0; tt < cp.term0 + cp.nterm; tt++) {
        const TermFlat f = a.tflat[tt];
        const int flags = a.terms[tt].flags;
        const Domain E = a.dom[a.cp[a.terms[tt].src].dom];
        const int2 bc = a.bcol[tt];
        const int ns = f.ns, ldT = f.ldT, ldM = f.ldM;
        const double *op = a.T + f.tsrc;
        const double *opT = (flags & 2) ? op - (long long)ldT * ldT : op + (long long)ldT * ldT;
        const double *Mst = a.M + f.moff;   // M(src, tgt), np_src x np_tgt
        // [P | P'] = M(tgt, src) [op(t_e) | op(t_e)^T]
        mma_tiles<NNT>(dt, 2 * ns, ns, [&](int i, int k) { return Mst[k * ldM + i]; },
                       [&](int k, int j) { return j < ns ? op[k * ldT + j] : opT[k * ldT + j - ns]; },
                       [&](int i, int j, double v) { PP[i * NLD2 + j] = v; });
        __syncthreads();
        // Z = tb P + tb^T P'
        mma_tiles<NNT>(dt, ns, 2 * dt, tbb,
                       [&](int k, int j) { return k < dt ? PP[k * NLD2 + j] : PP[(k - dt) * NLD2 + ns + j]; },
                       [&](int i, int j, double v) { Z[i * NLD + j] = v; });
        __syncthreads();
        // the source's LMO blocks of B += (c (-f) / 2) Z W_e^T
        const double sc = 0.5 * c * f.coef;
        const double *We = a.W + E.moff;
        const int ne = E.n, rpe = E.rp;
        mma_tiles<NNT>(dt, ne, ns, [&](int i, int k) { return Z[i * NLD + k]; },
                       [&](int k, int j) { return We[j * ne + k]; },
                       [&](int i, int j, double v) {
                         const int col = j < rpe ? bc.x + j : bc.y + j - rpe;
                         B[(long long)i * lb + col] += sc * v;
                       });
        __syncthreads();
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

hipError_t launch_nij(const NijArgs &a, int nwg, hipStream_t s) {
  if (a.ntg <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(a.counter, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nij, dim3(nwg), dim3(NNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace osv
