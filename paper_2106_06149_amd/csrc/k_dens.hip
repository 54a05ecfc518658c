// Densities of the MBE energy (exact derivative at fixed Q, Hylleraas stationarity).
//
// Per pair domain d = [pq], over every cluster X that holds the pair (fixed
// cluster order), with c_X the MBE coefficient and T~ the cluster amplitudes in
// the domain's pseudo-canonical basis:
//   A_d = sum_X c_X Tbar~,            Tbar~ = 2 T~ - T~^T
//   g_d = sum_X c_X (T~^T Tbar~ + Tbar~ T~^T)
// Then
//   G^K_pq = Y_p^T (2 A_d) Y_q        (dE/dK_pq; dE/dC_p = sum_q (G^K_pq + G^K_qp^T) C_q)
//   G^F_d  = W (g_d + g_d^T) W^T      (p < q; W g_d W^T for p = q): the domain's part of
//            the virtual density in its composite OSV basis (cf. eq:dv, D_(ij,kl)).
// Every term is written by one workgroup in a fixed order: no atomics.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int LDA = DMAX + 1;

__global__ __launch_bounds__(NTHREADS) void k_adjoint(const Domain *__restrict__ doms,
                                                      const int *__restrict__ rank,
                                                      const double *__restrict__ W,
                                                      const double *__restrict__ Y,
                                                      const double *__restrict__ Tall,
                                                      const long long *__restrict__ dcp_ptr,
                                                      const long long *__restrict__ dcp_toff,
                                                      const double *__restrict__ dcp_coef,
                                                      double *GK, long long ld, double *Gd) {
  __shared__ double L1[DMAX * LDA];
  __shared__ double L2[DMAX * LDA];
  const int d = blockIdx.x;
  const Domain D = doms[d];
  const int n = D.n, np = D.np, dt = rank[d];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool diag = (D.p == D.q);
  for (int e = tid; e < dt * dt; e += NTHREADS) {
    int i = e / dt, j = e % dt;
    L1[i * LDA + j] = 0.0;
    L2[i * LDA + j] = 0.0;
  }
  __syncthreads();
  const int tn = (dt + 15) >> 4;
  for (long long en = dcp_ptr[d]; en < dcp_ptr[d + 1]; en++) {
    const double c = dcp_coef[en];
    const double *T = Tall + dcp_toff[en];
    for (int e = tid; e < dt * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      L1[i * LDA + j] += c * (2.0 * T[i * np + j] - T[j * np + i]);
    }
    // g tiles: T^T Tbar + Tbar T^T
    for (int tile = wave; tile < tn * tn; tile += 4) {
      const int i0 = (tile / tn) * 16, j0 = (tile % tn) * 16;
      const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
      d4 acc = {0, 0, 0, 0};
      for (int k0 = 0; k0 < dt; k0 += 4) {
        const int k = k0 + (lane >> 4);
        double a1 = 0, b1 = 0, a2 = 0, b2 = 0;
        if (ia < dt && k < dt) {
          a1 = T[k * np + ia];                                 // (T^T)(i,k)
          a2 = 2.0 * T[ia * np + k] - T[k * np + ia];          // Tbar(i,k)
        }
        if (jb < dt && k < dt) {
          b1 = 2.0 * T[k * np + jb] - T[jb * np + k];         // Tbar(k,j)
          b2 = T[jb * np + k];                                 // (T^T)(k,j)
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2, acc, 0, 0, 0);
      }
      for (int v = 0; v < 4; v++) {
        const int i = i0 + (lane >> 4) + 4 * v, j = j0 + (lane & 15);
        if (i < dt && j < dt) L2[i * LDA + j] += c * acc[v];
      }
    }
    __syncthreads();
  }
  // symmetrise g for p < q (both orderings of the pair contribute)
  if (!diag) {
    for (int e = tid; e < dt * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      if (i < j) {
        double s = L2[i * LDA + j] + L2[j * LDA + i];
        L2[i * LDA + j] = s;
        L2[j * LDA + i] = s;
      } else if (i == j) {
        L2[i * LDA + i] *= 2.0;
      }
    }
    __syncthreads();
  }
  // T2 = W g' (n x dt) -> global Gd slot
  const double *Wd = W + D.moff;
  double *G = Gd + D.moff;
  for (int e = tid; e < n * dt; e += NTHREADS) {
    int i = e / dt, j = e % dt;
    double s = 0.0;
    for (int k = 0; k < dt; k++) s += Wd[i * n + k] * L2[k * LDA + j];
    G[i * n + j] = s;
  }
  __syncthreads();
  // Gd = T2 W^T (n x n) -> L2, then global
  for (int e = tid; e < n * n; e += NTHREADS) {
    int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k < dt; k++) s += G[i * n + k] * Wd[j * n + k];
    L2[i * LDA + j] = s;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += NTHREADS) {
    int i = e / n, j = e % n;
    G[i * n + j] = L2[i * LDA + j];
  }
  __syncthreads();
  // G^K block: T1 = 2 A Y_q (dt x rq) -> L2 ; Gamma = Y_p^T T1 (rp x rq)
  const double *Yd = Y + D.moff;
  const int rq = diag ? D.rp : D.rq, qcol = diag ? 0 : D.rp, offq = diag ? D.offp : D.offq;
  for (int e = tid; e < dt * rq; e += NTHREADS) {
    int a = e / rq, j = e % rq;
    double s = 0.0;
    for (int k = 0; k < dt; k++) s += L1[a * LDA + k] * Yd[k * n + qcol + j];
    L2[a * LDA + j] = 2.0 * s;
  }
  __syncthreads();
  for (int e = tid; e < D.rp * rq; e += NTHREADS) {
    int i = e / rq, j = e % rq;
    double s = 0.0;
    for (int k = 0; k < dt; k++) s += Yd[k * n + i] * L2[k * LDA + j];
    GK[(long long)(D.offp + i) * ld + (offq + j)] = s;
    if (!diag) GK[(long long)(offq + j) * ld + (D.offp + i)] = s;
  }
}

hipError_t launch_adjoint(const Domain *dom, int ndom, const int *rank, const double *W,
                          const double *Y, const double *T, const long long *dcp_ptr,
                          const long long *dcp_toff, const double *dcp_coef, double *GK,
                          long long ld, double *Gd, hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint, dim3(ndom), dim3(NTHREADS), 0, s, dom, rank, W, Y, T, dcp_ptr,
                     dcp_toff, dcp_coef, GK, ld, Gd);
  return hipGetLastError();
}

// G^F (sum r x sum r): off-diagonal orbital blocks (u < v) come from the one
// domain [uv]; a diagonal block (u, u) sums the (u, u) parts of every domain that
// holds u, in the listed order.  blocks[b] = (u, v); blk_ptr/blk_dom/blk_part list
// the contributing domains and which part (0: first LMO, 1: second) of each.
__global__ __launch_bounds__(NTHREADS) void k_assemble_gf(const Domain *__restrict__ doms,
                                                          const long long *__restrict__ blk_ptr,
                                                          const int *__restrict__ blk_dom,
                                                          const int *__restrict__ blk_part,
                                                          const int2 *__restrict__ blocks,
                                                          const int *__restrict__ off,
                                                          const int *__restrict__ r,
                                                          const double *__restrict__ Gd,
                                                          double *GF, long long ld) {
  const int b = blockIdx.x;
  const int u = blocks[b].x, v = blocks[b].y;
  const int ru = r[u], rv = r[v];
  for (int e = threadIdx.x; e < ru * rv; e += NTHREADS) {
    int i = e / rv, j = e % rv;
    double s = 0.0;
    for (long long t = blk_ptr[b]; t < blk_ptr[b + 1]; t++) {
      const Domain D = doms[blk_dom[t]];
      const double *G = Gd + D.moff;
      if (u != v) {
        s += G[i * D.n + D.rp + j];          // (p block, q block) of domain [uv]
      } else {
        const int o = blk_part[t] ? D.rp : 0;
        s += G[(o + i) * D.n + o + j];
      }
    }
    GF[(long long)(off[u] + i) * ld + off[v] + j] = s;
    if (u != v) GF[(long long)(off[v] + j) * ld + off[u] + i] = s;
  }
}

hipError_t launch_assemble_gf(const Domain *dom, const long long *blk_ptr, const int *blk_dom,
                              const int *blk_part, const int2 *blocks, int nblocks,
                              const int *off, const int *r, const double *Gd, double *GF,
                              long long ld, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble_gf, dim3(nblocks), dim3(NTHREADS), 0, s, dom, blk_ptr, blk_dom,
                     blk_part, blocks, off, r, Gd, GF, ld);
  return hipGetLastError();
}

}  // namespace osv
