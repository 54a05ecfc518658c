// Pair-domain preparation (one workgroup per domain [Q_p Q_q], or Q_p).
//
// The residual equations eq:rij live in the composite OSV basis of each pair
// domain (eq:aijkl).  Each domain is brought to a basis W with
//   W^T S_(pq,pq) W = 1   and   W^T F_(pq,pq) W = diag(e~)
// (canonical orthogonalisation, dropping overlap eigenvalues <= tau_S, then
// pseudo-canonicalisation), so that the same-pair Fock/overlap products of
// eq:rij become the diagonal factor (e~_a + e~_b - f_pp - f_qq).
// Also formed here:
//   Y   = W^T S_(pq,pq)                 (rows: kept functions; cols: p block | q block)
//   K~  = Y_p K_pq Y_q^T = W^T K_(pq,pq) W   with K_(pq,pq) = U_p K_pq U_q^T,
//         U_p = [Q_p Q_q]^T Q_p: the fitted integrals of each LMO in its own OSV span.
// and, per pair of domains A, B sharing an LMO, the coupling
//   M(A,B) = W_A^T S_(A,B) W_B
// through which eq:rij couples amplitudes of different pairs.
//
// Symmetric eigenproblems (n <= 100) are solved in LDS by the cyclic Jacobi
// method with a round-robin ordering: n/2 disjoint rotations per step, applied
// to both sides of A as independent 2x2 block updates.
#include "osv_internal.h"

namespace osv {

constexpr int LDM = DMAX + 1;  // LDS stride (doubles) of the 100x100 work matrices

// ---- block accessors of the orbital-pair matrices ------------------------------
// element (i, j) of the composite S_(A,B) (rows: domain A's OSVs, cols: domain B's)
__device__ __forceinline__ double comp_elem(const double *X, long long ld, const Domain &A,
                                            const Domain &B, int i, int j, bool unit_diag) {
  int a_orb, ai, b_orb, bj, a_off, b_off;
  if (i < A.rp) { a_orb = A.p; ai = i; a_off = A.offp; } else { a_orb = A.q; ai = i - A.rp; a_off = A.offq; }
  if (j < B.rp) { b_orb = B.p; bj = j; b_off = B.offp; } else { b_orb = B.q; bj = j - B.rp; b_off = B.offq; }
  if (unit_diag && a_orb == b_orb) return ai == bj ? 1.0 : 0.0;
  return X[(long long)(a_off + ai) * ld + (b_off + bj)];
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Cyclic Jacobi: A (n x n, stride LDM) is diagonalised in place, V receives the
// eigenvectors (columns).  Pair tables c/s/t/pp/qq have room for DMAX/2 pairs.
__device__ void jacobi_eig(double *A, double *V, int n, double *cs, double *sn, double *tn,
                           int *pp, int *qq, double *red) {
  const int tid = threadIdx.x;
  const int nE = n + (n & 1), h = nE / 2, m = nE - 1;
  for (int e = tid; e < n * n; e += NTHREADS) {
    int i = e / n, j = e % n;
    V[i * LDM + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n == 1) return;
  // scale for the stopping test
  double d2 = 0.0;
  for (int i = tid; i < n; i += NTHREADS) d2 += A[i * LDM + i] * A[i * LDM + i];
  double off2 = 0.0;
  for (int e = tid; e < n * n; e += NTHREADS) {
    int i = e / n, j = e % n;
    if (i != j) off2 += A[i * LDM + j] * A[i * LDM + j];
  }
  d2 = wave_sum(d2);
  off2 = wave_sum(off2);
  if ((tid & 63) == 0) { red[tid >> 6] = d2; red[4 + (tid >> 6)] = off2; }
  __syncthreads();
  double norm2 = red[0] + red[1] + red[2] + red[3] + red[4] + red[5] + red[6] + red[7];
  __syncthreads();
  const double tol2 = 1e-32 * norm2;
  for (int sweep = 0; sweep < 40; sweep++) {
    for (int st = 0; st < m; st++) {
      if (tid < h) {
        int a, b;
        if (tid == 0) { a = st % m; b = m; } else { a = (st + tid) % m; b = (st - tid + m) % m; }
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
          double apq = A[p * LDM + q];
          if (apq != 0.0) {
            double app = A[p * LDM + p], aqq = A[q * LDM + q];
            double theta = (aqq - app) / (2.0 * apq);
            double at = fabs(theta);
            if (at > 1e150) t = 0.5 / theta;
            else t = (theta >= 0.0 ? 1.0 : -1.0) / (at + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s; tn[tid] = t;
      }
      __syncthreads();
      // A <- J^T A J as 2x2 block updates over pairs (I <= J)
      const int nb = h * (h + 1) / 2;
      for (int bidx = tid; bidx < nb; bidx += NTHREADS) {
        // invert bidx -> (I, J) with I <= J, row-major over the upper triangle
        int I = 0, rem = bidx;
        while (rem >= h - I) { rem -= h - I; I++; }
        int J = I + rem;
        int pI = pp[I], qI = qq[I], pJ = pp[J], qJ = qq[J];
        double cI = cs[I], sI = sn[I], cJ = cs[J], sJ = sn[J];
        if (I == J) {
          if (qI < n && sI != 0.0) {
            double apq = A[pI * LDM + qI];
            A[pI * LDM + pI] -= tn[I] * apq;
            A[qI * LDM + qI] += tn[I] * apq;
            A[pI * LDM + qI] = 0.0;
            A[qI * LDM + pI] = 0.0;
          }
        } else {
          bool vqI = qI < n, vqJ = qJ < n;
          double b00 = A[pI * LDM + pJ];
          double b01 = vqJ ? A[pI * LDM + qJ] : 0.0;
          double b10 = vqI ? A[qI * LDM + pJ] : 0.0;
          double b11 = (vqI && vqJ) ? A[qI * LDM + qJ] : 0.0;
          // rows: R_I^T B  with R = [[c, s], [-s, c]]
          double r00 = cI * b00 - sI * b10, r01 = cI * b01 - sI * b11;
          double r10 = sI * b00 + cI * b10, r11 = sI * b01 + cI * b11;
          // cols: (.) R_J
          double n00 = r00 * cJ - r01 * sJ, n01 = r00 * sJ + r01 * cJ;
          double n10 = r10 * cJ - r11 * sJ, n11 = r10 * sJ + r11 * cJ;
          A[pI * LDM + pJ] = n00; A[pJ * LDM + pI] = n00;
          if (vqJ) { A[pI * LDM + qJ] = n01; A[qJ * LDM + pI] = n01; }
          if (vqI) { A[qI * LDM + pJ] = n10; A[pJ * LDM + qI] = n10; }
          if (vqI && vqJ) { A[qI * LDM + qJ] = n11; A[qJ * LDM + qI] = n11; }
        }
      }
      // V <- V J
      for (int e = tid; e < n * h; e += NTHREADS) {
        int i = e / h, k = e % h;
        int p = pp[k], q = qq[k];
        if (q < n) {
          double c = cs[k], s = sn[k];
          double vp = V[i * LDM + p], vq = V[i * LDM + q];
          V[i * LDM + p] = c * vp - s * vq;
          V[i * LDM + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    off2 = 0.0;
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      if (i != j) off2 += A[i * LDM + j] * A[i * LDM + j];
    }
    off2 = wave_sum(off2);
    if ((tid & 63) == 0) red[tid >> 6] = off2;
    __syncthreads();
    double tot = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    if (tot <= tol2) break;
  }
}

__global__ __launch_bounds__(NTHREADS) void k_domain_prep(const Domain *__restrict__ doms,
                                                          const double *__restrict__ S,
                                                          const double *__restrict__ F,
                                                          const double *__restrict__ K,
                                                          long long ld, double tau_S, double *W,
                                                          double *Y, double *Kt, double *epst,
                                                          int *rank, double *minev) {
  __shared__ double L1[DMAX * LDM];
  __shared__ double L2[DMAX * LDM];
  __shared__ double cs[DMAX / 2], sn[DMAX / 2], tn[DMAX / 2];
  __shared__ int pp[DMAX / 2], qq[DMAX / 2];
  __shared__ double red[8];
  __shared__ int keep_idx[DMAX];
  __shared__ int s_dt;
  const Domain D = doms[blockIdx.x];
  const int tid = threadIdx.x, n = D.n;
  const bool diag = (D.p == D.q);
  double *Wg = W + D.moff, *Yg = Y + D.moff, *Kg = Kt + D.moff, *eg = epst + D.voff;
  int dt;
  if (!diag) {
    // 1) S_(pq,pq) = U s U^T ; X = U_kept s_kept^{-1/2}
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      L1[i * LDM + j] = comp_elem(S, ld, D, D, i, j, true);
    }
    __syncthreads();
    jacobi_eig(L1, L2, n, cs, sn, tn, pp, qq, red);
    if (tid == 0) {
      int c = 0;
      double mn = 1e300;
      for (int k = 0; k < n; k++) {
        double sk = L1[k * LDM + k];
        if (sk < mn) mn = sk;
        if (sk > tau_S) keep_idx[c++] = k;
      }
      s_dt = c;
      minev[blockIdx.x] = mn;
    }
    __syncthreads();
    dt = s_dt;
    // X (n x dt) into the Y slot (global scratch)
    for (int e = tid; e < n * dt; e += NTHREADS) {
      int i = e / dt, c = e % dt;
      int k = keep_idx[c];
      Yg[i * n + c] = L2[i * LDM + k] / sqrt(L1[k * LDM + k]);
    }
    __syncthreads();
    // 2) L1 = F_(pq,pq) X (n x dt)
    for (int e = tid; e < n * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      double s = 0.0;
      for (int k = 0; k < n; k++) s += comp_elem(F, ld, D, D, i, k, false) * Yg[k * n + j];
      L1[i * LDM + j] = s;
    }
    __syncthreads();
    // H = X^T L1 (dt x dt) into L2
    for (int e = tid; e < dt * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      double s = 0.0;
      for (int k = 0; k < n; k++) s += Yg[k * n + i] * L1[k * LDM + j];
      L2[i * LDM + j] = s;
    }
    __syncthreads();
    for (int e = tid; e < dt * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      L1[i * LDM + j] = 0.5 * (L2[i * LDM + j] + L2[j * LDM + i]);
    }
    __syncthreads();
    jacobi_eig(L1, L2, dt, cs, sn, tn, pp, qq, red);
    for (int a = tid; a < dt; a += NTHREADS) eg[a] = L1[a * LDM + a];
    __syncthreads();
    // W = X V (n x dt) into L1, then to global
    for (int e = tid; e < n * dt; e += NTHREADS) {
      int i = e / dt, j = e % dt;
      double s = 0.0;
      for (int k = 0; k < dt; k++) s += Yg[i * n + k] * L2[k * LDM + j];
      L1[i * LDM + j] = s;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      Wg[i * n + j] = (j < dt) ? L1[i * LDM + j] : 0.0;
    }
    __syncthreads();
    // 3) Y = W^T S_(pq,pq) (dt x n) into L2 and global
    for (int e = tid; e < dt * n; e += NTHREADS) {
      int a = e / n, j = e % n;
      double s = 0.0;
      for (int k = 0; k < n; k++) s += L1[k * LDM + a] * comp_elem(S, ld, D, D, k, j, true);
      L2[a * LDM + j] = s;
    }
    __syncthreads();
  } else {
    // diagonal domain: S = 1, W = eigenvectors of F_pp
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      L1[i * LDM + j] = F[(long long)(D.offp + i) * ld + (D.offp + j)];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      L2[i * LDM + j] = 0.5 * (L1[i * LDM + j] + L1[j * LDM + i]);
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      L1[i * LDM + j] = L2[i * LDM + j];
    }
    __syncthreads();
    jacobi_eig(L1, L2, n, cs, sn, tn, pp, qq, red);
    dt = n;
    if (tid == 0) minev[blockIdx.x] = 1.0;
    for (int a = tid; a < n; a += NTHREADS) eg[a] = L1[a * LDM + a];
    for (int e = tid; e < n * n; e += NTHREADS) {
      int i = e / n, j = e % n;
      Wg[i * n + j] = L2[i * LDM + j];
    }
    __syncthreads();
    // Y = W^T
    for (int e = tid; e < n * n; e += NTHREADS) {
      int a = e / n, j = e % n;
      L1[a * LDM + j] = L2[j * LDM + a];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += NTHREADS) {
      int a = e / n, j = e % n;
      L2[a * LDM + j] = L1[a * LDM + j];
    }
    __syncthreads();
  }
  // Y (dt x n) is in L2: store it
  for (int e = tid; e < n * n; e += NTHREADS) {
    int a = e / n, j = e % n;
    Yg[a * n + j] = (a < dt) ? L2[a * LDM + j] : 0.0;
  }
  // 4) K~ = Y_p K_pq Y_q^T: L1 = Y_p K_pq (dt x rq), then K~ = L1 Y_q^T
  const int rq = diag ? D.rp : D.rq;
  const int offq = diag ? D.offp : D.offq;
  const int qcol = diag ? 0 : D.rp;
  for (int e = tid; e < dt * rq; e += NTHREADS) {
    int a = e / rq, j = e % rq;
    double s = 0.0;
    for (int k = 0; k < D.rp; k++) s += L2[a * LDM + k] * K[(long long)(D.offp + k) * ld + (offq + j)];
    L1[a * LDM + j] = s;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += NTHREADS) {
    int a = e / n, b = e % n;
    double s = 0.0;
    if (a < dt && b < dt)
      for (int k = 0; k < rq; k++) s += L1[a * LDM + k] * L2[b * LDM + qcol + k];
    Kg[a * n + b] = s;
  }
  if (tid == 0) rank[blockIdx.x] = dt;
}

hipError_t launch_domain_prep(const Domain *dom, int ndom, const double *S, const double *F,
                              const double *K, long long ld, double tau_S, double *W,
                              double *Y, double *Kt, double *epst, int *rank, double *minev,
                              hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_domain_prep, dim3(ndom), dim3(NTHREADS), 0, s, dom, S, F, K, ld, tau_S, W,
                     Y, Kt, epst, rank, minev);
  return hipGetLastError();
}

// M(A,B) = W_A^T S_(A,B) W_B   (dt_A x dt_B in an n_A x n_B slot)
__global__ __launch_bounds__(NTHREADS) void k_couplings(const Coupling *__restrict__ cpl,
                                                        const Domain *__restrict__ doms,
                                                        const int *__restrict__ rank,
                                                        const double *__restrict__ S, long long ld,
                                                        const double *__restrict__ W,
                                                        double *M) {
  __shared__ double G[DMAX * LDM];
  const Coupling c = cpl[blockIdx.x];
  const Domain A = doms[c.A], B = doms[c.B];
  const int dtA = rank[c.A], dtB = rank[c.B];
  const double *WA = W + A.moff, *WB = W + B.moff;
  const int tid = threadIdx.x;
  // G = S_(A,B) W_B  (n_A x dt_B)
  for (int e = tid; e < A.n * dtB; e += NTHREADS) {
    int i = e / dtB, j = e % dtB;
    double s = 0.0;
    for (int k = 0; k < B.n; k++) s += comp_elem(S, ld, A, B, i, k, true) * WB[k * B.n + j];
    G[i * LDM + j] = s;
  }
  __syncthreads();
  double *Mg = M + c.off;
  for (int e = tid; e < A.n * B.n; e += NTHREADS) {
    int a = e / B.n, b = e % B.n;
    double s = 0.0;
    if (a < dtA && b < dtB)
      for (int k = 0; k < A.n; k++) s += WA[k * A.n + a] * G[k * LDM + b];
    Mg[a * B.n + b] = s;
  }
}

hipError_t launch_couplings(const Coupling *cpl, int ncpl, const Domain *dom, const int *rank,
                            const double *S, long long ld, const double *W, double *M,
                            hipStream_t s) {
  if (ncpl <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_couplings, dim3(ncpl), dim3(NTHREADS), 0, s, cpl, dom, rank, S, ld, W, M);
  return hipGetLastError();
}

}  // namespace osv
