// Device helpers shared by the kernels that work on pair-domain matrices: the
// element accessor of composite orbital-pair matrices and a small FP64 MFMA tile
// product whose operands come from accessor functions.
#pragma once
#include "osv_internal.h"

namespace osv {

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

typedef double d4p __attribute__((ext_vector_type(4)));

// C(i, j) = sum_{k < K} A(i, k) B(k, j) for i < M, j < N on FP64
// MFMA 16x16x4: the 16x16 output tiles are spread over the block's waves, and the
// operands of 8 k-steps are loaded before their MFMAs, so that global loads are
// in flight together.  a(i, k), b(k, j) are called for in-range indices only;
// c(i, j, value) stores.  No barrier inside: the caller orders producers and
// consumers.
template <int NT, class FA, class FB, class FC>
__device__ __forceinline__ void mma_tiles(int M, int N, int K, FA a, FB b, FC c) {
  constexpr int KB = 8;    // k-steps of 4 per batch
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  for (int t = wave; t < tm * tn; t += NT / 64) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
    const int i = i0 + l15, j = j0 + l15;
    d4p acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 4 * KB) {
      double av[KB], bv[KB];
#pragma unroll
      for (int st = 0; st < KB; st++) {
        const int k = k0 + 4 * st + lhi;
        av[st] = (i < M && k < K) ? a(i, k) : 0.0;
        bv[st] = (j < N && k < K) ? b(k, j) : 0.0;
      }
#pragma unroll
      for (int st = 0; st < KB; st++)
        if (k0 + 4 * st < K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bv[st], acc, 0, 0, 0);
    }
    // accumulator: lane l, register v -> row 4v + (l >> 4), column l & 15
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int ii = i0 + 4 * v + lhi;
      if (ii < M && j < N) c(ii, j, acc[v]);
    }
  }
}

}  // namespace osv

namespace osv {

// A dense operand in global memory: element (r, c) is p[r ld + c], or p[c ld + r]
// when tr is set (the transpose of a row-major matrix); with p2 (a B operand
// that is not transposed) the element is p[r ld + c] + p2[r ld + c].
struct Mat {
  const double *p;
  long long ld;
  int tr;
  const double *p2 = nullptr;
};

// C(i, j) = sum_{k < K} A(i, k) B(k, j) for i < M <= 112, j < N <= 112 on FP64 MFMA
// 16x16x4 with both operands staged through LDS in chunks of 16 k: each chunk is
// read from global memory with 16-byte loads along the operand's contiguous
// direction (8-byte loads where the alignment does not allow them), stored as
// A[i][k] (row stride 18) and B[k][j] (row stride 112), so that the MFMA operand
// reads of a half-wave fall into distinct banks, and double-buffered: the loads of
// chunk c + 1 are in flight while chunk c is multiplied, one barrier per chunk.
// The 16x16 output tiles are spread over the block's waves; c(i, j, value) stores
// after the last chunk.  lds: gemm_lds_doubles() doubles.  Every thread of the
// block must call it; it begins and ends with a barrier.
constexpr int GKC = 16, GAP = GKC + 2, GBP = 112, GMAX = 112;
constexpr int GPR = GKC / 2;   // element pairs along k per row of a chunk
constexpr int GA_SZ = GMAX * GAP, GB_SZ = GKC * GBP;
__host__ __device__ constexpr int gemm_lds_doubles() { return 2 * (GA_SZ + GB_SZ); }

template <int NT, int TR, int SUM = 0>
struct ChunkLoader {
  static constexpr int NPAIR = (GMAX * GKC / 2 + NT - 1) / NT;  // element pairs per thread
  double2 v[NPAIR];
  // A chunk [0, M) x [k0, k0 + 16) into As[i][k]
  __device__ __forceinline__ void load_a(const Mat &A, int M, int K, int k0) {
    const int tid = threadIdx.x;
    const bool vec = ((A.ld & 1) == 0) && ((reinterpret_cast<uintptr_t>(A.p) & 15) == 0);
#pragma unroll
    for (int u = 0; u < NPAIR; u++) {
      const int q = tid + u * NT;
      double x0 = 0.0, x1 = 0.0;
      if (!TR) {   // pairs along k: (i, kk), (i, kk + 1)
        const int i = q / GPR, k = k0 + ((q % GPR) << 1);
        if (i < M) {
          const double *s = A.p + (long long)i * A.ld + k;
          if (vec && k + 1 < K) {
            const double2 w = *reinterpret_cast<const double2 *>(s);
            x0 = w.x;
            x1 = w.y;
          } else {
            if (k < K) x0 = s[0];
            if (k + 1 < K) x1 = s[1];
          }
        }
      } else {       // pairs along i: (i, k), (i + 1, k)
        const int mh = (M + 1) >> 1;
        const int kk = q / mh, i = (q - kk * mh) << 1, k = k0 + kk;
        if (kk < GKC && k < K) {
          const double *s = A.p + (long long)k * A.ld + i;
          if (vec && i + 1 < M) {
            const double2 w = *reinterpret_cast<const double2 *>(s);
            x0 = w.x;
            x1 = w.y;
          } else {
            if (i < M) x0 = s[0];
            if (i + 1 < M) x1 = s[1];
          }
        }
      }
      v[u] = make_double2(x0, x1);
    }
  }
  __device__ __forceinline__ void store_a(const Mat &A, int M, double *As) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < NPAIR; u++) {
      const int q = tid + u * NT;
      if (!TR) {
        const int i = q / GPR, kk = (q % GPR) << 1;
        if (i < GMAX) *reinterpret_cast<double2 *>(As + i * GAP + kk) = v[u];
      } else {
        const int mh = (M + 1) >> 1;
        const int kk = q / mh, i = (q - kk * mh) << 1;
        if (kk < GKC) {
          As[i * GAP + kk] = v[u].x;
          As[(i + 1) * GAP + kk] = v[u].y;
        }
      }
    }
  }
  // B chunk [k0, k0 + 16) x [0, N) into Bs[k][j]
  __device__ __forceinline__ void load_b(const Mat &B, int N, int K, int k0) {
    const int tid = threadIdx.x;
    const bool vec = ((B.ld & 1) == 0) && ((reinterpret_cast<uintptr_t>(B.p) & 15) == 0) &&
                     (!SUM || (reinterpret_cast<uintptr_t>(B.p2) & 15) == 0);
#pragma unroll
    for (int u = 0; u < NPAIR; u++) {
      const int q = tid + u * NT;
      double x0 = 0.0, x1 = 0.0;
      if (!TR) {   // pairs along j: (k, j), (k, j + 1)
        const int nh = (N + 1) >> 1;
        const int kk = q / nh, j = (q - kk * nh) << 1, k = k0 + kk;
        if (kk < GKC && k < K) {
          const double *s = B.p + (long long)k * B.ld + j;
          if (vec && j + 1 < N) {
            const double2 w = *reinterpret_cast<const double2 *>(s);
            x0 = w.x;
            x1 = w.y;
            if (SUM) {
              const double2 w2 = *reinterpret_cast<const double2 *>(B.p2 + (long long)k * B.ld + j);
              x0 += w2.x;
              x1 += w2.y;
            }
          } else {
            if (j < N) x0 = s[0] + (SUM ? B.p2[(long long)k * B.ld + j] : 0.0);
            if (j + 1 < N) x1 = s[1] + (SUM ? B.p2[(long long)k * B.ld + j + 1] : 0.0);
          }
        }
      } else {       // pairs along k: (k, j), (k + 1, j)
        const int j = q / GPR, k = k0 + ((q % GPR) << 1);
        if (j < N) {
          const double *s = B.p + (long long)j * B.ld + k;
          if (vec && k + 1 < K) {
            const double2 w = *reinterpret_cast<const double2 *>(s);
            x0 = w.x;
            x1 = w.y;
          } else {
            if (k < K) x0 = s[0];
            if (k + 1 < K) x1 = s[1];
          }
        }
      }
      v[u] = make_double2(x0, x1);
    }
  }
  __device__ __forceinline__ void store_b(const Mat &B, int N, double *Bs) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < NPAIR; u++) {
      const int q = tid + u * NT;
      if (!TR) {
        const int nh = (N + 1) >> 1;
        const int kk = q / nh, j = (q - kk * nh) << 1;
        if (kk < GKC) *reinterpret_cast<double2 *>(Bs + kk * GBP + j) = v[u];
      } else {
        const int j = q / GPR, kk = (q % GPR) << 1;
        if (j < GMAX) {
          Bs[kk * GBP + j] = v[u].x;
          Bs[(kk + 1) * GBP + j] = v[u].y;
        }
      }
    }
  }
};

template <int NT, int TRA, int TRB, int SUMB, class FC>
__device__ void gemm_lds_t(int M, int N, int K, const Mat A, const Mat B, double *lds, FC c) {
  constexpr int NW = NT / 64;
  constexpr int MAXTW = (7 * 7 + NW - 1) / NW;   // output tiles per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l15 = lane & 15, lhi = lane >> 4;
  const int tn = (N + 15) >> 4, nt = ((M + 15) >> 4) * tn;
  const int nch = (K + GKC - 1) / GKC;
  d4p acc[MAXTW];
#pragma unroll
  for (int u = 0; u < MAXTW; u++) acc[u] = d4p{0.0, 0.0, 0.0, 0.0};
  ChunkLoader<NT, TRA> la;
  ChunkLoader<NT, TRB, SUMB> lb;
  __syncthreads();
  if (nch > 0) {
    la.load_a(A, M, K, 0);
    lb.load_b(B, N, K, 0);
    la.store_a(A, M, lds);
    lb.store_b(B, N, lds + GA_SZ);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ch++) {
    const bool more = ch + 1 < nch;
    if (more) {
      la.load_a(A, M, K, (ch + 1) * GKC);
      lb.load_b(B, N, K, (ch + 1) * GKC);
    }
    const double *As = lds + (ch & 1) * (GA_SZ + GB_SZ), *Bs = As + GA_SZ;
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int t = wave + u * NW;
      if (t < nt) {
        const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
        const int kend = K - ch * GKC;   // k-steps past K multiply zeros: skipped
#pragma unroll
        for (int ks = 0; ks < GKC / 4; ks++) {
          if (4 * ks >= kend) break;
          const double av = As[(i0 + l15) * GAP + 4 * ks + lhi];
          const double bv = Bs[(4 * ks + lhi) * GBP + j0 + l15];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
        }
      }
      // one tile's operand reads at a time: keeps the reads of later tiles from
      // being hoisted into registers
      __builtin_amdgcn_sched_barrier(0);
    }
    if (more) {
      double *An = lds + ((ch + 1) & 1) * (GA_SZ + GB_SZ);
      la.store_a(A, M, An);
      lb.store_b(B, N, An + GA_SZ);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < MAXTW; u++) {
    const int t = wave + u * NW;
    if (t < nt) {
      const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int ii = i0 + 4 * v + lhi, jj = j0 + l15;
        if (ii < M && jj < N) c(ii, jj, acc[u][v]);
      }
    }
  }
}

// the transposition flags of A and B select the compiled loader
template <int NT, class FC>
__device__ __forceinline__ void gemm_lds(int M, int N, int K, const Mat A, const Mat B, double *lds, FC c) {
  if (A.tr) {
    if (B.tr) gemm_lds_t<NT, 1, 1, 0>(M, N, K, A, B, lds, c);
    else if (B.p2) gemm_lds_t<NT, 1, 0, 1>(M, N, K, A, B, lds, c);
    else gemm_lds_t<NT, 1, 0, 0>(M, N, K, A, B, lds, c);
  } else {
    if (B.tr) gemm_lds_t<NT, 0, 1, 0>(M, N, K, A, B, lds, c);
    else gemm_lds_t<NT, 0, 0, 0>(M, N, K, A, B, lds, c);
  }
}

}  // namespace osv
