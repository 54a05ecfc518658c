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
