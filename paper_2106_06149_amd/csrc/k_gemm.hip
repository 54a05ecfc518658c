// Dense tile kernels for the orbital-pair blocks and the back-transforms.
//
//   S_(i,j) = Q_i^T Q_j,  F_(i,j) = Q_i^T diag(eps) Q_j   (eq:aijkl, pair tasks of Algorithm 1)
//   K_ij    = C_i C_j^T                                    (pair tasks of Algorithm 1)
//   dE/dC   = 2 G^K C,  Z^T = G^F Q^T, D^v = Q Z^T          (back-transforms of the densities)
//
// FP64 products run on a 128x128-tile MFMA kernel fed by direct global-to-LDS
// loads (k_gemm_dma) whenever the leading dimensions and k are even and the
// operands 16-byte aligned, else on a 64x64-tile kernel that stages through
// registers (k_tile_f64); for the symmetric products a tile list skips tiles that
// hold no needed orbital-pair block.  FP64 tiles use v_mfma_f64_16x16x4f64; the
// mixed-precision K uses v_mfma_i32_16x16x64_i8 on exact int8 digit splits of
// the FP32 input with exact int32 accumulation, combined in FP64 at the end.
#include "osv_internal.h"

#include <type_traits>

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TB = 64;      // output tile edge
constexpr int KC = 16;      // k-chunk staged in LDS (FP64 kernel)
constexpr int LDT = KC + 1; // LDS row stride (doubles): conflict-free 16-row fragment reads

template <typename T>
__device__ __forceinline__ double ld_as_f64(const T *p) { return (double)(*p); }

// ---------------------------------------------------------------------------
// FP64 tile kernel.
//   A access: AK == 0 -> A(i,k) = A[i*lda + k];  AK == 1 -> A(i,k) = A[k*lda + i]
//   B access: BK == 0 -> B(k,j) = B[j*ldb + k];  BK == 1 -> B(k,j) = B[k*ldb + j]
//   C[i][j] = alpha * sum_k A(i,k) B(k,j);  C2[i][j] = alpha * sum_k A(i,k) w[k] B(k,j)
// Tiles come from `tiles` (tile row, tile col) or, if null, from the grid.
// mirror: also store the transposed tile at (j, i) when the tile is off-diagonal.
// ---------------------------------------------------------------------------
template <int AK, int BK, typename TA, typename TBt, bool DUAL>
__global__ __launch_bounds__(256) void k_tile_f64(const TA *__restrict__ A, long long lda,
                                                  const TBt *__restrict__ B, long long ldb,
                                                  const double *__restrict__ w, double *C,
                                                  double *C2, long long ldc, int M, int N, int K,
                                                  double alpha, const int2 *__restrict__ tiles,
                                                  int mirror) {
  __shared__ double As[TB * LDT];
  __shared__ double Bs[TB * LDT];
  __shared__ double Ws[KC];
  int ti, tj;
  if (tiles) {
    int2 t = tiles[blockIdx.x];
    ti = t.x;
    tj = t.y;
  } else {
    ti = blockIdx.y;
    tj = blockIdx.x;
  }
  const int i0 = ti * TB, j0 = tj * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  d4 acc[2][2], acc2[2][2];
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      acc[a][b] = (d4){0, 0, 0, 0};
      acc2[a][b] = (d4){0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < K; k0 += KC) {
    // stage A(i0..i0+63, k0..k0+15) and B(k0.., j0..j0+63) as [row][k]
    for (int e = tid; e < TB * KC; e += 256) {
      int r, k;
      if (AK == 0) { r = e / KC; k = e % KC; } else { k = e / TB; r = e % TB; }
      int gi = i0 + r, gk = k0 + k;
      double v = 0.0;
      if (gi < M && gk < K) v = ld_as_f64(AK == 0 ? &A[(long long)gi * lda + gk] : &A[(long long)gk * lda + gi]);
      As[r * LDT + k] = v;
      if (BK == 0) { r = e / KC; k = e % KC; } else { k = e / TB; r = e % TB; }
      int gj = j0 + r;
      gk = k0 + k;
      v = 0.0;
      if (gj < N && gk < K) v = ld_as_f64(BK == 0 ? &B[(long long)gj * ldb + gk] : &B[(long long)gk * ldb + gj]);
      Bs[r * LDT + k] = v;
    }
    if (DUAL && tid < KC) Ws[tid] = (k0 + tid < K) ? w[k0 + tid] : 0.0;
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kk = ks + (lane >> 4);
      double af[2], bfr[2];
#pragma unroll
      for (int a = 0; a < 2; a++) af[a] = As[(wr + a * 16 + (lane & 15)) * LDT + kk];
#pragma unroll
      for (int b = 0; b < 2; b++) bfr[b] = Bs[(wc + b * 16 + (lane & 15)) * LDT + kk];
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bfr[b], acc[a][b], 0, 0, 0);
          if (DUAL)
            acc2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a] * Ws[kk], bfr[b], acc2[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // f64 16x16 accumulator layout: lane l, reg v -> row (l>>4) + 4v, col l & 15
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int v = 0; v < 4; v++) {
        int i = i0 + wr + a * 16 + (lane >> 4) + 4 * v;
        int j = j0 + wc + b * 16 + (lane & 15);
        if (i < M && j < N) {
          C[(long long)i * ldc + j] = alpha * acc[a][b][v];
          if (DUAL) C2[(long long)i * ldc + j] = alpha * acc2[a][b][v];
          if (mirror && ti != tj) {
            C[(long long)j * ldc + i] = alpha * acc[a][b][v];
            if (DUAL) C2[(long long)j * ldc + i] = alpha * acc2[a][b][v];
          }
        }
      }
}

// ---------------------------------------------------------------------------
// FP64 128x128-tile kernel fed by direct global-to-LDS loads.
//   A(i,k) = A[i*lda + k] (rows i, k contiguous)
//   BK == 0: B(k,j) = B[j*ldb + k] (rows j, k contiguous)   -- C = A B^T (SYRK form)
//   BK == 1: B(k,j) = B[k*ldb + j] (rows k, j contiguous)   -- C = A B
//   C[i][j] = alpha sum_k A(i,k) B(k,j), or with WGT alpha sum_k A(i,k) w[k] B(k,j)
// Eight waves (two per SIMD: one wave alone cannot keep the FP64 MFMA pipe busy),
// each a 32x64 part of the tile as 2x4 MFMA 16x16x4 accumulators.
// k advances in stages of 16 through two LDS buffers (64 KB, so that two
// workgroups share a CU): the loads of stage s+1 (global_load_lds_dwordx4, 16
// bytes per lane, no registers) are issued before the MFMAs of stage s.  A
// [row][k] stage keeps a row's 16 doubles as eight 16-byte slots, slot index XOR
// (row mod 8), so that the 16 rows of an operand fragment spread over the LDS
// banks; a [k][j] stage pads its rows to 130 doubles.
// Rows and columns past M, N are clamped to the last valid one (they only feed
// outputs that are not stored); k past K is clamped on load and zeroed in LDS.
// Requirements (checked by the launchers): lda, ldb, K even, 16-byte aligned
// A and B, and for BK == 1 also N even.
// ---------------------------------------------------------------------------
constexpr int G = 128;             // output tile edge
constexpr int GRS = 130;           // LDS row stride of a [k][j] stage (doubles)
constexpr int GNS = 2;             // stages: the next one loads while this one is multiplied
constexpr int GNT = 512;           // threads (8 waves)
// the stage depth GKS (k per stage: 8, 16 or 32 doubles) is a template parameter,
// chosen at run time from the tuning table (16 by default: 64 KB of LDS, two
// workgroups per CU); GSL 16-byte slots per row of a [row][k] stage, GA and GB1
// doubles of a [row][k] and of a [k][j] stage
template <int GKS>
struct GemmStage {
  static constexpr int GSL = GKS / 2;
  static constexpr int GA = G * GKS;
  static constexpr int GB1 = GKS * GRS;
};

typedef __attribute__((address_space(3))) void *lds_ptr;

// issue the loads of stage k0 into buffer (As_b, Bs_b): GKS blocks of 1 KB per
// operand, GKS / 8 per wave
template <int GKS, int BK>
__device__ __forceinline__ void gemm_issue(const double *__restrict__ A, long long lda,
                                           const double *__restrict__ B, long long ldb, int i0,
                                           int j0, int k0, int M, int N, int K, double *As_b,
                                           double *Bs_b) {
  constexpr int GSL = GemmStage<GKS>::GSL;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < GKS / 8; v++) {
    const int u = wave + 8 * v;                 // 1 KB block of the stage
    const int p = u * 64 + lane;                // 16-byte slot in the stage
    const int row = p / GSL, kp = (p % GSL) ^ (row % GSL);
    const int gk = min(k0 + 2 * kp, K - 2);
    const int gi = min(i0 + row, M - 1);
    __builtin_amdgcn_global_load_lds((const void *)(A + (long long)gi * lda + gk),
                                     (lds_ptr)(As_b + u * 128), 16, 0, 0);
    if (BK == 0) {
      const int gj = min(j0 + row, N - 1);
      __builtin_amdgcn_global_load_lds((const void *)(B + (long long)gj * ldb + gk),
                                       (lds_ptr)(Bs_b + u * 128), 16, 0, 0);
    } else {
      const int kr = u;                          // k-row of the stage
      const int gkr = min(k0 + kr, K - 1);
      const int gj = min(j0 + 2 * lane, N - 2);
      __builtin_amdgcn_global_load_lds((const void *)(B + (long long)gkr * ldb + gj),
                                       (lds_ptr)(Bs_b + kr * GRS), 16, 0, 0);
    }
  }
}

template <int GKS, int BK, bool WGT>
__global__ __launch_bounds__(GNT) void k_gemm_dma(const double *__restrict__ A, long long lda,
                                                  const double *__restrict__ B, long long ldb,
                                                  const double *__restrict__ w, double *C,
                                                  long long ldc, int M, int N, int K,
                                                  double alpha, const int2 *__restrict__ tiles,
                                                  int mirror) {
  constexpr int GSL = GemmStage<GKS>::GSL, GA = GemmStage<GKS>::GA, GB1 = GemmStage<GKS>::GB1;
  constexpr int GBS = BK == 0 ? GA : GB1;
  __shared__ __attribute__((aligned(16))) double As[GNS * GA];
  __shared__ __attribute__((aligned(16))) double Bs[GNS * GBS];
  int ti, tj;
  if (tiles) {
    const int2 t = tiles[blockIdx.x];
    ti = t.x;
    tj = t.y;
  } else {
    ti = blockIdx.y;
    tj = blockIdx.x;
  }
  const int i0 = ti * G, j0 = tj * G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;
  d4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = (d4){0, 0, 0, 0};
  const int nst = (K + GKS - 1) / GKS;
  gemm_issue<GKS, BK>(A, lda, B, ldb, i0, j0, 0, M, N, K, As, Bs);
  for (int st = 0; st < nst; st++) {
    const int k0 = st * GKS, sb = st & 1;
    double *Ab = As + sb * GA, *Bb = Bs + sb * GBS;
    // this stage's loads have landed and every wave is done with the other buffer
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (st + 1 < nst)
      gemm_issue<GKS, BK>(A, lda, B, ldb, i0, j0, k0 + GKS, M, N, K, As + (sb ^ 1) * GA,
                     Bs + (sb ^ 1) * GBS);
    if (k0 + GKS > K) {
      // last, partial stage: zero k >= K
      const int kv = K - k0;
      for (int e = tid; e < G * GKS; e += GNT) {
        const int row = e / GKS, k = e % GKS;
        if (k >= kv) {
          const int idx = row * GKS + ((((k >> 1) ^ (row % GSL))) << 1) + (k & 1);
          Ab[idx] = 0.0;
          if (BK == 0) Bb[idx] = 0.0;
          else Bb[k * GRS + row] = 0.0;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int ks = 0; ks < GKS; ks += 4) {
      const int kk = ks + lhi;
      double af[2], bf[4];
#pragma unroll
      for (int a = 0; a < 2; a++) {
        const int row = wr + a * 16 + l15;
        af[a] = Ab[row * GKS + ((((kk >> 1) ^ (row % GSL))) << 1) + (kk & 1)];
      }
#pragma unroll
      for (int b = 0; b < 4; b++) {
        const int col = wc + b * 16 + l15;
        bf[b] = BK == 0 ? Bb[col * GKS + ((((kk >> 1) ^ (col % GSL))) << 1) + (kk & 1)]
                        : Bb[kk * GRS + col];
      }
      if (WGT) {
        const double wk = (k0 + kk < K) ? w[k0 + kk] : 0.0;
#pragma unroll
        for (int a = 0; a < 2; a++) af[a] *= wk;
      }
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 4; b++)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  }
  // accumulator layout: lane l, register v -> row 4v + (l >> 4), column l & 15
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 4; b++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = i0 + wr + a * 16 + lhi + 4 * v;
        const int j = j0 + wc + b * 16 + l15;
        if (i < M && j < N) {
          C[(long long)i * ldc + j] = alpha * acc[a][b][v];
          if (mirror && ti != tj) C[(long long)j * ldc + i] = alpha * acc[a][b][v];
        }
      }
}

// run f with the stage depth of the tuning table as a compile-time constant
template <class Fn>
static void dispatch_ks(Fn f) {
  switch (tuning().gemm_ks) {
    case 8: f(std::integral_constant<int, 8>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    default: f(std::integral_constant<int, 16>()); break;
  }
}

static bool dma_ok(const void *p, long long ld) {
  return ((size_t)p & 15) == 0 && (ld & 1) == 0;
}

hipError_t launch_syrk_f64(const void *A, int a_is_f32, long long lda, int M, int K,
                           const double *w, double *C, double *C2, long long ldc,
                           const int2 *tiles, int ntiles, const int2 *tiles128, int ntiles128,
                           hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dim3 block(256);
  if (!a_is_f32 && tiles128 && ntiles128 > 0 && dma_ok(A, lda) && (K & 1) == 0 && K >= 2) {
    // with a weight: C = A A^T and C2 = A diag(w) A^T as two passes over A
    dim3 grid(ntiles128), blk(GNT);
    auto run = [&](auto ks) {
      constexpr int KS = decltype(ks)::value;
      hipLaunchKernelGGL((k_gemm_dma<KS, 0, false>), grid, blk, 0, s, (const double *)A, lda,
                         (const double *)A, lda, nullptr, C, ldc, M, M, K, 1.0, tiles128, 1);
      if (w)
        hipLaunchKernelGGL((k_gemm_dma<KS, 0, true>), grid, blk, 0, s, (const double *)A, lda,
                           (const double *)A, lda, w, C2, ldc, M, M, K, 1.0, tiles128, 1);
    };
    dispatch_ks(run);
    return hipGetLastError();
  }
  dim3 grid(ntiles);
  if (w) {
    if (a_is_f32) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_tile_f64<0, 0, double, double, true>), grid, block, 0, s,
                       (const double *)A, lda, (const double *)A, lda, w, C, C2, ldc, M, M, K,
                       1.0, tiles, 1);
  } else if (a_is_f32) {
    hipLaunchKernelGGL((k_tile_f64<0, 0, float, float, false>), grid, block, 0, s,
                       (const float *)A, lda, (const float *)A, lda, nullptr, C, nullptr, ldc,
                       M, M, K, 1.0, tiles, 1);
  } else {
    hipLaunchKernelGGL((k_tile_f64<0, 0, double, double, false>), grid, block, 0, s,
                       (const double *)A, lda, (const double *)A, lda, nullptr, C, nullptr, ldc,
                       M, M, K, 1.0, tiles, 1);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_nn_f64(const double *A, long long lda, const double *B, int b_is_f32,
                              long long ldb, double *C, long long ldc, int M, int N, int K,
                              double alpha, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!b_is_f32 && dma_ok(A, lda) && dma_ok(B, ldb) && (K & 1) == 0 && K >= 2 && (N & 1) == 0) {
    dim3 grid((N + G - 1) / G, (M + G - 1) / G), block(GNT);
    auto run = [&](auto ks) {
      constexpr int KS = decltype(ks)::value;
      hipLaunchKernelGGL((k_gemm_dma<KS, 1, false>), grid, block, 0, s, A, lda, B, ldb, nullptr, C,
                         ldc, M, N, K, alpha, nullptr, 0);
    };
    dispatch_ks(run);
    return hipGetLastError();
  }
  dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB), block(256);
  if (b_is_f32)
    hipLaunchKernelGGL((k_tile_f64<0, 1, double, float, false>), grid, block, 0, s, A, lda,
                       (const float *)B, ldb, nullptr, C, nullptr, ldc, M, N, K, alpha,
                       nullptr, 0);
  else
    hipLaunchKernelGGL((k_tile_f64<0, 1, double, double, false>), grid, block, 0, s, A, lda, B,
                       ldb, nullptr, C, nullptr, ldc, M, N, K, alpha, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_gemm_tn_f64(const double *A, long long lda, const double *B, long long ldb,
                              double *C, long long ldc, int M, int N, int K, double alpha,
                              hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + TB - 1) / TB, (M + TB - 1) / TB), block(256);
  hipLaunchKernelGGL((k_tile_f64<1, 1, double, double, false>), grid, block, 0, s, A, lda, B,
                     ldb, nullptr, C, nullptr, ldc, M, N, K, alpha, nullptr, 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mixed precision K = C C^T from exact int8 digits.
//
// Each row i of the FP32 input C is scaled by a power of two s_i so that
// |x| = |C[i][P]| / s_i < 1/2, and x is split into ND signed integer digits
//   x = sum_k d_k 2^(-7(k+1)) + r,   |d_k| <= 64,   |r| <= 2^(-7 ND - 1)
// (round to nearest at each level; every step is exact in FP32).  The digits are
// int8, the int8 MFMA multiplies digit planes and accumulates in int32, exactly:
// one accumulator per level l = a + b <= NL - 1 = ND holds at most ND products of
// at most 2^12 per k, below 2^31 for up to 87,000 k (the launcher refuses more).
// At the end K_ij = s_i s_j 2^-14 sum_l 2^(-7 l) S_l in FP64.  Level ND is kept
// because an FP32 element at the top of its row fills four 7-bit digits and the
// square of its last digit lands there (dropping it biases K_ii by ~1e-11); the
// errors left are the truncation r of C and the levels l > ND, below 2^(-49) of
// the row scales: error-free splitting of a product into exact low-precision products
// (Ozaki, Ogita, Oishi and Rump, Numer. Algorithms 59 (2012) 95-118), here with
// per-row power-of-two scaling and integer arithmetic.
// ---------------------------------------------------------------------------
constexpr int ND = 6;       // int8 digits per element
constexpr int NL = ND + 1;  // levels a + b kept
constexpr int DKS = 64;     // k per stage (bytes of a digit row)
constexpr int DMAXK = 87000;

// per-row exponent: s_i = 2^e_i with max_P |C[i][P]| < 2^(e_i - 1) (FP32 or FP64 rows)
template <typename TF>
__global__ __launch_bounds__(256) void k_row_scale(const TF *__restrict__ C, long long ld,
                                                   int ncol, int *exps) {
  __shared__ TF red[4];
  const int i = blockIdx.x;
  TF m = 0;
  for (int c = threadIdx.x; c < ncol; c += 256) m = fmax(m, fabs(C[(long long)i * ld + c]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const TF t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = 0;
    if (t > 0) {
      int ex;
      frexp(t, &ex);  // t = f 2^ex, f in [0.5, 1)  ->  t < 2^ex
      e = ex + 1;     // |x| = |c| / 2^e < 1/2
    }
    exps[i] = e;
  }
}

// digit planes [ND][nrow][kp] (kp = ncol rounded up to DKS, zero beyond ncol);
// one thread per 4 consecutive elements of a row, stored as one 4-byte word per plane.
// Each digit is the rounded top 7 bits of what the earlier digits left, and the
// subtraction is exact in the element's own precision.
template <typename TF>
__global__ void k_split_i8(const TF *__restrict__ C, long long ld, int nrow, int ncol, int kp,
                           const int *__restrict__ exps, signed char *dig) {
  const long long plane = (long long)nrow * kp;
  const int q = kp / 4;
  const long long n = (long long)nrow * q;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / q), c0 = (int)(t - (long long)i * q) * 4;
    TF x[4];
#pragma unroll
    for (int e = 0; e < 4; e++)
      x[e] = (c0 + e < ncol) ? ldexp(C[(long long)i * ld + c0 + e], -exps[i]) : TF(0);
#pragma unroll
    for (int k = 0; k < ND; k++) {
      unsigned w = 0;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const TF d = rint(ldexp(x[e], 7 * (k + 1)));
        x[e] -= ldexp(d, -7 * (k + 1));
        w |= ((unsigned)(int)d & 0xffu) << (8 * e);
      }
      *(unsigned *)(dig + k * plane + (long long)i * kp + c0) = w;
    }
  }
}

int digit_kp(int ncol) { return (ncol + DKS - 1) / DKS * DKS; }
size_t digit_bytes(int nrow, int ncol) { return (size_t)ND * nrow * digit_kp(ncol); }
int digit_max_k() { return DMAXK; }

template <typename TF>
static hipError_t split_digits(const TF *C, long long ld, int nrow, int ncol, int *exps, void *dig,
                               hipStream_t s) {
  if (nrow <= 0 || ncol <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_scale<TF>, dim3(nrow), dim3(256), 0, s, C, ld, ncol, exps);
  const int kp = digit_kp(ncol);
  const long long n = (long long)nrow * (kp / 4);
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_split_i8<TF>, dim3((unsigned)nb), dim3(256), 0, s, C, ld, nrow, ncol, kp,
                     (const int *)exps, (signed char *)dig);
  return hipGetLastError();
}

hipError_t launch_split_digits(const float *C, int nrow, int ncol, int *exps, void *dig,
                               hipStream_t s) {
  return split_digits(C, (long long)ncol, nrow, ncol, exps, dig, s);
}

hipError_t launch_split_digits_f64(const double *A, long long lda, int nrow, int ncol, int *exps,
                                   void *dig, hipStream_t s) {
  return split_digits(A, lda, nrow, ncol, exps, dig, s);
}

// Products of digit planes on 128 x 64 output tiles (rows 128 ti.., columns 64 tj..):
// C_ij = s_i t_j 2^(eadd - 14) sum_l 2^(-7 l) S_l over the rows i of A's planes and
// the rows j of B's planes (both with k along the row), the SYRK K = C C^T when A
// and B are the same planes, or a general product (A B^T).  The SYRK
// with eight waves of 32 x 32 (2 x 2 MFMA 16x16x64 tiles, NL level accumulators
// each).  Stages of 64 k move all planes of the tile's 192 rows (72 KB) into LDS
// by direct global-to-LDS loads, double-buffered: the next stage is in flight
// while the current one is multiplied.  A stage is [plane][12 blocks][16 rows][64 B];
// blocks 0-7 hold the 128 A rows, 8-11 the 64 B rows; within a row the four 16-byte
// k segments are stored in the order s ^ dsw(row), so that the 16 rows of a
// fragment read hit distinct banks.  Each stage first reads the fragments of planes
// 0-2, then issues the reads of planes 3-5 between the 36 products that need only
// planes 0-2, then the other 68 products.  Every element is written
// at (i, j) and at (j, i): K is symmetric, so tiles that cross the diagonal or
// repeat a block only store the same values again.
constexpr int DNT = 512;
constexpr int DSTG = ND * 12 * 1024;   // bytes per stage
typedef int i4 __attribute__((ext_vector_type(4)));

// bank swizzle of the k segments of row r (r = 0..15 within a block)
__device__ __forceinline__ int dsw(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

template <bool SAMEB>
__device__ __forceinline__ void dig_issue(const signed char *__restrict__ digA, int MA,
                                          const signed char *__restrict__ digB, int MB,
                                          int kp, int i0, int j0, int k0, signed char *stage) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long planeA = (long long)MA * kp, planeB = (long long)MB * kp;
#pragma unroll
  for (int v = 0; v < 9; v++) {
    const int u = wave + 8 * v;            // 1 KB block: plane u / 12, block u % 12
    const int d = u / 12, rb = u - d * 12, rr = lane >> 2;
    const int seg = 16 * ((lane & 3) ^ dsw(rr));
    const signed char *src;
    if (SAMEB) {
      const int r = (rb < 8 ? i0 + 16 * rb : j0 + 16 * (rb - 8)) + rr;
      src = digA + d * planeA + (long long)min(r, MA - 1) * kp + k0 + seg;
    } else {
      src = rb < 8 ? digA + d * planeA + (long long)min(i0 + 16 * rb + rr, MA - 1) * kp + k0 + seg
                   : digB + d * planeB + (long long)min(j0 + 16 * (rb - 8) + rr, MB - 1) * kp + k0 + seg;
    }
    __builtin_amdgcn_global_load_lds((const void *)src, (lds_ptr)(stage + u * 1024), 16, 0, 0);
  }
}

// SYM: the listed tiles of a symmetric result (every element also stored at (j, i));
// otherwise the tile is blockIdx.x = ti * ntj + tj.  SAMEB: B's planes are A's (the
// same value then comes out for (i, j) and (j, i), so repeated stores agree).
template <bool SYM, bool SAMEB>
__global__ __launch_bounds__(DNT) void k_digit_mm(const signed char *__restrict__ digA, int MA,
                                                  const signed char *__restrict__ digB_, int MB_,
                                                  int kp, const int *__restrict__ expsA,
                                                  const int *__restrict__ expsB, int eadd,
                                                  double *C, long long ldc,
                                                  const int2 *__restrict__ tiles, int ntj) {
  __shared__ __attribute__((aligned(16))) signed char st_l[2 * DSTG];
  // (a SYRK reads both operands from A's planes)
  const signed char *__restrict__ digB = SAMEB ? digA : digB_;
  const int MB = SAMEB ? MA : MB_;
  int2 t;
  if (SYM) {
    t = tiles[blockIdx.x];
  } else {
    t.x = (int)(blockIdx.x / ntj);
    t.y = (int)(blockIdx.x - t.x * ntj);
  }
  const int i0 = t.x * 128, j0 = t.y * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const int soff = l15 * 64 + ((lhi ^ dsw(l15)) * 16);   // this lane's 16 bytes of a block
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  i4 lev[NL][2][2];
#pragma unroll
  for (int l = 0; l < NL; l++)
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) lev[l][a][b] = (i4){0, 0, 0, 0};
  const int nst = kp / DKS;
  dig_issue<SAMEB>(digA, MA, digB, MB, kp, i0, j0, 0, st_l);
  for (int st = 0; st < nst; st++) {
    const signed char *S = st_l + (st & 1) * DSTG;
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (st + 1 < nst) dig_issue<SAMEB>(digA, MA, digB, MB, kp, i0, j0, (st + 1) * DKS, st_l + ((st + 1) & 1) * DSTG);
    // fragment of 16 rows x 64 k: lane l reads row l & 15, bytes 16 (l >> 4) ..
    i4 af[ND][2], bf[ND][2];
#pragma unroll
    for (int d = 0; d < ND; d++) {
#pragma unroll
      for (int a = 0; a < 2; a++) af[d][a] = *(const i4 *)(S + (d * 12 + (wr >> 4) + a) * 1024 + soff);
#pragma unroll
      for (int b = 0; b < 2; b++) bf[d][b] = *(const i4 *)(S + (d * 12 + 8 + (wc >> 4) + b) * 1024 + soff);
    }
    // the products of planes 0-2, then the rest (each level's sum keeps the order
    // of its products within these two groups)
#pragma unroll
    for (int la = 0; la < 3; la++)
#pragma unroll
      for (int lb = 0; lb < 3; lb++)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
          for (int b = 0; b < 2; b++)
            lev[la + lb][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[la][a], bf[lb][b],
                                                                        lev[la + lb][a][b], 0, 0, 0);
#pragma unroll
    for (int la = 0; la < ND; la++)
#pragma unroll
      for (int lb = 0; lb < ND; lb++)
        if (la + lb < NL && (la >= 3 || lb >= 3))
#pragma unroll
          for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
              lev[la + lb][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[la][a], bf[lb][b],
                                                                          lev[la + lb][a][b], 0, 0, 0);
    // schedule: the 12 reads of planes 0-2, then one read of planes 3-5 after every
    // 3 of the 36 products of planes 0-2, then the other 68 products
    __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
#pragma unroll
    for (int g = 0; g < 12; g++) {
      __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 68, 0);
  }
  // int32 accumulator layout: lane l, register v -> row 4 (l >> 4) + v, column l & 15
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = i0 + wr + a * 16 + 4 * lhi + v;
        const int j = j0 + wc + b * 16 + l15;
        // a symmetric result from two different operands is stored from i <= j only
        // (its (j, i) value, from the other operand order, can differ in the last
        // bits); elements with i > j lie in diagonal blocks, with their (j, i) in the
        // same tile
        if (i < MA && j < MB && (SAMEB || !SYM || i <= j)) {
          double sum = 0.0;
#pragma unroll
          for (int l = NL - 1; l >= 0; l--) sum += ldexp((double)lev[l][a][b][v], -7 * l);
          const double val = ldexp(sum, expsA[i] + expsB[j] + eadd - 14);
          C[(long long)i * ldc + j] = val;
          if (SYM) C[(long long)j * ldc + i] = val;
        }
      }
}

hipError_t launch_syrk_digits(const void *dig, int M, int K, const int *exps, double *C,
                              long long ldc, const int2 *tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (K > DMAXK) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_digit_mm<true, true>), dim3(ntiles), dim3(DNT), 0, s, (const signed char *)dig,
                     M, (const signed char *)dig, M, digit_kp(K), exps, exps, 0, C, ldc, tiles, 0);
  return hipGetLastError();
}

hipError_t launch_syr2_digits(const void *digA, const void *digB, int M, int K, const int *expsA,
                              const int *expsB, double *C, long long ldc, const int2 *tiles,
                              int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (K > DMAXK) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_digit_mm<true, false>), dim3(ntiles), dim3(DNT), 0, s, (const signed char *)digA,
                     M, (const signed char *)digB, M, digit_kp(K), expsA, expsB, 0, C, ldc, tiles, 0);
  return hipGetLastError();
}

hipError_t launch_gemm_digits(const void *digA, int MA, const void *digB, int MB, int K,
                              const int *expsA, const int *expsB, int eadd, double *C,
                              long long ldc, hipStream_t s) {
  if (MA <= 0 || MB <= 0) return hipSuccess;
  if (K > DMAXK) return hipErrorInvalidValue;
  const int nti = (MA + 127) / 128, ntj = (MB + 63) / 64;
  hipLaunchKernelGGL((k_digit_mm<false, false>), dim3((unsigned)nti * ntj), dim3(DNT), 0, s,
                     (const signed char *)digA, MA, (const signed char *)digB, MB, digit_kp(K),
                     expsA, expsB, eadd, C, ldc, nullptr, ntj);
  return hipGetLastError();
}

// Xt (cols x rows) = X^T for a row-major X (rows x cols), through 32 x 32 LDS tiles
template <typename TF>
__global__ __launch_bounds__(256) void k_transpose(const TF *__restrict__ X, int rows, int cols,
                                                   TF *__restrict__ Xt) {
  __shared__ TF tl[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) tl[y][tx] = X[(long long)r * cols + c];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) Xt[(long long)c * rows + r] = tl[tx][y];
  }
}

hipError_t launch_transpose_f32(const float *X, int rows, int cols, float *Xt, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s, X, rows, cols, Xt);
  return hipGetLastError();
}

// Y = X diag(w) for a row-major X (rows x cols)
__global__ void k_scale_cols(const double *__restrict__ X, const double *__restrict__ w, int rows,
                             int cols, double *__restrict__ Y) {
  const long long n = (long long)rows * cols;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    Y[t] = X[t] * w[t % cols];
}

hipError_t launch_scale_cols(const double *X, const double *w, int rows, int cols, double *Y,
                             hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const long long n = (long long)rows * cols;
  const int nb = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_scale_cols, dim3(nb), dim3(256), 0, s, X, w, rows, cols, Y);
  return hipGetLastError();
}

hipError_t launch_transpose_f64(const double *X, int rows, int cols, double *Xt, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, s, X, rows, cols, Xt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_f32_to_f64(const float *__restrict__ x, double *__restrict__ y, long long n) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    y[t] = (double)x[t];
}

hipError_t launch_f32_to_f64(const float *x, double *y, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)nb), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}
__global__ void k_fill_i32(int *p, int v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
static unsigned nblk(long long n) {
  long long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}
hipError_t launch_fill_i32(int *p, int v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(nblk(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

template <typename T>
__global__ void k_check_finite(const T *x, long long n, int *flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v = (double)x[i];
    if (!(v - v == 0.0)) bad = 1;  // NaN or Inf
  }
  if (bad) atomicOr(flag, 1);
}
hipError_t launch_check_finite(const double *x, long long n, int *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite<double>, dim3(nblk(n)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}
hipError_t launch_check_finite_f32(const float *x, long long n, int *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite<float>, dim3(nblk(n)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

// out[j] = sum_i w[j*n + i] * x[i] in a fixed order (one workgroup per j):
// per-thread strided partial sums, then a fixed shared-memory tree.
__global__ __launch_bounds__(256) void k_wdot(const double *x, const double *w, long long n,
                                              double *out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) s += w[(long long)j * n + i] * x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}
hipError_t launch_wdot(const double *x, const double *w, long long n, int nw, double *out,
                       hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wdot, dim3(nw), dim3(256), 0, s, x, w, n, out);
  return hipGetLastError();
}

// out[a] = sum_y Qt[y][a] * Zt[y][a] (column dot over nosv rows) in two passes:
// part[c][a] sums the rows of chunk c (COLDOT_ROWS rows, in order), then out[a]
// sums the chunks in order: deterministic.
__global__ void k_coldot(const double *Qt, const double *Zt, int nosv, int nvir, double *part) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (a >= nvir) return;
  const int y1 = min(nosv, (c + 1) * COLDOT_ROWS);
  double s = 0.0;
  for (int y = c * COLDOT_ROWS; y < y1; y++)
    s += Qt[(long long)y * nvir + a] * Zt[(long long)y * nvir + a];
  part[(long long)c * nvir + a] = s;
}
__global__ void k_coldot_sum(const double *part, int nchunk, int nvir, double *out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nvir) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; c++) s += part[(long long)c * nvir + a];
  out[a] = s;
}
hipError_t launch_coldot(const double *Qt, const double *Zt, int nosv, int nvir, double *part,
                         double *out, hipStream_t s) {
  if (nvir <= 0) return hipSuccess;
  const int nchunk = (nosv + COLDOT_ROWS - 1) / COLDOT_ROWS;
  if (nchunk > 0)
    hipLaunchKernelGGL(k_coldot, dim3((nvir + 255) / 256, nchunk), dim3(256), 0, s, Qt, Zt, nosv,
                       nvir, part);
  hipLaunchKernelGGL(k_coldot_sum, dim3((nvir + 255) / 256), dim3(256), 0, s, part, nchunk, nvir,
                     out);
  return hipGetLastError();
}

// dE/df_uv = sum over the clusters holding u and v of c_X * Pl[entry]; the host
// lists, per (u,v), the (coefficient index, Pl index) pairs in cluster order.
__global__ void k_pocc(const long long *ptr, const long long *idx, const double *coef,
                       const double *Pl, int nocc, double *out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nocc * nocc) return;
  double s = 0.0;
  for (long long t = ptr[e]; t < ptr[e + 1]; t++) s += coef[idx[2 * t]] * Pl[idx[2 * t + 1]];
  out[e] = s;
}
hipError_t launch_pocc(const long long *ptr, const long long *idx, const double *coef,
                       const double *Pl, int nocc, double *out, hipStream_t s) {
  int n = nocc * nocc;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pocc, dim3((n + 255) / 256), dim3(256), 0, s, ptr, idx, coef, Pl, nocc,
                     out);
  return hipGetLastError();
}

}  // namespace osv

namespace osv {
// s[i][j] = sum over the (i, j) orbital block of S^2 (for the overlap metric
// eq:2bscreen); one thread per LMO pair i < j.
__global__ void k_block_sumsq(const double *S, long long ld, const int *off, const int *r,
                              int nocc, double *out) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nocc * nocc) return;
  int i = (int)(e / nocc), j = (int)(e % nocc);
  double s = 0.0;
  if (i < j)
    for (int a = 0; a < r[i]; a++)
      for (int b = 0; b < r[j]; b++) {
        double v = S[(long long)(off[i] + a) * ld + off[j] + b];
        s += v * v;
      }
  out[e] = s;
}
hipError_t launch_block_sumsq(const double *S, long long ld, const int *off, const int *r,
                              int nocc, double *out, hipStream_t s) {
  long long n = (long long)nocc * nocc;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_sumsq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, ld,
                     off, r, nocc, out);
  return hipGetLastError();
}
}  // namespace osv
