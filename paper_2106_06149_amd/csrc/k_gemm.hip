// Dense tile kernels for the orbital-pair blocks and the back-transforms.
//
//   S_(i,j) = Q_i^T Q_j,  F_(i,j) = Q_i^T diag(eps) Q_j   (eq:aijkl, pair tasks of Algorithm 1)
//   K_ij    = C_i C_j^T                                    (pair tasks of Algorithm 1)
//   dE/dC   = 2 G^K C,  Z^T = G^F Q^T, D^v = Q Z^T          (back-transforms of the densities)
//
// All of them are written as one 64x64-tile MFMA kernel over the full
// sum(r) x sum(r) (or sum(r) x n) index space; a tile list skips tiles that
// hold no needed orbital-pair block.  FP64 tiles use v_mfma_f64_16x16x4f64,
// the mixed-precision K uses v_mfma_f32_16x16x32_bf16 on hi/mid/lo bfloat16
// splits of the FP32 input, with each 32-long k-chunk flushed into FP64.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

hipError_t launch_syrk_f64(const void *A, int a_is_f32, long long lda, int M, int K,
                           const double *w, double *C, double *C2, long long ldc,
                           const int2 *tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(256);
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
// Mixed precision K = C C^T.  C (FP32) = hi + mid + lo exactly, each bfloat16
// (8 significant bits each).  Products of two bfloat16 are exact in FP32; the
// product set is chosen by nterms: 3 -> hh, hm, mh; 6 -> + hl, lh, mm; 9 -> all.
// Each 32-long k-chunk is accumulated by MFMA in FP32 and then added in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }  // round to nearest even

__global__ void k_split_bf16(const float *__restrict__ x, long long n, __bf16 *hi, __bf16 *mid,
                             __bf16 *lo) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float v = x[i];
    __bf16 h = f2bf(v);
    float r1 = v - (float)h;
    __bf16 m = f2bf(r1);
    float r2 = r1 - (float)m;
    hi[i] = h;
    mid[i] = m;
    lo[i] = f2bf(r2);
  }
}

hipError_t launch_split_bf16(const float *A, long long n, void *hi, void *mid, void *lo,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)nb), dim3(256), 0, s, A, n, (__bf16 *)hi,
                     (__bf16 *)mid, (__bf16 *)lo);
  return hipGetLastError();
}

constexpr int KB = 32;        // k per bf16 MFMA step
constexpr int LDB16 = KB + 8; // LDS row stride (bf16 elements): 80 bytes

template <int NT>
__global__ __launch_bounds__(256) void k_syrk_bf16x(const __bf16 *__restrict__ hi,
                                                    const __bf16 *__restrict__ mid,
                                                    const __bf16 *__restrict__ lo, long long lda,
                                                    int M, int K, double *C, long long ldc,
                                                    const int2 *__restrict__ tiles) {
  __shared__ __attribute__((aligned(16))) __bf16 As[3][TB * LDB16];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[3][TB * LDB16];
  int2 t = tiles[blockIdx.x];
  const int ti = t.x, tj = t.y;
  const int i0 = ti * TB, j0 = tj * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const __bf16 *src[3] = {hi, mid, lo};
  d4 acc[2][2];
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) acc[a][b] = (d4){0, 0, 0, 0};
  constexpr int NL = (NT == 3) ? 2 : 3;  // split levels that take part
  for (int k0 = 0; k0 < K; k0 += KB) {
    // stage 64 rows x 32 k of each level for the row tile and the column tile:
    // 64*32 = 2048 elements = 256 threads x 8
    {
      int r = tid >> 2, kq = (tid & 3) * 8;
      for (int lv = 0; lv < NL; lv++) {
        bf8 va, vb;
        for (int e = 0; e < 8; e++) {
          int gk = k0 + kq + e;
          int gi = i0 + r, gj = j0 + r;
          va[e] = (gi < M && gk < K) ? src[lv][(long long)gi * lda + gk] : (__bf16)0.0f;
          vb[e] = (gj < M && gk < K) ? src[lv][(long long)gj * lda + gk] : (__bf16)0.0f;
        }
        *(bf8 *)&As[lv][r * LDB16 + kq] = va;
        *(bf8 *)&Bs[lv][r * LDB16 + kq] = vb;
      }
    }
    __syncthreads();
    const int kq = (lane >> 4) * 8;
    f4 part[2][2];
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) part[a][b] = (f4){0, 0, 0, 0};
    // small products first, the hi*hi product last
#pragma unroll
    for (int pi = 0; pi < NT; pi++) {
      // product list ordered from smallest to largest magnitude
      const int la_tab[9] = {2, 1, 2, 0, 1, 2, 0, 1, 0};
      const int lb_tab[9] = {2, 2, 1, 2, 1, 0, 1, 0, 0};
      const int off = 9 - NT;
      const int la = la_tab[off + pi], lb = lb_tab[off + pi];
      bf8 af[2], bfv[2];
#pragma unroll
      for (int a = 0; a < 2; a++) af[a] = *(const bf8 *)&As[la][(wr + a * 16 + (lane & 15)) * LDB16 + kq];
#pragma unroll
      for (int b = 0; b < 2; b++) bfv[b] = *(const bf8 *)&Bs[lb][(wc + b * 16 + (lane & 15)) * LDB16 + kq];
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
          part[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfv[b], part[a][b], 0, 0, 0);
    }
    // f32 layout: lane l, reg v -> row 4(l>>4) + v, col l & 15.  Convert to the
    // f64 accumulator layout (row (l>>4) + 4v) by keeping the f32 layout and
    // storing with the f32 map below.
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++)
        for (int v = 0; v < 4; v++) acc[a][b][v] += (double)part[a][b][v];
    __syncthreads();
  }
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int v = 0; v < 4; v++) {
        int i = i0 + wr + a * 16 + 4 * (lane >> 4) + v;
        int j = j0 + wc + b * 16 + (lane & 15);
        if (i < M && j < M) {
          C[(long long)i * ldc + j] = acc[a][b][v];
          if (ti != tj) C[(long long)j * ldc + i] = acc[a][b][v];
        }
      }
}

hipError_t launch_syrk_bf16x(const void *hi, const void *mid, const void *lo, long long lda,
                             int M, int K, int nterms, double *C, long long ldc,
                             const int2 *tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(256);
  const __bf16 *h = (const __bf16 *)hi, *m = (const __bf16 *)mid, *l = (const __bf16 *)lo;
  if (nterms == 3)
    hipLaunchKernelGGL(k_syrk_bf16x<3>, grid, block, 0, s, h, m, l, lda, M, K, C, ldc, tiles);
  else if (nterms == 6)
    hipLaunchKernelGGL(k_syrk_bf16x<6>, grid, block, 0, s, h, m, l, lda, M, K, C, ldc, tiles);
  else if (nterms == 9)
    hipLaunchKernelGGL(k_syrk_bf16x<9>, grid, block, 0, s, h, m, l, lda, M, K, C, ldc, tiles);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
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

// out[a] = sum_y Qt[y][a] * Zt[y][a]  (column dot over nosv rows; one thread per a,
// rows in order -> deterministic)
__global__ void k_coldot(const double *Qt, const double *Zt, int nosv, int nvir, double *out) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nvir) return;
  double s = 0.0;
  for (int y = 0; y < nosv; y++) s += Qt[(long long)y * nvir + a] * Zt[(long long)y * nvir + a];
  out[a] = s;
}
hipError_t launch_coldot(const double *Qt, const double *Zt, int nosv, int nvir, double *out,
                         hipStream_t s) {
  if (nvir <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coldot, dim3((nvir + 255) / 256), dim3(256), 0, s, Qt, Zt, nosv, nvir,
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
