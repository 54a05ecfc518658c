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
// Every term is written by one workgroup in a fixed order: no atomics.  The
// cluster amplitudes stream through LDS by direct global-to-LDS loads and all
// products run on FP64 MFMA 16x16x4.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int ANT = 1024;            // threads per domain (16 wave64, four per SIMD)
constexpr int ANW = ANT / 64;
constexpr int ALD = DMAX + 1;        // odd LDS stride of the transform matrices
constexpr int ARS = 130;             // LDS row stride of a staged amplitude row (>= 128)
constexpr int ASTG = 32 * ARS;       // stage: T~ rows 0..15, T~^T rows 16..31
constexpr int ANSTG = 4;             // ring stages (loads run three chunks ahead)
constexpr int MAXTW = (49 + ANW - 1) / ANW;   // 16x16 output tiles per wave (7 x 7)
constexpr int AROWS = 16 / ANW;      // rows of T~ (and of T~^T) each wave loads per chunk
static_assert(ANW == 16, "the chunk wait below counts 2 * AROWS loads per wave");
static_assert(ANSTG * ASTG <= 2 * DMAX * ALD, "the ring overlays the transform buffers");

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16 rows of T~ and of T~^T (rows 16q..16q+15 of the slot pair at toff, np wide) into
// a ring stage: 2 AROWS direct global-to-LDS loads per wave; lanes past the row end are
// clamped onto its last 16 bytes and fill LDS columns that are never read.
__device__ __forceinline__ void adj_issue(const double *T, long long toff, int np, int q,
                                          double *ring, int stage) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = min(2 * lane, np - 2);
  const double *Ts = T + toff + (long long)(16 * q + wave) * np + col;
  const double *Tt = Ts + (long long)np * np;
  const int lbase = __builtin_amdgcn_readfirstlane(
      (int)(size_t)(__attribute__((address_space(3))) void *)ring + (stage * ASTG + wave * ARS) * 8);
#pragma unroll
  for (int u = 0; u < AROWS; u++) {
    __builtin_amdgcn_global_load_lds((const void *)(Ts + u * ANW * np),
                                     (__attribute__((address_space(3))) void *)(size_t)(lbase + u * ANW * ARS * 8),
                                     16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void *)(Tt + u * ANW * np),
                                     (__attribute__((address_space(3))) void *)(size_t)(lbase + (16 + u * ANW) * ARS * 8),
                                     16, 0, 0);
  }
}

// Per pair domain d = [pq], over every cluster X that holds the pair (fixed order),
// with c_X the MBE coefficient and T~ the cluster amplitudes (T~ and T~^T slots):
//   A_d = sum_X c_X Tbar~,      Tbar~ = 2 T~ - T~^T
//   g_d = sum_X c_X (T~^T Tbar~ + Tbar~ T~^T) = sum_X 2 c_X (Ts^T (Ts - Tt) + Tt^T Tt)
// with Ts = T~ and Tt = T~^T as row-major slots, so every product is X^T Y of two
// row-major matrices and both MFMA operands are read along rows.  Then
//   G^F_d = W g' W^T   (g' = g + g^T for p < q, g for p = q)  -> Gd slot
//   G^K_pq = Y_p^T (2 A_d) Y_q                                  -> GK block (and transpose)
__global__ __launch_bounds__(ANT) void k_adjoint(const Domain *__restrict__ doms,
                                                 const int *__restrict__ order,
                                                 const int *__restrict__ rank,
                                                 const double *__restrict__ W,
                                                 const double *__restrict__ Y,
                                                 const double *__restrict__ Tall,
                                                 const long long *__restrict__ dcp_ptr,
                                                 const long long *__restrict__ dcp_toff,
                                                 const double *__restrict__ dcp_coef,
                                                 double *GK, long long ld, double *Gd) {
  __shared__ __attribute__((aligned(16))) double buf[2 * DMAX * ALD];
  double *L1 = buf, *L2 = buf + DMAX * ALD;
  const int d = order[blockIdx.x];   // domains in order of cost, largest first
  const Domain D = doms[d];
  const int n = D.n, np = D.np, dt = rank[d];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const bool diag = (D.p == D.q);
  const int tn = (dt + 15) >> 4, nt2 = tn * tn;

  // ---- phase 1: accumulate g and A over the domain's cluster entries -------------
  d4 g[MAXTW], A[MAXTW];
#pragma unroll
  for (int u = 0; u < MAXTW; u++) {
    g[u] = (d4){0, 0, 0, 0};
    A[u] = (d4){0, 0, 0, 0};
  }
  const long long e0 = dcp_ptr[d], e1 = dcp_ptr[d + 1];
  const long long nchunk = (e1 - e0) * tn;
  // producer: chunk k = (entry e0 + k / tn, rows 16 (k % tn) ..)
  auto issue_k = [&](long long k) {
    const long long en = e0 + k / tn;
    adj_issue(Tall, dcp_toff[en], np, (int)(k % tn), buf, (int)(k % ANSTG));
  };
  for (int k = 0; k < ANSTG - 1; k++)
    if (k < nchunk) issue_k(k);
  for (long long k = 0; k < nchunk; k++) {
    // this wave's loads of chunk k are done once at most those of the chunks issued
    // after it (2 loads each, up to two chunks) remain; then every wave is done
    // with the stage the next issue overwrites
    const long long later = nchunk - 1 - k;
    if (later >= 2)
      asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else if (later == 1)
      asm volatile("s_waitcnt vmcnt(2) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (k + ANSTG - 1 < nchunk) issue_k(k + ANSTG - 1);
    const long long en = e0 + k / tn;
    const int q = (int)(k % tn);
    const double c = dcp_coef[en], c2 = 2.0 * c;
    const double *Ts = buf + (k % ANSTG) * ASTG, *Tt = Ts + 16 * ARS;
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int tau = wave + ANW * u;
      if (tau < nt2) {
        const int ib = tau / tn, jb = tau - ib * tn;
        const int ci = 16 * ib + l15, cj = 16 * jb + l15;
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int rr = (4 * kk + lhi) * ARS;
          const double tsj = Ts[rr + cj], ttj = Tt[rr + cj];
          g[u] = mfma64(Ts[rr + ci], c2 * (tsj - ttj), g[u]);
          g[u] = mfma64(Tt[rr + ci], c2 * ttj, g[u]);
        }
        if (ib == q) {
          // A tile rows 16 ib + 4v + lhi are rows 4v + lhi of this chunk
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int rr = (4 * v + lhi) * ARS;
            A[u][v] += c * (2.0 * Ts[rr + cj] - Tt[rr + cj]);
          }
        }
      }
    }
  }
  __syncthreads();   // ring free: buf becomes L1 / L2

  // ---- phase 2: g' -> L1 (dt x dt), W -> L2 (n x n) --------------------------------
#pragma unroll
  for (int u = 0; u < MAXTW; u++) {
    const int tau = wave + ANW * u;
    if (tau < nt2) {
      const int ib = tau / tn, jb = tau - ib * tn;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = 16 * ib + 4 * v + lhi, j = 16 * jb + l15;
        if (i < dt && j < dt) L1[i * ALD + j] = g[u][v];
      }
    }
  }
  for (int e = tid; e < n * n; e += ANT) {
    const int i = e / n, a = e - i * n;
    L2[i * ALD + a] = W[D.moff + e];
  }
  __syncthreads();
  if (!diag) {
    // g' = g + g^T, through registers
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int tau = wave + ANW * u;
      if (tau < nt2) {
        const int ib = tau / tn, jb = tau - ib * tn;
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int i = 16 * ib + 4 * v + lhi, j = 16 * jb + l15;
          g[u][v] = (i < dt && j < dt) ? L1[i * ALD + j] + L1[j * ALD + i] : 0.0;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int tau = wave + ANW * u;
      if (tau < nt2) {
        const int ib = tau / tn, jb = tau - ib * tn;
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int i = 16 * ib + 4 * v + lhi, j = 16 * jb + l15;
          if (i < dt && j < dt) L1[i * ALD + j] = g[u][v];
        }
      }
    }
    __syncthreads();
  }

  // ---- phase 3: Z = W g' (n x dt) -> L1, then G^F = Z W^T (n x n) -> Gd -----------
  const int tnn = (n + 15) >> 4;
  {
    d4 Z[MAXTW];
    const int nz = tnn * tn;
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      Z[u] = (d4){0, 0, 0, 0};
      const int tau = wave + ANW * u;
      if (tau < nz) {
        const int ib = tau / tn, jb = tau - ib * tn;
        const int i = 16 * ib + l15, b = 16 * jb + l15;
        for (int a0 = 0; a0 < dt; a0 += 4) {
          const int a = a0 + lhi;
          const double w = (i < n && a < dt) ? L2[i * ALD + a] : 0.0;
          const double gv = (a < dt && b < dt) ? L1[a * ALD + b] : 0.0;
          Z[u] = mfma64(w, gv, Z[u]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int tau = wave + ANW * u;
      if (tau < nz) {
        const int ib = tau / tn, jb = tau - ib * tn;
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int i = 16 * ib + 4 * v + lhi, b = 16 * jb + l15;
          if (i < n && b < dt) L1[i * ALD + b] = Z[u][v];
        }
      }
    }
    __syncthreads();
  }
  {
    double *G = Gd + D.moff;
    for (int tau = wave; tau < tnn * tnn; tau += ANW) {
      const int ib = tau / tnn, jb = tau - ib * tnn;
      const int i = 16 * ib + l15, j = 16 * jb + l15;
      d4 acc = {0, 0, 0, 0};
      for (int b0 = 0; b0 < dt; b0 += 4) {
        const int b = b0 + lhi;
        const double z = (i < n && b < dt) ? L1[i * ALD + b] : 0.0;
        const double w = (j < n && b < dt) ? L2[j * ALD + b] : 0.0;
        acc = mfma64(z, w, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int r = 16 * ib + 4 * v + lhi;
        if (r < n && j < n) G[r * n + j] = acc[v];
      }
    }
  }
  __syncthreads();

  // ---- phase 4: G^K_pq = Y_p^T (2A) Y_q -------------------------------------------
  const int rq = diag ? D.rp : D.rq, qcol = diag ? 0 : D.rp, offq = diag ? D.offp : D.offq;
#pragma unroll
  for (int u = 0; u < MAXTW; u++) {
    const int tau = wave + ANW * u;
    if (tau < nt2) {
      const int ib = tau / tn, jb = tau - ib * tn;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = 16 * ib + 4 * v + lhi, j = 16 * jb + l15;
        if (i < dt && j < dt) L1[i * ALD + j] = 2.0 * A[u][v];
      }
    }
  }
  for (int e = tid; e < dt * n; e += ANT) {
    const int a = e / n, j = e - a * n;
    L2[a * ALD + j] = Y[D.moff + e];
  }
  __syncthreads();
  const int tq = (rq + 15) >> 4, tp = (D.rp + 15) >> 4;
  {
    // T1 = (2A) Y_q (dt x rq) -> L1
    d4 T1[MAXTW];
    const int n1 = tn * tq;
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      T1[u] = (d4){0, 0, 0, 0};
      const int tau = wave + ANW * u;
      if (tau < n1) {
        const int ib = tau / tq, jb = tau - ib * tq;
        const int a = 16 * ib + l15, j = 16 * jb + l15;
        for (int b0 = 0; b0 < dt; b0 += 4) {
          const int b = b0 + lhi;
          const double x = (a < dt && b < dt) ? L1[a * ALD + b] : 0.0;
          const double y = (b < dt && j < rq) ? L2[b * ALD + qcol + j] : 0.0;
          T1[u] = mfma64(x, y, T1[u]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXTW; u++) {
      const int tau = wave + ANW * u;
      if (tau < n1) {
        const int ib = tau / tq, jb = tau - ib * tq;
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int a = 16 * ib + 4 * v + lhi, j = 16 * jb + l15;
          if (a < dt && j < rq) L1[a * ALD + j] = T1[u][v];
        }
      }
    }
    __syncthreads();
  }
  // Gamma = Y_p^T T1 (rp x rq) -> GK at (offp, offq), and its transpose for p < q
  for (int tau = wave; tau < tp * tq; tau += ANW) {
    const int ib = tau / tq, jb = tau - ib * tq;
    const int i = 16 * ib + l15, j = 16 * jb + l15;
    d4 acc = {0, 0, 0, 0};
    for (int a0 = 0; a0 < dt; a0 += 4) {
      const int a = a0 + lhi;
      const double y = (a < dt && i < D.rp) ? L2[a * ALD + i] : 0.0;
      const double t = (a < dt && j < rq) ? L1[a * ALD + j] : 0.0;
      acc = mfma64(y, t, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int r = 16 * ib + 4 * v + lhi;
      if (r < D.rp && j < rq) {
        GK[(long long)(D.offp + r) * ld + (offq + j)] = acc[v];
        if (!diag) GK[(long long)(offq + j) * ld + (D.offp + r)] = acc[v];
      }
    }
  }
}

hipError_t launch_adjoint(const Domain *dom, int ndom, const int *order, const int *rank, const double *W,
                          const double *Y, const double *T, const long long *dcp_ptr,
                          const long long *dcp_toff, const double *dcp_coef, double *GK,
                          long long ld, double *Gd, hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint, dim3(ndom), dim3(ANT), 0, s, dom, order, rank, W, Y, T, dcp_ptr,
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
