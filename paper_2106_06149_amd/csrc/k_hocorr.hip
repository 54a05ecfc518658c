// One-step high-order correction of the MBE(3) amplitudes (section on the
// high-order MBE(n) contribution).
//
// 1. Collective amplitudes per pair domain d = [pq], in its pseudo-canonical basis:
//      T~c_d = sum over the clusters X holding the pair of c_X T~^X_d
//    (eq:tmbediag / eq:tmbeoff with the inclusion-exclusion coefficients), both
//    orientations, zero-padded np x np slots, summed in cluster order.
// 2. Per target domain d, the residual eq:rij at the collective amplitudes with k
//    over the LMOs that share a cluster with p and q:
//      R~ = K~ + (e~_a + e~_b - f_pp - f_qq) T~c + sum_terms (-f) M op(T~c_src) M^T,
//    then one Jacobi step dT~ = -R~ / Delta on the kept rank, and per domain
//      dE_d = w <K~, 2 dT~ - dT~^T>,  E_d = w <K~, 2 T~c - T~c^T>,  ||R~||_F^2
//    (w = 1 for p = q, 2 otherwise).  Each term runs as two FP64 MFMA products:
//    X = M(tgt,src) op(T~c) into LDS, then R~ += coef X M(tgt,src)^T with R~ in
//    the accumulators of the wave that owns its 16 x 16 tile.
#include "osv_internal.h"
#include "tiles.h"

namespace osv {

typedef double d4h __attribute__((ext_vector_type(4)));

constexpr int HNT = 256;           // threads per domain
constexpr int HNW = HNT / 64;
constexpr int HMT = 7;             // 16-tiles per dimension (np <= 112)
constexpr int HLD = 16 * HMT + 1;  // LDS stride of X
constexpr int HTPW = (HMT * HMT + HNW - 1) / HNW;   // R~ tiles per wave

__global__ __launch_bounds__(HNT) void k_collective(const Domain *__restrict__ doms,
                                                    const long long *__restrict__ ptr,
                                                    const long long *__restrict__ toff,
                                                    const double *__restrict__ coef,
                                                    const double *__restrict__ T,
                                                    const long long *__restrict__ coff, double *Tc) {
  const int d = blockIdx.x;
  const int np = doms[d].np;
  const long long n2 = 2LL * np * np;
  double *out = Tc + coff[d];
  const long long x0 = ptr[d], x1 = ptr[d + 1];
  for (long long e = threadIdx.x; e < n2; e += HNT) {
    // four clusters' loads in flight; the sum keeps the cluster order
    double s = 0.0;
    long long x = x0;
    for (; x + 4 <= x1; x += 4) {
      const double v0 = T[toff[x] + e], v1 = T[toff[x + 1] + e];
      const double v2 = T[toff[x + 2] + e], v3 = T[toff[x + 3] + e];
      s += coef[x] * v0;
      s += coef[x + 1] * v1;
      s += coef[x + 2] * v2;
      s += coef[x + 3] * v3;
    }
    for (; x < x1; x++) s += coef[x] * T[toff[x] + e];
    out[e] = s;
  }
}

hipError_t launch_collective(const Domain *dom, int ndom, const long long *ptr, const long long *toff,
                             const double *coef, const double *T, const long long *coff, double *Tc,
                             hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_collective, dim3(ndom), dim3(HNT), 0, s, dom, ptr, toff, coef, T, coff, Tc);
  return hipGetLastError();
}

__device__ __forceinline__ double hsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(HNT) void k_collective_step(const Domain *__restrict__ doms,
                                                         const int *__restrict__ rank,
                                                         const long long *__restrict__ tptr,
                                                         const CTerm *__restrict__ terms,
                                                         const double *__restrict__ Tc,
                                                         const long long *__restrict__ coff,
                                                         const double *__restrict__ M,
                                                         const double *__restrict__ Kep,
                                                         const double *__restrict__ F, int nocc,
                                                         double *out) {
  __shared__ double X[16 * HMT * HLD];
  __shared__ double red[3 * HNW];
  const int d = blockIdx.x;
  const Domain D = doms[d];
  const int np = D.np, nt = rank[d];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const int tb = np >> 4;                  // 16-tiles per dimension of the target
  d4h R[HTPW];
#pragma unroll
  for (int u = 0; u < HTPW; u++) R[u] = (d4h){0, 0, 0, 0};
  for (long long t = tptr[d]; t < tptr[d + 1]; t++) {
    const CTerm tm = terms[t];
    const double cf = -F[(long long)tm.fa * nocc + tm.fb];
    const int ns = rank[tm.src], nps = tm.ldT, sb = (ns + 15) >> 4;
    const double *Tg = Tc + tm.tsrc;       // op(T~c_src), np_s x np_s row-major
    const double *Mg = M + tm.moff;        // M(src, tgt), np_s x np_t row-major
    // X(i, k) = sum_j M(tgt,src)(i, j) op(T)(j, k) = sum_j Mg[j np_t + i] Tg[j np_s + k]
    // for the target's kept rows (rows of X past nt feed only rows of R~ that are
    // never read); the operands of 8 k-steps are loaded before their MFMAs
    (void)sb;
    mma_tiles<HNT>(nt, ns, ns, [&](int i, int j) { return Mg[(long long)j * np + i]; },
                   [&](int j, int k) { return Tg[(long long)j * nps + k]; },
                   [&](int i, int k, double v) { X[i * HLD + k] = v; });
    __syncthreads();
    // R(i, l) += cf sum_k X(i, k) M(tgt,src)(l, k) = cf sum_k X(i, k) Mg[k np_t + l]
#pragma unroll
    for (int u = 0; u < HTPW; u++) {
      const int tau = wave + HNW * u;
      if (tau < tb * tb) {
        const int ib = tau / tb, lb = tau - ib * tb;
        const int i = 16 * ib + l15, l = 16 * lb + l15;
        // 8 k-steps of operands loaded before their MFMAs
        for (int k0 = 0; k0 < ns; k0 += 32) {
          double a[8], b[8];
#pragma unroll
          for (int st = 0; st < 8; st++) {
            const int k = k0 + 4 * st + lhi;
            a[st] = (k < ns) ? X[i * HLD + k] : 0.0;
            b[st] = (k < ns) ? cf * Mg[(long long)k * np + l] : 0.0;
          }
#pragma unroll
          for (int st = 0; st < 8; st++)
            if (k0 + 4 * st < ns) R[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], R[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // epilogue: R~ = terms + K~ + Delta T~c, the step -R~ / Delta and the sums
  const double *Kt = Kep + D.voff, *ev = Kt + (long long)np * np;   // Kt[b np + a] = K~(a, b)
  const double *Td = Tc + coff[d];
  const double fd = F[(long long)D.p * nocc + D.p] + F[(long long)D.q * nocc + D.q];
  const double w = (D.p == D.q) ? 1.0 : 2.0;
  double sE = 0.0, sC = 0.0, sR = 0.0;
#pragma unroll
  for (int u = 0; u < HTPW; u++) {
    const int tau = wave + HNW * u;
    if (tau < tb * tb) {
      const int ib = tau / tb, lb = tau - ib * tb;
      const int l = 16 * lb + l15;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = 16 * ib + 4 * v + lhi;
        if (i < nt && l < nt) {
          const double kil = Kt[(long long)l * np + i], kli = Kt[(long long)i * np + l];
          const double delta = ev[i] + ev[l] - fd;
          const double tc = Td[(long long)i * np + l];
          const double r = R[u][v] + kil + delta * tc;
          const double dt = -r / delta;
          sE += dt * (2.0 * kil - kli);
          sC += tc * (2.0 * kil - kli);
          sR += r * r;
        }
      }
    }
  }
  sE = hsum(sE);
  sC = hsum(sC);
  sR = hsum(sR);
  if (lane == 0) {
    red[wave] = sE;
    red[HNW + wave] = sC;
    red[2 * HNW + wave] = sR;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = 0; q < HNW; q++) {
      a += red[q];
      b += red[HNW + q];
      c += red[2 * HNW + q];
    }
    out[3LL * d] = w * a;
    out[3LL * d + 1] = w * b;
    out[3LL * d + 2] = c;
  }
}

hipError_t launch_collective_step(const Domain *dom, int ndom, const int *rank, const long long *tptr,
                                  const CTerm *terms, const double *Tc, const long long *coff,
                                  const double *M, const double *Kep, const double *F, int nocc,
                                  double *out, hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_collective_step, dim3(ndom), dim3(HNT), 0, s, dom, rank, tptr, terms, Tc, coff, M,
                     Kep, F, nocc, out);
  return hipGetLastError();
}

}  // namespace osv
