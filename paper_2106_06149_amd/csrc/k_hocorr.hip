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
//    (w = 1 for p = q, 2 otherwise).  Each term runs as two FP64 MFMA products on
//    the LDS-staged tile product, X = M(tgt,src) op(T~c), then
//    R~ += coef X M(tgt,src)^T, in per-workgroup scratch.
#include "osv_internal.h"
#include "tiles.h"

namespace osv {

constexpr int HNT = 256;           // threads per domain of the collective sums

__global__ __launch_bounds__(HNT) void k_collective(const Domain *__restrict__ doms,
                                                   const int *__restrict__ order,
                                                    const long long *__restrict__ ptr,
                                                    const long long *__restrict__ toff,
                                                    const double *__restrict__ coef,
                                                    const double *__restrict__ T,
                                                    const long long *__restrict__ coff, double *Tc) {
  const int d = order[blockIdx.x];   // domains in order of cost, largest first
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

hipError_t launch_collective(const Domain *dom, int ndom, const int *order, const long long *ptr,
                             const long long *toff,
                             const double *coef, const double *T, const long long *coff, double *Tc,
                             hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_collective, dim3(ndom), dim3(HNT), 0, s, dom, order, ptr, toff, coef, T, coff, Tc);
  return hipGetLastError();
}

__device__ __forceinline__ double hsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The residual step: one persistent workgroup of eight waves per CU takes target
// domains from a queue (most terms first).  Per term, X = M(tgt,src) op(T~c) and
// R~ += coef X M(tgt,src)^T run on the LDS-staged tile product (gemm_lds), X and
// R~ (kept rows and columns only) in the workgroup's scratch; then the epilogue.
constexpr int CNT = 512;
constexpr int CLD = 112;   // row stride of X and R~ in scratch

__global__ __launch_bounds__(CNT) void k_collective_step(const Domain *__restrict__ doms,
                                                         const int *__restrict__ rank,
                                                         const long long *__restrict__ tptr,
                                                         const CTerm *__restrict__ terms,
                                                         const double *__restrict__ Tc,
                                                         const long long *__restrict__ coff,
                                                         const double *__restrict__ M,
                                                         const double *__restrict__ Kep,
                                                         const double *__restrict__ F, int nocc,
                                                         const int *__restrict__ queue, int ndom,
                                                         int *counter, double *scr, double *out) {
  __shared__ int s_next;
  __shared__ __align__(16) double lds[gemm_lds_doubles()];
  __shared__ double red[3 * (CNT / 64)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *R = scr + (long long)blockIdx.x * 2 * CLD * CLD, *X = R + CLD * CLD;
  for (;;) {
    if (tid == 0) s_next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_next;
    __syncthreads();
    if (it >= ndom) break;
    const int d = queue[it];
    const Domain D = doms[d];
    const int np = D.np, nt = rank[d];
    for (int e = tid; e < nt * CLD; e += CNT) R[e] = 0.0;
    __syncthreads();
    for (long long t = tptr[d]; t < tptr[d + 1]; t++) {
      const CTerm tm = terms[t];
      const double cf = -F[(long long)tm.fa * nocc + tm.fb];
      const int ns = rank[tm.src], nps = tm.ldT;
      const double *Tg = Tc + tm.tsrc;   // op(T~c_src), np_s x np_s row-major
      const double *Mg = M + tm.moff;    // M(src, tgt), np_s x np_t row-major
      // X(i, k) = sum_j M(tgt,src)(i, j) op(T)(j, k), M(tgt,src)(i, j) = Mg[j np_t + i]
      gemm_lds<CNT>(nt, ns, ns, Mat{Mg, np, 1}, Mat{Tg, nps, 0}, lds,
                    [&](int i, int k, double v) { X[i * CLD + k] = v; });
      // R(i, l) += cf sum_k X(i, k) M(tgt,src)(l, k) = cf sum_k X(i, k) Mg[k np_t + l]
      gemm_lds<CNT>(nt, nt, ns, Mat{X, CLD, 0}, Mat{Mg, np, 0}, lds,
                    [&](int i, int l, double v) { R[i * CLD + l] += cf * v; });
    }
    __syncthreads();
    // epilogue: R~ = terms + K~ + Delta T~c, the step -R~ / Delta and the sums
    const double *Kt = Kep + D.voff, *ev = Kt + (long long)np * np;   // Kt[b np + a] = K~(a, b)
    const double *Td = Tc + coff[d];
    const double fd = F[(long long)D.p * nocc + D.p] + F[(long long)D.q * nocc + D.q];
    const double w = (D.p == D.q) ? 1.0 : 2.0;
    double sE = 0.0, sC = 0.0, sR = 0.0;
    for (int e = tid; e < nt * nt; e += CNT) {
      const int i = e / nt, l = e - i * nt;
      const double kil = Kt[(long long)l * np + i], kli = Kt[(long long)i * np + l];
      const double delta = ev[i] + ev[l] - fd;
      const double tc = Td[(long long)i * np + l];
      const double r = R[i * CLD + l] + kil + delta * tc;
      const double dt = -r / delta;
      sE += dt * (2.0 * kil - kli);
      sC += tc * (2.0 * kil - kli);
      sR += r * r;
    }
    sE = hsum(sE);
    sC = hsum(sC);
    sR = hsum(sR);
    if (lane == 0) {
      red[wave] = sE;
      red[CNT / 64 + wave] = sC;
      red[2 * (CNT / 64) + wave] = sR;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0, c = 0.0;
      for (int q = 0; q < CNT / 64; q++) {
        a += red[q];
        b += red[CNT / 64 + q];
        c += red[2 * (CNT / 64) + q];
      }
      out[3LL * d] = w * a;
      out[3LL * d + 1] = w * b;
      out[3LL * d + 2] = c;
    }
    __syncthreads();
  }
}

long long collective_step_scratch(int nwg) { return (long long)nwg * 2 * CLD * CLD; }

hipError_t launch_collective_step(const Domain *dom, int ndom, const int *rank, const long long *tptr,
                                  const CTerm *terms, const double *Tc, const long long *coff,
                                  const double *M, const double *Kep, const double *F, int nocc,
                                  const int *queue, int *counter, double *scr, int nwg, double *out,
                                  hipStream_t s) {
  if (ndom <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(counter, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_collective_step, dim3(nwg), dim3(CNT), 0, s, dom, rank, tptr, terms, Tc, coff, M, Kep,
                     F, nocc, queue, ndom, counter, scr, out);
  return hipGetLastError();
}

}  // namespace osv
