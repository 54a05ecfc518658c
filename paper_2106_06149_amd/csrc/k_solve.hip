// Cluster residual solve: eq:rij for every pair of every cluster, Jacobi
// sweeps in each pair domain's pseudo-canonical basis, Hylleraas energy eq:ec.
//
// In the basis W of domain [pq] (W^T S W = 1, W^T F W = diag(e~)) the residual of
// the unordered pair p <= q of cluster X reads
//   R~_pq = K~_pq + (e~_a + e~_b - f_pp - f_qq) T~_pq
//         + sum_terms (-f_ab) M op(T~_src) M^T,     M = W_pq^T S_(pq,src) W_src,
// with one term per LMO m of X in each of the two k-sums of eq:rij, except the
// m = q (first sum) and m = p (second sum) terms, which are the diagonal factor.
// op is a transpose when the source pair is ordered (a, b) with a > b, because
// the canonical amplitudes satisfy T^{ba} = (T^{ab})^T.
//
// One workgroup owns one cluster at a time: it pops clusters from a
// cost-sorted queue, zeroes the cluster's amplitudes, and iterates
//   R~ from the current T~ for every pair; stop if max ||R~||_F < tau_R;
//   otherwise T~ <- T~ - R~ / (e~_a + e~_b - f_pp - f_qq)
// to convergence inside the kernel.  At the stopping sweep it records
//   E^X = sum_pairs w <2 T~ - T~^T, K~ + R~>       (eq:ec; w = 1 for p = q, 2 for p < q)
// and the inner products that make up dE/df_ab.  Every reduction has a fixed
// order, so results are bitwise reproducible.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int LDX = DMAX + 1;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// logical element (i, k) of a matrix stored row-major with leading dimension ld,
// or of its transpose
__device__ __forceinline__ double at(const double *p, int ld, int tr, int i, int k) {
  return tr ? p[(long long)k * ld + i] : p[(long long)i * ld + k];
}

__global__ __launch_bounds__(NTHREADS) void k_solve(SolveArgs a) {
  __shared__ double Xs[DMAX * LDX];
  __shared__ double red[16];
  __shared__ int s_cur;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *Rs = a.Rs + (long long)blockIdx.x * a.rs_stride;
  for (;;) {
    if (tid == 0) s_cur = atomicAdd(a.counter, 1);
    __syncthreads();
    const int qi = s_cur;
    __syncthreads();
    if (qi >= a.n_clusters) break;
    const int X = a.queue[qi];
    const Cluster cl = a.cl[X];
    const int nl = cl.nlmo;
    double *Pl = a.Pl + cl.poff;
    // zero the cluster's amplitudes
    for (int c = 0; c < cl.ncp; c++) {
      const CPair P = a.cp[cl.cp0 + c];
      const int n = a.dom[P.dom].n;
      double *T = a.T + P.toff;
      for (int e = tid; e < n * n; e += NTHREADS) T[e] = 0.0;
    }
    __syncthreads();
    int sweep = 0;
    double maxn = 0.0, E = 0.0;
    for (;;) {
      maxn = 0.0;
      E = 0.0;
      if (tid == 0)
        for (int e = 0; e < nl * nl; e++) Pl[e] = 0.0;
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const Domain D = a.dom[P.dom];
        const int n = D.n, nt = a.dom_rank[P.dom];
        const double *T = a.T + P.toff;
        const double *Kt = a.Kt + D.moff;
        const double *ep = a.epst + D.voff;
        double *R = Rs + (P.toff - cl.toff0);
        const double fd = a.F_occ[D.p * a.nocc + D.p] + a.F_occ[D.q * a.nocc + D.q];
        // R~ = K~ + Delta T~
        for (int e = tid; e < nt * nt; e += NTHREADS) {
          int i = e / nt, j = e % nt;
          R[i * n + j] = Kt[i * n + j] + (ep[i] + ep[j] - fd) * T[i * n + j];
        }
        __syncthreads();
        if (sweep > 0) {
          for (int t = P.term0; t < P.term0 + P.nterm; t++) {
            const Term tm = a.terms[t];
            const Coupling cp = a.cpl[tm.cpl];
            const CPair Ps = a.cp[tm.src];
            const int ns = a.dom_rank[Ps.dom];
            const int nsl = a.dom[Ps.dom].n;
            const double *Ts = a.T + Ps.toff;
            const double *Mp = a.M + cp.off;
            const int ldM = a.dom[cp.B].n;
            const int trM = tm.flags & 1, trT = (tm.flags >> 1) & 1;
            const double coef = -a.F_occ[tm.fa * a.nocc + tm.fb];
            // Xs = M op(T_src)   (nt x ns)
            const int ti_n = (nt + 15) >> 4, tj_n = (ns + 15) >> 4;
            for (int tile = wave; tile < ti_n * tj_n; tile += 4) {
              const int i0 = (tile / tj_n) * 16, j0 = (tile % tj_n) * 16;
              d4 acc = {0, 0, 0, 0};
              const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
              for (int k0 = 0; k0 < ns; k0 += 4) {
                const int k = k0 + (lane >> 4);
                double av = 0.0, bv = 0.0;
                if (ia < nt && k < ns) av = at(Mp, ldM, trM, ia, k);
                if (jb < ns && k < ns) bv = at(Ts, nsl, trT, k, jb);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
              }
              for (int v = 0; v < 4; v++) {
                const int i = i0 + (lane >> 4) + 4 * v, j = j0 + (lane & 15);
                if (i < nt && j < ns) Xs[i * LDX + j] = acc[v];
              }
            }
            __syncthreads();
            // Y = Xs M^T  (nt x nt); R~ += coef Y; val = <Tbar_tgt, Y>
            double val = 0.0;
            for (int tile = wave; tile < ti_n * ti_n; tile += 4) {
              const int i0 = (tile / ti_n) * 16, j0 = (tile % ti_n) * 16;
              d4 acc = {0, 0, 0, 0};
              const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
              for (int k0 = 0; k0 < ns; k0 += 4) {
                const int k = k0 + (lane >> 4);
                double av = 0.0, bv = 0.0;
                if (ia < nt && k < ns) av = Xs[ia * LDX + k];
                if (jb < nt && k < ns) bv = at(Mp, ldM, trM, jb, k);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
              }
              for (int v = 0; v < 4; v++) {
                const int i = i0 + (lane >> 4) + 4 * v, j = j0 + (lane & 15);
                if (i < nt && j < nt) {
                  R[i * n + j] += coef * acc[v];
                  val += (2.0 * T[i * n + j] - T[j * n + i]) * acc[v];
                }
              }
            }
            val = wsum(val);
            if (lane == 0) red[wave] = val;
            __syncthreads();
            if (tid == 0) {
              const double tv = red[0] + red[1] + red[2] + red[3];
              Pl[tm.la * nl + tm.lb] -= tv;
              if (P.la != P.lb) Pl[tm.lb * nl + tm.la] -= tv;
            }
          }
        }
        // norm, energy and same-pair dE/df pieces
        double s_nrm = 0.0, s_e = 0.0, s_v = 0.0;
        for (int e = tid; e < nt * nt; e += NTHREADS) {
          int i = e / nt, j = e % nt;
          double r = R[i * n + j];
          double tb = 2.0 * T[i * n + j] - T[j * n + i];
          s_nrm += r * r;
          s_e += tb * (Kt[i * n + j] + r);
          s_v += tb * T[i * n + j];
        }
        s_nrm = wsum(s_nrm);
        s_e = wsum(s_e);
        s_v = wsum(s_v);
        if (lane == 0) { red[4 + wave] = s_nrm; red[8 + wave] = s_e; red[12 + wave] = s_v; }
        __syncthreads();
        const double nrm = sqrt(red[4] + red[5] + red[6] + red[7]);
        const double ec = red[8] + red[9] + red[10] + red[11];
        const double vv = red[12] + red[13] + red[14] + red[15];
        maxn = (nrm > maxn || nrm != nrm) ? nrm : maxn;
        E += P.w * ec;
        if (tid == 0) {
          Pl[P.la * nl + P.la] -= 2.0 * vv;
          if (P.la != P.lb) Pl[P.lb * nl + P.lb] -= 2.0 * vv;
        }
        __syncthreads();
      }
      if (maxn < a.tau_R || maxn != maxn || sweep >= a.max_sweeps) break;
      // Jacobi update of every pair of the cluster
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const Domain D = a.dom[P.dom];
        const int n = D.n, nt = a.dom_rank[P.dom];
        double *T = a.T + P.toff;
        const double *ep = a.epst + D.voff;
        const double *R = Rs + (P.toff - cl.toff0);
        const double fd = a.F_occ[D.p * a.nocc + D.p] + a.F_occ[D.q * a.nocc + D.q];
        for (int e = tid; e < nt * nt; e += NTHREADS) {
          int i = e / nt, j = e % nt;
          T[i * n + j] -= R[i * n + j] / (ep[i] + ep[j] - fd);
        }
      }
      __syncthreads();
      sweep++;
    }
    if (tid == 0) {
      a.Ecl[X] = E;
      a.sweeps[X] = sweep;
      a.maxres[X] = maxn;
    }
    __syncthreads();
  }
}

hipError_t launch_solve(const SolveArgs &a, int nwg, hipStream_t s) {
  if (a.n_clusters <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve, dim3(nwg), dim3(NTHREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace osv
