// OSV generation (eq:svd): for every LMO k the orthonormal eigenvectors of the
// diagonal MP2 amplitudes [T_kk]_ab = (ka|kb) / (f_aa + f_bb - 2 f_kk) whose
// eigenvalues exceed l_osv, largest first.
//
// (ka|kb) = B_k B_k^T comes from the FP64 MFMA product kernel; here, one workgroup
// per LMO (the nvir x nvir matrix in its own global slot):
//   1. Householder reduction to a symmetric tridiagonal matrix (reflector k is
//      stored in row k of the slot, right of the diagonal, its leading 1 implicit);
//   2. bisection with Sturm counts for the wanted eigenvalues (the number above
//      l_osv, at most r_max), one thread per eigenvalue;
//   3. (second kernel, after the host has packed the LMOs' output offsets) inverse
//      iteration on the tridiagonal matrix for each eigenvalue, re-orthogonalised
//      against the earlier vectors of its cluster of close eigenvalues, then the
//      reflectors applied in reverse order, and each vector's entry of largest
//      magnitude made positive.
// Every reduction is in a fixed order.
#include "osv_internal.h"

namespace osv {

constexpr int GNT_EIG = 1024;              // threads per LMO
constexpr int GNW_EIG = GNT_EIG / 64;

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// fixed-order block sum (red: GNW_EIG doubles)
__device__ __forceinline__ double bsum(double v, double *red) {
  v = wsum64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < GNW_EIG; w++) t += red[w];
  __syncthreads();
  return t;
}

// T_kk = K_kk / (eps_a + eps_b - 2 f_kk) in place, every LMO's nvir x nvir slot
__global__ void k_osv_denom(double *T, int nvir, const double *__restrict__ eps,
                            const double *__restrict__ F, int nocc) {
  const int k = blockIdx.y;
  const long long n2 = (long long)nvir * nvir;
  const double f2 = 2.0 * F[(long long)k * nocc + k];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (long long)gridDim.x * blockDim.x) {
    const int a = (int)(e / nvir), b = (int)(e - (long long)a * nvir);
    T[(long long)k * n2 + e] /= (eps[a] + eps[b] - f2);
  }
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence; pivots
// smaller than pivmin in magnitude are replaced by -pivmin)
__device__ double sturm_count(const double *d, const double *e, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < n; i++) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return (double)c;
}

// Per LMO: Householder tridiagonalisation of T (n x n, row-major, in place), then the
// wanted eigenvalues by bisection.  Outputs per LMO k: d, e (n each), tau (n), the
// count rk[k] = min(r_max, #{omega > l_osv}) and omega (r_max, descending).
// Each column's rank-2 update of the trailing matrix is fused with the next
// column's product p = tau A22 v: the row holding the next reflector is updated
// first, the reflector formed, and then one pass over the other rows updates each
// row and takes its dot product with the new reflector (the trailing matrix is
// read and written once per column instead of read twice and written once).
__global__ __launch_bounds__(GNT_EIG) void k_osv_tridiag(double *Tall, int n, double l_osv, int r_max,
                                                        double *dall, double *eall, double *tauall,
                                                        int *rk, double *omall) {
  extern __shared__ double sh[];
  double *vb[2] = {sh, sh + n};            // reflectors of this column and the next
  double *pb[2] = {sh + 2 * n, sh + 3 * n};  // p (then w) of this column and the next
  __shared__ double red[GNW_EIG];
  __shared__ double s_tau, s_beta;
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *A = Tall + (long long)k * n * n;
  double *d = dall + (long long)k * n, *e = eall + (long long)k * n, *tau = tauall + (long long)k * n;
  // reflector of column c from row c right of the diagonal (all updates of earlier
  // columns applied): d[c], e[c], tau[c], and v (leading 1) into vv; returns tau
  auto reflector = [&](int c, double *vv) -> double {
    const int m = n - c - 1;
    const double *x = A + (long long)c * n + c + 1;
    double ss = 0.0;
    for (int i = 1 + tid; i < m; i += GNT_EIG) ss += x[i] * x[i];
    const double xn2 = bsum(ss, red);
    if (tid == 0) {
      const double alpha = x[0];
      if (xn2 == 0.0) {
        s_tau = 0.0;
        s_beta = alpha;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        s_tau = (beta - alpha) / beta;
        s_beta = beta;
      }
      d[c] = A[(long long)c * n + c];
      e[c] = s_beta;
      tau[c] = s_tau;
    }
    __syncthreads();
    const double tc = s_tau;
    if (tc != 0.0) {
      const double scale = 1.0 / (x[0] - s_beta);
      for (int i = tid; i < m; i += GNT_EIG) vv[i] = (i == 0) ? 1.0 : x[i] * scale;
    }
    __syncthreads();
    return tc;
  };
  int cur = 0;
  double tc = 0.0;
  if (n >= 3) {
    // the first column: reflector and p = tau A22 v (one wave per row)
    tc = reflector(0, vb[0]);
    if (tc != 0.0) {
      const int m = n - 1;
      const double *v = vb[0];
      for (int i = wave; i < m; i += GNW_EIG) {
        const double *row = A + (long long)(1 + i) * n + 1;
        double t = 0.0;
        for (int j = lane; j < m; j += 64) t += row[j] * v[j];
        t = wsum64(t);
        if (lane == 0) pb[0][i] = tc * t;
      }
      __syncthreads();
    }
  }
  for (int c = 0; c + 2 < n; c++) {
    const int m = n - c - 1;   // the trailing matrix A22: rows and columns c + 1 ..
    double *v = vb[cur], *w = pb[cur];
    if (tc != 0.0) {
      double pv = 0.0;
      for (int i = tid; i < m; i += GNT_EIG) pv += w[i] * v[i];
      const double K = -0.5 * tc * bsum(pv, red);
      for (int i = tid; i < m; i += GNT_EIG) w[i] += K * v[i];
      __syncthreads();
    }
    double tn = 0.0;
    if (c + 3 < n) {
      // row 0 of A22 (row c + 1) first: it holds the next reflector
      if (tc != 0.0) {
        double *row = A + (long long)(c + 1) * n + c + 1;
        const double vi = v[0], wi = w[0];
        for (int j = tid; j < m; j += GNT_EIG) row[j] -= vi * w[j] + wi * v[j];
        __syncthreads();
      }
      double *vn = vb[cur ^ 1], *pn = pb[cur ^ 1];
      tn = reflector(c + 1, vn);
      // rows 1.. of A22: the update and, with the updated row, p of the next column
      // (columns 1.. of A22 are the next trailing matrix; column 0 is not read again)
      // (four rows per wave at a time, 16 lanes along each row)
      const int mn = m - 1, l16 = lane & 15;
      for (int i0 = 1 + 4 * wave; i0 < m; i0 += 4 * GNW_EIG) {
        const int i = i0 + (lane >> 4);
        double t = 0.0;
        if (i < m) {
          double *row = A + (long long)(c + 1 + i) * n + c + 2;
          const double vi = v[i], wi = w[i];
#pragma unroll 8
          for (int j = l16; j < mn; j += 16) {
            double a = row[j];
            if (tc != 0.0) {
              a -= vi * w[j + 1] + wi * v[j + 1];
              row[j] = a;
            }
            t += a * vn[j];
          }
        }
        if (tn != 0.0) {
          for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
          if (l16 == 0 && i < m) pn[i - 1] = tn * t;
        }
      }
    } else if (tc != 0.0) {
      // the last column: the plain update
      for (int i = wave; i < m; i += GNW_EIG) {
        double *row = A + (long long)(c + 1 + i) * n + c + 1;
        const double vi = v[i], wi = w[i];
        for (int j = lane; j < m; j += 64) row[j] -= vi * w[j] + wi * v[j];
      }
    }
    // the reflector, kept in row c right of the diagonal (leading 1 implicit)
    if (tc != 0.0) {
      double *xr = A + (long long)c * n + c + 1;
      for (int i = 1 + tid; i < m; i += GNT_EIG) xr[i] = v[i];
    }
    __syncthreads();
    cur ^= 1;
    tc = tn;
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(long long)(n - 2) * n + n - 2];
      e[n - 2] = A[(long long)(n - 2) * n + n - 1];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = A[(long long)(n - 1) * n + n - 1];
    tau[n - 1] = 0.0;
    e[n - 1] = 0.0;
  }
  __syncthreads();
  // bisection: Gerschgorin interval, then the (n-1-j)-th smallest eigenvalue for
  // thread j < r (descending order)
  __shared__ double s_lo, s_hi, s_piv;
  __shared__ int s_r;
  if (tid == 0) {
    double lo = 1e300, hi = -1e300, emax = 0.0;
    for (int i = 0; i < n; i++) {
      const double el = i > 0 ? fabs(e[i - 1]) : 0.0, er = i + 1 < n ? fabs(e[i]) : 0.0;
      lo = fmin(lo, d[i] - el - er);
      hi = fmax(hi, d[i] + el + er);
      if (i + 1 < n) emax = fmax(emax, e[i] * e[i]);
    }
    const double span = fmax(fabs(lo), fabs(hi));
    s_lo = lo - 2.2e-16 * span - 1e-300;
    s_hi = hi + 2.2e-16 * span + 1e-300;
    s_piv = 2.3e-308 * fmax(1.0, emax);
    const int above = n - (int)sturm_count(d, e, n, l_osv, s_piv);
    int r = above < r_max ? above : r_max;
    s_r = r < 0 ? 0 : r;
    rk[k] = s_r;
  }
  __syncthreads();
  const int r = s_r;
  for (int j = tid; j < r; j += GNT_EIG) {
    const int idx = n - 1 - j;      // ascending index of the wanted eigenvalue
    double lo = s_lo, hi = s_hi;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(d, e, n, mid, s_piv) > idx) hi = mid;
      else lo = mid;
      if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi))) break;
    }
    omall[(long long)k * r_max + j] = 0.5 * (lo + hi);
  }
}

// Per LMO: eigenvectors of the tridiagonal matrix by inverse iteration (LU with
// partial pivoting by one thread, three iterations from a fixed start vector, each
// followed by modified Gram-Schmidt against the earlier vectors whose eigenvalues
// lie within 1e-3 ||T||), the reflectors applied from the last to the first, the
// sign fixed, and the result written as rows off[k] + j of Qt (ld n) with omega.
__global__ __launch_bounds__(GNT_EIG) void k_osv_vectors(const double *Tall, int n, int r_max,
                                                        const double *dall, const double *eall,
                                                        const double *tauall, const int *rk,
                                                        const double *omall, const int *off,
                                                        double *Zall, double *Qt, double *omega) {
  extern __shared__ double sh[];
  double *u1 = sh, *u2 = u1 + n, *u3 = u2 + n, *ml = u3 + n, *y = ml + n;
  double *dl = y + n, *el = dl + n;   // the tridiagonal matrix, in LDS for the serial LU
  unsigned char *pv = (unsigned char *)(el + n);
  __shared__ double red[GNW_EIG];
  __shared__ double s_nrm;
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = rk[k];
  if (r == 0) return;
  const double *A = Tall + (long long)k * n * n;
  const double *d = dall + (long long)k * n, *e = eall + (long long)k * n, *tau = tauall + (long long)k * n;
  const double *om = omall + (long long)k * r_max;
  double *Z = Zall + (long long)k * n * r_max;     // column j at Z + j n
  for (int i = tid; i < n; i += GNT_EIG) {
    dl[i] = d[i];
    el[i] = e[i];
  }
  __syncthreads();
  // ||T|| (1-norm of the tridiagonal matrix) for the pivot floor and the cluster test
  double tn = 0.0;
  for (int i = tid; i < n; i += GNT_EIG)
    tn = fmax(tn, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0));
  {
    double t = tn;
    for (int o = 32; o > 0; o >>= 1) t = fmax(t, __shfl_xor(t, o, 64));
    if (lane == 0) red[wave] = t;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < GNW_EIG; w++) m = fmax(m, red[w]);
      s_nrm = m;
    }
    __syncthreads();
  }
  const double tnorm = s_nrm, pfloor = 2.2e-16 * fmax(tnorm, 1e-300), ortol = 1e-3 * tnorm;
  int c0 = 0;   // first vector of the current cluster
  for (int j = 0; j < r; j++) {
    const double lam = om[j];
    if (j > 0 && fabs(om[j - 1] - lam) > ortol) c0 = j;
    double *zj = Z + (long long)j * n;
    if (tid == 0) {
      // LU with partial pivoting of (tridiagonal - lam): rows (p, q, s) at columns (i, i+1, i+2)
      double p = dl[0] - lam, q = n > 1 ? el[0] : 0.0, s3 = 0.0;
      for (int i = 0; i + 1 < n; i++) {
        const double ci = el[i], ai1 = dl[i + 1] - lam, bi1 = (i + 2 < n) ? el[i + 1] : 0.0;
        if (fabs(p) >= fabs(ci)) {
          const double pp = (fabs(p) < pfloor) ? copysign(pfloor, p) : p;
          const double mlt = ci / pp;
          u1[i] = pp; u2[i] = q; u3[i] = s3; ml[i] = mlt; pv[i] = 0;
          p = ai1 - mlt * q;
          q = bi1 - mlt * s3;
          s3 = 0.0;
        } else {
          const double mlt = p / ci;
          u1[i] = ci; u2[i] = ai1; u3[i] = bi1; ml[i] = mlt; pv[i] = 1;
          p = q - mlt * ai1;
          q = s3 - mlt * bi1;
          s3 = 0.0;
        }
      }
      u1[n - 1] = (fabs(p) < pfloor) ? copysign(pfloor, p) : p;
      u2[n - 1] = 0.0;
      u3[n - 1] = 0.0;
    }
    // fixed start vector
    for (int i = tid; i < n; i += GNT_EIG) y[i] = 1.0 + 0.37 * (double)((i * 7919 + j * 104729) % 1000) / 1000.0;
    __syncthreads();
    for (int it = 0; it < 3; it++) {
      if (tid == 0) {
        for (int i = 0; i + 1 < n; i++) {
          if (pv[i]) {
            const double t = y[i];
            y[i] = y[i + 1];
            y[i + 1] = t;
          }
          y[i + 1] -= ml[i] * y[i];
        }
        for (int i = n - 1; i >= 0; i--) {
          double t = y[i];
          if (i + 1 < n) t -= u2[i] * y[i + 1];
          if (i + 2 < n) t -= u3[i] * y[i + 2];
          y[i] = t / u1[i];
        }
      }
      __syncthreads();   // the solve is done before anyone reads y
      // rescale to keep the entries of order one (largest magnitude 1)
      {
        double mx = 0.0;
        for (int i = tid; i < n; i += GNT_EIG) mx = fmax(mx, fabs(y[i]));
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        double m2 = 0.0;
        for (int w = 0; w < GNW_EIG; w++) m2 = fmax(m2, red[w]);
        const double sc = m2 > 0.0 ? 1.0 / m2 : 1.0;
        __syncthreads();
        for (int i = tid; i < n; i += GNT_EIG) y[i] *= sc;
        __syncthreads();
      }
      // modified Gram-Schmidt against the earlier vectors of the cluster
      for (int t = c0; t < j; t++) {
        const double *zt = Z + (long long)t * n;
        double pd = 0.0;
        for (int i = tid; i < n; i += GNT_EIG) pd += zt[i] * y[i];
        const double dot = bsum(pd, red);
        for (int i = tid; i < n; i += GNT_EIG) y[i] -= dot * zt[i];
        __syncthreads();
      }
      double ps = 0.0;
      for (int i = tid; i < n; i += GNT_EIG) ps += y[i] * y[i];
      const double nr = sqrt(bsum(ps, red));
      for (int i = tid; i < n; i += GNT_EIG) y[i] /= nr;
      __syncthreads();
    }
    for (int i = tid; i < n; i += GNT_EIG) zj[i] = y[i];
    __syncthreads();
  }
  __threadfence();
  __syncthreads();
  // back-transformation x = H_0 H_1 ... H_{n-3} z: reflector c (u = (1, A[c][c+2..])
  // on rows c+1..) applied from the last to the first; one wave per vector
  for (int c = n - 3; c >= 0; c--) {
    const double tc = tau[c];
    if (tc != 0.0) {
      const double *ur = A + (long long)c * n + c + 1;   // ur[0] is not the reflector's 1
      for (int j = wave; j < r; j += GNW_EIG) {
        double *zj = Z + (long long)j * n + c + 1;
        double t = 0.0;
        for (int i = lane; i < n - c - 1; i += 64) t += (i == 0 ? 1.0 : ur[i]) * zj[i];
        t = tc * wsum64(t);
        for (int i = lane; i < n - c - 1; i += 64) zj[i] -= t * (i == 0 ? 1.0 : ur[i]);
      }
    }
    __syncthreads();
  }
  // sign (entry of largest magnitude positive, first on ties), output
  for (int j = wave; j < r; j += GNW_EIG) {
    const double *zj = Z + (long long)j * n;
    double best = -1.0;
    int bi = n;
    for (int i = lane; i < n; i += 64) {
      const double a = fabs(zj[i]);
      if (a > best) { best = a; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sg = zj[bi] < 0.0 ? -1.0 : 1.0;
    double *q = Qt + (long long)(off[k] + j) * n;
    for (int i = lane; i < n; i += 64) q[i] = sg * zj[i];
    if (lane == 0) omega[(long long)k * r_max + j] = om[j];
  }
}

size_t osvgen_lds_tridiag(int n) { return (size_t)4 * n * sizeof(double); }
size_t osvgen_lds_vectors(int n) { return (size_t)7 * n * sizeof(double) + (size_t)n; }

hipError_t launch_osv_denom(double *T, int nvir, const double *eps, const double *F, int nocc,
                            hipStream_t s) {
  const long long n2 = (long long)nvir * nvir;
  const int bx = (int)std::min<long long>((n2 + 255) / 256, 1024);
  hipLaunchKernelGGL(k_osv_denom, dim3(bx, nocc), dim3(256), 0, s, T, nvir, eps, F, nocc);
  return hipGetLastError();
}

hipError_t launch_osv_tridiag(double *T, int nocc, int n, double l_osv, int r_max, double *d,
                              double *e, double *tau, int *rk, double *om, hipStream_t s) {
  hipLaunchKernelGGL(k_osv_tridiag, dim3(nocc), dim3(GNT_EIG), osvgen_lds_tridiag(n), s, T, n, l_osv,
                     r_max, d, e, tau, rk, om);
  return hipGetLastError();
}

hipError_t launch_osv_vectors(const double *T, int nocc, int n, int r_max, const double *d,
                              const double *e, const double *tau, const int *rk, const double *om,
                              const int *off, double *Z, double *Qt, double *omega, hipStream_t s) {
  hipLaunchKernelGGL(k_osv_vectors, dim3(nocc), dim3(GNT_EIG), osvgen_lds_vectors(n), s, T, n, r_max, d,
                     e, tau, rk, om, off, Z, Qt, omega);
  return hipGetLastError();
}

}  // namespace osv
