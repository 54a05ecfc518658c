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
// to both sides of A as independent 2x2 block updates.  The Fock eigenproblem of
// an off-diagonal domain first gets an approximate eigenbasis (Householder
// reduction, bisection, twisted-factorisation eigenvectors), which one
// first-order step (or, failing its test, the Jacobi sweeps) finishes.
#include "osv_internal.h"
#include "tiles.h"

namespace osv {

constexpr int LDM = DMAX + 1;  // LDS stride (doubles) of the 100x100 work matrices
constexpr int FOCK_START_MIN = 8;   // smallest domain given an approximate starting basis

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum over NT threads (fixed order); red has room for NT/64 values
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NT / 64; w++) t += red[w];
  __syncthreads();
  return t;
}

// Rotation t of step st of a round-robin sweep over m + 1 indices (m odd): the
// pair (p, q), p < q; index m is a dummy when n is odd.
__device__ __forceinline__ void rr_pair(int st, int t, int m, int &p, int &q) {
  int a, b;
  if (t == 0) {
    a = st;
    b = m;
  } else {
    a = st + t;
    a -= (a >= m) ? m : 0;
    b = st - t;
    b += (b < 0) ? m : 0;
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// index of element (a, b) of a symmetric matrix of which only the upper triangle
// is kept
template <int LD>
__device__ __forceinline__ int up(int a, int b) {
  return a < b ? a * LD + b : b * LD + a;
}

// Cyclic Jacobi: A (n x n, stride LD) is diagonalised in place, V receives the
// eigenvectors (columns).  Round-robin ordering: in step st the n/2 disjoint
// pairs rotate simultaneously; A <- J^T A J is applied as independent 2x2 block
// updates.  A step has two phases separated by barriers: (1) wave 0 forms the
// step's rotation table and applies each rotation to its own diagonal 2x2 block
// while the other waves apply the previous step's rotations to the rows of V (V
// is not read by the A updates), (2) every thread updates its off-diagonal 2x2
// blocks of A.
// A is read in full on entry; during the sweeps only its upper triangle is kept
// (each 2x2 block is read and written once), so on return only the diagonal
// (the eigenvalues) and the upper triangle are meaningful.
// Threshold rule: a_pq^2 <= 1e-34 |a_pp a_qq| or |a_pq| <= 1e-18 ||A||_F is set
// to zero without a rotation.  After a sweep with rotations every pair is tested
// against that rule; the solve ends when no pair would rotate (a further sweep
// would change no diagonal element and no element of V).
// Requires NT >= 128 and n/2 <= 64; rt holds n/2 entries.
template <int LD, int NT, int MAXB, int MAXV>
__device__ void jacobi_eig(double *A, double *V, int n, double2 *rt, double *red, int *flag) {
  const int tid = threadIdx.x;
  const int nE = n + (n & 1), h = nE / 2, m = nE - 1;
  for (int e = tid; e < n * n; e += NT) {
    int i = e / n, j = e - i * n;
    V[i * LD + j] = (i == j) ? 1.0 : 0.0;
  }
  double f2 = 0.0;
  for (int e = tid; e < n * n; e += NT) {
    int i = e / n, j = e - i * n;
    f2 += A[i * LD + j] * A[i * LD + j];
  }
  const double absthr = 1e-18 * sqrt(block_sum<NT>(f2, red));
  if (n == 1) return;
  // Each thread owns the same off-diagonal 2x2 blocks (I, J), I < J < h, in every
  // step (only the rotation table changes): block b = tid + NT u, row-major over
  // the strict upper triangle of the h x h block grid.  The diagonal blocks are
  // updated by the rotation threads themselves.
  const int nb = h * (h - 1) / 2;
  int bI[MAXB], bJ[MAXB];
#pragma unroll
  for (int u = 0; u < MAXB; u++) {
    const int b = tid + NT * u;
    int I = 0, rem = b;
    while (I < h && rem >= h - 1 - I) { rem -= h - 1 - I; I++; }
    bI[u] = (b < nb) ? I : -1;
    bJ[u] = I + 1 + rem;
  }
  // V entries: thread vt = tid - 64 of waves 1.. applies rotation k = vt mod h to
  // rows r0 + R u, r0 = vt / h, R = (NT - 64) / h (threads vt >= R h have none)
  const int vt = tid - 64;
  const int R = (NT - 64) / h;
  const int vk = (vt >= 0 && vt < R * h) ? vt % h : -1;
  const int r0 = vt >= 0 ? vt / h : 0;
  // table entries: (cosine, sine); (1, 0) where no rotation takes place.  A V
  // thread copies its entry of step st to registers during the A updates of
  // that step and applies it while the table of the next step is formed.
  auto v_update = [&](const double2 r, int st) {
    if (vk < 0) return;
    if (r.y == 0.0) return;   // a rotation implies q < n
    int p, q;
    rr_pair(st, vk, m, p, q);
#pragma unroll
    for (int u = 0; u < MAXV; u++) {
      const int i = r0 + R * u;
      if (i < n) {
        const double vp = V[i * LD + p], vq = V[i * LD + q];
        V[i * LD + p] = r.x * vp - r.y * vq;
        V[i * LD + q] = r.y * vp + r.x * vq;
      }
    }
  };
  double2 vr = make_double2(1.0, 0.0);   // this thread's pending V rotation, of step vst
  int vst = 0;
  for (int sweep = 0; sweep < 60; sweep++) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int st = 0; st < m; st++) {
      double2 *tab = rt;
      if (tid < h) {
        int p, q;
        rr_pair(st, tid, m, p, q);
        double c = 1.0, sv = 0.0;
        if (q < n) {
          const double apq = A[p * LD + q];
          if (apq != 0.0) {
            const double app = A[p * LD + p], aqq = A[q * LD + q];
            if (!(apq * apq <= 1e-34 * fabs(app * aqq) || fabs(apq) <= absthr)) {
              const double theta = (aqq - app) / (2.0 * apq);
              const double at = fabs(theta);
              double t;
              if (at > 1e150) t = 0.5 / theta;
              else t = (theta >= 0.0 ? 1.0 : -1.0) / (at + sqrt(theta * theta + 1.0));
              c = 1.0 / sqrt(t * t + 1.0);
              sv = t * c;
              *flag = 1;
              // this pair's diagonal block: a_pp, a_qq take the rotation, and a_pq
              // (zeroed below) is below the threshold when there is none
              A[p * LD + p] = app - t * apq;
              A[q * LD + q] = aqq + t * apq;
            }
            A[p * LD + q] = 0.0;
          }
        }
        tab[tid] = make_double2(c, sv);
      } else {
        v_update(vr, vst);
      }
      __syncthreads();
      if (vk >= 0) {
        vr = tab[vk];
        vst = st;
      }
#pragma unroll
      for (int u = 0; u < MAXB; u++) {
        const int I = bI[u], J = bJ[u];
        if (I < 0) continue;
        const double2 rI = tab[I];
        int pI, qI;
        rr_pair(st, I, m, pI, qI);
        const double2 rJ = tab[J];
        if (rI.y != 0.0 || rJ.y != 0.0) {
          int pJ, qJ;
          rr_pair(st, J, m, pJ, qJ);
          const double cI = rI.x, sI = rI.y, cJ = rJ.x, sJ = rJ.y;
          const bool vqI = qI < n, vqJ = qJ < n;
          const int i00 = up<LD>(pI, pJ), i01 = up<LD>(pI, qJ), i10 = up<LD>(qI, pJ),
                    i11 = up<LD>(qI, qJ);
          const double b00 = A[i00];
          const double b01 = vqJ ? A[i01] : 0.0;
          const double b10 = vqI ? A[i10] : 0.0;
          const double b11 = (vqI && vqJ) ? A[i11] : 0.0;
          const double r00 = cI * b00 - sI * b10, r01 = cI * b01 - sI * b11;
          const double r10 = sI * b00 + cI * b10, r11 = sI * b01 + cI * b11;
          A[i00] = r00 * cJ - r01 * sJ;
          if (vqJ) A[i01] = r00 * sJ + r01 * cJ;
          if (vqI) A[i10] = r10 * cJ - r11 * sJ;
          if (vqI && vqJ) A[i11] = r10 * sJ + r11 * cJ;
        }
      }
      __syncthreads();
    }
    // would any pair rotate in another sweep?  (none did in this one: done)
    bool more = false;
    if (*flag) {
      for (int e = tid; e < n * n; e += NT) {
        const int p = e / n, q = e - p * n;
        if (p < q) {
          const double apq = A[p * LD + q];
          if (apq != 0.0 &&
              !(apq * apq <= 1e-34 * fabs(A[p * LD + p] * A[q * LD + q]) || fabs(apq) <= absthr))
            more = true;
        }
      }
    }
    if (!__syncthreads_or(more)) break;
  }
  v_update(vr, vst);
  __syncthreads();
}

// Lane exchanges within rows of 16 lanes (DPP): quad_perm [1,0,3,2], [2,3,0,1],
// row_ror 4 and 8.  row_sum16 leaves the sum of its row in every lane of the row
// (lanes of different quads may differ in the last bit: each lane's order of
// additions is fixed).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp64<0xB1>(v);
  v += dpp64<0x4E>(v);
  v += dpp64<0x124>(v);
  v += dpp64<0x128>(v);
  return v;
}
// sum over a whole wave, the same value in every lane and every wave that sums
// the same data: the row sums of lanes 0, 16, 32, 48 added in that order
__device__ __forceinline__ double wave_sum_fixed(double v) {
  v = row_sum16(v);
  const long long b = __double_as_longlong(v);
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int lo = __builtin_amdgcn_readlane((int)b, 16 * k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * k);
    r[k] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return (r[0] + r[1]) + (r[2] + r[3]);
}
// 1 / x from the hardware reciprocal and one Newton step (x normal and finite)
__device__ __forceinline__ double recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Starting basis for the Fock eigensolve of an off-diagonal domain.  The cyclic
// Jacobi method converges quadratically once the off-diagonal part is small, so
// an approximate eigenbasis V1 (orthonormal to rounding) leaves it one sweep
// instead of five to eight, and in practice a single first-order step.  V1 is formed in four steps, all in LDS:
//   1. Householder reduction H = Q T Q^T (T tridiagonal): every wave forms the
//      reflector of column c from row c (the same arithmetic in every wave), the
//      product p = tau A22 v goes to row 0 of Z, then A22 -= v w^T + w v^T with
//      w = p - (tau/2)(p.v) v: two barriers per column.  Teams of 16 lanes take
//      rows; a lane holds its entries j = l, l + 16, ... of v and w in registers.
//      Reflector c is then kept in row c right of the superdiagonal (leading 1
//      implicit) and tau_c in the spare column LD - 1 of A; d and e stay on the
//      diagonal and superdiagonal;
//   2. every eigenvalue of T by multisection on Sturm counts, one team of 4 lanes
//      per eigenvalue testing 4 points at a time (five-section, 20 rounds: the width
//      shrinks by 5^20 = 9.5e13), kept in the spare column of Z.  A count is the
//      number of sign changes of the leading principal minors of T - x (one fused
//      multiply-add per step on the serial path, no division);
//   3. each eigenvector of T from a twisted factorisation T - lambda = N_r D_r N_r^T
//      (Dhillon and Parlett, LAA 387 (2004) 1-28), one thread per vector: the
//      stationary LDL^T pivots D+ forward, the UDU^T pivots D- backward, the twist
//      r where |gamma_r| = |D+_r + D-_r - (d_r - lambda)| is smallest, and
//      z_r = 1, z_i = -(e_i / D+_i) z_{i+1} (i < r), z_{i+1} = -(e_i / D-_{i+1}) z_i
//      (i >= r), with pivots of magnitude below eps ||T|| replaced by +-eps ||T||;
//      then V0 = Q Z, each team of 16 lanes keeping its columns of Z in registers
//      through all reflectors (no barriers);
//   4. one Newton-Schulz step V1 = V0 (3/2 - G/2), G = V0^T V0 (in place of the
//      polar factor of V0): the error 1 - G of order 1e-11 becomes 1e-22.
// The serial recurrences take reciprocals from the hardware estimate and one
// Newton step: the basis is a starting point, which the Jacobi sweep makes exact.
// Sums within a team may differ in the last bit between its lanes (each lane's
// order of additions is fixed, so results are reproducible).
// On return A holds 3/2 - G/2 and Z holds V0, both n x n; false (uniform) when
// max |1 - G| exceeds 1e-8 or is not finite (eigenvalues too close for the
// vectors to be told apart): the caller then keeps its basis.
template <int LD, int NT>
__device__ bool fock_start(double *A, double *Z, int n) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // 1. tridiagonalisation; (pc, pbeta, pt, psc): reflector of the previous column,
  // written into its row by wave 0 once no wave reads that row any more
  int pc = -1;
  double pbeta = 0.0, pt = 0.0, psc = 0.0;
  auto finish_row = [&]() {
    if (wave == 0 && pc >= 0) {
      double *xr = A + pc * LD + pc + 1;
      const int pm = n - pc - 1;
      if (pt != 0.0)
        for (int i = 1 + lane; i < pm; i += 64) xr[i] *= psc;
      if (lane == 0) {
        xr[0] = pbeta;
        A[pc * LD + LD - 1] = pt;
      }
    }
  };
  double *p = Z;   // p of the current column (row 0 of Z, free until step 2)
  const int team = tid >> 4, tl = tid & 15;
  constexpr int EPL = (LD - 1 + 15) / 16;   // entries of a row per lane of a team
  for (int c = 0; c + 2 < n; c++) {
    const int m = n - c - 1;
    const double *x = A + c * LD + c + 1;
    finish_row();
    double ss = 0.0;
    for (int i = 1 + lane; i < m; i += 64) ss += x[i] * x[i];
    ss = wave_sum_fixed(ss);
    const double alpha = x[0];
    double t = 0.0, beta = alpha, sc = 0.0;
    if (ss != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      // |beta| >= sqrt(ss) and |alpha - beta| >= |beta| are normal: the
      // reciprocal estimate and one Newton step, off the serial path's divisions
      t = (beta - alpha) * recip(beta);
      sc = recip(alpha - beta);
    }
    pc = c;
    pbeta = beta;
    pt = t;
    psc = sc;
    if (t == 0.0) continue;   // uniform; the next column's finish_row runs after a barrier
    // this lane's entries j = tl + 16 s of v (zero past m), all loads first
    double vr[EPL];
#pragma unroll
    for (int u = 0; u < EPL; u++) {
      const int j = tl + 16 * u;
      vr[u] = j < m ? x[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EPL; u++) vr[u] = (tl + 16 * u == 0) ? 1.0 : vr[u] * sc;
    // p = t A22 v: team g takes rows g, g + NT/16, ...
    for (int i = team; i < m; i += NT / 16) {
      const double *ar = A + (c + 1 + i) * LD + c + 1;
      double av[EPL];
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int j = tl + 16 * u;
        av[u] = j < m ? ar[j] : 0.0;
      }
      double sa = 0.0;
#pragma unroll
      for (int u = 0; u < EPL; u++) sa += av[u] * vr[u];
      sa = row_sum16(sa);
      if (tl == 0) p[i] = t * sa;
    }
    __syncthreads();
    // K = -(t/2) p.v within each team (the team's lanes hold every entry); w = p + K v
    double pr[EPL];
#pragma unroll
    for (int u = 0; u < EPL; u++) {
      const int j = tl + 16 * u;
      pr[u] = j < m ? p[j] : 0.0;
    }
    double pv = 0.0;
#pragma unroll
    for (int u = 0; u < EPL; u++) pv += pr[u] * vr[u];
    const double K = -0.5 * t * row_sum16(pv);
#pragma unroll
    for (int u = 0; u < EPL; u++) pr[u] += K * vr[u];
    for (int i = team; i < m; i += NT / 16) {
      const double vi = i == 0 ? 1.0 : x[i] * sc, wi = p[i] + K * vi;
      double *ar = A + (c + 1 + i) * LD + c + 1;
      double av[EPL];
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int j = tl + 16 * u;
        av[u] = j < m ? ar[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int j = tl + 16 * u;
        if (j < m) ar[j] = av[u] - (vi * pr[u] + wi * vr[u]);
      }
    }
    __syncthreads();
  }
  __syncthreads();
  finish_row();
  __syncthreads();
  // Gerschgorin interval, ||T||_1 and the largest e^2 (every thread, same order)
  auto dg = [&](int i) { return A[i * LD + i]; };
  auto ev = [&](int i) { return A[i * LD + i + 1]; };
  // (a thread per row, then the block's min and max, which are exact in any
  // order; the wave partials go to row 2 of Z, left of its spare column)
  double lo = 1e300, hi = -1e300, tn = 0.0;
  for (int i = tid; i < n; i += NT) {
    const double el = i > 0 ? fabs(ev(i - 1)) : 0.0, er = i + 1 < n ? fabs(ev(i)) : 0.0;
    lo = fmin(lo, dg(i) - el - er);
    hi = fmax(hi, dg(i) + el + er);
    tn = fmax(tn, fabs(dg(i)) + el + er);
  }
  {
    constexpr int NW = NT / 64;
    static_assert(3 * NW < LD - 1, "partials left of the spare column");
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
      tn = fmax(tn, __shfl_xor(tn, o, 64));
    }
    double *gp = Z + 2 * LD;
    if (lane == 0) {
      gp[wave] = lo;
      gp[NW + wave] = hi;
      gp[2 * NW + wave] = tn;
    }
    __syncthreads();
    for (int w = 0; w < NW; w++) {
      lo = fmin(lo, gp[w]);
      hi = fmax(hi, gp[NW + w]);
      tn = fmax(tn, gp[2 * NW + w]);
    }
  }
  const double span = fmax(fabs(lo), fabs(hi));
  lo -= 2.2e-16 * span + 1e-300;
  hi += 2.2e-16 * span + 1e-300;
  const double pfloor = 2.2e-16 * fmax(tn, 1e-300);
  // 2. eigenvalues (ascending): the BL lanes of a team test a + (l + 1) h,
  //    h = (b - a) / (BL + 1).  The number of eigenvalues below x is the number of
  //    sign changes in p_(-1) = 1, p_0, .., p_(n-1), the leading principal minors
  //    of T - x: p_i = (d_i - x) p_(i-1) - e_(i-1)^2 p_(i-2).  An isolated zero
  //    minor differs in sign from one of its neighbours and so is counted once;
  //    e^2 is kept at least 2^-400 (of the scaled norm) so that zeros stay isolated.
  //    T is scaled by the power of two 2^-E that brings ||T||_1 into [1/2, 1), and
  //    the two latest minors are rescaled by a power of two every 8 steps (the
  //    minors grow by at most a factor 3 per step).  d and e^2 go to rows 0 and 1 of Z.
  {
    constexpr int BL = 4, ROUNDS = 20;
    int E;
    (void)frexp(fmax(tn, 1e-300), &E);
    for (int i = tid; i < n; i += NT) {
      Z[i] = ldexp(dg(i), -E);
      const double es = i > 0 ? ldexp(ev(i - 1), -E) : 0.0;
      Z[LD + i] = fmax(es * es, 0x1p-400);
    }
    __syncthreads();
    const double los = ldexp(lo, -E), his = ldexp(hi, -E);
    constexpr double RB = 1.0 / (BL + 1);
    const int bt = tid / BL, bl = tid % BL;
    for (int k = bt; k < n; k += NT / BL) {
      double a = los, b = his;
      for (int rd = 0; rd < ROUNDS; rd++) {
        const double h = (b - a) * RB, xq = a + (bl + 1) * h;
        double pm = 1.0, pc = Z[0] - xq;
        unsigned cnt = (unsigned)__double2hiint(pc) >> 31;
        auto step = [&](int i) {
          const double pn = fma(Z[i] - xq, pc, -Z[LD + i] * pm);
          cnt += ((unsigned)__double2hiint(pn) ^ (unsigned)__double2hiint(pc)) >> 31;
          pm = pc;
          pc = pn;
        };
        int i = 1;
        for (; i + 7 < n; i += 8) {
#pragma unroll
          for (int u = 0; u < 8; u++) step(i + u);
          int ep;
          (void)frexp(fmax(fabs(pc), fabs(pm)), &ep);
          pc = ldexp(pc, -ep);
          pm = ldexp(pm, -ep);
        }
        for (; i < n; i++) step(i);
        const unsigned long long bal = __ballot((int)cnt > k);
        const int j = BL - __popcll((bal >> (lane & (64 - BL))) & ((1ull << BL) - 1));   // points below lambda_k
        const double na = a + j * h, nb = j < BL ? a + (j + 1) * h : b;
        a = na;
        b = nb;
      }
      if (bl == 0) Z[k * LD + LD - 1] = ldexp(0.5 * (a + b), E);
    }
  }
  __syncthreads();
  // 3. eigenvectors of T, thread j -> column j of Z (pivots, then the vector, in place)
  for (int j = tid; j < n; j += NT) {
    const double lam = Z[j * LD + LD - 1];
    double *zc = Z + j;
    auto fl = [&](double v) { return fabs(v) < pfloor ? (v < 0.0 ? -pfloor : pfloor) : v; };
    double Dp = fl(dg(0) - lam);
    zc[0] = Dp;
    for (int i = 0; i + 1 < n; i++) {
      const double ei = ev(i);
      Dp = fl(dg(i + 1) - lam - ei * ei * recip(Dp));
      zc[(i + 1) * LD] = Dp;
    }
    double Dm = fl(dg(n - 1) - lam);
    double best = fabs(zc[(n - 1) * LD] + Dm - (dg(n - 1) - lam));
    int r = n - 1;
    for (int k = n - 2; k >= 0; k--) {
      const double ek = ev(k);
      Dm = fl(dg(k) - lam - ek * ek * recip(Dm));
      const double g = fabs(zc[k * LD] + Dm - (dg(k) - lam));
      if (g < best) {
        best = g;
        r = k;
      }
    }
    Dm = fl(dg(n - 1) - lam);
    for (int i = n - 2; i >= r; i--) {
      const double ei = ev(i), rD = recip(Dm);
      zc[(i + 1) * LD] = ei * rD;
      Dm = fl(dg(i) - lam - ei * ei * rD);
    }
    double zv = 1.0, ss = 1.0;
    for (int i = r - 1; i >= 0; i--) {
      zv = -(ev(i) * recip(zc[i * LD])) * zv;
      zc[i * LD] = zv;
      ss += zv * zv;
    }
    zc[r * LD] = 1.0;
    zv = 1.0;
    for (int i = r; i + 1 < n; i++) {
      zv = -zc[(i + 1) * LD] * zv;
      zc[(i + 1) * LD] = zv;
      ss += zv * zv;
    }
    const double sc = 1.0 / sqrt(ss);
    for (int i = 0; i < n; i++) zc[i * LD] *= sc;
  }
  __syncthreads();
  // V0 = H_0 H_1 ... H_{n-3} Z: team g keeps columns g, g + NT/16, ... of Z in
  // registers (entry i = tl + 16 u) through all reflectors
  {
    constexpr int NTM = NT / 16, CPT = (LD - 1 + NTM - 1) / NTM;   // teams, columns per team
    double zr[CPT][EPL];
#pragma unroll
    for (int q = 0; q < CPT; q++) {
      const int j = team + NTM * q;
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int i = tl + 16 * u;
        zr[q][u] = (j < n && i < n) ? Z[i * LD + j] : 0.0;
      }
    }
    for (int c = n - 3; c >= 0; c--) {
      const double t = A[c * LD + LD - 1];
      if (t == 0.0) continue;
      // reflector c on rows c + 1 ..: u_(c+1) = 1, u_i = A[c][i] for i > c + 1
      double ur[EPL];
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int i = tl + 16 * u;
        ur[u] = (i > c + 1 && i < n) ? A[c * LD + i] : (i == c + 1 ? 1.0 : 0.0);
      }
#pragma unroll
      for (int q = 0; q < CPT; q++) {
        double sa = 0.0;
#pragma unroll
        for (int u = 0; u < EPL; u++) sa += ur[u] * zr[q][u];
        sa = t * row_sum16(sa);
#pragma unroll
        for (int u = 0; u < EPL; u++) zr[q][u] -= sa * ur[u];
      }
    }
#pragma unroll
    for (int q = 0; q < CPT; q++) {
      const int j = team + NTM * q;
#pragma unroll
      for (int u = 0; u < EPL; u++) {
        const int i = tl + 16 * u;
        if (j < n && i < n) Z[i * LD + j] = zr[q][u];
      }
    }
  }
  __syncthreads();
  // 4. G = V0^T V0 into A, the test, then 3/2 - G/2
  mma_tiles<NT>(n, n, n, [&](int i, int k) { return Z[k * LD + i]; },
                [&](int k, int j) { return Z[k * LD + j]; },
                [&](int i, int j, double v) { A[i * LD + j] = v; });
  __syncthreads();
  bool bad = false;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    bad = bad || !(fabs(((i == j) ? 1.0 : 0.0) - A[i * LD + j]) <= 1e-8);
  }
  if (__syncthreads_or(bad)) return false;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    A[i * LD + j] = ((i == j) ? 1.5 : 0.0) - 0.5 * A[i * LD + j];
  }
  __syncthreads();
  return true;
}

// Pair-domain preparation, one workgroup of NT threads per domain of dimension
// n <= NM (LDS work matrices NM x (NM+1)).
template <int NM, int NT>
__global__ __launch_bounds__(NT) void k_domain_prep(const Domain *__restrict__ doms,
                                                    const int *__restrict__ ids,
                                                    const double *__restrict__ S,
                                                    const double *__restrict__ F,
                                                    const double *__restrict__ K, long long ld,
                                                    double tau_S,
                                                    const long long *__restrict__ dmoff,
                                                    double *W, double *Y,
                                                    double *Kep, int *rank,
                                                    double *minev) {
  constexpr int LD = NM + 1;
  constexpr int HM = NM / 2;
  constexpr int MAXB = (HM * (HM - 1) / 2 + NT - 1) / NT;   // off-diagonal blocks per thread
  constexpr int MAXV = (NM + (NT - 64) / HM - 1) / ((NT - 64) / HM);   // V rows per thread
  static_assert(NT >= 128 && HM <= 64, "jacobi_eig needs a rotation wave and V waves");
  __shared__ double L1[NM * LD];
  __shared__ double L2[NM * LD];
  __shared__ double2 rt[HM];
  __shared__ double red[NT / 64];
  __shared__ int keep_idx[NM];
  __shared__ int s_dt, s_flag;
  const int dom_id = ids[blockIdx.x];
  const Domain D = doms[dom_id];
  const int tid = threadIdx.x, n = D.n;
  const bool diag = (D.p == D.q);
  // K~^T (np x np, ld np) and the pseudo-canonical energies (np) share one
  // zero-padded slot at voff
  const int np = D.np;
  double *Wg = W + D.moff, *Yg = Y + D.moff, *Kg = Kep + D.voff, *eg = Kg + np * np;
  int dt;
  if (!diag) {
    const int rp = D.rp, rq = D.rq;
    const double *Bg = S + (long long)D.offp * ld + D.offq;   // B = S_pq (rp x rq, ld)
    // 1) canonical orthogonalisation.  Block Gram-Schmidt: Q_q' = Q_q - Q_p B has
    //    overlap A = 1 - B^T B = L L^T, so X = [[1, -B L^-T], [0, L^-T]] gives
    //    X^T S X = 1.  The overlap eigenvalues are 1 +- sigma_k(B) (and 1), so all of
    //    them exceed tau_S iff lambda_min(A) > tau_S (2 - tau_S); since
    //    lambda_min(A) >= 1 / trace(A^-1) = 1 / ||L^-1||_F^2, that bound certifies
    //    that nothing is dropped.  Otherwise the overlap eigenvalues are cut
    //    explicitly (eigendecomposition of S_(pq,pq)).
    mma_tiles<NT>(rq, rq, rp, [&](int i, int k) { return Bg[(long long)k * ld + i]; },
                  [&](int k, int j) { return Bg[(long long)k * ld + j]; },
                  [&](int i, int j, double v) { L1[i * LD + j] = ((i == j) ? 1.0 : 0.0) - v; });
    __syncthreads();
    // right-looking Cholesky (lower triangle of L1)
    for (int j = 0; j < rq; j++) {
      const double d = L1[j * LD + j];
      __syncthreads();
      if (!(d > 0.0)) break;  // uniform: every thread read the same d
      const double sd = sqrt(d);
      for (int i = j + 1 + tid; i < rq; i += NT) L1[i * LD + j] /= sd;
      __syncthreads();
      if (tid == 0) L1[j * LD + j] = sd;
      for (int e = tid; e < (rq - j - 1) * (rq - j - 1); e += NT) {
        int i = j + 1 + e / (rq - j - 1), k = j + 1 + e % (rq - j - 1);
        if (k <= i) L1[i * LD + k] -= L1[i * LD + j] * L1[k * LD + j];
      }
      __syncthreads();
    }
    bool chol_ok = true;
    for (int j = 0; j < rq; j++) chol_ok = chol_ok && (L1[j * LD + j] > 0.0);
    // L^-1 by forward substitution (lower triangle of L2): one column per team of
    // 16 lanes of a wave, each row's dot product split over the team and summed
    // by shuffles (fixed order); the team's first lane stores the element, which
    // the team reads back in later rows (one wave: LDS operations stay in order)
    double tr = 0.0;
    if (chol_ok) {
      const int team = tid >> 4, tl = tid & 15;
      for (int c = team; c < rq; c += NT / 16) {
        for (int i = 0; i < rq; i++) {
          double x = 0.0;
          if (i >= c) {
            double sd = 0.0;
            for (int k = c + tl; k < i; k += 16) sd += L1[i * LD + k] * L2[k * LD + c];
            for (int o = 8; o > 0; o >>= 1) sd += __shfl_xor(sd, o, 16);
            x = ((i == c) ? 1.0 : 0.0) - sd;
            x = x / L1[i * LD + i];
          }
          if (tl == 0) {
            L2[i * LD + c] = x;
            tr += x * x;
          }
        }
      }
    }
    tr = block_sum<NT>(tr, red);
    // (the certificate's bound assumes tau_S < 1; the eigenvalues of S_(pq,pq) are
    // 1 +- sigma_k <= 2, so a larger tau_S always takes the eigenvalue cut)
    const bool gs = chol_ok && tau_S < 1.0 && (1.0 / tr > tau_S * (2.0 - tau_S));
    if (gs) {
      // X = [[1, -B Z], [0, Z]], Z = L^-T (upper): X into the Y slot (global scratch);
      // the block -B Z (rp x rq) as FP64 MFMA tiles, the rest elementwise
      for (int e = tid; e < n * n; e += NT) {
        int i = e / n, j = e - i * n;
        if (j >= rp && i < rp) continue;
        double x;
        if (j < rp) {
          x = (i == j) ? 1.0 : 0.0;
        } else {
          const int jj = j - rp, ii = i - rp;
          x = (ii <= jj) ? L2[jj * LD + ii] : 0.0;
        }
        Yg[i * n + j] = x;
      }
      mma_tiles<NT>(rp, rq, rq, [&](int i, int k) { return Bg[(long long)i * ld + k]; },
                    [&](int k, int jj) { return k <= jj ? L2[jj * LD + k] : 0.0; },
                    [&](int i, int jj, double v) { Yg[i * n + rp + jj] = -v; });
      if (tid == 0) { s_dt = n; minev[dom_id] = 1.0 / tr; }
      __syncthreads();
      dt = n;
    } else {
      // eigenvalue cut of S_(pq,pq) = U s U^T: X = U_kept s_kept^{-1/2}
      for (int e = tid; e < n * n; e += NT) {
        int i = e / n, j = e - i * n;
        L1[i * LD + j] = comp_elem(S, ld, D, D, i, j, true);
      }
      __syncthreads();
      jacobi_eig<LD, NT, MAXB, MAXV>(L1, L2, n, rt, red, &s_flag);
      if (tid == 0) {
        int c = 0;
        double mn = 1e300;
        for (int k = 0; k < n; k++) {
          double sk = L1[k * LD + k];
          if (sk < mn) mn = sk;
          if (sk > tau_S) keep_idx[c++] = k;
        }
        s_dt = c;
        minev[dom_id] = mn;
      }
      __syncthreads();
      dt = s_dt;
      for (int e = tid; e < n * dt; e += NT) {
        int i = e / dt, c = e - i * dt;
        int k = keep_idx[c];
        Yg[i * n + c] = L2[i * LD + k] / sqrt(L1[k * LD + k]);
      }
      __syncthreads();
    }
    // Fallback start of the Fock eigensolve (block Gram-Schmidt X only): X <- X
    // diag(V_p, V_q) with the eigenvectors of the prepared diagonal domains, so that
    // the p block of X^T F X is already diagonal and the q block nearly so (X^T S X
    // = 1 still); used when the approximate eigenbasis below is not taken
    const long long mp = (gs && dmoff) ? dmoff[D.p] : -1, mq = (gs && dmoff) ? dmoff[D.q] : -1;
    auto warm_start = [&]() {
      if (mp < 0 || mq < 0) return;
      const int rp = D.rp, rq = D.rq;
      const double *Vp = W + mp, *Vq = W + mq;
      mma_tiles<NT>(n, n, n, [&](int i, int k) { return Yg[i * n + k]; },
                    [&](int k, int j) {
                      return k < rp ? (j < rp ? Vp[k * rp + j] : 0.0)
                                    : (j >= rp ? Vq[(k - rp) * rq + (j - rp)] : 0.0);
                    },
                    [&](int i, int j, double v) { L1[i * LD + j] = v; });
      __syncthreads();
      for (int e = tid; e < n * n; e += NT) {
        int i = e / n, j = e - i * n;
        Yg[i * n + j] = L1[i * LD + j];
      }
      __syncthreads();
    };
    // 2) H = X^T F_(pq,pq) X (dt x dt) into L1: L1 = F X (n x dt), L2 = X^T L1,
    //    symmetrised into L1
    auto form_h = [&]() {
      mma_tiles<NT>(n, dt, n, [&](int i, int k) { return comp_elem(F, ld, D, D, i, k, false); },
                    [&](int k, int j) { return Yg[k * n + j]; },
                    [&](int i, int j, double v) { L1[i * LD + j] = v; });
      __syncthreads();
      mma_tiles<NT>(dt, dt, n, [&](int i, int k) { return Yg[k * n + i]; },
                    [&](int k, int j) { return L1[k * LD + j]; },
                    [&](int i, int j, double v) { L2[i * LD + j] = v; });
      __syncthreads();
      for (int e = tid; e < dt * dt; e += NT) {
        int i = e / dt, j = e - i * dt;
        L1[i * LD + j] = 0.5 * (L2[i * LD + j] + L2[j * LD + i]);
      }
      __syncthreads();
    };
    form_h();
    // approximate eigenbasis V1 of H: X <- X V1 (V1 = V0 (3/2 - G/2) through the W
    // slot, not yet written) and H formed again, nearly diagonal
    bool started = false;
    if (dt == n && n >= FOCK_START_MIN && fock_start<LD, NT>(L1, L2, n)) {
      started = true;
      mma_tiles<NT>(n, n, n, [&](int i, int k) { return L2[i * LD + k]; },
                    [&](int k, int j) { return L1[k * LD + j]; },
                    [&](int i, int j, double v) { Wg[i * n + j] = v; });
      __syncthreads();
      mma_tiles<NT>(n, n, n, [&](int i, int k) { return Yg[i * n + k]; },
                    [&](int k, int j) { return Wg[k * n + j]; },
                    [&](int i, int j, double v) { L1[i * LD + j] = v; });
      __syncthreads();
      for (int e = tid; e < n * n; e += NT) {
        int i = e / n, j = e - i * n;
        Yg[i * n + j] = L1[i * LD + j];
      }
      __syncthreads();
      form_h();
    } else {
      warm_start();
      if ((dt == n && n >= FOCK_START_MIN) || (mp >= 0 && mq >= 0)) form_h();   // H overwritten, or X changed
    }
    // From the approximate eigenbasis the off-diagonal elements a_pq of H are of
    // the order of 1e-14 ||H||: one first-order step finishes the eigenproblem,
    // V = 1 + E, E_pq = a_pq / (a_qq - a_pp), eigenvalues a_pp.  E is exactly
    // antisymmetric (H is symmetrised), so V^T V = 1 + E^T E, and what the step
    // leaves out is of order |E|^2, below rounding when every |a_pq| <= 1e-8
    // |a_qq - a_pp|; otherwise (or without the approximate basis) the Jacobi
    // sweeps run.
    bool finished = false;
    if (started) {
      bool bad = false;
      for (int e = tid; e < n * n; e += NT) {
        const int i = e / n, j = e - i * n;
        if (i != j) bad = bad || !(fabs(L1[i * LD + j]) <= 1e-8 * fabs(L1[j * LD + j] - L1[i * LD + i]));
      }
      if (!__syncthreads_or(bad)) {
        for (int e = tid; e < n * n; e += NT) {
          const int i = e / n, j = e - i * n;
          const double a = L1[i * LD + j];
          L2[i * LD + j] = (i == j) ? 1.0 : (a == 0.0 ? 0.0 : a / (L1[j * LD + j] - L1[i * LD + i]));
        }
        __syncthreads();
        finished = true;
      }
    }
    if (!finished) jacobi_eig<LD, NT, MAXB, MAXV>(L1, L2, dt, rt, red, &s_flag);
    for (int a = tid; a < np; a += NT) eg[a] = (a < dt) ? L1[a * LD + a] : 0.0;
    __syncthreads();
    // W = X V (n x dt) into L1, then to global
    mma_tiles<NT>(n, dt, dt, [&](int i, int k) { return Yg[i * n + k]; },
                  [&](int k, int j) { return L2[k * LD + j]; },
                  [&](int i, int j, double v) { L1[i * LD + j] = v; });
    __syncthreads();
    for (int e = tid; e < n * n; e += NT) {
      int i = e / n, j = e - i * n;
      Wg[i * n + j] = (j < dt) ? L1[i * LD + j] : 0.0;
    }
    __syncthreads();
    // 3) Y = W^T S_(pq,pq) (dt x n) into L2
    mma_tiles<NT>(dt, n, n, [&](int a, int k) { return L1[k * LD + a]; },
                  [&](int k, int j) { return comp_elem(S, ld, D, D, k, j, true); },
                  [&](int a, int j, double v) { L2[a * LD + j] = v; });
    __syncthreads();
  } else {
    // diagonal domain: S = 1, W = eigenvectors of F_pp
    for (int e = tid; e < n * n; e += NT) {
      int i = e / n, j = e - i * n;
      L1[i * LD + j] = 0.5 * (F[(long long)(D.offp + i) * ld + (D.offp + j)] +
                              F[(long long)(D.offp + j) * ld + (D.offp + i)]);
    }
    __syncthreads();
    jacobi_eig<LD, NT, MAXB, MAXV>(L1, L2, n, rt, red, &s_flag);
    // S_(p,p) = 1: every overlap eigenvalue is 1, kept unless tau_S >= 1
    dt = (1.0 > tau_S) ? n : 0;
    if (tid == 0) minev[dom_id] = 1.0;
    for (int a = tid; a < np; a += NT) eg[a] = (a < dt) ? L1[a * LD + a] : 0.0;
    for (int e = tid; e < n * n; e += NT) {
      int i = e / n, j = e - i * n;
      Wg[i * n + j] = L2[i * LD + j];
    }
    __syncthreads();
    // Y = W^T
    for (int e = tid; e < n * n; e += NT) {
      int a = e / n, j = e - a * n;
      L1[a * LD + j] = L2[j * LD + a];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += NT) {
      int a = e / n, j = e - a * n;
      L2[a * LD + j] = L1[a * LD + j];
    }
    __syncthreads();
  }
  // Y (dt x n) is in L2: store it
  for (int e = tid; e < n * n; e += NT) {
    int a = e / n, j = e - a * n;
    Yg[a * n + j] = (a < dt) ? L2[a * LD + j] : 0.0;
  }
  // 4) K~ = Y_p K_pq Y_q^T: L1 = Y_p K_pq (dt x rq), then K~ = L1 Y_q^T (stored as K~^T)
  const int rq = diag ? D.rp : D.rq;
  const int offq = diag ? D.offp : D.offq;
  const int qcol = diag ? 0 : D.rp;
  mma_tiles<NT>(dt, rq, D.rp, [&](int a, int k) { return L2[a * LD + k]; },
                [&](int k, int j) { return K[(long long)(D.offp + k) * ld + (offq + j)]; },
                [&](int a, int j, double v) { L1[a * LD + j] = v; });
  __syncthreads();
  // stored transposed and zero-padded: Kg[b np + a] = K~(a, b)
  for (int e = tid; e < np * np; e += NT) {
    const int b = e / np, a = e - b * np;
    if (a >= dt || b >= dt) Kg[b * np + a] = 0.0;
  }
  mma_tiles<NT>(dt, dt, rq, [&](int a, int k) { return L1[a * LD + k]; },
                [&](int k, int b) { return L2[b * LD + qcol + k]; },
                [&](int a, int b, double v) { Kg[b * np + a] = v; });
  if (tid == 0) rank[dom_id] = dt;
}

hipError_t launch_domain_prep(const Domain *dom, const int *ids, const int *counts,
                              const double *S, const double *F, const double *K, long long ld,
                              double tau_S, const long long *diag_moff, double *W, double *Y,
                              double *Kep, int *rank, double *minev, hipStream_t s) {
  // counts: number of domains with n <= 32, 32 < n <= 64, 64 < n <= PREP_N3,
  // PREP_N3 < n <= DMAX, in that order in ids[]; threads per class from the tuning
  // table, except the third class (512 threads: two workgroups share a CU's LDS)
  int o = 0;
  const int *nt = tuning().prep_nt;
#define OSV_PREP(NM, NT, c)                                                                      \
  hipLaunchKernelGGL((k_domain_prep<NM, NT>), dim3(counts[c]), dim3(NT), 0, s, dom, ids + o, S, F, \
                     K, ld, tau_S, diag_moff, W, Y, Kep, rank, minev)
  if (counts[0] > 0) {
    if (nt[0] == 128) OSV_PREP(32, 128, 0);
    else OSV_PREP(32, 256, 0);
  }
  o += counts[0];
  if (counts[1] > 0) {
    if (nt[1] == 256) OSV_PREP(64, 256, 1);
    else if (nt[1] == 1024) OSV_PREP(64, 1024, 1);
    else OSV_PREP(64, 512, 1);
  }
  o += counts[1];
  if (counts[2] > 0) OSV_PREP(PREP_N3, 512, 2);
  o += counts[2];
  if (counts[3] > 0) {
    if (nt[2] == 512) OSV_PREP(DMAX, 512, 3);
    else OSV_PREP(DMAX, 1024, 3);
  }
#undef OSV_PREP
  return hipGetLastError();
}

// Couplings M(A,B) = W_A^T S_(A,B) W_B, one workgroup (8 wave64) per coupling,
// FP64 MFMA 16x16x4.  G = S_(A,B) W_B (n_A x dt_B) is formed in LDS; the product
// W_A^T G is then taken once per orientation, so that M(A,B) and M(B,A) =
// M(A,B)^T are both written with row-contiguous stores over their whole
// zero-padded np x np slots.  G keeps only the dt_B columns that can be nonzero,
// so that several workgroups share a CU and one coupling's loads overlap another's
// products.  Two size classes by the larger of the two domain dimensions: up to
// 64 (4 waves, G 33 KB, four workgroups per CU) and up to DMAX (8 waves, G
// 80.8 KB, two per CU); ids lists the couplings of the class.
typedef double d4c __attribute__((ext_vector_type(4)));

template <int NM, int CNT>
__global__ __launch_bounds__(CNT) void k_couplings(const Coupling *__restrict__ cpl,
                                                   const int *__restrict__ ids,
                                                   const Domain *__restrict__ doms,
                                                   const int *__restrict__ rank,
                                                   const double *__restrict__ S, long long ld,
                                                   const double *__restrict__ W,
                                                   double *M) {
  constexpr int LDG = NM + 1;   // LDS stride of G (columns < dt_B <= NM)
  __shared__ double G[NM * LDG];
  const Coupling c = cpl[ids[blockIdx.x]];
  const Domain A = doms[c.A], B = doms[c.B];
  const int dtA = rank[c.A], dtB = rank[c.B];
  const double *WA = W + A.moff, *WB = W + B.moff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  constexpr int NWV = CNT / 64;
  // 1) G(i, j) = sum_k S_(A,B)(i, k) W_B(k, j); S_(A,B)(i, k) is read as S_(B,A)(k, i),
  //    which is contiguous in i for a fixed k (S holds both orientations of its blocks).
  //    A wave keeps one row tile of S_(A,B) in registers for its whole k range and
  //    walks over column tiles of W_B, loading each one's k range in two batches.
  constexpr int KST = (NM + 3) / 4;   // k-steps of 4 covering the class's dimensions
  constexpr int KH = (KST + 1) / 2;
  const int ti = (A.n + 15) >> 4, tjn = (dtB + 15) >> 4;   // column tiles holding G's dt_B columns
  {
    const int grp = NWV / ti, it = wave % ti, g = wave / ti;
    if (g < grp) {
      const int i = it * 16 + l15;
      double av[KST];
#pragma unroll
      for (int st = 0; st < KST; st++) {
        const int k = 4 * st + lhi;
        av[st] = (i < A.n && k < B.n) ? comp_elem(S, ld, B, A, k, i, true) : 0.0;
      }
      for (int jt = g; jt < tjn; jt += grp) {
        const int j = jt * 16 + l15;
        d4c acc = {0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < 2; h++) {
          double bv[KH];
#pragma unroll
          for (int u = 0; u < KH; u++) {
            const int st = h * KH + u, k = 4 * st + lhi;
            bv[u] = (st < KST && j < dtB && k < B.n) ? WB[k * B.n + j] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < KH; u++) {
            const int st = h * KH + u;
            if (st < KST && 4 * st < B.n)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bv[u], acc, 0, 0, 0);
          }
        }
        // accumulator: lane l, register v -> row 4v + (l >> 4), column l & 15
        for (int v = 0; v < 4; v++) {
          const int ii = it * 16 + 4 * v + lhi;
          if (ii < A.n && j < dtB) G[ii * LDG + j] = acc[v];
        }
      }
    }
  }
  __syncthreads();
  // 2) M(A,B)(a, b) = sum_k W_A(k, a) G(k, b) and M(B,A)(b, a) = sum_k G(k, b) W_A(k, a)
  //    over the padded ranges (W_A columns beyond dt_A and G columns beyond dt_B are
  //    taken as 0).
  //    A wave keeps one column tile of W_A in registers and walks over column tiles
  //    of G; each G fragment read from LDS feeds both orientations.
  const int ta = A.np >> 4, tb = B.np >> 4;
  double *Mab = M + c.offAB, *Mba = M + c.offBA;
  {
    const int grp = NWV / ta, at = wave % ta, g = wave / ta;
    if (g < grp) {
      const int a0 = at * 16, a = a0 + l15;
      double wv[KST];
#pragma unroll
      for (int st = 0; st < KST; st++) {
        const int k = 4 * st + lhi;
        wv[st] = (a < dtA && k < A.n) ? WA[k * A.n + a] : 0.0;
      }
      for (int bt = g; bt < tb; bt += grp) {
        const int b0 = bt * 16, b = b0 + l15;
        d4c acc = {0, 0, 0, 0}, acct = {0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < KST; st++) {
          if (4 * st < A.n) {
            const int k = 4 * st + lhi;
            const double gv = (k < A.n && b < dtB) ? G[k * LDG + b] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[st], gv, acc, 0, 0, 0);
            acct = __builtin_amdgcn_mfma_f64_16x16x4f64(gv, wv[st], acct, 0, 0, 0);
          }
        }
        for (int v = 0; v < 4; v++) {
          Mab[(long long)(a0 + 4 * v + lhi) * B.np + b] = acc[v];
          Mba[(long long)(b0 + 4 * v + lhi) * A.np + a] = acct[v];
        }
      }
    }
  }
}

hipError_t launch_couplings(const Coupling *cpl, const int *ids, int n64, int nbig,
                            const Domain *dom, const int *rank, const double *S, long long ld,
                            const double *W, double *M, hipStream_t s) {
  if (n64 > 0)
    hipLaunchKernelGGL((k_couplings<64, 256>), dim3(n64), dim3(256), 0, s, cpl, ids, dom, rank, S, ld,
                       W, M);
  if (nbig > 0)
    hipLaunchKernelGGL((k_couplings<DMAX, 512>), dim3(nbig), dim3(512), 0, s, cpl, ids + n64, dom,
                       rank, S, ld, W, M);
  return hipGetLastError();
}

// Cross-projected integrals of one pair domain in its pseudo-canonical basis:
// K~(a, b) = sum_P Gp[a][P] Gq[b][P] with Gp = V^T B_p, Gq = V^T B_q (dt x naux,
// V = [Q_p Q_q] W the domain's pseudo-canonical virtuals), stored as K~^T in the
// domain's zero-padded slot (Kt[b np + a]).
__global__ __launch_bounds__(256) void k_exact_ktilde(const double *__restrict__ Gp,
                                                      const double *__restrict__ Gq, int dt, int naux,
                                                      double *Kt, int np) {
  mma_tiles<256>(dt, dt, naux, [&](int a, int k) { return Gp[(long long)a * naux + k]; },
                 [&](int k, int b) { return Gq[(long long)b * naux + k]; },
                 [&](int a, int b, double v) { Kt[(long long)b * np + a] = v; });
}

hipError_t launch_exact_ktilde(const double *Gp, const double *Gq, int dt, int naux, double *Kt, int np,
                               hipStream_t s) {
  if (dt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exact_ktilde, dim3(1), dim3(256), 0, s, Gp, Gq, dt, naux, Kt, np);
  return hipGetLastError();
}

// Weak 2b clusters, one-block dispersion scheme: pair (i, j) keeps only the block
// T_(i,j) in the pseudo-canonical bases of the diagonal domains (i, i) and (j, j)
// (their W slots, ranks and eigenvalues e~ from the preparation), where the
// one-block residual K~ + (e~_a + e~_b - f_ii - f_jj) T~ vanishes in one step:
// T~ = -K~ / Delta with K~ = W_i^T K_ij W_j.  The pair's energy over both
// orderings is 4 <T~, K~> = -4 sum K~^2 / Delta.  One workgroup per pair, every
// product on FP64 MFMA tiles (mma_tiles):
//   G = K_ij W_j (LDS), K~ = W_i^T G, T~ and the sums e = 4 <T~, K~>, tt = <T~, T~>;
// with STORE_T also the amplitudes in the OSV bases, T = W_i T~ W_j^T (r_i x r_j,
// row-major at toff[w]), through the pair's own slot: T~, then W_i T~, then T.
constexpr int WNT = 256;
constexpr int WLD = DMAX + 1;

template <bool STORE_T>
__global__ __launch_bounds__(WNT) void k_weak(const int2 *__restrict__ wp,
                                              const Domain *__restrict__ doms,
                                              const int *__restrict__ rank,
                                              const double *__restrict__ K, long long ld,
                                              const double *__restrict__ W,
                                              const double *__restrict__ Kep,
                                              const double *__restrict__ F, int nocc,
                                              const long long *__restrict__ toff, double *Tw,
                                              double *out_e, double *out_tt) {
  __shared__ double X[DMAX * WLD];   // W_j, then W_i, then W_j
  __shared__ double Y[DMAX * WLD];   // K_ij W_j, then T~, then W_i T~
  __shared__ double red[2 * (WNT / 64)];
  const int2 pr = wp[blockIdx.x];
  const Domain Di = doms[pr.x], Dj = doms[pr.y];
  const int ri = Di.n, rj = Dj.n, dti = rank[pr.x], dtj = rank[pr.y];
  const int tid = threadIdx.x;
  for (int e = tid; e < rj * rj; e += WNT) {
    const int b = e / rj, d = e - b * rj;
    X[b * WLD + d] = W[Dj.moff + e];
  }
  __syncthreads();
  mma_tiles<WNT>(ri, dtj, rj, [&](int a, int b) { return K[(long long)(Di.offp + a) * ld + Dj.offp + b]; },
                 [&](int b, int d) { return X[b * WLD + d]; },
                 [&](int a, int d, double v) { Y[a * WLD + d] = v; });
  __syncthreads();
  for (int e = tid; e < ri * ri; e += WNT) {
    const int a = e / ri, c = e - a * ri;
    X[a * WLD + c] = W[Di.moff + e];
  }
  __syncthreads();
  const double *ei = Kep + Di.voff + (long long)Di.np * Di.np;
  const double *ej = Kep + Dj.voff + (long long)Dj.np * Dj.np;
  const double fd = F[Di.p * nocc + Di.p] + F[Dj.p * nocc + Dj.p];
  double *T = STORE_T ? Tw + toff[blockIdx.x] : nullptr;
  double acc = 0.0, tt = 0.0;
  // K~(c, d) = sum_a W_i(a, c) G(a, d)
  mma_tiles<WNT>(dti, dtj, ri, [&](int c, int a) { return X[a * WLD + c]; },
                 [&](int a, int d) { return Y[a * WLD + d]; },
                 [&](int c, int d, double kt) {
                   const double t = -kt / (ei[c] + ej[d] - fd);
                   acc += t * kt;
                   tt += t * t;
                   if (STORE_T) T[c * rj + d] = t;
                 });
  acc = wave_sum(acc);
  tt = wave_sum(tt);
  if ((tid & 63) == 0) {
    red[tid >> 6] = acc;
    red[WNT / 64 + (tid >> 6)] = tt;
  }
  __syncthreads();
  if (tid == 0) {
    double e = 0.0, t2 = 0.0;
    for (int w = 0; w < WNT / 64; w++) {
      e += red[w];
      t2 += red[WNT / 64 + w];
    }
    out_e[blockIdx.x] = 4.0 * e;
    if (STORE_T) out_tt[blockIdx.x] = t2;
  }
  if (STORE_T) {
    // T~ (written by every wave) back into LDS: the device-scope fence makes the
    // slot's stores visible to the whole workgroup after the barrier
    __threadfence();
    __syncthreads();
    for (int e = tid; e < dti * dtj; e += WNT) {
      const int c = e / dtj, d = e - c * dtj;
      Y[c * WLD + d] = T[c * rj + d];
    }
    __syncthreads();
    // H = W_i T~ (ri x dtj) into the slot
    mma_tiles<WNT>(ri, dtj, dti, [&](int a, int c) { return X[a * WLD + c]; },
                   [&](int c, int d) { return Y[c * WLD + d]; },
                   [&](int a, int d, double v) { T[a * rj + d] = v; });
    __threadfence();
    __syncthreads();
    for (int e = tid; e < ri * dtj; e += WNT) {
      const int a = e / dtj, d = e - a * dtj;
      Y[a * WLD + d] = T[a * rj + d];
    }
    for (int e = tid; e < rj * rj; e += WNT) {
      const int b = e / rj, d = e - b * rj;
      X[b * WLD + d] = W[Dj.moff + e];
    }
    __syncthreads();
    // T = H W_j^T (ri x rj): columns past dt_j of W_j are not used
    mma_tiles<WNT>(ri, rj, dtj, [&](int a, int d) { return Y[a * WLD + d]; },
                   [&](int d, int b) { return X[b * WLD + d]; },
                   [&](int a, int b, double v) { T[a * rj + b] = v; });
  }
}

hipError_t launch_weak(const int2 *wp, int nweak, const Domain *dom, const int *rank,
                       const double *K, long long ld, const double *W, const double *Kep,
                       const double *F, int nocc, double *out, hipStream_t s) {
  if (nweak <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weak<false>, dim3(nweak), dim3(WNT), 0, s, wp, dom, rank, K, ld, W, Kep, F, nocc,
                     (const long long *)nullptr, (double *)nullptr, out, (double *)nullptr);
  return hipGetLastError();
}

hipError_t launch_weak_amplitudes(const int2 *wp, int nweak, const Domain *dom, const int *rank,
                                  const double *K, long long ld, const double *W, const double *Kep,
                                  const double *F, int nocc, const long long *toff, double *Tw,
                                  double *out_e, double *out_tt, hipStream_t s) {
  if (nweak <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weak<true>, dim3(nweak), dim3(WNT), 0, s, wp, dom, rank, K, ld, W, Kep, F, nocc,
                     toff, Tw, out_e, out_tt);
  return hipGetLastError();
}

// Densities of the weak pairs' one-block energies (stationary one-block Hylleraas
// functional 8 <T, K_ij> + 4 <T, F_(i,i) T + T F_(j,j) - (f_ii + f_jj) T>, OSV
// bases, S_(i,i) = 1):
//   dE/dK_ij = 8 T  ->  G^K_ij = 4 T, G^K_ji = 4 T^T (dE/dC = 2 G^K C);
//   dE/dF_(i,i) = 4 T T^T, dE/dF_(j,j) = 4 T^T T  ->  G^F diagonal blocks;
//   dE/df_ii = dE/df_jj = -4 <T, T>.
// G^K: the (i, j) blocks of weak pairs belong to no pair domain, so they are
// written once, by the pair's workgroup.
__global__ __launch_bounds__(WNT) void k_weak_gk(const int2 *__restrict__ lmo, const int *__restrict__ off,
                                                 const int *__restrict__ r, const long long *__restrict__ toff,
                                                 const double *__restrict__ Tw, double *GK, long long ld) {
  const int2 ij = lmo[blockIdx.x];
  const int ri = r[ij.x], rj = r[ij.y], oi = off[ij.x], oj = off[ij.y];
  const double *T = Tw + toff[blockIdx.x];
  for (int e = threadIdx.x; e < ri * rj; e += WNT) {
    const int a = e / rj, b = e - a * rj;
    const double v = 4.0 * T[e];
    GK[(long long)(oi + a) * ld + oj + b] = v;
    GK[(long long)(oj + b) * ld + oi + a] = v;
  }
}

// G^F_(p,p) += 4 sum over the weak pairs holding p, in pair order, of T T^T (p first)
// or T^T T (p second); one workgroup per LMO, output tiles on FP64 MFMA with each
// tile's sum over pairs and k in a fixed order.
__global__ __launch_bounds__(WNT) void k_weak_gf(const long long *__restrict__ lptr,
                                                 const int *__restrict__ lidx,
                                                 const int2 *__restrict__ lmo, const int *__restrict__ off,
                                                 const int *__restrict__ r, const long long *__restrict__ toff,
                                                 const double *__restrict__ Tw, double *GF, long long ld) {
  const int p = blockIdx.x;
  const long long w0 = lptr[p], w1 = lptr[p + 1];
  if (w0 == w1) return;
  const int rp = r[p], op = off[p];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l15 = lane & 15, lhi = lane >> 4;
  const int tn = (rp + 15) >> 4;
  for (int t = wave; t < tn * tn; t += WNT / 64) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
    const int i = i0 + l15, j = j0 + l15;
    d4p acc = {0, 0, 0, 0};
    for (long long w = w0; w < w1; w++) {
      const int pw = lidx[w];
      const int2 ij = lmo[pw];
      const bool first = ij.x == p;
      const int rq = r[first ? ij.y : ij.x];
      const double *T = Tw + toff[pw];
      // first: C(i, j) = sum_k T(i, k) T(j, k), T is rp x rq;
      // second: C(i, j) = sum_k T(k, i) T(k, j), T is rq x rp
      for (int k0 = 0; k0 < rq; k0 += 4) {
        const int k = k0 + lhi;
        double av = 0.0, bv = 0.0;
        if (k < rq) {
          if (first) {
            av = i < rp ? T[i * rq + k] : 0.0;
            bv = j < rp ? T[j * rq + k] : 0.0;
          } else {
            av = i < rp ? T[k * rp + i] : 0.0;
            bv = j < rp ? T[k * rp + j] : 0.0;
          }
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int ii = i0 + 4 * v + lhi;
      if (ii < rp && j < rp) GF[(long long)(op + ii) * ld + op + j] += 4.0 * acc[v];
    }
  }
}

// dE/df_pp -= 4 sum over the weak pairs holding p, in pair order, of <T, T>
__global__ void k_weak_focc(const long long *__restrict__ lptr, const int *__restrict__ lidx,
                            const double *__restrict__ tt, int nocc, double *dF) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nocc) return;
  double s = 0.0;
  for (long long w = lptr[p]; w < lptr[p + 1]; w++) s += tt[lidx[w]];
  if (lptr[p + 1] > lptr[p]) dF[(long long)p * nocc + p] -= 4.0 * s;
}

hipError_t launch_weak_densities(int nweak, int nocc, const int2 *lmo, const int *off, const int *r,
                                  const long long *toff, const double *Tw, const double *tt,
                                  const long long *lptr, const int *lidx, double *GK, double *GF,
                                  long long ld, double *dF, hipStream_t s) {
  if (nweak <= 0) return hipSuccess;
  if (GK)
    hipLaunchKernelGGL(k_weak_gk, dim3(nweak), dim3(WNT), 0, s, lmo, off, r, toff, Tw, GK, ld);
  if (GF)
    hipLaunchKernelGGL(k_weak_gf, dim3(nocc), dim3(WNT), 0, s, lptr, lidx, lmo, off, r, toff, Tw, GF, ld);
  if (dF)
    hipLaunchKernelGGL(k_weak_focc, dim3((nocc + 255) / 256), dim3(256), 0, s, lptr, lidx, tt, nocc, dF);
  return hipGetLastError();
}

}  // namespace osv
