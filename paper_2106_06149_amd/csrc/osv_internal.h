// Internal layout shared by the host orchestration and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osv {

constexpr int DMAX = 100;      // largest pair-domain dimension r_p + r_q
constexpr int PREP_N3 = 70;    // domains of 64 < n <= PREP_N3 are prepared two per CU
// clusters with at most SOLVE_MAXT pairs and SOLVE_MAXTERM terms run in the solve
// kernel that keeps their descriptors in LDS (every MBE(3) cluster does)
constexpr int SOLVE_MAXT = 16, SOLVE_MAXTERM = 64;
constexpr int NTHREADS = 256;  // threads of every per-item workgroup (4 wave64)

// One pair domain [Q_p Q_q] (p < q) or Q_p (p == q).  Every per-domain square
// matrix (W, Y = W^T S, the OSV-basis virtual density) lives in an n x n slot at
// moff (row-major, ld n); K~ (transposed) and the pseudo-canonical energies e~
// live in a zero-padded slot at voff (np x np, ld np, then np values).  The
// kept rank dt <= n is written by the preparation kernel into dom_rank[].
// np = n rounded up to a multiple of 16: the leading dimension of the zero-padded
// amplitude and coupling slots used by the solve.
struct Domain {
  int p, q, rp, rq, n, offp, offq, np;
  long long moff;   // n*n slot offset
  long long voff;   // offset of the zero-padded slot holding K~^T (np x np) then e~ (np)
};

// Coupling between domains A < B that share an LMO, stored in both orientations
// as zero-padded row-major slots:
//   offAB: M(A,B) = W_A^T S_(A,B) W_B   (np_A x np_B, ld np_B)
//   offBA: M(B,A) = M(A,B)^T            (np_B x np_A, ld np_A)
// entries beyond the kept ranks are zero.
struct Coupling {
  int A, B;
  long long offAB, offBA;
};

// One residual term of eq:rij in pseudo-canonical coordinates:
//   R~_tgt += -f[fa][fb] * M op(T~_src) M^T,   M = M(tgt, src)
// flags bit0: the target is the coupling's B domain (the source is A)
//       bit1: op = transpose (ordered source pair (a,b) with a > b)
struct Term {
  int src;    // absolute cluster-pair index of the source amplitudes
  int cpl;    // coupling index
  int flags;
  int fa, fb; // global LMO indices of the coefficient f[fa][fb]
  int la, lb; // the same LMOs as cluster-local indices (dE/dF bookkeeping)
  int pad;
};

// One unordered LMO pair (p <= q) of one cluster.
struct CPair {
  int dom;
  int la, lb;         // cluster-local LMO indices of p and q
  int term0, nterm;   // range in the term array
  int w;              // 1 for p == q, 2 for p < q (ordered-pair multiplicity)
  long long toff;     // offset of the amplitude slots: T~ (np x np, ld np) at toff,
                      // T~^T at toff + np*np; zero beyond the kept rank
  long long init;     // amplitude slots of the same pair in a cluster solved by an
                      // earlier launch (its final amplitudes start this pair's
                      // sweeps), or -1: the sweeps start from zero
};

struct Cluster {
  int cp0, ncp;       // range of cluster pairs
  int nlmo, lmo0;     // LMOs: cl_lmo[lmo0 .. lmo0+nlmo)
  long long toff0;    // amplitude offset of the first pair (scratch base)
  int term0, term1;   // the cluster's terms (contiguous, in pair order)
  long long poff;     // offset of the nlmo x nlmo block of dE/dF inner products
};

// Everything the solve kernel needs about one term, gathered once after the
// pair domains are prepared (one aligned 32-byte load per term).
struct TermFlat {
  long long tsrc;   // slot of op(T~_src) as a row-major np_src x np_src matrix
                    // (the T~ slot, or the T~^T slot when op is a transpose)
  long long moff;   // slot of M(src, tgt) (np_src x np_tgt, row-major)
  double coef;      // -f[fa][fb]
  short ldT, ldM;   // np_src, np_tgt
  int ns;           // kept rank of the source domain
};

// One term of the collective residual of the one-step correction: the source
// domain's collective amplitudes op(T~c_src) at tsrc (its T~c or T~c^T slot), the
// coupling M(src, tgt) at moff, the coefficient -f[fa][fb].
struct CTerm {
  long long tsrc;
  long long moff;
  int src;      // source domain
  int fa, fb;
  int ldT;      // np of the source domain
};

struct SolveArgs {
  const TermFlat *tflat;
  const Cluster *cl;
  const CPair *cp;
  const Term *terms;
  const Domain *dom;
  const int *dom_rank;
  const Coupling *cpl;
  const double *M;      // couplings
  const double *Kep;    // per domain: K~^T (np x np) then e~ (np), zero-padded
  const double *F_occ;  // nocc x nocc
  int nocc;
  double *T;            // amplitudes per cluster pair (final values)
  double *T2;           // second buffer of the same layout: sweeps alternate T -> T2 -> T
  double *Rs;           // per-workgroup scratch (the P pass's per-term products)
  long long rs_stride;  // doubles per workgroup
  double *Ecl;          // [n_clusters] Hylleraas energies
  double *Pl;           // dE/dF inner products per cluster (nlmo x nlmo)
  int *sweeps;          // [n_clusters]
  double *maxres;       // [n_clusters]
  const int *queue;     // cluster order (cost descending)
  int *counter;         // work-queue heads (three: large clusters, clusters of <= 2
                        // LMOs, the rest)
  int n_clusters;
  double tau_R;
  int max_sweeps;
  int split;            // 1: balanced (column block, source block) work split over the
                        // waves (sweeps that take no per-term products); 0: one wave per
                        // column block
};

// OSV response N_ij (eq:nij) of one stored pair domain d = [pq] and, for p < q,
// of the reversed pair (q, p): the clusters holding the pair with nonzero MBE
// coefficient (entries ent0 .. ent1: cluster pair index and c_X, cluster order),
// the LMOs that its k-sums reach (lmo_tab[lmo0 .. lmo0 + nlmo): LMO and its column
// offset in the per-LMO accumulator, lb columns in all) and the output offsets of
// N_pq and N_qp (n x n row-major each; -1 for p == q).
struct NijTarget {
  int dom, nlmo, lb, pad;
  long long ent0, ent1, lmo0;
  long long outF, outR;
};

struct NijArgs {
  const NijTarget *tg;
  int ntg;
  const int *ent_cp;      // cluster pair of each entry
  const double *ent_c;    // c_X of each entry
  const int2 *lmo_tab;    // (LMO, column offset in the accumulator)
  const int2 *bcol;       // per residual term: accumulator columns of the source's
                          // first and second LMO blocks (-1: diagonal source)
  const int *tmate;       // per residual term of a diagonal target (p, p): the sum-2
                          // term of the same source and coefficient (the pair is
                          // taken at once), -2 for that sum-2 term, else -1
  const CPair *cp;
  const Term *terms;
  const TermFlat *tflat;
  const Domain *dom;
  const int *rank;
  const double *W, *Y;    // per-domain slots (moff)
  const double *Kep;      // per domain: K~^T then e~ (voff)
  const double *M;        // couplings
  const double *T;        // converged cluster amplitudes
  const double *S, *F, *K;
  long long ld;
  const double *F_occ;
  int nocc;
  const int *off, *r;     // per LMO: first OSV row, number of OSVs
  double *scr;            // per-workgroup scratch of scr_stride doubles
  long long scr_stride;
  int *counter;           // work-queue head
  double *N;              // output
};

// Launch parameters chosen at run time among compiled variants: defaults are the
// hand-measured choices; a tuning file written by the autotuner (key value lines,
// read once per process: $OSV_TUNING_FILE, else osv_tuning.txt beside the library)
// or osv_set_tuning overrides them.  Every variant computes the same quantities.
struct Tuning {
  int gemm_ks = 16;                     // FP64 tile GEMM k per stage: 8, 16, 32
  int prep_nt[3] = {256, 512, 1024};    // domain preparation threads for n <= 32 {128, 256},
                                        // 32 < n <= 64 {256, 512, 1024}, PREP_N3 < n <= DMAX
                                        // {512, 1024} (64 < n <= PREP_N3: 512)
  int cpl_split = 64;                   // couplings with both domains <= this run in the
                                        // 4-wave class: 0 (none) or 64
  int solve_split = 1;                  // residual solve: balanced work split of each
                                        // target over the waves (1) or one wave per
                                        // 16-column block (0)
};
Tuning &tuning();

}  // namespace osv

// ---- launch wrappers (defined next to their kernels) -----------------------
namespace osv {
// C[i][j] = sum_k A[i][k] A[j][k] (and C2 with weight w[k]) on the listed output
// tiles (ti <= tj; the transposed tile is written too); A row-major.  FP64 A with
// even lda and K runs on the 128x128 tiles of tiles128, anything else on the
// 64x64 tiles of tiles.
hipError_t launch_syrk_f64(const void *A, int a_is_f32, long long lda, int M, int K,
                           const double *w, double *C, double *C2, long long ldc,
                           const int2 *tiles, int ntiles, const int2 *tiles128, int ntiles128,
                           hipStream_t s);
hipError_t launch_f32_to_f64(const float *x, double *y, long long n, hipStream_t s);
// mixed-precision K: exact int8 digit planes of the FP32 rows with per-row
// power-of-two exponents (digit_bytes(nrow, ncol) bytes), then the digit SYRK on
// 128 x 64 output tiles (tile row ti covers rows 128 ti.., column tj columns 64 tj..);
// K (ncol) at most digit_max_k()
size_t digit_bytes(int nrow, int ncol);
int digit_max_k();
hipError_t launch_split_digits(const float *C, int nrow, int ncol, int *exps, void *dig,
                               hipStream_t s);
hipError_t launch_syrk_digits(const void *dig, int M, int K, const int *exps, double *C,
                              long long ldc, const int2 *tiles, int ntiles, hipStream_t s);
// dE/dC-type products from digit planes: C (MA x MB, ldc) = 2^eadd A B^T with the
// rows of A and of B split by launch_split_digits* over the same K
hipError_t launch_gemm_digits(const void *digA, int MA, const void *digB, int MB, int K,
                              const int *expsA, const int *expsB, int eadd, double *C,
                              long long ldc, hipStream_t s);
hipError_t launch_split_digits_f64(const double *A, long long lda, int nrow, int ncol, int *exps,
                                   void *dig, hipStream_t s);
hipError_t launch_transpose_f32(const float *X, int rows, int cols, float *Xt, hipStream_t s);
hipError_t launch_transpose_f64(const double *X, int rows, int cols, double *Xt, hipStream_t s);
// the listed 128 x 64 tiles of a symmetric C = A B^T (both orientations stored), from
// the digit planes of A and B (M rows each, the same K)
hipError_t launch_syr2_digits(const void *digA, const void *digB, int M, int K, const int *expsA,
                              const int *expsB, double *C, long long ldc, const int2 *tiles,
                              int ntiles, hipStream_t s);
hipError_t launch_scale_cols(const double *X, const double *w, int rows, int cols, double *Y,
                             hipStream_t s);
// C[i][j] = alpha * sum_k A[i][k] B[k][j]  (A row-major M x K, B row-major K x N)
hipError_t launch_gemm_nn_f64(const double *A, long long lda, const double *B, int b_is_f32,
                              long long ldb, double *C, long long ldc, int M, int N, int K,
                              double alpha, hipStream_t s);
// C[i][j] = alpha * sum_k A[k][i] B[k][j]  (A row-major K x M)
hipError_t launch_gemm_tn_f64(const double *A, long long lda, const double *B, long long ldb,
                              double *C, long long ldc, int M, int N, int K, double alpha,
                              hipStream_t s);
// diag_moff (may be null): per LMO p the W slot of the prepared domain (p, p) or
// -1; off-diagonal domains then start their Fock eigensolve from those
// eigenvectors
hipError_t launch_domain_prep(const Domain *dom, const int *ids, const int *counts,
                              const double *S, const double *F, const double *K, long long ld,
                              double tau_S, const long long *diag_moff, double *W, double *Y,
                              double *Kep, int *rank, double *minev, hipStream_t s);
// both orientations of every coupling, zero-padded (FP64 MFMA); ids: the n64
// couplings whose domains both have n <= 64, then the nbig others
hipError_t launch_couplings(const Coupling *cpl, const int *ids, int n64, int nbig,
                            const Domain *dom, const int *rank, const double *S, long long ld,
                            const double *W, double *M, hipStream_t s);
constexpr double OSV_WEAK_MIN = 1e-7;   // weak pairs below this s2b are discarded
// weak 2b clusters: per pair (diagonal domain of i, of j) the one-block
// dispersion energy into out[nweak]
hipError_t launch_weak(const int2 *wp, int nweak, const Domain *dom, const int *rank,
                       const double *K, long long ld, const double *W, const double *Kep,
                       const double *F, int nocc, double *out, hipStream_t s);
// the same pairs with their amplitudes kept: T = W_i T~ W_j^T (r_i x r_j, row-major
// at toff[w]), pair energies out_e and <T, T> out_tt
hipError_t launch_weak_amplitudes(const int2 *wp, int nweak, const Domain *dom, const int *rank,
                                  const double *K, long long ld, const double *W, const double *Kep,
                                  const double *F, int nocc, const long long *toff, double *Tw,
                                  double *out_e, double *out_tt, hipStream_t s);
// the weak pairs' density contributions: G^K (i, j) blocks (written), G^F diagonal
// blocks (added, per LMO over lptr/lidx in pair order) and dE/df_pp (added); any
// of GK, GF, dF may be null
hipError_t launch_weak_densities(int nweak, int nocc, const int2 *lmo, const int *off, const int *r,
                                 const long long *toff, const double *Tw, const double *tt,
                                 const long long *lptr, const int *lidx, double *GK, double *GF,
                                 long long ld, double *dF, hipStream_t s);
// queue: [0, n_big) global descriptors; [n_big, n_first) and [n_first, n) LDS
// descriptors in two launches (the second one's clusters may start from amplitudes
// of the first one's)
hipError_t launch_solve(const SolveArgs &a, int n_big, int n_first, int nwg, hipStream_t s);
hipError_t launch_term_flat(const Term *terms, long long nterms, const CPair *cp,
                            const Coupling *cpl, const Domain *dom, const int *rank,
                            const double *F_occ, int nocc, TermFlat *out, hipStream_t s);
hipError_t launch_fill_i32(int *p, int v, long long n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, long long n, hipStream_t s);
hipError_t launch_check_finite(const double *x, long long n, int *flag, hipStream_t s);
hipError_t launch_check_finite_f32(const float *x, long long n, int *flag, hipStream_t s);
// fixed-order weighted sums: out[j] = sum_i w[j*n + i] * x[i], j < nw
hipError_t launch_wdot(const double *x, const double *w, long long n, int nw, double *out,
                       hipStream_t s);
// adjoint per domain: G^K blocks into GK (ld), virtual density in OSV basis into Gd
hipError_t launch_adjoint(const Domain *dom, int ndom, const int *order, const int *rank, const double *W,
                          const double *Y, const double *T, const long long *dcp_ptr,
                          const long long *dcp_toff, const double *dcp_coef, double *GK,
                          long long ld, double *Gd, hipStream_t s);
// assemble G^F (nosv x nosv) from per-domain OSV-basis blocks (fixed order)
hipError_t launch_assemble_gf(const Domain *dom, const long long *blk_ptr,
                              const int *blk_dom, const int *blk_part, const int2 *blocks,
                              int nblocks, const int *off, const int *r, const double *Gd,
                              double *GF, long long ld, hipStream_t s);
// dE/deps_a = sum_y Qt[y][a] Zt[y][a]
// part: scratch of ceil(nosv / COLDOT_ROWS) * nvir doubles
constexpr int COLDOT_ROWS = 64;
hipError_t launch_coldot(const double *Qt, const double *Zt, int nosv, int nvir, double *part,
                         double *out, hipStream_t s);
// dE/dF: out[u][v] = sum over clusters of c_X * Pl (CSR per entry, fixed order)
hipError_t launch_pocc(const long long *ptr, const long long *idx, const double *coef,
                       const double *Pl, int nocc, double *out, hipStream_t s);
}  // namespace osv
namespace osv {
// process-wide cache of device allocations (one free list per device); see devpool.hip
hipError_t pool_alloc(void **p, size_t bytes);  // on the current device
void pool_free(void *p);                         // back to its device's cache
void pool_release(int device);                   // hipFree the cached blocks (-1: every device)
size_t pool_cached_bytes(int device);
// OSV generation (eq:svd): T_kk = K_kk / (eps_a + eps_b - 2 f_kk) in place in every
// LMO's nvir x nvir slot; Householder tridiagonalisation and bisection of the
// wanted eigenvalues (count rk[k], values om[k r_max ..]); eigenvectors into rows
// off[k] .. of Qt (ld n) and omega (scratch Z: nocc n r_max doubles)
constexpr int OSV_GEN_MAX_NVIR = 1024;
hipError_t launch_osv_denom(double *T, int nvir, const double *eps, const double *F, int nocc,
                            hipStream_t s);
hipError_t launch_osv_tridiag(double *T, int nocc, int n, double l_osv, int r_max, double *d,
                              double *e, double *tau, int *rk, double *om, hipStream_t s);
hipError_t launch_osv_vectors(const double *T, int nocc, int n, int r_max, const double *d,
                              const double *e, const double *tau, const int *rk, const double *om,
                              const int *off, double *Z, double *Qt, double *omega, hipStream_t s);
// one-step high-order correction: collective amplitudes per domain (slots of
// 2 np^2 at coff[d], both orientations), then per domain the residual at them,
// one Jacobi step and out[3 d ..] = (dE_d, E_d, ||R~_d||_F^2)
hipError_t launch_collective(const Domain *dom, int ndom, const int *order, const long long *ptr, const long long *toff,
                             const double *coef, const double *T, const long long *coff, double *Tc,
                             hipStream_t s);
// (persistent: nwg workgroups take the domains in queue order; scr holds
// collective_step_scratch(nwg) doubles, counter one int)
long long collective_step_scratch(int nwg);
hipError_t launch_collective_step(const Domain *dom, int ndom, const int *rank, const long long *tptr,
                                  const CTerm *terms, const double *Tc, const long long *coff,
                                  const double *M, const double *Kep, const double *F, int nocc,
                                  const int *queue, int *counter, double *scr, int nwg, double *out,
                                  hipStream_t s);
// K~ of one pair domain from Gp = V^T B_p and Gq = V^T B_q (dt x naux), into K~^T of
// its zero-padded slot (leading dimension np)
hipError_t launch_exact_ktilde(const double *Gp, const double *Gq, int dt, int naux, double *Kt, int np,
                               hipStream_t s);
// OSV response N_ij: per-workgroup scratch (doubles) for accumulators of at most
// lb_max columns, and the persistent launch over the targets in a.tg order
long long nij_scratch_doubles(int lb_max);
hipError_t launch_nij(const NijArgs &a, int nwg, hipStream_t s);
// weak pairs: N^up_ij = T_(i,j) K_(j,i) (r_i x r_i row-major at noff[w])
hipError_t launch_weak_nup(const int2 *lmo, int nweak, const int *off, const int *r, const long long *toff,
                           const double *T, const double *K, long long ld, const long long *noff, double *N,
                           hipStream_t s);
hipError_t launch_block_sumsq(const double *S, long long ld, const int *off, const int *r,
                              int nocc, double *out, hipStream_t s);
}
