/*
 * osv.h -- C ABI of libosvmbe: the per-cluster hot path of MBE(3)-OSV-MP2 on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Liang & Yang, "Third-order many-body expansion of OSV-MP2
 * wavefunction for low-order scaling analytical gradient computation"
 * (arXiv 2106.06149).  The library computes, for every selected 1-, 2- and
 * 3-LMO cluster, the OSV pair amplitudes that solve the residual equations
 * (eq:rij), the Hylleraas cluster energies (eq:ec), their many-body
 * inclusion-exclusion (eq:mbe1; equivalent to the cluster amplitude
 * expansions eq:tmbediag/eq:tmbeoff), and the exact first derivatives of the
 * MBE energy with respect to the OSV-projected fitted integrals C_i, the
 * occupied Fock matrix and the virtual orbital energies (the occupied and
 * virtual density contributions of eq:do/eq:dv and the C-space analogue of
 * eq:ec2eY), by Hylleraas stationarity.
 *
 * General conventions
 *   - All functions return OSV_OK (0) or a negative status; nothing throws
 *     across the ABI.  osv_last_error(ctx) returns a message for the last
 *     failed call on that context (or on no context, for NULL).
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory.
 *   - All work (kernels and the copies of tables built on the host) is
 *     enqueued on the caller's HIP stream (NULL = default stream).  Calls that
 *     return host values synchronise the caller's stream before returning.
 *   - Indices are 0-based.  Matrices are dense with the layout stated.
 *   - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef OSV_H
#define OSV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  OSV_OK = 0,
  OSV_E_ARG = -1,            /* bad size, NULL pointer, r_i out of range, unknown enum  */
  OSV_E_HIP = -2,            /* HIP runtime error (message has the HIP error string)     */
  OSV_E_NOMEM = -3,          /* device or host allocation failed                         */
  OSV_E_NOT_CONVERGED = -4,  /* solve hit max_sweeps; info and amplitudes remain valid   */
  OSV_E_NONFINITE = -5,      /* NaN/Inf in an input or in the residual                   */
  OSV_E_STATE = -6,          /* energy/densities requested before a converged solve      */
  OSV_E_DOMAIN = -7          /* a pair domain has rank 0 after the tau_S cut             */
};

/* arithmetic of the fitted-integral contraction K_ij = C_i C_j^T */
enum {
  OSV_FP64 = 0,   /* every step in FP64 (FP64 MFMA)                                      */
  OSV_MIXED = 1   /* K_ij from FP32 C split into exact int8 digits (per-row power-of-two */
                  /* scale) on int8 MFMA with exact int32 accumulation, combined in      */
                  /* FP64; S, F, dE/dC = 2 G^K C and G^F Q^T likewise from six-digit    */
                  /* splits of their operands' rows; FP64 elsewhere.  Needs C_dtype =   */
                  /* FP32; a product whose contraction exceeds 87000 (int32 range) is   */
                  /* computed in FP64.                                                  */
};

/* cluster selection */
enum {
  OSV_SEL_DISTANCE = 0,  /* 2b: |x_i-x_j| <= cut2; 3b: all three distances <= cut3      */
  OSV_SEL_OVERLAP = 1,   /* 2b: s2b_ij > l2b (eq:2bscreen); 3b: mean s2b > l3b (eq:3bscreen) */
  OSV_SEL_FULL = 2       /* one cluster holding every LMO: plain OSV-MP2, no MBE          */
};

/* C dtype */
enum { OSV_DT_F64 = 0, OSV_DT_F32 = 1 };

typedef struct osv_ctx osv_ctx;  /* opaque; owns all internal device memory */

/*
 * The OSV-MP2 problem (statement of eq:rij, eq:ec and eq:osv).
 *   nocc, nvir, naux   numbers of LMOs, canonical virtuals, fitting functions.
 *   r        host  [nocc]   OSVs per LMO, 1 <= r_i; r_i + r_j <= OSV_MAX_DOMAIN for
 *                           every selected pair (r_i <= OSV_MAX_DOMAIN for r_i alone).
 *   Q        device nvir x sum(r), column-major (ld = nvir): block i = columns
 *                           off_i .. off_i + r_i - 1 with off_i = sum_{k<i} r_k,
 *                           orthonormal columns (Q_i^T Q_i = 1, eq:svd).
 *   C        device sum(r) x naux, row-major (ld = naux): rows off_i.. hold
 *                           C_i = Q_i^T B_i, the OSV-projected fitted integrals.
 *   C_dtype  OSV_DT_F64 or OSV_DT_F32.
 *   eps_vir  device [nvir]  canonical virtual orbital energies f_aa.
 *   F_occ    device nocc x nocc row-major, symmetric; diagonal = f_ii.
 *   centroid host  nocc x 3 (bohr); read by OSV_SEL_DISTANCE only, may be NULL otherwise.
 * The library reads Q, C, eps_vir and F_occ in osv_build_pairs and again in
 * osv_solve_clusters and osv_densities: they are borrowed, not copied, and must
 * stay allocated and unchanged until osv_destroy (or the next build).
 */
typedef struct {
  int32_t nocc, nvir, naux;
  const int32_t *r;
  const double *Q;
  const void *C;
  int32_t C_dtype;
  const double *eps_vir;
  const double *F_occ;
  const double *centroid;
} osv_system;

/* Cluster selection (MBE(3) partitioning; screening eq:2bscreen/eq:3bscreen). */
typedef struct {
  int32_t mode;      /* OSV_SEL_*                                                   */
  double cut2, cut3; /* bohr, inclusive, DISTANCE mode                              */
  double l2b, l3b;   /* OVERLAP mode thresholds (paper defaults 1e-2 and 0.2)       */
  double tau_S;      /* pair-domain overlap eigenvalues <= tau_S are dropped (1e-8) */
} osv_select;

typedef struct {
  int64_t n1b, n2b, n3b;     /* selected clusters per order (FULL: n1b = n2b = n3b = 0) */
  int64_t n_clusters;        /* all clusters (FULL: 1)                                  */
  int64_t n_pair_blocks;     /* sum over clusters of its unordered LMO pairs incl. i=i  */
  int64_t n_domains;         /* distinct orbital pairs (i <= j) with a pair domain      */
  int64_t n_couplings;       /* distinct domain pairs coupled by eq:rij                 */
} osv_counts;

typedef struct {
  int32_t sweeps;            /* largest number of Jacobi steps of any cluster           */
  double max_residual;       /* largest final max_pairs ||W^T R W||_F of any cluster    */
  int32_t converged;         /* 1 if every cluster met tau_R                             */
  int64_t n_not_converged;   /* clusters that hit max_sweeps                             */
} osv_solve_info;

#define OSV_MAX_DOMAIN 100   /* largest pair-domain dimension r_i + r_j supported */

/*
 * osv_build_pairs -- Algorithm 1, pair tasks: select clusters, compute the
 * orbital-pair blocks S_(i,j) = Q_i^T Q_j, F_(i,j) = Q_i^T diag(eps) Q_j and
 * K_ij = C_i C_j^T for every orbital pair that shares a cluster, and prepare
 * each pair domain [Q_i Q_j] (eq:aijkl): canonical orthogonalisation (tau_S),
 * pseudo-canonical basis, K in that basis, and the domain-to-domain couplings
 * that eq:rij needs.
 *   sys, sel   problem and selection (see above); precision = OSV_FP64 / OSV_MIXED.
 *   stream     HIP stream for all kernels and copies.
 *   out        host: receives a new context (NULL on failure).  Free with osv_destroy.
 * Errors: OSV_E_ARG, OSV_E_NONFINITE (NaN/Inf in Q, C, eps_vir or F_occ),
 * OSV_E_DOMAIN, OSV_E_NOMEM, OSV_E_HIP.  Synchronises the stream.
 */
int osv_build_pairs(const osv_system *sys, const osv_select *sel, int32_t precision,
                    hipStream_t stream, osv_ctx **out);

/*
 * osv_build_pairs_exact -- osv_build_pairs with the pair-domain integrals of the
 * strong pairs taken as the cross-projected four blocks of eq:aijkl,
 *   K_(pq,pq) = [Q_p Q_q]^T B_p B_q^T [Q_p Q_q],  (p mu|q nu) over both OSV sets,
 * instead of the OSV-projected C_p given in osv_system.  The diagonal domains and
 * the weak pairs' one-block integrals are the same in both: C_p = Q_p^T B_p is
 * formed here from B.  sys->C may be NULL; B is device nocc x nvir x naux row-major
 * (B_p = rows p nvir ..), read only in this call.  FP64 only (precision OSV_FP64).
 * The other calls work as after osv_build_pairs, except that osv_densities gives
 * no dE/dC (OSV_E_ARG if asked: E then depends on B, not on C); dE/dF_occ,
 * dE/deps and the virtual density keep their meaning.
 * Errors: as osv_build_pairs, and OSV_E_NONFINITE for NaN/Inf in B.
 */
int osv_build_pairs_exact(const osv_system *sys, const double *B, const osv_select *sel, int32_t precision,
                          hipStream_t stream, osv_ctx **out);

/* osv_query -- counts of the built context (host out).  OSV_E_ARG on NULL. */
int osv_query(const osv_ctx *ctx, osv_counts *out);

/*
 * osv_solve_clusters -- solve eq:rij for every cluster (k restricted to the
 * cluster's LMOs) by Jacobi sweeps preconditioned in each domain's
 * pseudo-canonical basis.  Clusters of one or two LMOs start from T = 0; each
 * pair of a three-LMO cluster starts from the converged amplitudes of the same
 * pair in one of its two-LMO clusters (solved first).  A cluster stops when the
 * largest ||W^T R W||_F over its pairs is below tau_R; its amplitudes are those
 * at which that residual was evaluated, and info->sweeps counts the Jacobi steps
 * taken (the largest over the clusters).  Also evaluates each cluster's
 * Hylleraas energy (eq:ec) and the inner products that dE/dF_occ needs.
 *   tau_R       convergence threshold (e.g. 1e-10); max_sweeps >= 1.
 *   info        host, may be NULL.
 * Errors: OSV_E_ARG, OSV_E_NOT_CONVERGED (info filled, results usable but not
 * converged), OSV_E_NONFINITE (residual not finite), OSV_E_HIP.  Synchronises.
 */
int osv_solve_clusters(osv_ctx *ctx, double tau_R, int32_t max_sweeps, hipStream_t stream,
                       osv_solve_info *info);

/*
 * osv_energy -- MBE(3) inclusion-exclusion of the cluster energies (eq:mbe1):
 *   E = sum_X c_X E^X with c_X = 1 (3b), 1 - n3(IJ) (2b), 1 - n2(I) + n3(I) (1b),
 *   plus, with OSV_SEL_OVERLAP, the one-block energies of the weak 2b clusters
 *   (see osv_weak_pairs; their amplitudes are formed by osv_solve_clusters).
 *   E         host, required.
 *   E_orders  host [3] or NULL: E_1b, dE_2b (weak pairs included), dE_3b (NaN for
 *             OSV_SEL_FULL).
 *   E_cluster device [n_clusters] or NULL: E^X in canonical cluster order
 *             (all 1b ascending, 2b lexicographic, 3b lexicographic).
 * Errors: OSV_E_STATE before a successful solve, OSV_E_ARG, OSV_E_HIP.  Synchronises.
 */
int osv_energy(osv_ctx *ctx, hipStream_t stream, double *E, double *E_orders, double *E_cluster);

/*
 * osv_weak_pairs -- weak 2b clusters by the one-block scheme (section on the
 * correlation scheme for weak 2b clusters; selection by eq:2bscreen).  With
 * OSV_SEL_OVERLAP, the pairs i < j with 1e-7 <= s2b_ij <= l2b are neither
 * strong clusters nor discarded; each keeps only its dispersion block T_(i,j)
 * (i to OSVs of i, j to OSVs of j) in the pseudo-canonical bases of the diagonal
 * domains, where the projected one-block residual
 *   K~_(i,j) + (e~_i[a] + e~_j[b] - f_ii - f_jj) T = 0,   K~ = W_i^T K_ij W_j,
 * is solved in one step, and the pair adds 4 <T, K~> to the energy (both
 * orderings; the exchange block is not represented).  osv_energy includes the
 * sum in E and osv_densities the weak pairs' densities (after a solve); this
 * call gives the pair energies alone and needs only osv_build_pairs (their K_ij
 * blocks are formed there).  Other selection modes have no weak pairs.
 *   E_weak   host, required: sum of the pair energies in pair order.
 *   n_weak   host or NULL: number of weak pairs.
 *   E_pairs  device [n_weak] or NULL: the pair energies, pairs in (i, j)
 *            lexicographic order.
 *   pairs    host int32 [2 n_weak] or NULL: (i, j) of each pair.
 * Call once with E_pairs and pairs NULL to learn n_weak.
 * Errors: OSV_E_ARG, OSV_E_NOMEM, OSV_E_HIP.  Synchronises the stream.
 */
int osv_weak_pairs(osv_ctx *ctx, hipStream_t stream, double *E_weak, int64_t *n_weak,
                   double *E_pairs, int32_t *pairs);

/*
 * osv_weak_pairs_noalloc -- osv_weak_pairs for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as osv_weak_pairs, but it calls no
 * hipMalloc, hipFree or other allocating routine: the per-pair domain table, the
 * pair energies and their sum live in a static device array of the library
 * (16 MiB + 256 B per device, held until the process ends), so it takes at most
 * OSV_NOALLOC_MAX_WEAK weak pairs (OSV_E_ARG beyond, before any device work).
 * Every call on one device shares that array and finds what the last call left
 * in it: calls that overlap on one device (any contexts, any streams) race, and
 * the caller must order them.  E_weak is summed on the device in a fixed order
 * (256 strided partial sums, then a fixed tree), so it equals osv_weak_pairs'
 * host sum in pair order to rounding; E_pairs are bitwise the same.
 */
#define OSV_NOALLOC_MAX_WEAK 1048576
int osv_weak_pairs_noalloc(osv_ctx *ctx, hipStream_t stream, double *E_weak, int64_t *n_weak,
                           double *E_pairs, int32_t *pairs);

/*
 * osv_densities -- exact derivatives of the MBE energy at fixed Q (Hylleraas
 * stationarity: the amplitudes contribute nothing), the weak pairs' one-block
 * energies included (OSV_SEL_OVERLAP: dE/dK_ij = 8 T, dE/dF_(i,i) = 4 T T^T,
 * dE/dF_(j,j) = 4 T^T T, dE/df_ii = dE/df_jj = -4 <T, T>, T in the OSV bases):
 *   dE_dC     device sum(r) x naux row-major FP64: dE/dC_i = sum_j (G_ij + G_ji^T) C_j
 *             with G_ij = sum_X c_X U_i^T (2 Tbar_ij) U_j   (cf. eq:ec2eY).
 *   dE_dFocc  device nocc x nocc row-major: dE/df_uv, every entry taken as an
 *             independent variable (the result is symmetric; cf. eq:do).
 *   dE_deps   device [nvir]: dE/deps_a = diag of the virtual density (cf. eq:dv).
 *   Dvir_full device nvir x nvir row-major or NULL: sum_uv Q_u G^F_uv Q_v^T.
 * Any of the first three may be NULL to skip it.  Outputs are overwritten.
 * Errors: OSV_E_STATE before a successful solve, OSV_E_ARG, OSV_E_HIP.
 */
int osv_densities(osv_ctx *ctx, hipStream_t stream, double *dE_dC, double *dE_dFocc,
                  double *dE_deps, double *Dvir_full);

/*
 * osv_generate_osvs -- the OSVs of every LMO from the fitted integrals (eq:svd,
 * eq:osv): Q_k holds the orthonormal eigenvectors of the diagonal MP2 amplitudes
 *   [T_kk]_ab = (ka|kb) / (f_aa + f_bb - 2 f_kk),  (ka|kb) = sum_P B_k[a,P] B_k[b,P],
 * whose eigenvalues omega exceed l_osv, largest first, at most r_max of them; each
 * column's entry of largest magnitude is positive.  C_k = Q_k^T B_k are the
 * OSV-projected fitted integrals osv_system takes.  (ka|kb) on FP64 MFMA, then per
 * LMO a Householder reduction, bisection and inverse iteration in FP64.
 *   nocc, nvir, naux  sizes; 1 <= nvir <= 1024.
 *   B        device nocc x nvir x naux row-major (B_k = rows k nvir .. of naux).
 *   eps_vir  device [nvir]; F_occ device nocc x nocc row-major (its diagonal f_kk).
 *   l_osv    eigenvalue cut (the paper's default 1e-4); r_max in [1, min(nvir, OSV_MAX_DOMAIN)].
 *   r        host out [nocc]: OSVs kept per LMO (may be 0).
 *   omega    device out nocc x r_max or NULL: row k holds the r_k kept eigenvalues, zeros after.
 *   Q        device out, nvir x (nocc r_max) column-major capacity (ld nvir): the first
 *            sum(r) columns receive Q in the osv_system layout (block k at off_k).
 *   C        device out or NULL, (nocc r_max) x naux row-major capacity: the first
 *            sum(r) rows receive C in the osv_system layout.
 * Errors: OSV_E_ARG, OSV_E_NONFINITE (NaN/Inf in B, eps_vir, F_occ), OSV_E_NOMEM,
 * OSV_E_HIP.  Synchronises the stream; device work memory comes from the block cache.
 */
int osv_generate_osvs(int32_t nocc, int32_t nvir, int32_t naux, const double *B, const double *eps_vir,
                      const double *F_occ, double l_osv, int32_t r_max, hipStream_t stream, int32_t *r,
                      double *omega, double *Q, double *C);

/*
 * osv_high_order_correction -- the one-step posterior correction of the MBE(3)
 * amplitudes (section on the high-order MBE(n) contribution).  From the converged
 * cluster amplitudes it forms the collective amplitudes of every pair domain,
 *   T_(pq) = sum over the clusters X holding p and q of c_X T^X_pq
 * (eq:tmbediag / eq:tmbeoff), evaluates the residual eq:rij of every pair at them
 * with k over the LMOs that share a cluster with p and q (so that every cluster's
 * couplings enter at once), takes one Jacobi step dT in each pair domain's
 * pseudo-canonical basis, and returns the energy change it makes,
 *   dE = sum_pairs w <K_(pq,pq), 2 dT - dT^T>   (w = 1 for p = q, 2 otherwise).
 *   dE          host, required.
 *   E_coll      host or NULL: sum_pairs w <K_(pq,pq), 2 T_(pq) - T_(pq)^T> (equals the
 *               MBE energy of the strong clusters at convergence).
 *   max_dR      host or NULL: the largest ||W^T dR W||_F over the pairs.
 *   per_domain  host [3 n_domains] or NULL: per pair domain (p <= q, lexicographic)
 *               its dE, E_coll and ||W^T dR W||_F.
 * The weak pairs of OSV_SEL_OVERLAP are not part of it.  Errors: OSV_E_STATE
 * before a converged solve, OSV_E_ARG, OSV_E_NOMEM, OSV_E_HIP.  Synchronises.
 */
int osv_high_order_correction(osv_ctx *ctx, hipStream_t stream, double *dE, double *E_coll,
                              double *max_dR, double *per_domain);

/*
 * osv_response_layout -- the layout of the OSV response intermediates of
 * osv_response (host only; valid once the pairs are built).  One n x n block per
 * ordered pair (i, j) of every pair domain [ij] (n = r_i + r_j, or r_i for i == j):
 * the domains in (p <= q) lexicographic order, for p < q first (p, q) then (q, p).
 *   n_pairs    host out or NULL: number of ordered pairs.
 *   n_doubles  host out or NULL: doubles the output of osv_response needs.
 *   pairs      host out or NULL, 2 int32 per ordered pair (capacity n_pairs): (i, j).
 *   offsets    host out or NULL, per ordered pair (capacity n_pairs): first double of
 *              its block.
 * Errors: OSV_E_ARG.
 */
int osv_response_layout(const osv_ctx *ctx, int64_t *n_pairs, int64_t *n_doubles, int32_t *pairs,
                        int64_t *offsets);

/*
 * osv_response -- the OSV response intermediate N_ij of eq:nij for every ordered
 * pair (i, j) of the strong clusters, combined over the clusters with the MBE
 * coefficients (eq:nmbeii for i == j, eq:nmbeij otherwise, written with the
 * inclusion-exclusion coefficients c_X):
 *   N_ij = sum_X c_X [ Tbar K_(ij,ij) + D_(ij,ij) F_(ij,ij) + D'_(ij,ij) S_(ij,ij)
 *                      - sum_{k in X} ( f_jk D_(ij,ik) S_(ik,ij) + f_ik D_(ij,kj) S_(kj,ij) ) ],
 *   D_(ij,kl) = 1/2 (Tbar_ij S_(ij,kl) T_kl + Tbar_ij^T S_(ij,kl) T_kl^T), D' the same
 *   with F_(ij,kl), at each cluster's converged amplitudes (Tbar = 2T - T^T), in the
 * composite OSV basis [Q_i Q_j] of the ordered pair (row-major blocks, layout of
 * osv_response_layout; a pair held only by clusters with c_X = 0 gets zeros).
 * The weak pairs of OSV_SEL_OVERLAP are not part of it.
 *   N         device out, n_doubles FP64 (overwritten).
 *   ms_flops  host [2] or NULL: device time of the evaluation (ms) and the flops of
 *             its tile products at the kept ranks.
 * Errors: OSV_E_STATE before a converged solve; OSV_E_ARG for a NULL N or for a
 * context of osv_build_pairs_exact; OSV_E_NOMEM, OSV_E_HIP.  Runs on stream and
 * synchronises it; work memory (per-workgroup scratch) is kept by the context.
 */
int osv_response(osv_ctx *ctx, hipStream_t stream, double *N, double *ms_flops);

/*
 * osv_weak_response -- the weak pairs' part of the OSV response in the one-block
 * approximation of eq:nij2b: for each weak pair (i, j) of OSV_SEL_OVERLAP (pair
 * order of osv_weak_pairs) the upper block N^up_ij = T_(i,j) K_(j,i) (r_i x r_i,
 * OSV basis of LMO i, row-major; the lower block is taken as zero), with T_(i,j)
 * the pair's one-block amplitudes of the last solve in the OSV bases.
 *   n_doubles  host or NULL: doubles N_up needs (sum of r_i^2 over the weak pairs;
 *              the blocks follow one another in pair order).
 *   N_up       device out or NULL (NULL: only n_doubles is written).
 * Errors: OSV_E_STATE before a converged solve (when N_up is given), OSV_E_ARG,
 * OSV_E_HIP.  Synchronises the stream.  Other selection modes have no weak pairs
 * (n_doubles 0).
 */
int osv_weak_response(osv_ctx *ctx, hipStream_t stream, int64_t *n_doubles, double *N_up);

/*
 * osv_correction_stats -- device times and algorithmic work of the last
 * osv_high_order_correction call on this context:
 *   out4  host [4]: the collective sums (ms, bytes they must read and write: every
 *         cluster slot of a domain once, the domain's two slots once), then the
 *         residual step (ms, flops: 2 (dt n_s^2 + dt^2 n_s) per term at the kept ranks).
 * Errors: OSV_E_ARG.  Zeros before the first call.
 */
int osv_correction_stats(const osv_ctx *ctx, double *out4);

/*
 * osv_generation_stats -- device times and algorithmic flops of the last
 * osv_generate_osvs call of the calling thread:
 *   out8  host [8]: (ms, flops) of the products (ka|kb) (nvir^2 naux per LMO,
 *         symmetric), of the Householder reduction with the eigenvalue bisection
 *         (4/3 nvir^3 per LMO), of the eigenvectors (inverse iteration and the
 *         reflectors applied to the kept vectors, 4 nvir^2 r_k), and of C = Q^T B
 *         (2 r_k nvir naux).
 * Errors: OSV_E_ARG.  Zeros before the first call.
 */
int osv_generation_stats(double *out8);

/*
 * osv_plan_clusters -- host-only cluster selection for OSV_SEL_DISTANCE and
 * OSV_SEL_FULL (no device work; usable without a GPU).
 *   nocc, centroid (host nocc x 3), sel: as above.
 *   counts     host out (n_couplings included).
 *   lmos       host out or NULL: 3 int32 per cluster (unused slots -1), canonical order;
 *              capacity cap clusters (OSV_E_ARG if too small).  FULL writes nothing here.
 *   coef       host out or NULL: MBE coefficient c_X per cluster (capacity cap).
 */
int osv_plan_clusters(int32_t nocc, const double *centroid, const osv_select *sel,
                      osv_counts *counts, int32_t *lmos, double *coef, int64_t cap);

/* osv_destroy -- free a context; NULL is a no-op.  Waits for the device to finish
 * queued work, then returns the context's device blocks to the library's cache. */
void osv_destroy(osv_ctx *ctx);

/*
 * Device memory cache.  Every context takes its device buffers from a
 * process-wide cache (one per device): blocks freed by osv_destroy are kept and
 * handed to later contexts that ask for the same size class (requests round up
 * to 512 B below 1 MiB, to 2 MiB above; a cached block may be up to 1/8 larger),
 * so a caller that builds one context per geometry step allocates only in its
 * first step.  A failed allocation releases the device's cache and retries.
 * Reused blocks are not cleared; the environment variable OSV_POOL_POISON=1
 * fills every block handed out with 0xFF bytes (a debugging aid).
 *   osv_release_cached_memory(device)  hipFree the cached blocks of device
 *                                      (-1: of every device).  Blocks held by
 *                                      live contexts are not touched.  Returns
 *                                      OSV_OK, or OSV_E_ARG for device < -1.
 *   osv_cached_bytes(device)           bytes held in the cache (-1: all devices).
 */
int osv_release_cached_memory(int32_t device);
int64_t osv_cached_bytes(int32_t device);

/*
 * Launch tuning.  Some kernels exist in several compiled variants that compute the
 * same quantities with different tile or workgroup shapes; which one runs is a
 * process-wide table, read once from $OSV_TUNING_FILE, else from osv_tuning.txt
 * beside the library (written by the package's autotuner; "key value" lines), else
 * left at its defaults.  Keys and allowed values:
 *   gemm_ks          8, 16, 32      k per LDS stage of the FP64 tile GEMM (S/F, K, dE/dC in FP64 mode)
 *   prep_nt_small    128, 256       threads per pair domain of n <= 32 in the preparation
 *   prep_nt_mid      256, 512, 1024 the same for 32 < n <= 64
 *   prep_nt_big      512, 1024      the same for n > 70 (64 < n <= 70: 512, fixed)
 *   cpl_split        0, 64          couplings whose domains both have n <= this run as
 *                                   4-wave workgroups, the others as 8-wave ones
 *   solve_split      0, 1           residual solve: 1 spreads each target's (column
 *                                   block, source block) products evenly over the
 *                                   four waves of a workgroup, 0 gives each wave
 *                                   whole 16-column blocks (energies agree to
 *                                   rounding; each setting is bitwise reproducible)
 * Set the table before building contexts; changing it while another thread builds
 * or solves is not supported.  OSV_E_ARG for an unknown key or value, an unreadable
 * file or a bad line (entries before a bad line stay applied).
 */
int osv_set_tuning(const char *key, int32_t value);
int osv_get_tuning(const char *key, int32_t *value);
int osv_load_tuning(const char *path);

/* message of a status code (static string) */
const char *osv_status_string(int status);

/* last error message recorded on ctx (or the library-wide one for NULL); never NULL */
const char *osv_last_error(const osv_ctx *ctx);

/* stage timings of the last build/solve/energy/densities on ctx, milliseconds,
 * from HIP events on the caller's stream (stage 8 is host wall time); host out [9]:
 *   0 S/F blocks, 1 K blocks, 2 domain prep, 3 couplings, 4 solve, 5 energy,
 *   6 adjoint (per domain), 7 back-transforms, 8 host cluster selection + plan.
 * Values of stages not run are 0. */
int osv_stage_times(const osv_ctx *ctx, double *ms9);

/* algorithmic floating-point operations of the same stages (host out [9]):
 * the flops of the mathematical contractions at the kept (unpadded) sizes,
 * e.g. 2*r_p*r_q*naux per K_pq block and 2*(n_t*n_s^2 + n_t^2*n_s) per residual
 * term per sweep; stage 2 counts the products around the eigensolvers and 9 m^3 per
 * symmetric eigendecomposition of order m; the host stage 8 counts 0. */
int osv_stage_flops(const osv_ctx *ctx, double *flops9);

#ifdef __cplusplus
}
#endif
#endif /* OSV_H */
