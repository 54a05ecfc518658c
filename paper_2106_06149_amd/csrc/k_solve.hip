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
// One workgroup (8 wave64, two per SIMD) owns one cluster at a time: it pops
// clusters from a cost-sorted queue, zeroes the cluster's amplitudes, and iterates
//   R~ from the current T~ for every pair; stop if max ||R~||_F < tau_R;
//   otherwise T~ <- T~ - R~ / (e~_a + e~_b - f_pp - f_qq)
// to convergence inside the kernel.  At the final amplitudes the kernel records
//   E^X = sum_pairs w <Tbar~, K~ + R~>   (eq:ec; w = 1 for p = q, 2 for p < q)
// split into <Tbar~, 2 K~ + Delta T~> and the terms' <Tbar~, M op(T~_src) M^T>,
// which are also the inner products that make up dE/df_ab.  They come from the
// stopping sweep itself when its convergence was predicted from the two previous
// norms (geometric rate), else from one more pass over the terms (P pass).
//
// A term Y = M op(T) M^T runs on FP64 MFMA 16x16x4 tiles as X' = coef op(T)^T M^T
// (pass 1), then Y^T = M X' (pass 2).  The f64 MFMA accumulator layout (lane l,
// register v -> row 4v + (l >> 4), column l & 15) equals the B-operand layout of
// the k-rows 4v..4v+3, so a tile X'(kb, i) feeds the second product straight from
// its accumulators, and R~ of the target stays in MFMA accumulators across its
// terms.  The unit of work is a pair (16-wide target block i, 16-row source block
// kb): the tile X'(kb, i) in pass 1 and its product M(kb rows, :)^T X'(kb, i) into
// the column block R~^T(:, i) in pass 2; every unit costs the same.  Each SIMD
// has two slots, one per wave, each a block i and the source blocks kb = rs
// (mod md) (a fixed table per number of target blocks, balanced over the four
// SIMDs); a block split over several waves leaves partial sums of R~^T(:, i) that
// are added through LDS, in a fixed order, by the wave that owns the block's
// epilogue.  Sweeps that store per-term products (the energy passes) keep one wave
// per block (blocks w, w + 4).
//
// Operands are zero-padded row-major slots (leading dimension np = n rounded up
// to 16): op(T~) is a T~ or T~^T slot and M(tgt, src)^T = M(src, tgt) is stored,
// so every chunk of 16 k-rows is 16 contiguous rows of two matrices.  After a
// target's terms its epilogue chunks bring 16 rows of K~^T and of T~^T plus e~, so
// the residual R~ = terms + K~ + Delta T~, its norm and the Jacobi step
// -R~ / Delta are formed from LDS and registers only.  Sweeps alternate between
// two amplitude buffers: a sweep reads T~ and T~^T from one and writes the
// stepped amplitudes, in both orientations, to the other, so no step goes
// through scratch; after the last sweep the final amplitudes are moved to T if
// they are in the second buffer.  The epilogue's owner of a 16 x 16 block writes
// T~^T rows directly and T~ rows through a transpose in the part of the stage
// only it reads, so both stores are row-contiguous.  All chunks stream through a
// 4-stage LDS ring by direct global-to-LDS loads (16 bytes per lane, no
// registers), used as two pairs of stages: one wait and one barrier per pair of
// chunks, the next pair loading while this one is consumed, across term and
// target boundaries.  The second wave of each SIMD issues the loads and stalls
// on the address unit while the first one multiplies.  Every reduction has a
// fixed order, so results are bitwise reproducible.
#include "osv_internal.h"

namespace osv {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int SNT = 512;        // threads per workgroup (8 wave64, two per SIMD)
constexpr int NWAVE = SNT / 64; // waves
constexpr int NW = 4;           // SIMDs: wave w runs on SIMD w % NW; waves NW.. load the ring
constexpr int NS = NWAVE / NW;  // waves (work slots) per SIMD
constexpr int MT = 7;           // 16-tiles per dimension covering DMAX = 100
constexpr int RS = 130;         // LDS row stride (doubles) of a staged row
constexpr int NSTG = 4;         // ring stages: loads run three chunks ahead
constexpr int STG = 33 * RS;    // doubles per stage: rows 0..15, 16..31, and row 32
constexpr int PLMAX = 64;       // clusters with nlmo^2 <= PLMAX keep dE/df sums in LDS
constexpr int MAXT = SOLVE_MAXT;        // clusters with <= MAXT pairs and <= MAXTERM terms
constexpr int MAXTERM = SOLVE_MAXTERM;  //   keep their pair and term descriptors in LDS
constexpr int NTG = 6;          // P pass: terms per reduction group
constexpr int FMAXTERM = 64;    // clusters with at most this many terms may take the
                                // energy and dE/df products in their last sweep

// What the sweep needs about one target pair of the current cluster.
struct TgtDesc {
  long long toff;    // amplitude slots (T~ then T~^T)
  long long kslot;   // K~^T / e~ slot
  double fd;         // f_pp + f_qq
  int np, nt, term0, nterm, w, la, lb, dom;
};

// Descriptor source: LDS tables filled at the start of each cluster (DLDS), or
// the global arrays for clusters too large for the tables.
template <bool DLDS>
struct Desc {
  const SolveArgs *a;
  const Cluster *cl;
  const TgtDesc *tg;
  const TermFlat *tm;
  __device__ __forceinline__ TgtDesc target(int c) const {
    if (DLDS) return tg[c];
    return make_target(*a, *cl, c);
  }
  __device__ __forceinline__ TermFlat term(int t) const {
    if (DLDS) return tm[t - cl->term0];
    return a->tflat[t];
  }
  static __device__ __forceinline__ TgtDesc make_target(const SolveArgs &a, const Cluster &cl, int c) {
    const CPair P = a.cp[cl.cp0 + c];
    const Domain D = a.dom[P.dom];
    TgtDesc g;
    g.toff = P.toff;
    g.kslot = D.voff;
    g.fd = a.F_occ[D.p * a.nocc + D.p] + a.F_occ[D.q * a.nocc + D.q];
    g.np = D.np;
    g.nt = a.dom_rank[P.dom];
    g.term0 = P.term0;
    g.nterm = P.nterm;
    g.w = P.w;
    g.la = P.la;
    g.lb = P.lb;
    g.dom = P.dom;
    return g;
  }
};

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Slot s of a SIMD: target block col (-1: none), source blocks kb with
// kb & (md - 1) == rs, partial-sum slot ps it writes (-1: it owns the block), and
// for an owner the partial slots rd it adds, in this order (-1: none).
struct SlotMap {
  signed char col, md, rs, ps, rd[3];
};
constexpr int NPART = 5;   // partial-sum tiles exchanged per target block row
// balanced split, indexed [njb - 1][SIMD][slot]
__constant__ SlotMap kSplit[MT][NW][NS] = {
    // njb = 1: the block over all four waves (kb mod 4)
    {{{0, 4, 0, -1, {0, 1, 2}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{0, 4, 1, 0, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{0, 4, 2, 1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{0, 4, 3, 2, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}}},
    // njb = 2: each block over two waves (kb mod 2)
    {{{0, 2, 0, -1, {0, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{0, 2, 1, 0, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{1, 2, 0, -1, {1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{1, 2, 1, 1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}}},
    // njb = 3: blocks 0, 1 over two waves each, block 2 over all four
    {{{0, 2, 0, -1, {0, -1, -1}}, {2, 4, 2, 3, {-1, -1, -1}}},
     {{0, 2, 1, 0, {-1, -1, -1}}, {2, 4, 0, -1, {2, 3, 4}}},
     {{1, 2, 0, -1, {1, -1, -1}}, {2, 4, 3, 4, {-1, -1, -1}}},
     {{1, 2, 1, 1, {-1, -1, -1}}, {2, 4, 1, 2, {-1, -1, -1}}}},
    // njb = 4: one block per wave
    {{{0, 1, 0, -1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{1, 1, 0, -1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{2, 1, 0, -1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}},
     {{3, 1, 0, -1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}}},
    // njb = 5: one block per wave, block 4 over all four
    {{{0, 1, 0, -1, {-1, -1, -1}}, {4, 4, 0, -1, {0, 1, 2}}},
     {{1, 1, 0, -1, {-1, -1, -1}}, {4, 4, 1, 0, {-1, -1, -1}}},
     {{2, 1, 0, -1, {-1, -1, -1}}, {4, 4, 2, 1, {-1, -1, -1}}},
     {{3, 1, 0, -1, {-1, -1, -1}}, {4, 4, 3, 2, {-1, -1, -1}}}},
    // njb = 6: one block per wave, blocks 4 and 5 over two waves each
    {{{0, 1, 0, -1, {-1, -1, -1}}, {4, 2, 0, -1, {0, -1, -1}}},
     {{1, 1, 0, -1, {-1, -1, -1}}, {4, 2, 1, 0, {-1, -1, -1}}},
     {{2, 1, 0, -1, {-1, -1, -1}}, {5, 2, 0, -1, {1, -1, -1}}},
     {{3, 1, 0, -1, {-1, -1, -1}}, {5, 2, 1, 1, {-1, -1, -1}}}},
    // njb = 7: blocks w and w + 4 (no split)
    {{{0, 1, 0, -1, {-1, -1, -1}}, {4, 1, 0, -1, {-1, -1, -1}}},
     {{1, 1, 0, -1, {-1, -1, -1}}, {5, 1, 0, -1, {-1, -1, -1}}},
     {{2, 1, 0, -1, {-1, -1, -1}}, {6, 1, 0, -1, {-1, -1, -1}}},
     {{3, 1, 0, -1, {-1, -1, -1}}, {-1, 1, 0, -1, {-1, -1, -1}}}},
};

// The slot of wave w for a target of njb blocks: entry [njb - 1][w % NW][w / NW] of
// the table, so the two waves of a SIMD hold the two slots of one table row
// (wave-uniform values).
struct Slot {
  int col, msk, rs, ps, rd[3];
  bool xch;   // some block of the target is split: partial sums are exchanged
  __device__ __forceinline__ bool has(int kb) const { return col >= 0 && (kb & msk) == rs; }
};

__device__ __forceinline__ Slot make_slot(int njb, int wave, bool split) {
  Slot S;
  const int v = wave % NW, s = wave / NW;
  S.xch = split && njb != 4 && njb != 7;
  if (split) {
    const SlotMap m = kSplit[njb - 1][v][s];
    S.col = uni(m.col);
    S.msk = uni(m.md - 1);
    S.rs = uni(m.rs);
    S.ps = uni(m.ps);
#pragma unroll
    for (int r = 0; r < 3; r++) S.rd[r] = uni(m.rd[r]);
  } else {
    const int c = v + NW * s;
    S.col = c < njb ? c : -1;
    S.msk = 0;
    S.rs = 0;
    S.ps = -1;
#pragma unroll
    for (int r = 0; r < 3; r++) S.rd[r] = -1;
  }
  return S;
}

// fixed-order block sums of NV values (red: NWAVE * NV doubles)
template <int NV>
__device__ __forceinline__ void block_sums(double *v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; c++) {
    double x = wsum(v[c]);
    if (lane == 0) red[c * NWAVE + wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; c++) {
    double t = 0.0;
    for (int w = 0; w < NWAVE; w++) t += red[c * NWAVE + w];
    v[c] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// dst[0, n) = src[0, n) (or 0 when src is null) by the whole workgroup: 16-byte
// accesses, four loads of a thread in flight before its stores.  n is even and
// both slots 16-byte aligned (slot sizes are multiples of 2 np^2 doubles).
__device__ __forceinline__ void block_copy(double *dst, const double *src, int n) {
  const int n2 = n >> 1;
  double2 *d = reinterpret_cast<double2 *>(dst);
  const double2 *s = reinterpret_cast<const double2 *>(src);
  for (int e0 = threadIdx.x; e0 < n2; e0 += 4 * SNT) {
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (e0 + u * SNT < n2) v[u] = s ? s[e0 + u * SNT] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (e0 + u * SNT < n2) d[e0 + u * SNT] = v[u];
  }
}

// Producer of the chunk stream of one sweep of a cluster.  For every target pair
// (in cluster order): the chunks of its terms (term t: nkb pass-1 chunks holding
// op(T) rows and M(src,tgt) rows 16q.., then ceil(nkb / 2) pass-2 chunks holding
// the M(src,tgt) rows of two 16-row tiles), then, unless this is the P pass, njb epilogue chunks holding K~^T rows,
// T~^T rows and e~.  Every field is wave-uniform.
struct Producer {
  int c, ncp;           // target pair, pairs in the cluster
  int t, tend;          // term, end of the target's terms
  int q, nq;            // chunk within the term (or epilogue), chunks in it
  int nkb, ldT, ldM;    // current term
  long long tsrc, moff;
  int epi;              // 1 while issuing the target's epilogue
  int np;               // target's padded dimension
  long long kslot, ttslot;
  int use_terms, use_epi;
  const double *Tb;     // amplitude buffer this sweep reads
};

// Load the next target with something to issue (or run off the end).
template <bool DLDS>
__device__ __forceinline__ void next_target(const Desc<DLDS> &ds, Producer &p) {
  for (; p.c < p.ncp; p.c++) {
    const TgtDesc g = ds.target(p.c);
    p.np = uni(g.np);
    p.kslot = g.kslot;
    p.ttslot = g.toff + (long long)p.np * p.np;
    p.t = uni(g.term0);
    p.tend = p.use_terms ? p.t + uni(g.nterm) : p.t;
    p.q = 0;
    if (p.t < p.tend) {
      const TermFlat f = ds.term(p.t);
      p.nkb = uni((f.ns + 15) >> 4);
      p.nq = p.nkb + ((p.nkb + 1) >> 1);
      p.ldT = uni(f.ldT);
      p.ldM = uni(f.ldM);
      p.tsrc = f.tsrc;
      p.moff = f.moff;
      p.epi = 0;
      return;
    }
    if (p.use_epi) {
      p.epi = 1;
      p.nq = uni((g.nt + 15) >> 4);
      return;
    }
  }
}

template <bool DLDS>
__device__ __forceinline__ void advance(const Desc<DLDS> &ds, Producer &p) {
  if (++p.q < p.nq) return;
  p.q = 0;
  if (!p.epi) {
    if (++p.t < p.tend) {
      const TermFlat f = ds.term(p.t);
      p.nkb = uni((f.ns + 15) >> 4);
      p.nq = p.nkb + ((p.nkb + 1) >> 1);
      p.ldT = uni(f.ldT);
      p.ldM = uni(f.ldM);
      p.tsrc = f.tsrc;
      p.moff = f.moff;
      return;
    }
    if (p.use_epi) {
      p.epi = 1;
      p.nq = uni((ds.target(p.c).nt + 15) >> 4);
      return;
    }
  }
  p.c++;
  next_target(ds, p);
}

// Issue the producer's chunk into a ring stage and advance (loading waves only:
// wave NW + w loads rows w, w + 4, w + 8, w + 12 of each 16-row group); returns the
// number of load instructions each loading wave issued for it (8 pass 1, 8 or 4
// pass 2, 9 epilogue, 0 past the end).  Every lane takes part: lane l moves doubles 2l, 2l+1 of a row,
// clamped to the row's last 16 bytes, so lanes past the row end only fill LDS
// columns that are never read.  stage_off is the stage's LDS byte offset from the
// ring base (uniform).
template <bool DLDS>
__device__ __forceinline__ int issue(const SolveArgs &a, const Desc<DLDS> &ds, Producer &p,
                                     double *ring, int stage_off) {
  if (p.c >= p.ncp) return 0;
  const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) - NW;
  // LDS byte address of row rr of this stage: uniform, kept in a scalar register
  const int lbase = uni((int)(size_t)(__attribute__((address_space(3))) void *)ring + stage_off +
                        wave * RS * 8);
  int cnt;
  if (!p.epi) {
    const int ldT = p.ldT, ldM = p.ldM;
    if (p.q < p.nkb) {
      // pass 1: rows 16q.. of op(T) into stage rows 0..15, of M into rows 16..31
      const int c = p.q;
      const double *Tg = p.Tb + p.tsrc + (16 * c + wave) * ldT + min(2 * lane, ldT - 2);
      const double *Mg = a.M + p.moff + (16 * c + wave) * ldM + min(2 * lane, ldM - 2);
#pragma unroll
      for (int u = 0; u < 4; u++) {
        __builtin_amdgcn_global_load_lds((const void *)(Tg + u * NW * ldT),
                                         (__attribute__((address_space(3))) void *)(size_t)(lbase + u * NW * RS * 8),
                                         16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(Mg + u * NW * ldM),
                                         (__attribute__((address_space(3))) void *)(size_t)(lbase + (16 + u * NW) * RS * 8),
                                         16, 0, 0);
      }
      cnt = 8;
    } else {
      // pass 2: M rows of tiles 2c and 2c + 1 (if there is one) into stage rows
      // 0..15 and 16..31
      const int c = p.q - p.nkb;
      const bool two = 2 * c + 1 < p.nkb;
      const double *Mg = a.M + p.moff + (32 * c + wave) * ldM + min(2 * lane, ldM - 2);
#pragma unroll
      for (int u = 0; u < 4; u++)
        __builtin_amdgcn_global_load_lds((const void *)(Mg + u * NW * ldM),
                                         (__attribute__((address_space(3))) void *)(size_t)(lbase + u * NW * RS * 8),
                                         16, 0, 0);
      if (two) {
#pragma unroll
        for (int u = 0; u < 4; u++)
          __builtin_amdgcn_global_load_lds((const void *)(Mg + (16 + u * NW) * ldM),
                                           (__attribute__((address_space(3))) void *)(size_t)(lbase + (16 + u * NW) * RS * 8),
                                           16, 0, 0);
      }
      cnt = two ? 8 : 4;
    }
  } else {
    const int np = p.np;
    const int col = min(2 * lane, np - 2);
    const double *Kg = a.Kep + p.kslot + (16 * p.q + wave) * np + col;
    const double *Tg = p.Tb + p.ttslot + (16 * p.q + wave) * np + col;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      __builtin_amdgcn_global_load_lds((const void *)(Kg + u * NW * np),
                                       (__attribute__((address_space(3))) void *)(size_t)(lbase + u * NW * RS * 8),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void *)(Tg + u * NW * np),
                                       (__attribute__((address_space(3))) void *)(size_t)(lbase + (16 + u * NW) * RS * 8),
                                       16, 0, 0);
    }
    // e~: every wave loads the whole row (same bytes), keeping the count uniform
    __builtin_amdgcn_global_load_lds((const void *)(a.Kep + p.kslot + (long long)np * np + col),
                                     (__attribute__((address_space(3))) void *)(size_t)(lbase - wave * RS * 8 + 32 * RS * 8),
                                     16, 0, 0);
    cnt = 9;
  }
  advance(ds, p);
  return cnt;
}

// A loading wave waits until all of its loads (the two chunks of the pair) have
// landed, every wave until its LDS reads are done, then barrier: afterwards both
// chunks are in LDS and every wave has finished the previous pair.
__device__ __forceinline__ void stage_wait() {
  if (uni(threadIdx.x >> 6) < NW) asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__global__ void k_term_flat(const Term *terms, long long nterms, const CPair *cp,
                            const Coupling *cpl, const Domain *dom, const int *rank,
                            const double *F_occ, int nocc, TermFlat *out) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nterms) return;
  const Term tm = terms[t];
  const CPair ps = cp[tm.src];
  const Coupling c = cpl[tm.cpl];
  const Domain Ds = dom[ps.dom];
  const bool tgt_is_B = tm.flags & 1;   // then the source is A and M(src,tgt) = M(A,B)
  const Domain Dt = dom[tgt_is_B ? c.B : c.A];
  TermFlat f;
  f.tsrc = ps.toff + ((tm.flags & 2) ? (long long)Ds.np * Ds.np : 0LL);
  f.moff = tgt_is_B ? c.offAB : c.offBA;
  f.coef = -F_occ[tm.fa * nocc + tm.fb];
  f.ldT = (short)Ds.np;
  f.ldM = (short)Dt.np;
  f.ns = rank[ps.dom];
  out[t] = f;
}

hipError_t launch_term_flat(const Term *terms, long long nterms, const CPair *cp,
                            const Coupling *cpl, const Domain *dom, const int *rank,
                            const double *F_occ, int nocc, TermFlat *out, hipStream_t s) {
  if (nterms <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_term_flat, dim3((unsigned)((nterms + 255) / 256)), dim3(256), 0, s, terms,
                     nterms, cp, cpl, dom, rank, F_occ, nocc, out);
  return hipGetLastError();
}

// The consumer's step to the next chunk.  The four stages are used in pairs: at
// an even step the pair (seq, seq + 1), issued one pair earlier, is waited for
// together, and the loading waves issue chunks seq + 2 and seq + 3 into the two
// stages the previous pair used; an odd step neither waits nor synchronises.  The
// loading waves stall on the address unit while the other wave of their SIMD
// multiplies.  Returns the chunk's stage.
struct Ring {
  double *base;
  int seq;
};

template <bool DLDS>
__device__ __forceinline__ const double *next_chunk(const SolveArgs &a, const Desc<DLDS> &ds,
                                                    Producer &p, Ring &r) {
  if ((r.seq & 1) == 0) {
    // chunks seq and seq + 1 (issued two steps ago) are waited for together; the
    // two stages the previous pair used are then free for chunks seq + 2, seq + 3
    stage_wait();
    if (uni(threadIdx.x >> 6) >= NW) {
      issue(a, ds, p, r.base, ((r.seq + 2) & 3) * STG * 8);
      issue(a, ds, p, r.base, ((r.seq + 3) & 3) * STG * 8);
    }
  }
  const double *st = r.base + (r.seq & 3) * STG;
  r.seq++;
  return st;
}

template <bool DLDS>
__global__ __launch_bounds__(SNT) void k_solve(SolveArgs a) {
  __shared__ __attribute__((aligned(16))) double ring[NSTG * STG];
  __shared__ double red[(NTG + 2) * NWAVE];
  __shared__ double plds[PLMAX];
  __shared__ double nrm[MAXT * NWAVE];
  __shared__ TgtDesc tg_l[MAXT];
  __shared__ TermFlat tm_l[MAXTERM];
  __shared__ double fpart[FMAXTERM];   // predicted last sweep: <Tbar~, Z_u> per term
  __shared__ double fe[MAXT * 2];      //   and <Tbar~, 2K~ + Delta T~>, <Tbar~, T~> per target
  __shared__ double part[2 * NPART * 256];   // partial sums of split target blocks, one
                                             // buffer per parity of the tile row
  __shared__ int s_cur;
  const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
  const int l15 = lane & 15, lhi = lane >> 4;
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
    const bool small = nl * nl <= PLMAX;
    const bool lds_norms = cl.ncp <= MAXT;
    double *Pl = small ? plds : a.Pl + cl.poff;
    const Desc<DLDS> ds{&a, &cl, tg_l, tm_l};
    if (DLDS) {
      // the previous cluster's readers of the tables finished at its last barrier
      for (int c = tid; c < cl.ncp; c += SNT) tg_l[c] = Desc<DLDS>::make_target(a, cl, c);
      for (int t = tid; t < cl.term1 - cl.term0; t += SNT) tm_l[t] = a.tflat[cl.term0 + t];
    }
    // Every sweep's epilogue writes the whole m x m corner (m = kept rank rounded
    // up to 16) of the stepped slots, zeros included; the band of rows and columns
    // m .. np-1 is never written by a sweep, so it is cleared here in both buffers.
    // Sweep 0 takes the current amplitudes as zero without reading them.
    for (int c = 0; c < cl.ncp; c++) {
      const CPair P = a.cp[cl.cp0 + c];
      const int np = a.dom[P.dom].np, m = ((a.dom_rank[P.dom] + 15) >> 4) * 16;
      if (m < np) {
        double *T = a.T + P.toff, *T2 = a.T2 + P.toff;
        for (int e = tid; e < 2 * np * np; e += SNT) {
          const int r = (e / np) % np, col = e % np;
          if (r >= m || col >= m) {
            T[e] = 0.0;
            T2[e] = 0.0;
          }
        }
      }
    }
    // Warm start: pairs with init >= 0 take the final amplitudes of the same pair
    // from a cluster of an earlier launch, the others start from zero; the
    // sweeps then take the terms from sweep 0 on.
    bool warm = false;
    for (int c = 0; c < cl.ncp; c++) warm = warm || a.cp[cl.cp0 + c].init >= 0;
    if (warm) {
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const int np = a.dom[P.dom].np;
        double *T = a.T + P.toff;
        if (P.init >= 0) {
          block_copy(T, a.T + P.init, 2 * np * np);
        } else {
          block_copy(T, nullptr, 2 * np * np);
        }
      }
    }
    int sweep = 0, cur = 0;   // cur: the buffer holding the current amplitudes
    double maxn = 0.0, E = 0.0;
    bool pmode = false;  // after convergence: the pass for energies and dE/df
    // A sweep predicted to be the last one (fmode) also stores, after each term,
    // the target's residual terms so far Z_u = sum_{v <= u} coef_v Y_v, and after
    // the target's epilogue takes <Tbar~, Z_u>, <Tbar~, 2K~ + Delta T~> and
    // <Tbar~, T~>; if it converges, the energy and the dE/df products follow from
    // these and the P pass is skipped.  A term's own product is the difference
    // of two consecutive partial sums divided by its coefficient, so a cluster
    // qualifies only if every term's |coef| is at least 2^-10 of the largest one
    // of its target (no cancellation worse than 2^10 ulp), and if its terms and
    // pairs fit the LDS tables.
    bool fm_ok = false;
    if (DLDS) {
      int ok = (cl.term1 - cl.term0 <= FMAXTERM && cl.ncp <= MAXT) ? 1 : 0;
      __syncthreads();   // tables written
      if (ok && tid < cl.ncp) {
        const TgtDesc P = tg_l[tid];
        double cmax = 0.0;
        for (int u = 0; u < P.nterm; u++) cmax = fmax(cmax, fabs(tm_l[P.term0 - cl.term0 + u].coef));
        for (int u = 0; u < P.nterm; u++) {
          const double cu = tm_l[P.term0 - cl.term0 + u].coef;
          if (!(cu != 0.0 && fabs(cu) >= 0x1p-10 * cmax)) ok = 0;
        }
      }
      fm_ok = __syncthreads_and(ok) != 0;
    }
    double n1 = 0.0, n2 = 0.0;   // norms of the previous two sweeps
    for (;;) {
      __syncthreads();   // amplitudes written, ring and scratch free
      Producer pr;
      pr.c = 0;
      pr.ncp = cl.ncp;
      pr.use_terms = (sweep > 0 || pmode || warm) ? 1 : 0;
      pr.use_epi = pmode ? 0 : 1;
      double *const Tcur = cur ? a.T2 : a.T, *const Tnext = cur ? a.T : a.T2;
      pr.Tb = Tcur;
      // geometric prediction of this sweep's norm: n1^2 / n2 below tau_R (a wrong
      // guess costs the products' stores and sums, a missed one the whole P pass)
      const bool fmode = fm_ok && !pmode && sweep >= 2 && n1 * n1 < a.tau_R * n2;
      next_target(ds, pr);
      Ring rg{ring, 0};
      if (wave >= NW) {
        issue(a, ds, pr, ring, 0);
        issue(a, ds, pr, ring, STG * 8);
      }
      double maxn_s = 0.0;   // norms when they do not fit in LDS
      for (int c = 0; c < cl.ncp; c++) {
        const TgtDesc P = ds.target(c);
        const int np = uni(P.np), nt = uni(P.nt);
        const double fd = P.fd;
        const int njb = (nt + 15) >> 4;
        const int nterm = pr.use_terms ? uni(P.nterm) : 0;
        const Slot sl = make_slot(njb, wave, a.split && !pmode && !fmode);
        // coupling-term accumulators of R~^T(j, i) for (a partial sum of) target
        // block ib = sl.col: tile jb covers rows j = 16 jb + lhi + 4v, lane column
        // i = 16 ib + l15
        d4 Racc[MT];
#pragma unroll
        for (int jb = 0; jb < MT; jb++) Racc[jb] = (d4){0, 0, 0, 0};
        for (int u = 0; u < nterm; u++) {
          const TermFlat f = ds.term(P.term0 + u);
          // in the P pass each term is accumulated alone with unit weight
          const double coef = pmode ? 1.0 : f.coef;
          const int nkb = uni((f.ns + 15) >> 4);
          if (pmode) {
#pragma unroll
            for (int jb = 0; jb < MT; jb++) Racc[jb] = (d4){0, 0, 0, 0};
          }
          // pass 1: X'(kb, ib) = coef op(T)^T M^T over chunks of 16 source rows, for
          // the source blocks kb of the slot
          d4 Xp[MT];
#pragma unroll
          for (int kb = 0; kb < MT; kb++) Xp[kb] = (d4){0, 0, 0, 0};
          for (int cc = 0; cc < nkb; cc++) {
            const double *ts = next_chunk(a, ds, pr, rg), *mc = ts + 16 * RS;
            if (sl.col < 0) continue;
            double bv[4];
#pragma unroll
            for (int kk = 0; kk < 4; kk++) bv[kk] = coef * mc[(4 * kk + lhi) * RS + sl.col * 16 + l15];
#pragma unroll
            for (int kb = 0; kb < MT; kb++) {
              if (kb < nkb && sl.has(kb)) {
                double av[4];
#pragma unroll
                for (int kk = 0; kk < 4; kk++) av[kk] = ts[(4 * kk + lhi) * RS + kb * 16 + l15];
#pragma unroll
                for (int kk = 0; kk < 4; kk++) Xp[kb] = mfma(av[kk], bv[kk], Xp[kb]);
              }
            }
          }
          // pass 2: R~^T(:, ib) += M X'(:, ib), X' tile kc; a chunk holds the M rows
          // of two tiles
          const double *mst = nullptr;
#pragma unroll
          for (int kc = 0; kc < MT; kc++) {
            if (kc < nkb) {
              if ((kc & 1) == 0) mst = next_chunk(a, ds, pr, rg);
              if (!sl.has(kc)) continue;
              const double *mc = mst + (kc & 1) * 16 * RS;
#pragma unroll
              for (int jb = 0; jb < MT; jb++) {
                if (jb < njb) {
                  double av[4];
#pragma unroll
                  for (int kk = 0; kk < 4; kk++) av[kk] = mc[(4 * kk + lhi) * RS + jb * 16 + l15];
#pragma unroll
                  for (int kk = 0; kk < 4; kk++) Racc[jb] = mfma(av[kk], Xp[kc][kk], Racc[jb]);
                }
              }
            }
          }
          if (pmode || fmode) {
            // Y^T of this term (P pass), or R~^T of the terms so far (predicted last
            // sweep), to scratch slot u, read back after the target's epilogue
            double *Y = Rs + (long long)u * np * np;
            const int ib = sl.col, i = ib * 16 + l15;
            if (ib >= 0) {
#pragma unroll
              for (int jb = 0; jb < MT; jb++)
                if (jb < njb)
#pragma unroll
                  for (int v = 0; v < 4; v++) Y[(jb * 16 + lhi + 4 * v) * np + i] = Racc[jb][v];
            }
          }
        }
        if (!pmode) {
          // epilogue: R~ = terms + K~ + Delta T~ tile row by tile row from the ring;
          // norm, and the stepped amplitudes T~ - R~ / Delta into the other buffer
          // (both orientations); a converged sweep's step is never read
          double *Tn = Tnext + P.toff, *TnT = Tn + (long long)np * np;
          double ss = 0.0;
#pragma unroll
          for (int jb = 0; jb < MT; jb++) {
            if (jb < njb) {
              const double *st = next_chunk(a, ds, pr, rg);
              const double *ev = st + 32 * RS;
              if (sl.xch) {
                // partial sums of split blocks: written to LDS, added by the owner in
                // the order of its list
                // (two buffers: the write of row jb + 2 comes after row jb + 1's barrier,
                // which every owner passes only when it has read row jb)
                double *pb = part + (jb & 1) * NPART * 256;
                if (sl.ps >= 0)
#pragma unroll
                  for (int v = 0; v < 4; v++) pb[sl.ps * 256 + v * 64 + lane] = Racc[jb][v];
                asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                if (sl.col >= 0 && sl.ps < 0)
#pragma unroll
                  for (int r = 0; r < 3; r++)
                    if (sl.rd[r] >= 0)
#pragma unroll
                      for (int v = 0; v < 4; v++) Racc[jb][v] += pb[sl.rd[r] * 256 + v * 64 + lane];
              }
              const int ib = sl.col, i = ib * 16 + l15;
              if (ib >= 0 && sl.ps < 0) {
                const double ei = ev[i] - fd;
                // the 16 x 16 block (rows jb, columns ib) of the stage's K~^T rows is
                // read by this wave only: the stepped tile goes back there, so that
                // its transpose can be stored row-contiguous
                double *blk = const_cast<double *>(st) + ib * 16;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                  const int jl = lhi + 4 * v, j = jb * 16 + jl;
                  const double delta = ei + ev[j];
                  // T~(i, j) from the T~^T row j (zero in a cold sweep 0)
                  const double tij = (sweep > 0 || warm) ? st[(16 + jl) * RS + i] : 0.0;
                  const double r = Racc[jb][v] + blk[jl * RS + l15] + delta * tij;
                  const bool in = (i < nt) && (j < nt);
                  const double tn = in ? tij - r / delta : 0.0;
                  ss += in ? r * r : 0.0;
                  TnT[j * np + i] = tn;
                  blk[jl * RS + l15] = tn;
                }
                // T~ rows ib: lane (il, jl) = (4v + lhi, l15) stores T~(16 ib + il, 16 jb + jl)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                  const int il = 4 * v + lhi;
                  Tn[(ib * 16 + il) * np + jb * 16 + l15] = blk[l15 * RS + il];
                }
              }
            }
          }
          ss = wsum(ss);
          if (lds_norms) {
            if (lane == 0) nrm[c * NWAVE + wave] = ss;
          } else {
            double v1[1] = {lane == 0 ? ss : 0.0};   // ss is already the wave's sum
            block_sums<1>(v1, red);
            const double nr = sqrt(v1[0]);
            maxn_s = (nr > maxn_s || nr != nr) ? nr : maxn_s;
          }
        }
        if (pmode || fmode) {
          // P pass: <Tbar~, 2 K~ + Delta T~>, <Tbar~, T~> and <Tbar~, Y_u> per term
          // (predicted last sweep: <Tbar~, Z_u> of the partial sums Z_u, kept in LDS)
          __syncthreads();
          const double *Tt = Tcur + P.toff, *TT = Tt + (long long)np * np;
          const double *Kg = a.Kep + P.kslot, *ev = Kg + (long long)np * np;
          for (int g0 = 0; g0 == 0 || g0 < P.nterm; g0 += NTG) {
            double acc[NTG + 2];
#pragma unroll
            for (int k = 0; k < NTG + 2; k++) acc[k] = 0.0;
            for (int e = tid; e < nt * nt; e += SNT) {
              const int j = e / nt, i = e - j * nt;
              const double tij = TT[j * np + i], tji = Tt[j * np + i];
              const double tb = 2.0 * tij - tji;
              if (g0 == 0) {
                acc[0] += tb * (2.0 * Kg[j * np + i] + (ev[i] + ev[j] - fd) * tij);
                acc[1] += tb * tij;
              }
#pragma unroll
              for (int k = 0; k < NTG; k++)
                if (g0 + k < P.nterm) acc[2 + k] += tb * Rs[(long long)(g0 + k) * np * np + j * np + i];
            }
            block_sums<NTG + 2>(acc, red);
            if (fmode) {
              if (tid == 0) {
                if (g0 == 0) {
                  fe[c * 2] = acc[0];
                  fe[c * 2 + 1] = acc[1];
                }
                for (int k = 0; k < NTG && g0 + k < P.nterm; k++)
                  fpart[P.term0 - cl.term0 + g0 + k] = acc[2 + k];
              }
              continue;
            }
            if (g0 == 0) {
              E += P.w * acc[0];
              if (tid == 0) {
                Pl[P.la * nl + P.la] -= 2.0 * acc[1];
                if (P.la != P.lb) Pl[P.lb * nl + P.lb] -= 2.0 * acc[1];
              }
            }
            for (int k = 0; k < NTG && g0 + k < P.nterm; k++) {
              const TermFlat f = ds.term(P.term0 + g0 + k);
              E += P.w * f.coef * acc[2 + k];
              if (tid == 0) {
                const Term tm = a.terms[P.term0 + g0 + k];
                Pl[tm.la * nl + tm.lb] -= acc[2 + k];
                if (P.la != P.lb) Pl[tm.lb * nl + tm.la] -= acc[2 + k];
              }
            }
          }
        }
      }
      if (pmode) break;
      __syncthreads();   // steps in scratch, norms in LDS
      maxn = maxn_s;
      if (lds_norms) {
        for (int c = 0; c < cl.ncp; c++) {
          double t = 0.0;
          for (int w = 0; w < NWAVE; w++) t += nrm[c * NWAVE + w];
          const double nr = sqrt(t);
          maxn = (nr > maxn || nr != nr) ? nr : maxn;
        }
      }
      if (fmode && maxn < a.tau_R) {
        // the predicted last sweep converged: energy and dE/df from its partial
        // sums, in the fixed order of the P pass (targets, then their terms)
        if (tid == 0)
          for (int e = 0; e < nl * nl; e++) Pl[e] = 0.0;
        E = 0.0;
        for (int c = 0; c < cl.ncp; c++) {
          const TgtDesc P = tg_l[c];
          const double ek = fe[c * 2], et = fe[c * 2 + 1];
          E += P.w * ek;
          if (tid == 0) {
            Pl[P.la * nl + P.la] -= 2.0 * et;
            if (P.la != P.lb) Pl[P.lb * nl + P.lb] -= 2.0 * et;
          }
          double prev = 0.0;
          for (int u = 0; u < P.nterm; u++) {
            const int t = P.term0 - cl.term0 + u;
            const double pu = fpart[t];
            const double d = pu - prev;   // coef_u <Tbar~, Y_u>
            prev = pu;
            E += P.w * d;
            if (tid == 0) {
              const double y = d / tm_l[t].coef;
              const Term tm = a.terms[P.term0 + u];
              Pl[tm.la * nl + tm.lb] -= y;
              if (P.la != P.lb) Pl[tm.lb * nl + tm.la] -= y;
            }
          }
        }
        break;
      }
      // a norm that is NaN or infinite ends the sweeps too (the host reports it)
      if (maxn < a.tau_R || !(maxn <= 1.7976931348623157e308) || sweep >= a.max_sweeps) {
        if (sweep == 0 && !warm) {
          // stopped before any step: the final amplitudes are zero
          for (int c = 0; c < cl.ncp; c++) {
            const TgtDesc P = ds.target(c);
            double *T = a.T + P.toff;
            block_copy(T, nullptr, 2 * P.np * P.np);
          }
          __syncthreads();
        }
        pmode = true;  // amplitudes final: energies and inner products at this T
        if (tid == 0)
          for (int e = 0; e < nl * nl; e++) Pl[e] = 0.0;
        E = 0.0;
        continue;
      }
      cur ^= 1;   // the stepped amplitudes become current
      n2 = n1;
      n1 = maxn;
      sweep++;
    }
    if (cur) {
      // the final amplitudes are in the second buffer: move them to T
      __syncthreads();
      for (int c = 0; c < cl.ncp; c++) {
        const CPair P = a.cp[cl.cp0 + c];
        const int np = a.dom[P.dom].np;
        block_copy(a.T + P.toff, a.T2 + P.toff, 2 * np * np);
      }
    }
    if (small) {
      __syncthreads();
      for (int e = tid; e < nl * nl; e += SNT) a.Pl[cl.poff + e] = plds[e];
    }
    if (tid == 0) {
      a.Ecl[X] = E;
      a.sweeps[X] = sweep;
      a.maxres[X] = maxn;
    }
    __syncthreads();
  }
}

// Clusters whose descriptors fit the LDS tables run in the DLDS instantiation;
// the queue holds the others first (cost order puts large clusters there), so
// a.queue[0 .. n_big) goes to the global-descriptor instantiation with
// counter[0] and the rest to the LDS one in two launches, [n_big, n_first) with
// counter[1] and [n_first, n) with counter[2]: clusters of the second launch may
// start from amplitudes the first one wrote.
hipError_t launch_solve(const SolveArgs &a, int n_big, int n_first, int nwg, hipStream_t s) {
  if (a.n_clusters <= 0) return hipSuccess;
  if (n_big > 0) {
    SolveArgs b = a;
    b.n_clusters = n_big;
    hipLaunchKernelGGL(k_solve<false>, dim3(nwg < n_big ? nwg : n_big), dim3(SNT), 0, s, b);
  }
  const int bounds[3] = {n_big, n_first, a.n_clusters};
  for (int g = 0; g < 2; g++) {
    if (bounds[g + 1] <= bounds[g]) continue;
    SolveArgs b = a;
    b.queue = a.queue + bounds[g];
    b.n_clusters = bounds[g + 1] - bounds[g];
    b.counter = a.counter + 1 + g;
    hipLaunchKernelGGL(k_solve<true>, dim3(nwg < b.n_clusters ? nwg : b.n_clusters), dim3(SNT), 0, s, b);
  }
  return hipGetLastError();
}

}  // namespace osv
