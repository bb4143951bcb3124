// Device building blocks shared by the depth-first kernels: row streaming
// through scalar registers, the fused and+popcount folds, the bound test, the
// per-lane best leaf and the depth-4 expansion of one prefix per lane.
#pragma once
#include "pdfs_dev.h"

namespace pdfs {
namespace {

// Read-only view of the round's rows.  The rows do not change while a DFS
// kernel runs, so reading them through the constant address space lets the
// compiler fetch a wave-uniform row with scalar loads (one copy per wave,
// held in SGPRs, used directly as VALU operands).
typedef const __attribute__((address_space(4))) uint32_t cu32;

// A launch's problem and workspace where a kernel reads them again: its own
// arguments (through the kernel-argument segment) or a batch descriptor,
// both unchanged while it runs, so read through the constant address space.
typedef const __attribute__((address_space(4))) Problem cProblem;
typedef const __attribute__((address_space(4))) Work cWork;

// p, opaque to the optimiser: loads through the result are made where they
// are written instead of being hoisted out of loops and held in scalar
// registers (or spilled) across them.
template <class T>
__device__ __forceinline__ T* fresh(T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// *p by 32-bit words (scalar loads; the words of fields left unused are
// never loaded).
template <class T>
__device__ __forceinline__ T load_const(const __attribute__((address_space(4))) T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  union {
    T t;
    uint32_t u[sizeof(T) / 4];
  } r;
  const __attribute__((address_space(4))) uint32_t* s =
      (const __attribute__((address_space(4))) uint32_t*)p;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) r.u[i] = s[i];
  return r.t;
}

// d = (a & b) | c with b a wave-uniform (SGPR) operand.
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
  return d;
}

// acc + popcount(x)
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t d;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(d) : "v"(x), "v"(acc));
  return d;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// OR over k of (y[k] & row[k]) with four independent chains.
template <int W>
__device__ __forceinline__ uint32_t fold_nonempty(const uint32_t (&y)[W], cu32* row) {
  uint32_t r[W];
#pragma unroll
  for (int k = 0; k < W; ++k) r[k] = row[k];
  uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
  for (int k = 0; k < W; k += 4) {
    a0 = and_or(y[k], r[k], a0);
    if (k + 1 < W) a1 = and_or(y[k + 1], r[k + 1], a1);
    if (k + 2 < W) a2 = and_or(y[k + 2], r[k + 2], a2);
    if (k + 3 < W) a3 = and_or(y[k + 3], r[k + 3], a3);
  }
  return a0 | a1 | a2 | a3;
}

// OR over k of (y[k] & r[k]) for a row already in (scalar) registers, as one
// dependent chain (W operations; a wave's dependent VALU operations issue
// back to back).
template <int W>
__device__ __forceinline__ uint32_t fold_chain_r(const uint32_t (&y)[W], const uint32_t (&r)[W]) {
  uint32_t a = y[0] & r[0];
#pragma unroll
  for (int k = 1; k < W; ++k) a = and_or(y[k], r[k], a);
  return a;
}

// sum over k of popcount(y[k] & row[k]), four accumulator chains.
template <int W>
__device__ __forceinline__ int popc_and(const uint32_t (&y)[W], cu32* row) {
  uint32_t r[W];
#pragma unroll
  for (int k = 0; k < W; ++k) r[k] = row[k];
  uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
  for (int k = 0; k < W; k += 4) {
    c0 = bcnt_acc(y[k] & r[k], c0);
    if (k + 1 < W) c1 = bcnt_acc(y[k + 1] & r[k + 1], c1);
    if (k + 2 < W) c2 = bcnt_acc(y[k + 2] & r[k + 2], c2);
    if (k + 3 < W) c3 = bcnt_acc(y[k + 3] & r[k + 3], c3);
  }
  return (int)(c0 + c1 + c2 + c3);
}

__device__ __forceinline__ int popc_and_n(const uint32_t (&z)[kMaxWN32], cu32* row) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) c += __popc(z[k] & row[k]);
  return c;
}

// Normals joined into a prefix: carrying every gene (AND), or under the
// literal reading of T- any of them (OR).
__device__ __forceinline__ uint32_t nrm_join(uint32_t a, uint32_t b, bool literal) {
  return literal ? (a | b) : (a & b);
}

// FP of a leaf from its prefix's normals z and the last gene's normal row.
__device__ __forceinline__ int leaf_fp(const uint32_t (&z)[kMaxWN32], cu32* row, bool literal) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) c += __popc(nrm_join(z[k], row[k], literal));
  return c;
}

// Rows of at least this many 64-bit words keep the normal prefixes in LDS.
#ifndef PDFS_ZLDS_MIN_W64
#define PDFS_ZLDS_MIN_W64 10
#endif
constexpr int kZLdsMinW64 = PDFS_ZLDS_MIN_W64;

// A lane's normal-sample prefix (its genes' normal rows joined, kMaxWN32
// words): in registers, or -- for the widest tumour rows, whose depth-first
// kernels are bound by registers -- in the wave's LDS slice, stored
// [word][lane] so that a word of all 64 lanes is one conflict-free access.
template <bool kLds>
struct NrmPre;

template <>
struct NrmPre<false> {
  uint32_t z[kMaxWN32];
  __device__ uint32_t get(int k, int /*lane*/) const { return z[k]; }
  __device__ void set(int k, int /*lane*/, uint32_t v) { z[k] = v; }
};

template <>
struct NrmPre<true> {
  uint32_t* s;   // [kMaxWN32][kWave] words of the wave's LDS slice
  __device__ uint32_t get(int k, int lane) const { return s[k * kWave + lane]; }
  __device__ void set(int k, int lane, uint32_t v) { s[k * kWave + lane] = v; }
};

// FP of a leaf from its prefix's normals z (lane `lane`) and the last gene's
// normal row.
template <bool kLds>
__device__ __forceinline__ int leaf_fp_z(const NrmPre<kLds>& z, int lane, cu32* row, bool literal) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) c += __popc(nrm_join(z.get(k, lane), row[k], literal));
  return c;
}

// sum over k of popcount(y[k] & r[k]) for a row already in (scalar) registers
template <int W>
__device__ __forceinline__ int popc_and_r(const uint32_t (&y)[W], const uint32_t (&r)[W]) {
  if (W <= 4) {   // one chain: no final add
    uint32_t c0 = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) c0 = bcnt_acc(y[k] & r[k], c0);
    return (int)c0;
  }
  uint32_t c0 = 0, c1 = 0;
#pragma unroll
  for (int k = 0; k < W; k += 2) {
    c0 = bcnt_acc(y[k] & r[k], c0);
    if (k + 1 < W) c1 = bcnt_acc(y[k + 1] & r[k + 1], c1);
  }
  return (int)(c0 + c1);
}

// Rows d .. d+KR-1 (clamped to `last`) into scalar registers.
template <int W, int KR>
__device__ __forceinline__ void load_rows(uint32_t (&r)[KR][W], cu32* base, int d, int last) {
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int dj = d + j < last ? d + j : last;
#pragma unroll
    for (int k = 0; k < W; ++k) r[j][k] = base[(size_t)dj * W + k];
  }
}

// Makes `next` (the next row index) depend on the rows of the current group.
// Scalar loads may complete out of order, so waiting for one waits for every
// load in flight; tying the next group's addresses to the current group's
// data places that wait before the next loads are issued, which then overlap
// the current group's arithmetic.
template <int W, int KR>
__device__ __forceinline__ void after_arrival(int& next, const uint32_t (&r)[KR][W]) {
  asm volatile("; rows arrived %1" : "+s"(next) : "s"(r[KR - 1][W - 1]));
}

// KR consecutive rows starting at p into scalar registers (no clamping).
template <int W, int KR>
__device__ __forceinline__ void load_group(uint32_t (&r)[KR][W], cu32* p) {
#pragma unroll
  for (int j = 0; j < KR; ++j)
#pragma unroll
    for (int k = 0; k < W; ++k) r[j][k] = p[j * W + k];
}

// after_arrival for a row pointer.
template <int W, int KR>
__device__ __forceinline__ void group_arrived(cu32*& next, const uint32_t (&r)[KR][W]) {
  asm volatile("; rows arrived %1" : "+s"(next) : "s"(r[KR - 1][W - 1]));
}

__device__ __forceinline__ unsigned long long load_incumbent(RoundState* st) {
  return __hip_atomic_load(&st->incumbent, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true when a prefix with first indices (a, b) and score bound ub cannot
// produce the round's answer.
__device__ __forceinline__ bool dominated(int ub, int a, int b, unsigned long long inc) {
  if (inc == 0) return false;
  const int s = (int)(inc >> 32) - 1;
  if (ub != s) return ub < s;
  const int g1 = 0xffff - (int)((inc >> 16) & 0xffff);
  const int g2 = 0xffff - (int)(inc & 0xffff);
  return a > g1 || (a == g1 && b > g2);
}

__device__ __forceinline__ unsigned long long leaf_key(int s, int a, int b) {
  return ((unsigned long long)(s + 1) << 32) | ((unsigned long long)(0xffff - a) << 16) |
         (unsigned long long)(0xffff - b);
}

// Orders this wave's LDS writes before its later LDS reads of other lanes'
// entries.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A lane's best leaf: score, TP, FP and the tuple of active indices, packed
// i0 << 48 | i1 << 32 | i2 << 16 | i3 (every index < 65536), so that the
// order (S desc, tuple asc) is two integer comparisons and the update is
// plain selects -- no branches in the candidate loops.
struct Best {
  int s, tp, fp;
  unsigned long long t;
  __device__ void init() { s = -1; tp = fp = 0; t = ~0ull; }
  __device__ int idx(int k) const { return (int)((t >> (48 - 16 * k)) & 0xffffull); }
  __device__ void offer(int s2, int tp2, int fp2, int j0, int j1, int j2, int j3) {
    const unsigned long long t2 = ((unsigned long long)j0 << 48) | ((unsigned long long)j1 << 32) |
                                  ((unsigned long long)j2 << 16) | (unsigned long long)j3;
    const bool take = s2 > s || (s2 == s && t2 < t);
    s = take ? s2 : s;
    tp = take ? tp2 : tp;
    fp = take ? fp2 : fp;
    t = take ? t2 : t;
  }
};

struct Tally {
  unsigned long long ne3, ne4, vis3, vis4, bp2, bp3;
  unsigned long long xv3, xv4, xfp;   // active-candidate visits, FP-counted leaves
  __device__ void init() { ne3 = ne4 = vis3 = vis4 = bp2 = bp3 = xv3 = xv4 = xfp = 0; }
};

// base + the number of lanes below this one whose bit is set in m.
__device__ __forceinline__ int rank_below(unsigned long long m, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
}

// Largest v over the wave.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return uniform(v);
}

// Smallest TP with which a leaf can still replace a best leaf of score s.  A
// leaf scores at most p*TP + q*N_n (no false positives); it replaces the best
// if it scores more, or the same with a smaller tuple.  tie_wins says whether
// the leaves in question can have the smaller tuple.  Always >= 1, so it also
// implies a non-empty leaf.
__device__ __forceinline__ int min_tp_for(const Problem& P, int s, bool tie_wins) {
  const int e = s - P.q * P.n_normal;   // p*TP must reach e (tie) or pass it
  if (e < 0) return 1;
  const uint32_t p = (uint32_t)P.p;
  if (p == 0) return tie_wins && e == 0 ? 1 : 0x7fffffff;   // TP does not count
  const uint32_t t = tie_wins ? ((uint32_t)e + p - 1u) / p : (uint32_t)e / p + 1u;
  return t > 1u ? (int)t : 1;
}

// Depth-4 expansion of one prefix per lane: y3 (tumour) and z3 (normal)
// given, c = the lane's depth-3 index, c_first <= every valid lane's c.  The
// wave streams the candidates d > c_first through scalar loads; each lane
// masks the d at or below its own c.  Every non-empty leaf is counted; only
// those whose TP reaches the lane's threshold (min_tp_for of the lane's best)
// are scored and offered, which leaves the answer unchanged: a leaf below it
// cannot replace the leaf the lane already holds.
template <int W, bool kBound, bool kZL>
__device__ __forceinline__ void expand4(const Problem& P, const Work& w, RoundState* st,
                                        uint32_t (&y3)[W], const NrmPre<kZL>& z3,
                                        uint32_t znz, bool valid, int a3, int b3, int c,
                                        int c_first, Best& best, Tally& tl,
                                        unsigned long long& inc) {
  const int lane = threadIdx.x & 63;
  const int nA = uniform(st->nA);
  cu32* TA = (cu32*)w.TA;
  cu32* NA = (cu32*)w.NA;
  bool live = valid;
  if (kBound) {
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) cnt += __popc(y3[k]);
    inc = load_incumbent(st);
    const bool drop = live && dominated(P.p * cnt + P.q * P.n_normal, a3, b3, inc);
    tl.bp3 += __popcll(__ballot(drop));
    live = live && !drop;
    if (!__any(live)) return;
  }
  // a leaf's FP needs counting unless no normal is left in the prefix (under
  // the literal reading the last gene's normals add on, so always)
  const bool zlive = live && (znz != 0 || P.tn_literal);
  if (live) tl.xv4 += (unsigned long long)(nA - 1 - c);
  // a dead lane's TP is 0 at every d: it never counts nor offers
  uint32_t (&y)[W] = y3;
#pragma unroll
  for (int k = 0; k < W; ++k) y[k] = live ? y[k] : 0u;
  const int cmax = wave_max(live ? c : -1);   // d > cmax: no lane masks d
  // the prefix's leaves all have a smaller tuple than the best exactly when
  // (a3, b3, c) precedes the best's first three indices
  const unsigned long long pre = ((unsigned long long)a3 << 32) | ((unsigned long long)b3 << 16) |
                                 (unsigned long long)c;
  int thr = min_tp_for(P, best.s, pre < (best.t >> 16));
  uint32_t ne = 0;   // non-empty leaves of this pass (< 64 * nA)
  // leaves of candidate d in lanes m (TP >= thr): score and offer
  auto offer = [&](int d, int tp, unsigned long long m) {
    const bool hit = __builtin_amdgcn_inverse_ballot_w64(m);
    int fp = 0;
    if (__any(hit && zlive)) {
      if (hit && zlive) {
        fp = leaf_fp_z(z3, lane, NA + (size_t)d * kMaxWN32, P.tn_literal);
        tl.xfp++;
      }
    }
    if (hit) {
      const int sc = P.p * tp + P.q * (P.n_normal - fp);
      best.offer(sc, tp, fp, a3, b3, c, d);
      // a best from this prefix has a smaller tuple than its later leaves
      thr = min_tp_for(P, best.s, pre < (best.t >> 16));
      if (kBound) {
        const unsigned long long key = leaf_key(sc, a3, b3);
        if (key > inc) {
          const unsigned long long old = atomicMax(&st->incumbent, key);
          inc = old > key ? old : key;
        }
      }
    }
  };
  int d = c_first + 1;
  // d <= cmax: lanes with c >= d mask it
  for (; d <= cmax && d < nA; ++d) {
    uint32_t row[W];
#pragma unroll
    for (int k = 0; k < W; ++k) row[k] = TA[(size_t)d * W + k];
    const int tp = popc_and_r<W>(y, row);
    const unsigned long long dm = __ballot(d > c);
    ne += (uint32_t)__popcll(__ballot(tp > 0) & dm);
    const unsigned long long m = __ballot(tp >= thr) & dm;
    if (m) offer(d, tp, m);
  }
  if (d >= nA) {
    tl.ne4 += ne;
    return;
  }
  // d > cmax: every lane tests every d.  Candidates stream through two
  // register buffers of KR rows each, the next group in flight while the
  // current one is tested.  TA holds at least 128 rows past the last active
  // one (whole 128-row tiles plus 128), so groups are read unclamped; rows
  // at or past nA are zeroed before use (TP 0: neither counted nor offered).
  constexpr int KR = W <= 4 ? 4 : (W <= 16 ? 2 : 1);
  auto step = [&](int dd, const uint32_t (&row)[W]) {
    const int tp = popc_and_r<W>(y, row);
    ne += (uint32_t)__popcll(__ballot(tp > 0));
    const unsigned long long m = __ballot(tp >= thr);
    if (m) offer(dd, tp, m);
  };
  auto group = [&](uint32_t (&r)[KR][W]) {
    if (d + KR > nA) {
#pragma unroll
      for (int j = 1; j < KR; ++j)
#pragma unroll
        for (int k = 0; k < W; ++k) r[j][k] = d + j < nA ? r[j][k] : 0u;
    }
#pragma unroll
    for (int j = 0; j < KR; ++j) step(d + j, r[j]);
    d += KR;
  };
  cu32* ptr = TA + (size_t)d * W;
  uint32_t ra[KR][W], rb[KR][W];
  load_group<W, KR>(ra, ptr);
  for (;;) {
    cu32* pn = ptr + KR * W;
    group_arrived<W, KR>(pn, ra);
    load_group<W, KR>(rb, pn);
    group(ra);
    if (d >= nA) break;
    ptr = pn;
    pn = ptr + KR * W;
    group_arrived<W, KR>(pn, rb);
    load_group<W, KR>(ra, pn);
    group(rb);
    if (d >= nA) break;
    ptr = pn;
  }
  tl.ne4 += ne;
}

// ---- listing of long-stream depth-3 prefixes (two-phase depth 4)
constexpr int kStage = 256;   // listed prefixes staged per wave before one global append

__device__ __forceinline__ unsigned long long triple_entry(int a, int b, int c) {
  return (unsigned long long)a | ((unsigned long long)b << 16) | ((unsigned long long)c << 32);
}

// Appends q[0, n) to the round's list (one atomic per call) and adds the
// per-c counts, one atomic per run of equal c among 64 consecutive entries;
// the count an atomic returns is the run's first rank among the entries of
// its c, kept with each entry so that the bucketing needs no atomics.
__device__ __forceinline__ void append_staged(const Work& w, RoundState* st,
                                              const unsigned long long* q, int n, int lane) {
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&st->n_tri, (unsigned long long)n);
  base = __shfl(base, 0, 64);
  for (int i0 = 0; i0 < n; i0 += kWave) {
    const int i = i0 + lane;
    const bool v = i < n && base + i < w.tri_cap;
    const unsigned long long e = v ? q[i] : 0ull;
    if (v) w.tri[base + i] = e;
    const int c = v ? (int)(e >> 32) : -1;
    const int cprev = __shfl_up(c, 1, 64);
    const bool head = v && (lane == 0 || c != cprev);
    const unsigned long long H = __ballot(head);
    // valid lanes form a prefix; counted with the whole wave active
    const int nvalid = __popcll(__ballot(v));
    uint32_t r0 = 0;
    if (head) {
      const unsigned long long above = H & ~((2ull << lane) - 1ull);
      const int next = above ? __builtin_ctzll(above) : nvalid;
      r0 = atomicAdd(&w.c_hist[c], (uint32_t)(next - lane));
    }
    // the run's head: highest head at or below this lane (lane 0 always is one)
    const unsigned long long below = H & ((2ull << lane) - 1ull);
    const int hl = below ? 63 - __builtin_clzll(below) : 0;
    const uint32_t rank = (uint32_t)__shfl((int)r0, hl, 64) + (uint32_t)(lane - hl);
    if (v) w.tri_rank[base + i] = rank;
  }
}

}  // namespace
}  // namespace pdfs
