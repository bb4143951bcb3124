// Depth-first expansion of the non-empty pairs (Alg. 2 depths 3..h, h <= 4).
//
// Work unit (the lambda subtree of Sec. III-D, batched): 64 consecutive
// non-empty pairs (one per lane) x a contiguous range of depth-3 candidates.
// Ranges are cut into chunks so that waves pulling items from one atomic
// cursor stay balanced (the paper hands out fixed-size lambda intervals on
// request for the same reason).
//
// Inner loop: each lane keeps its prefix intersection y (and the normal
// prefix z) in VGPRs; the wave walks candidates c in ascending order, the
// candidate row arrives through scalar loads (one copy for all 64 lanes) and
// every lane folds y & row into an emptiness test with v_and_or_b32.  A lane
// whose y_l & row is empty backtracks (Alg. 2: the prefix is not extended).
//
// h = 3: a non-empty y3 is a leaf, scored at once.
// h = 4: a non-empty (lane, c) is a depth-3 prefix; it is staged in an LDS
//   queue in ascending c.  Each full queue of 64 prefixes becomes a depth-4
//   pass with one prefix per lane (y3 = y2[s] & T_c built with cross-lane
//   permutes), again streaming candidates d > c through scalar loads; a
//   non-empty y4 is a leaf.
//
// Leaves: TP = |y_h| (popcount), FP = |z_{h-1} & N_g| (skipped when the
// normal prefix is already empty), S = p*TP + q*(N_n - FP); each lane keeps
// the best (S desc, tuple asc), reduced per wave into a slot.
//
// Bound mode (Sec. III-E, exact): a prefix covering c uncovered samples
// cannot score above p*c + q*N_n.  The best leaf found so far is kept in one
// 64-bit atomic key (S+1)<<32 | (0xffff-a)<<16 | (0xffff-b) (a, b = first two
// indices); a prefix is dropped when its bound is below that score, or equal
// to it with first two indices lexicographically above the key's -- then
// every tuple under it loses to a tuple already found.
#include "dfs_core.h"
#include "pdfs_dev.h"
#include "slot_reduce.h"

namespace pdfs {

namespace {

// Depth-4 pass over n <= 64 staged prefixes (queue entries lane | c << 6,
// ascending c): prefix s's y2 and z2 come from lane s by cross-lane reads.
template <int W, bool kBound, bool kZL>
__device__ __forceinline__ void depth4(const Problem& P, const Work& w, RoundState* st,
                                       const uint32_t* q, int n, const uint32_t (&y2)[W],
                                       const NrmPre<kZL>& z2, uint32_t* zl3, int a, int b,
                                       Best& best, Tally& tl, unsigned long long& inc, int lane) {
  const bool valid = lane < n;
  const uint32_t e = q[valid ? lane : 0];
  const int s = e & 63;
  const int c = (int)(e >> 6);
  cu32* TA = (cu32*)w.TA;
  cu32* NA = (cu32*)w.NA;
  uint32_t y3[W];
  NrmPre<kZL> z3;
  if constexpr (kZL) z3.s = zl3;
  const uint32_t vmask = valid ? ~0u : 0u;
  const int cc = valid ? c : 0;   // any in-range row for idle lanes
#pragma unroll
  for (int k = 0; k < W; ++k) {
    uint32_t v = __shfl(y2[k], s, 64);
    y3[k] = v & TA[(size_t)cc * W + k] & vmask;
  }
  uint32_t znz = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) {
    uint32_t v;
    if constexpr (kZL) v = z2.get(k, s);   // lane s's word, from the LDS slice
    else v = __shfl(z2.z[k], s, 64);
    const uint32_t z = nrm_join(v, NA[(size_t)cc * kMaxWN32 + k], P.tn_literal) & vmask;
    z3.set(k, lane, z);
    znz |= z;
  }
  const int a3 = __shfl(a, s, 64);
  const int b3 = __shfl(b, s, 64);
  // visited at depth 4 below the prefix: sorted indices in (idx(c), G-1]
  if (valid) tl.vis4 += (unsigned long long)(P.G - 1 - w.act[c]);
  const int c_first = uniform((int)(q[0] >> 6));
  expand4<W, kBound, kZL>(P, w, st, y3, z3, znz, valid, a3, b3, c, c_first, best, tl, inc);
}

// The per-round values the depth-first walk of one instance reads.
struct DfsView {
  const unsigned long long* plist;   // phase 1: the seed list, 2: the work list
  unsigned long long npairs;
  int nA_all;
  int c_long;       // c < c_long: at least w.long_stream depth-4 candidates
  bool all_pre;     // exhaustive mode (h = 4): every depth-3 prefix is extended
  bool list_long;   // two-phase depth 4: long-stream prefixes are listed
};

template <int H>
__device__ __forceinline__ DfsView dfs_view(const Problem& P, const Work& w, const RoundState* st,
                                            int phase) {
  DfsView v;
  v.plist = phase == 1 ? w.seed_pairs : w.work_pairs;
  v.npairs = phase == 1 ? (st->n_seed < kSeedCap ? st->n_seed : kSeedCap) : st->n_work_pairs;
  v.nA_all = uniform(st->nA);
  v.c_long = v.nA_all - w.long_stream;
  v.all_pre = H == 4 && P.mode == kPruneNone;
  // Two-phase depth 4 (empty-prefix pruning, list allocated): prefixes whose
  // candidate stream d > c is long are listed for the sorted tile kernel;
  // the short ones are expanded here.
  v.list_long = H == 4 && P.mode == kPruneEmpty && w.tri_cap > 0;
  return v;
}

// One walk: the 64 pairs of a batch (one per lane) x the depth-3 candidates
// [c_lo, c_hi) -- one work item, or a run of consecutive items of the batch
// -- each non-empty depth-3 prefix scored (h = 3), listed or queued and
// expanded at depth 4 (h = 4).  first_chunk: the range starts at the batch's
// first candidate (its pair-level counts are taken there).
//
// Pp, wp: where the instance's problem and workspace are read (the kernel's
// arguments or its batch descriptor).  They are read at the item's start and
// again for every depth-4 pass or append, so the walk holds only what it
// uses in scalar registers.
template <int H, int W64, bool kBound>
__device__ __forceinline__ void dfs_item(cProblem* Pp, cWork* wp, int phase, uint32_t batch,
                                         int c_lo, int c_hi, uint32_t first_chunk,
                                         uint32_t* q, unsigned long long* sq, int& sn,
                                         uint32_t* zl, Best& best, Tally& tl,
                                         unsigned long long& inc, int lane) {
  constexpr int W = 2 * W64;
  constexpr bool kZL = W64 >= kZLdsMinW64;
  constexpr bool kPipe = W <= 16;
  constexpr int KG = W <= 8 ? 16 / W : 1;
  const Problem P = load_const(fresh(Pp));
  const Work w = load_const(fresh(wp));
  RoundState* st = w.st;
  const DfsView v = dfs_view<H>(P, w, st, phase);
  const unsigned long long* __restrict__ plist = v.plist;
  const unsigned long long npairs = v.npairs;
  const int nA_all = v.nA_all;
  const int c_long = v.c_long;
  const bool all_pre = v.all_pre;
  const bool list_long = v.list_long;
  cu32* TA = (cu32*)w.TA;
  cu32* NA = (cu32*)w.NA;
  if (c_lo >= c_hi) return;   // never made by the item builder
  const unsigned long long pi = (unsigned long long)batch * kPairBatch + lane;
  bool valid = pi < npairs;
  const unsigned long long e = valid ? plist[pi] : 0ull;
  const int a = (int)(e & 0xffff);
  const int b = (int)((e >> 16) & 0xffff);
  const int ct = (int)((e >> 32) & 0xffff);
  valid = valid && a < b && b < nA_all;   // list entries always satisfy this
  if (kBound) {
    inc = load_incumbent(st);
    const bool drop = valid && dominated(P.p * ct + P.q * P.n_normal, a, b, inc);
    if (first_chunk) {
      tl.bp2 += __popcll(__ballot(drop));
      if (valid && !drop) tl.vis3 += (unsigned long long)(P.G - H + 2 - w.act[b]);
    }
    valid = valid && !drop;
  }
  if (!__any(valid)) return;
  uint32_t y2[W];
  NrmPre<kZL> z2;
  if constexpr (kZL) z2.s = zl;
  const uint32_t vmask = valid ? ~0u : 0u;
  const int ra = valid ? a : 0, rb = valid ? b : 0;   // in-range rows for idle lanes
#pragma unroll
  for (int k = 0; k < W; ++k)
    y2[k] = TA[(size_t)ra * W + k] & TA[(size_t)rb * W + k] & vmask;
  uint32_t znz = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) {
    const uint32_t z = nrm_join(NA[(size_t)ra * kMaxWN32 + k], NA[(size_t)rb * kMaxWN32 + k],
                                P.tn_literal) & vmask;
    z2.set(k, lane, z);
    znz |= z;
  }
  if constexpr (kZL) wave_lds_sync();   // the depth-4 passes read other lanes' words
  if (valid) {
    const int lo = c_lo > b + 1 ? c_lo : b + 1;
    if (c_hi > lo) tl.xv3 += (unsigned long long)(c_hi - lo);
  }

  int qn = 0;
  // Non-empty depth-3 prefixes (lane, c) of candidate c, m = their lanes:
  // scored (h = 3), or bound-tested and then listed or queued (h = 4).
  // m_hit: the lanes whose (lane, c) is non-empty; m: the prefixes to
  // extend -- the non-empty ones, or every (lane, c) in exhaustive mode.
  // Lane flags are taken from the masks as they are (inverse ballot), and a
  // lane's slot in a queue is its rank among the wave's extended prefixes
  // (mbcnt).
  const unsigned long long valid_m = __ballot(valid);
  const int b_max = wave_max(valid ? b : -1);   // c > b_max: every valid lane takes c
  const unsigned long long ab_entry = triple_entry(a, b, 0);
  uint32_t ne3 = 0;   // this item's non-empty depth-3 prefixes (< 64 * 65536)
  auto on_hits = [&](int c, unsigned long long m_hit, unsigned long long m) {
    cu32* row = TA + (size_t)c * W;
    ne3 += (uint32_t)__popcll(m_hit);
    bool hit = __builtin_amdgcn_inverse_ballot_w64(m);
    if (H == 3) {
      int fp = 0;
      const bool zn = znz != 0 || P.tn_literal;
      if (__any(hit && zn)) {
        if (hit && zn) {
          fp = leaf_fp_z(z2, lane, NA + (size_t)c * kMaxWN32, P.tn_literal);
          tl.xfp++;
        }
      }
      if (hit) {
        const int tp = popc_and<W>(y2, row);
        const int sc = P.p * tp + P.q * (P.n_normal - fp);
        best.offer(sc, tp, fp, a, b, c, 0);
        if (kBound) {
          const unsigned long long key = leaf_key(sc, a, b);
          if (key > inc) {
            const unsigned long long old = atomicMax(&st->incumbent, key);
            inc = old > key ? old : key;
          }
        }
      }
      return;
    }
    if (kBound) {
      bool drop = false;
      if (hit) {
        const int cnt = popc_and<W>(y2, row);
        drop = dominated(P.p * cnt + P.q * P.n_normal, a, b, inc);
      }
      tl.bp3 += __popcll(__ballot(drop));
      hit = hit && !drop;
      m = __ballot(hit);
      if (m == 0) return;
    }
    const int r = rank_below(m, 0);
    if (list_long && c < c_long) {
      if (hit) sq[sn + r] = ab_entry | ((unsigned long long)c << 32);
      sn += __popcll(m);
      wave_lds_sync();
      return;
    }
    if (hit) q[qn + r] = (uint32_t)lane | ((uint32_t)c << 6);
    qn += __popcll(m);
    wave_lds_sync();
  };
  // Staged long-stream prefixes go out once kStage are waiting; every full
  // wave of queued prefixes becomes a depth-4 pass.
  auto drain = [&]() {
    if (H != 4) return;
    if (sn < kStage && qn < kWave) return;
    const Problem P2 = load_const(fresh(Pp));
    const Work w2 = load_const(fresh(wp));
    if (sn >= kStage) {
      append_staged(w2, w2.st, sq, sn, lane);
      sn = 0;
    }
    int off = 0;
    while (qn - off >= kWave) {
      depth4<W, kBound, kZL>(P2, w2, w2.st, q + off, kWave, y2, z2, zl + kMaxWN32 * kWave, a,
                             b, best, tl, inc, lane);
      off += kWave;
    }
    if (off > 0) {
      const int rest = qn - off;   // < kWave
      const uint32_t moved = (lane < rest) ? q[off + lane] : 0u;
      wave_lds_sync();
      if (lane < rest) q[lane] = moved;
      wave_lds_sync();
      qn = rest;
    }
  };
  // The walk stops as soon as a full wave of prefixes is queued or the
  // staging buffer is full; the depth-4 passes and the append run outside
  // it and the walk resumes at the next candidate.  So no candidate rows in
  // flight (nor the walk's lane masks) stay live across a depth-4 pass,
  // whose own row buffers then fit the scalar registers.
  auto full = [&]() { return H == 4 && (qn >= kWave || sn >= kStage); };
  int c = c_lo;
  while (c < c_hi) {
    if (!kPipe) {
      while (c < c_hi) {
        const uint32_t acc = fold_nonempty<W>(y2, TA + (size_t)c * W);
        unsigned long long m_in = valid_m;
        if (c <= b_max) m_in &= __ballot(c > b);
        const unsigned long long m_hit = __ballot(acc != 0) & m_in;
        const unsigned long long m = all_pre ? m_in : m_hit;
        const int cc = c++;
        if (m == 0) continue;
        on_hits(cc, m_hit, m);
        if (full()) break;
      }
    } else {
      // Rows past c_hi are loaded (inside the round's row allocation: at
      // least 128 rows past the last active one) but never tested.  Each
      // row of a group is tested and acted on before the next, so only one
      // row's lane masks are live.
      auto group = [&](int c0, const uint32_t (&rows)[KG][W]) {
#pragma unroll
        for (int j = 0; j < KG; ++j) {
          const int cj = c0 + j;
          if (cj >= c_hi) break;
          const uint32_t acc = fold_chain_r<W>(y2, rows[j]);
          unsigned long long m_in = valid_m;
          if (cj <= b_max) m_in &= __ballot(cj > b);
          const unsigned long long m_hit = __ballot(acc != 0) & m_in;
          const unsigned long long m = all_pre ? m_in : m_hit;
          if (m) on_hits(cj, m_hit, m);
        }
      };
      constexpr int kNoClamp = 0x7fffffff;
      uint32_t rA[KG][W], rB[KG][W];
      load_rows<W, KG>(rA, TA, c, kNoClamp);
      for (;;) {
        int cn = c + KG;
        after_arrival<W, KG>(cn, rA);
        load_rows<W, KG>(rB, TA, cn, kNoClamp);
        group(c, rA);
        c += KG;
        if (c >= c_hi || full()) break;
        cn = c + KG;
        after_arrival<W, KG>(cn, rB);
        load_rows<W, KG>(rA, TA, cn, kNoClamp);
        group(c, rB);
        c += KG;
        if (c >= c_hi || full()) break;
      }
    }
    drain();
  }
  if (H == 4 && qn > 0) {
    const Problem P2 = load_const(fresh(Pp));
    const Work w2 = load_const(fresh(wp));
    depth4<W, kBound, kZL>(P2, w2, w2.st, q, qn, y2, z2, zl + kMaxWN32 * kWave, a, b, best,
                           tl, inc, lane);
    qn = 0;
  }
  tl.ne3 += ne3;
}

// kBound: bound pruning (Sec. III-E) compiled in; the other modes run the
// instantiation without it.
constexpr unsigned long long kMinChunk = 16;   // depth-3 candidates per work item at least
constexpr unsigned long long kGuide = 4;   // a run: 1/kGuide of a wave's share of the rest
constexpr unsigned long long kMaxRun = 4;   // items per cursor step at most

// The argument layout of k_dfs in its kernel-argument segment (in order,
// each at its natural alignment).
struct DfsArgs {
  Problem P;
  Work w;
  int phase;
};

template <int H, int W64, bool kBound>
__global__ __launch_bounds__(256, (W64 <= 5 || (W64 <= 16 && !kBound) ? 3 : 2)) void k_dfs(Problem P, Work w, int phase) {
  constexpr int W = 2 * W64;
  // Rows of up to 8 words: candidate rows arrive in groups of KG (one
  // 16-dword scalar load for up to 4 words, one row above that), the next
  // group in flight while the current one is tested; a group's prefixes are
  // queued before any depth-4 pass, so the queues hold up to KG more waves'
  // worth.  (Wider rows one at a time: a double-buffered row measured 13 %
  // slower at 16 words.)
  constexpr int KG = W <= 8 ? 16 / W : 1;
  __shared__ uint32_t qbuf[kBlock / kWave][kWave * (KG + 1)];
  // h = 4, two-phase: staged long-stream prefixes before a global append
  __shared__ unsigned long long sbuf[kBlock / kWave][H == 4 ? kStage + KG * kWave : 1];
  // the widest rows: the pairs' and the pass's normal prefixes
  constexpr bool kZL = W64 >= kZLdsMinW64;
  __shared__ uint32_t zbuf[kBlock / kWave][kZL ? 2 * kMaxWN32 * kWave : 1];
  RoundState* st = w.st;
  if (st->done) return;
  const auto* args = (const __attribute__((address_space(4))) DfsArgs*)
      __builtin_amdgcn_kernarg_segment_ptr();
  cProblem* Pp = &args->P;
  cWork* wp = &args->w;
  // the arguments read back through the segment must be the ones passed
  if (fresh(wp)->st != st || fresh(Pp)->G != P.G || fresh(wp)->TA != w.TA) {
    if (threadIdx.x == 0) atomicOr(&st->overflow, 2);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wib = uniform(threadIdx.x >> 6);
  uint32_t* q = qbuf[wib];
  unsigned long long* sq = sbuf[wib];
  int sn = 0;
  // phase 1 expands the seed list, phase 2 the (filtered) work list
  const unsigned long long nit = st->n_items;
  const uint32_t nitems = (uint32_t)uniform((int)(nit < w.item_cap ? nit : w.item_cap));
  if (blockIdx.x == 0 && threadIdx.x == 0 && nit > w.item_cap) st->overflow |= 1;

  Best best;
  best.init();
  Tally tl;
  tl.init();
  unsigned long long inc = 0;

  // Scheduling: the grid is sized to what the device holds at once, so every
  // wave starts at launch.  The items are split into kSubQueues contiguous
  // ranges, each with its own cursor (256 bytes apart, so that the atomics
  // of different ranges do not queue on one address -- one address serves
  // its atomics one at a time).  Wave g belongs to range g % kSubQueues: it
  // takes its first item there without an atomic, then runs of consecutive
  // items from that range's cursor (guided self-scheduling: about 1/kGuide
  // of a wave's share of what is left in the range, at most kMaxRun), and
  // once the range is done, runs from the following ranges in turn; it
  // leaves when every range is done.  A plain read before each atomic, so
  // that a done range costs no atomic.  Consecutive items of one batch in a
  // run are walked as one range of candidates.
  const auto* items = (const __attribute__((address_space(4))) Item*)w.items;
  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  const uint32_t gw = blockIdx.x * (kBlock / kWave) + wib;
  auto range_lo = [&](uint32_t r) {
    return (uint32_t)((unsigned long long)nitems * r / kSubQueues);
  };
  // waves g with g % kSubQueues == r
  auto range_waves = [&](uint32_t r) { return (nwaves + kSubQueues - 1 - r) / kSubQueues; };
  uint32_t qs = gw % kSubQueues;
  uint32_t q_left = kSubQueues;   // ranges not yet found done
  uint32_t t_next = range_lo(qs) + gw / kSubQueues;
  uint32_t t_end = t_next + 1;
  if (t_end > range_lo(qs + 1)) t_end = t_next;   // the range has fewer items than waves
  for (;;) {
    if (t_next >= t_end) {
      uint32_t start = 0, cnt = 0;
      while (q_left > 0) {
        const uint32_t hi = range_lo(qs + 1);
        const uint32_t nw = range_waves(qs);
        const uint32_t base = range_lo(qs) + nw;
        if (lane == 0) {
          unsigned long long* cur_p = w.cursors + (size_t)qs * kCursorStride;
          const unsigned long long cur =
              __hip_atomic_load(cur_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (base + cur < hi) {
            const unsigned long long left = hi - base - cur;
            const unsigned long long run = left / (kGuide * (unsigned long long)(nw > 0 ? nw : 1));
            cnt = run < 1 ? 1u : (run > kMaxRun ? (uint32_t)kMaxRun : (uint32_t)run);
            start = (uint32_t)(base + atomicAdd(cur_p, (unsigned long long)cnt));
          }
        }
        start = (uint32_t)uniform((int)start);
        cnt = (uint32_t)uniform((int)cnt);
        if (cnt > 0 && start < hi) {
          if (start + cnt > hi) cnt = hi - start;
          break;
        }
        cnt = 0;
        qs = qs + 1 == kSubQueues ? 0 : qs + 1;
        --q_left;
      }
      if (cnt == 0) break;
      t_next = start;
      t_end = start + cnt;
    }
    // the longest same-batch stretch of the run from t_next
    const uint32_t batch = (uint32_t)uniform((int)items[t_next].batch);
    uint32_t t_last = t_next;
    while (t_last + 1 < t_end && (uint32_t)uniform((int)items[t_last + 1].batch) == batch) ++t_last;
    const int c_lo = uniform((int)items[t_next].c_lo);
    const int c_hi = uniform((int)items[t_last].c_hi);
    const uint32_t first_chunk = (uint32_t)uniform((int)items[t_next].pad) & 1u;
    t_next = t_last + 1;
    dfs_item<H, W64, kBound>(Pp, wp, phase, batch, c_lo, c_hi, first_chunk, q, sq, sn,
                             zbuf[wib], best, tl, inc, lane);
  }
  if (H == 4 && sn > 0) append_staged(load_const(fresh(wp)), st, sq, sn, lane);

  // block argmax -> slot
  Slot sl = empty_slot();
  if (best.s >= 0) {
    sl.s = best.s; sl.tp = best.tp; sl.fp = best.fp;
    sl.idx[0] = best.idx(0); sl.idx[1] = best.idx(1); sl.idx[2] = best.idx(2); sl.idx[3] = best.idx(3);
  }
  block_best_to(&w.slots[(size_t)phase * kSlotsPerPhase + blockIdx.x], sl);
  // wave-uniform counts are held by lane 0 only, per-lane ones by every lane
  unsigned long long v[kTallyN] = {0};
  if (lane == 0) {
    v[kTNe3] = tl.ne3;
    v[kTNe4] = H == 4 ? tl.ne4 : 0;
    v[kTBp2] = tl.bp2;
    v[kTBp3] = tl.bp3;
    v[kTLeaves] = H == 3 ? tl.ne3 : tl.ne4;
  }
  v[kTVis3] = tl.vis3;
  v[kTVis4] = H == 4 ? tl.vis4 : 0;
  v[kTXv3] = tl.xv3;
  v[kTXv4] = tl.xv4;
  v[kTXfp] = tl.xfp;
  block_tally_to(w.tallies + ((size_t)phase * kPersistBlocks + blockIdx.x) * kTallyN, v);
  // slots and tally rows of blocks beyond a smaller grid read as empty
  for (int vb = blockIdx.x + gridDim.x; vb < kPersistBlocks; vb += gridDim.x) {
    if (threadIdx.x == 0) w.slots[(size_t)phase * kSlotsPerPhase + vb] = empty_slot();
    if (threadIdx.x < kTallyN)
      w.tallies[((size_t)phase * kPersistBlocks + vb) * kTallyN + threadIdx.x] = 0ull;
  }
}

// The depth-first step of a batched launch: one persistent grid drains the
// shared queue of every live instance's work items (instance i owns the queue
// positions [base[i], base[i+1])).  A wave works on one instance at a time;
// its queue positions only grow, so when it moves past an instance it sends
// that instance its staged prefixes, best leaf and counts, and never returns
// to it within the launch.
template <int H, int W64, bool kBound>
__global__ __launch_bounds__(256, (W64 <= 6 || (W64 <= 16 && !kBound) ? 3 : 2)) void k_dfs_multi(
    const BatchDesc* __restrict__ bd, BatchQueue* __restrict__ bq, int phase) {
  constexpr int W = 2 * W64;
  constexpr int KG = W <= 8 ? 16 / W : 1;
  __shared__ uint32_t qbuf[kBlock / kWave][kWave * (KG + 1)];
  __shared__ unsigned long long sbuf[kBlock / kWave][H == 4 ? kStage + KG * kWave : 1];
  constexpr bool kZL = W64 >= kZLdsMinW64;
  __shared__ uint32_t zbuf[kBlock / kWave][kZL ? 2 * kMaxWN32 * kWave : 1];
  const int lane = threadIdx.x & 63;
  const int wib = uniform(threadIdx.x >> 6);
  uint32_t* q = qbuf[wib];
  unsigned long long* sq = sbuf[wib];
  int sn = 0;
  const uint32_t total = (uint32_t)uniform((int)bq->total);
  int cur = -1;
  uint32_t lo = 0, hi = 0;
  const auto* cbd = (const __attribute__((address_space(4))) BatchDesc*)bd;
  cProblem* Pp = nullptr;
  cWork* wp = nullptr;
  Best best;
  Tally tl;
  unsigned long long inc = 0;
  auto flush = [&]() {
    const Work w = load_const(fresh(wp));
    RoundState* st = w.st;
    if (H == 4 && sn > 0) {
      append_staged(w, st, sq, sn, lane);
      sn = 0;
    }
    Slot sl = empty_slot();
    if (best.s >= 0) {
      sl.s = best.s; sl.tp = best.tp; sl.fp = best.fp;
      sl.idx[0] = best.idx(0); sl.idx[1] = best.idx(1); sl.idx[2] = best.idx(2);
      sl.idx[3] = best.idx(3);
    }
    unsigned long long v[kTallyN] = {0};
    if (lane == 0) {
      v[kTNe3] = tl.ne3;
      v[kTNe4] = H == 4 ? tl.ne4 : 0;
      v[kTBp2] = tl.bp2;
      v[kTBp3] = tl.bp3;
      v[kTLeaves] = H == 3 ? tl.ne3 : tl.ne4;
    }
    v[kTVis3] = tl.vis3;
    v[kTVis4] = H == 4 ? tl.vis4 : 0;
    v[kTXv3] = tl.xv3;
    v[kTXv4] = tl.xv4;
    v[kTXfp] = tl.xfp;
    wave_flush(w, st, phase, sl, v);
  };
  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  const uint32_t gw = blockIdx.x * (kBlock / kWave) + wib;
  bool first = true;
  for (;;) {
    uint32_t g = total;
    if (first) {
      g = gw;
      first = false;
    } else if (lane == 0) {
      const unsigned long long c =
          __hip_atomic_load(&bq->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c + nwaves < total) g = (uint32_t)(nwaves + atomicAdd(&bq->cursor, 1ull));
    }
    g = (uint32_t)uniform((int)g);
    if (g >= total) break;
    if (g >= hi) {
      if (cur >= 0) flush();
      int i = cur + 1;   // g < total = base[n]: the scan stops at an instance below n
      while ((uint32_t)uniform((int)bq->base[i + 1]) <= g) ++i;
      cur = i;
      lo = (uint32_t)uniform((int)bq->base[i]);
      hi = (uint32_t)uniform((int)bq->base[i + 1]);
      Pp = &cbd[i].P;
      wp = &cbd[i].w;
      best.init();
      tl.init();
      inc = 0;
    }
    {
      const auto* items = (const __attribute__((address_space(4))) Item*)fresh(wp)->items;
      const uint32_t it = g - lo;
      dfs_item<H, W64, kBound>(Pp, wp, phase, (uint32_t)uniform((int)items[it].batch),
                               uniform((int)items[it].c_lo), uniform((int)items[it].c_hi),
                               (uint32_t)uniform((int)items[it].pad) & 1u, q, sq, sn, zbuf[wib],
                               best, tl, inc, lane);
    }
  }
  if (cur >= 0) flush();
}

// One wave: the shared queue of a batched depth-first launch over the live
// instances' work items (kind 0) or 64-prefix depth-4 tiles (kind 1), and the
// phase's per-round log and counter row of every live instance cleared.
__global__ __launch_bounds__(64) void k_batch_queue(const BatchDesc* __restrict__ bd, int n,
                                                   BatchQueue* __restrict__ bq, int phase,
                                                   int kind) {
  const int lane = threadIdx.x;
  unsigned long long cnt = 0;
  if (lane < n) {
    const Work& w = bd[lane].w;
    RoundState* st = w.st;
    if (!st->done) {
      if (kind == 0) {
        cnt = st->n_items;
        if (cnt > w.item_cap) {
          st->overflow |= 1;
          cnt = w.item_cap;
        }
      } else {
        const unsigned long long nt = st->n_tri < w.tri_cap ? st->n_tri : w.tri_cap;
        cnt = (nt + kWave - 1) / kWave;
      }
      st->nlog[phase] = 0u;
      for (int f = 0; f < kTallyN; ++f)
        w.tallies[(size_t)phase * kPersistBlocks * kTallyN + f] = 0ull;
    }
  }
  unsigned long long incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long x = __shfl_up(incl, o, 64);
    if (lane >= o) incl += x;
  }
  if (lane < n) bq->base[lane + 1] = (uint32_t)incl;
  if (lane == 0) {
    bq->base[0] = 0u;
    bq->n = (uint32_t)n;
    bq->cursor = 0ull;
  }
  if (lane == 63) bq->total = (uint32_t)incl;
}

// Work items: batches of kPairBatch consecutive list pairs, each batch's
// depth-3 candidate range (min b + 1 .. amax[3]) cut into chunks.  One wave
// handles 64 batches (lane j holds batch j's range) and reserves their items
// with a single atomic.
__device__ __forceinline__ void make_items_body(const Problem& P, const Work& w, int seed, int chunk0) {
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  // the walk's range cursors start from zero (this kernel runs before every walk)
  if (blockIdx.x == 0 && threadIdx.x < kSubQueues) w.cursors[threadIdx.x * kCursorStride] = 0ull;
  const unsigned long long* __restrict__ list = seed ? w.seed_pairs : w.work_pairs;
  const unsigned long long np =
      seed ? (st->n_seed < kSeedCap ? st->n_seed : kSeedCap) : st->n_work_pairs;
  const unsigned long long nb = (np + kPairBatch - 1) / kPairBatch;
  const int amax3 = st->amax[3];
  // chunk length: shorter for a small round, so that its work still spreads
  // over the grid (about 4 items per wave of a full grid; batches average
  // about nA/2 candidates), and long enough that the item list cannot
  // overflow
  unsigned long long chunk = (unsigned long long)(chunk0 > 0 ? chunk0 : w.chunk);
  const unsigned long long spread = nb * (unsigned long long)st->nA / (8ull * kWavesPerGrid);
  if (spread < chunk) chunk = spread < kMinChunk ? kMinChunk : spread;
  const unsigned long long room = w.item_cap > nb ? w.item_cap - nb : 1;
  const unsigned long long need = (nb * (unsigned long long)st->nA + room - 1) / room;
  if (need > chunk) chunk = need;
  for (unsigned long long blk = (unsigned long long)gw * 64; blk < nb;
       blk += (unsigned long long)gridDim.x * (blockDim.x >> 6) * 64) {
    int mylo = 0, mylen = 0;
    const int nbat = (int)((nb - blk) < 64 ? (nb - blk) : 64);
    // 16 batches' loads in flight before their reductions
    for (int j0 = 0; j0 < nbat; j0 += 16) {
      int bv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const unsigned long long pi = (blk + j0 + u) * kPairBatch + lane;
        bv[u] = (j0 + u < nbat && pi < np) ? (int)((list[pi] >> 16) & 0xffff) : 0x7fffffff;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        int b = bv[u];
        for (int o = 32; o > 0; o >>= 1) b = min(b, __shfl_xor(b, o, 64));
        if (lane == j0 + u && j0 + u < nbat) {
          mylo = b + 1;
          mylen = amax3 > mylo ? amax3 - mylo : 0;
        }
      }
    }
    const unsigned long long n = mylen > 0 ? ((unsigned long long)mylen + chunk - 1) / chunk : 0;
    unsigned long long incl = n;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const unsigned long long total = __shfl(incl, 63, 64);
    if (total == 0) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&st->n_items, total);
    base = __shfl(base, 0, 64) + incl - n;
    for (unsigned long long k = 0; k < n; ++k) {
      if (base + k < w.item_cap) {
        Item it;
        it.batch = (uint32_t)(blk + lane);
        it.c_lo = (uint32_t)(mylo + k * chunk);
        const unsigned long long e = mylo + (k + 1) * chunk;
        it.c_hi = (uint32_t)(e < (unsigned long long)amax3 ? e : (unsigned long long)amax3);
        it.pad = (k == 0) ? 1u : 0u;
        w.items[base + k] = it;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_make_items(Problem P, Work w, int seed, int chunk0) {
  make_items_body(P, w, seed, chunk0);
}

__global__ __launch_bounds__(256) void k_make_items_m(const BatchDesc* __restrict__ bd, int seed, int chunk0) {
  make_items_body(bd[blockIdx.y].P, bd[blockIdx.y].w, seed, chunk0);
}

// Bound mode: the pair list is final; the seed and work lists and the item
// list start empty.
__device__ __forceinline__ void begin_bound_lists_body(const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;
  if (st->n_pairs > w.pair_cap) st->overflow |= kOverflowPairs;   // n_pairs: the count emitted
  st->n_work_pairs = 0;
  st->n_seed = 0;
  st->n_items = 0;
  st->cursor = 0;
}

__global__ void k_begin_bound_lists(Work w) {
  begin_bound_lists_body(w);
}

__global__ void k_begin_bound_lists_m(const BatchDesc* __restrict__ bd) {
  begin_bound_lists_body(bd[blockIdx.y].w);
}

// Empty-only mode: every emitted pair is expanded.
__device__ __forceinline__ void use_all_pairs_body(const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;
  unsigned long long n = st->n_pairs;
  if (n > w.pair_cap) {
    st->overflow |= kOverflowPairs;   // n_pairs keeps the count emitted
    n = w.pair_cap;
  } else {
    st->n_pairs = n;
  }
  st->n_work_pairs = n;
  st->n_items = 0;
  st->cursor = 0;
}

__global__ void k_use_all_pairs(Work w) {
  use_all_pairs_body(w);
}

__global__ void k_use_all_pairs_m(const BatchDesc* __restrict__ bd) {
  use_all_pairs_body(bd[blockIdx.y].w);
}

// ---- bound mode: seed selection and pair filtering -------------------------
// Histogram of the pair counts (C_T) of all emitted pairs.
__device__ __forceinline__ void pair_hist_body(const Work& w) {
  __shared__ uint32_t h[kMaxCount + 1];
  if (w.st->done) return;
  for (int v = threadIdx.x; v <= kMaxCount; v += blockDim.x) h[v] = 0u;
  __syncthreads();
  const unsigned long long np = w.st->n_pairs < w.pair_cap ? w.st->n_pairs : w.pair_cap;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < np;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const int ct = (int)((w.pairs[i] >> 32) & 0xffff);
    atomicAdd(&h[ct < kMaxCount ? ct : kMaxCount], 1u);
  }
  __syncthreads();
  for (int v = threadIdx.x; v <= kMaxCount; v += blockDim.x)
    if (h[v]) atomicAdd(&w.hist[v], h[v]);
}

__global__ __launch_bounds__(256) void k_pair_hist(Work w) {
  pair_hist_body(w);
}

__global__ __launch_bounds__(256) void k_pair_hist_m(const BatchDesc* __restrict__ bd) {
  pair_hist_body(bd[blockIdx.y].w);
}

// Threshold t: the largest count such that at least `want` pairs reach it (1
// if fewer pairs exist).  Every block computes it from the histogram.
__device__ int seed_threshold(const uint32_t* __restrict__ hist, int want) {
  constexpr int kPer = (kMaxCount + kBlock) / kBlock;   // bins per thread, from the top
  __shared__ unsigned int part[kBlock];
  __shared__ int t_sh;
  const int tid = threadIdx.x;
  unsigned int sum = 0;
  for (int k = 0; k < kPer; ++k) {
    const int v = kMaxCount - tid * kPer - k;
    if (v >= 1) sum += hist[v];
  }
  part[tid] = sum;
  if (tid == 0) t_sh = 1;
  __syncthreads();
  if (tid == 0) {
    unsigned long long cum = 0;
    for (int i = 0; i < kBlock; ++i) {
      if (cum + part[i] >= (unsigned long long)want) {
        for (int k = 0; k < kPer; ++k) {
          const int v = kMaxCount - i * kPer - k;
          if (v < 1) break;
          cum += hist[v];
          if (cum >= (unsigned long long)want) { t_sh = v; break; }
        }
        break;
      }
      cum += part[i];
    }
  }
  __syncthreads();
  return t_sh;
}

// Pairs with count >= t go to the seed list (up to kSeedCap) and are marked
// (bit 63) in the full list so that the main phase skips them.
__device__ __forceinline__ void seed_select_body(const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const unsigned long long np = st->n_pairs < w.pair_cap ? st->n_pairs : w.pair_cap;
  const int t = seed_threshold(w.hist, w.seed_n);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->seed_t = t;
  for (unsigned long long i0 = (unsigned long long)gw * 64; i0 < np;
       i0 += (unsigned long long)gridDim.x * (blockDim.x >> 6) * 64) {
    const unsigned long long i = i0 + lane;
    unsigned long long e = i < np ? w.pairs[i] : 0ull;
    const bool sel = i < np && (int)((e >> 32) & 0xffff) >= t;
    const unsigned long long m = __ballot(sel);
    if (!m) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&st->n_seed, (unsigned long long)__popcll(m));
    base = __shfl(base, 0, 64);
    const unsigned long long pos = base + __popcll(m & ((1ull << lane) - 1));
    if (sel && pos < kSeedCap) {
      w.seed_pairs[pos] = e;
      w.pairs[i] = e | (1ull << 63);
    }
  }
}

__global__ __launch_bounds__(256) void k_seed_select(Work w) {
  seed_select_body(w);
}

__global__ __launch_bounds__(256) void k_seed_select_m(const BatchDesc* __restrict__ bd) {
  seed_select_body(bd[blockIdx.y].w);
}

// Main-phase list: every unmarked pair whose bound can still reach the
// incumbent found by the seed phase.  Waves append their survivors in list
// order, so batches keep the locality of the pair table's tiles.
__device__ __forceinline__ void filter_pairs_body(const Problem& P, const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const unsigned long long np = st->n_pairs < w.pair_cap ? st->n_pairs : w.pair_cap;
  const unsigned long long inc = load_incumbent(st);
  unsigned long long dropped = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the seed phase's items are consumed; the main phase builds new ones
    st->n_items = 0;
    st->cursor = 0;
  }
  for (unsigned long long i0 = (unsigned long long)gw * 64; i0 < np;
       i0 += (unsigned long long)gridDim.x * (blockDim.x >> 6) * 64) {
    const unsigned long long i = i0 + lane;
    const unsigned long long e = i < np ? w.pairs[i] : (1ull << 63);
    const int a = (int)(e & 0xffff), b = (int)((e >> 16) & 0xffff);
    const int ct = (int)((e >> 32) & 0xffff);
    const bool seeded = (e >> 63) != 0;
    const bool drop = !seeded && dominated(P.p * ct + P.q * P.n_normal, a, b, inc);
    const bool keep = !seeded && !drop;
    const unsigned long long dm = __ballot(drop);
    if (lane == 0) dropped += __popcll(dm);
    const unsigned long long m = __ballot(keep);
    if (!m) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&st->n_work_pairs, (unsigned long long)__popcll(m));
    base = __shfl(base, 0, 64);
    if (keep) w.work_pairs[base + __popcll(m & ((1ull << lane) - 1))] = e;
  }
  // one atomic per block
  __shared__ unsigned long long bsum;
  if (threadIdx.x == 0) bsum = 0;
  __syncthreads();
  if (lane == 0 && dropped) atomicAdd(&bsum, dropped);
  __syncthreads();
  if (threadIdx.x == 0 && bsum) atomicAdd(&st->cnt.bound_pruned[2], bsum);
}

__global__ __launch_bounds__(256) void k_filter_pairs(Problem P, Work w) {
  filter_pairs_body(P, w);
}

__global__ __launch_bounds__(256) void k_filter_pairs_m(const BatchDesc* __restrict__ bd) {
  filter_pairs_body(bd[blockIdx.y].P, bd[blockIdx.y].w);
}

// Blocks of one DFS instantiation resident per compute unit (register use
// differs by row width), queried once.
template <int H, int W64, bool kBound>
int resident_blocks() {
  static const int n = [] {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_dfs<H, W64, kBound>), kBlock, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    return per_cu;
  }();
  return n;
}

template <int H, int W64, bool kBound>
hipError_t launch_mode(const Problem& P, const Work& w, int phase, hipStream_t s) {
  int blocks = resident_blocks<H, W64, kBound>() * (P.n_cu > 0 ? P.n_cu : 1);
  if (blocks > kPersistBlocks) blocks = kPersistBlocks;
  k_dfs<H, W64, kBound><<<blocks, kBlock, 0, s>>>(P, w, phase);
  return hipGetLastError();
}

template <int H, int W64>
hipError_t launch_one(const Problem& P, const Work& w, int phase, hipStream_t s) {
  return P.mode == kPruneBound ? launch_mode<H, W64, true>(P, w, phase, s)
                               : launch_mode<H, W64, false>(P, w, phase, s);
}

template <int H>
hipError_t dispatch(const Problem& P, const Work& w, int phase, hipStream_t s) {
  switch (w.w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_one<H, n>(P, w, phase, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

// ---- batched launches
template <int H, int W64, bool kBound>
hipError_t launch_multi_mode(const BatchDesc* bd, BatchQueue* bq, int phase, int n_cu,
                             hipStream_t s) {
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &v, reinterpret_cast<const void*>(&k_dfs_multi<H, W64, kBound>), kBlock, 0) !=
            hipSuccess ||
        v < 1)
      v = 1;
    return v;
  }();
  int blocks = per_cu * (n_cu > 0 ? n_cu : 1);
  if (blocks > kPersistBlocks) blocks = kPersistBlocks;
  k_dfs_multi<H, W64, kBound><<<blocks, kBlock, 0, s>>>(bd, bq, phase);
  return hipGetLastError();
}

template <int H>
hipError_t dispatch_multi(int w64, bool bound, const BatchDesc* bd, BatchQueue* bq, int phase,
                          int n_cu, hipStream_t s) {
  switch (w64) {
#define PDFS_CASE(n)                                                                   \
  case n:                                                                              \
    return bound ? launch_multi_mode<H, n, true>(bd, bq, phase, n_cu, s)               \
                 : launch_multi_mode<H, n, false>(bd, bq, phase, n_cu, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Row width (64-bit words) the DFS kernels are built for: the smallest
// instantiated width that holds n words.
int dfs_row_words(int n) {
  static const int widths[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 18, 20};
  for (int v : widths)
    if (v >= n) return v;
  return -1;
}

hipError_t launch_use_all_pairs(const Work& w, hipStream_t s) {
  k_use_all_pairs<<<1, 1, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_make_items(const Problem& P, const Work& w, bool seed, hipStream_t s) {
  k_make_items<<<kPersistBlocks / 4, kBlock, 0, s>>>(P, w, seed ? 1 : 0, seed ? 32 : w.chunk);
  return hipGetLastError();
}

hipError_t launch_seed_select(const Problem& P, const Work& w, hipStream_t s) {
  (void)P;
  k_begin_bound_lists<<<1, 1, 0, s>>>(w);
  k_pair_hist<<<256, 256, 0, s>>>(w);
  k_seed_select<<<kPersistBlocks / 2, kBlock, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_filter_pairs(const Problem& P, const Work& w, hipStream_t s) {
  k_filter_pairs<<<kPersistBlocks / 2, kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

hipError_t launch_batch_queue(const BatchDesc* bd, int n, BatchQueue* bq, int phase, int kind,
                              hipStream_t s) {
  k_batch_queue<<<1, 64, 0, s>>>(bd, n, bq, phase, kind);
  return hipGetLastError();
}

hipError_t launch_dfs_m(int h, int w64, bool bound, const BatchDesc* bd, BatchQueue* bq,
                        int phase, int n_cu, hipStream_t s) {
  if (h == 3) return dispatch_multi<3>(w64, bound, bd, bq, phase, n_cu, s);
  if (h == 4) return dispatch_multi<4>(w64, bound, bd, bq, phase, n_cu, s);
  return hipErrorInvalidValue;
}

hipError_t launch_make_items_m(const BatchDesc* bd, int n, bool seed, hipStream_t s) {
  // seed phase: 32 candidates per item; main phase: each instance's own chunk
  k_make_items_m<<<dim3(kPersistBlocks / 4, n), kBlock, 0, s>>>(bd, seed ? 1 : 0, seed ? 32 : -1);
  return hipGetLastError();
}

hipError_t launch_seed_select_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_begin_bound_lists_m<<<dim3(1, n), 1, 0, s>>>(bd);
  k_pair_hist_m<<<dim3(64, n), 256, 0, s>>>(bd);
  k_seed_select_m<<<dim3(kPersistBlocks / 4, n), kBlock, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_filter_pairs_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_filter_pairs_m<<<dim3(kPersistBlocks / 4, n), kBlock, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_use_all_pairs_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_use_all_pairs_m<<<dim3(1, n), 1, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_dfs(const Problem& P, const Work& w, int phase, hipStream_t s) {
  if (P.h == 3) return dispatch<3>(P, w, phase, s);
  if (P.h == 4) return dispatch<4>(P, w, phase, s);
  return hipErrorInvalidValue;
}

}  // namespace pdfs
