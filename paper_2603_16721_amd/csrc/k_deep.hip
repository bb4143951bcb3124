// Depth-first expansion for h = 5..9 (Alg. 2 depths 3..h, Sec. III-C).
//
// Every depth is expanded wave-wide, as the h <= 4 depth-4 loop does: a wave
// holds 64 prefixes of one depth (one per lane) and streams the candidate
// rows of the next depth through scalar loads, each lane masking the
// candidates at or below its own last index; the candidate row is loaded
// once per wave instead of once per lane, and no lane waits for another's
// subtree.  Depth 3 comes from the work items (64 pairs x a range of
// depth-3 candidates); a prefix of depth l (3 <= l < h) that is extended --
// non-empty, or any in exhaustive mode -- goes into the wave's ring for
// depth l in device memory ([word][entry] intersections, [depth][entry]
// indices), and 64 entries of that ring make the next depth-(l+1) expansion.
// When a ring holds 64 or more entries the expansion filling it is
// suspended (its intersections, indices and position saved in the wave's
// frame for that depth) and the deeper level runs first; so each ring stays
// below 128 entries and at most one suspended expansion exists per depth.
// Once the items are exhausted the rings are flushed shallowest first with
// partial batches.
//
// Leaves (depth h) whose TP reaches the lane's threshold (the least TP that
// can still replace its best, ties included when the prefix precedes the
// best's) are scored S = p*TP + q*(N_n - FP) and compared under (S desc,
// tuple asc); the normal join of a prefix is formed at its first such leaf.
//
// Bound mode: a prefix whose score bound p*TP + q*N_n cannot reach the
// round's incumbent (or ties it with larger first two indices) is not
// extended; leaves that become a lane's best raise the incumbent.
//
// Counters: non-empty prefixes per depth, bound-pruned prefixes per depth,
// and for every extended depth-l prefix the depth-(l+1) visits of Alg. 2's
// loop bounds (sorted indices in (idx(g_l), G-h+l]), per wave in LDS, then
// one atomic per wave and depth.  The depth-2 and depth-3 visit counts come
// from the pair kernel, as for h <= 4.
#include <algorithm>

#include "dfs_core.h"
#include "pdfs_dev.h"
#include "slot_reduce.h"

namespace pdfs {

namespace {

constexpr int kLv = kMaxH - 3;   // rings of depths 3..kMaxH-1, frames of depths 3..kMaxH-1

// kBound: bound mode (an instance of its own, so that the other modes do
// not carry its registers)
template <int W64, bool kBound>
__global__ __launch_bounds__(256) void k_dfs_deep(Problem P, Work w, int phase) {
  constexpr int W = 2 * W64;
  constexpr int KR = W <= 4 ? 4 : (W <= 16 ? 2 : 1);
  constexpr int kNone = 0x7fffffff;   // "last index" of an idle lane: masks every candidate
  constexpr int kWib = kBlock / kWave;
  __shared__ int s_amax[kMaxH + 1];
  __shared__ unsigned long long s_cnt[kWib][3][kMaxH + 1];   // non-empty, visited, bound-pruned
  // per ring: entries taken, entries queued (running counts, modulo 2^32)
  __shared__ uint32_t s_q[kWib][2][kLv];
  __shared__ int s_f[kWib][2][kLv];   // per suspended frame: next candidate, end
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  if (threadIdx.x <= kMaxH) s_amax[threadIdx.x] = st->amax[threadIdx.x];
  if (lane <= kMaxH) s_cnt[wib][0][lane] = s_cnt[wib][1][lane] = s_cnt[wib][2][lane] = 0ull;
  if (lane < kLv) s_q[wib][0][lane] = s_q[wib][1][lane] = 0u;
  __syncthreads();
  unsigned long long* cne = s_cnt[wib][0];
  unsigned long long* cvis = s_cnt[wib][1];
  unsigned long long* cbp = s_cnt[wib][2];
  uint32_t* q_taken = s_q[wib][0];
  uint32_t* q_queued = s_q[wib][1];
  const int h = P.h;
  const bool all_pre = P.mode == kPruneNone;
  constexpr bool bound = kBound;
  unsigned long long inc = 0;   // the round's incumbent key as last seen by this lane
  const bool lit = P.tn_literal != 0;
  // bound mode: phase 1 expands the seed list, phase 2 the filtered work
  // list; the other modes run phase 2 over every pair
  const unsigned long long* __restrict__ plist = phase == 1 ? w.seed_pairs : w.work_pairs;
  const unsigned long long npairs =
      phase == 1 ? (st->n_seed < kSeedCap ? st->n_seed : kSeedCap) : st->n_work_pairs;
  const unsigned long long nit = st->n_items;
  const uint32_t nitems = (uint32_t)uniform((int)(nit < w.item_cap ? nit : w.item_cap));
  const int nA_all = uniform(st->nA);
  if (blockIdx.x == 0 && threadIdx.x == 0 && nit > w.item_cap) st->overflow |= 1;
  const uint32_t* __restrict__ TA = w.TA;
  const uint32_t* __restrict__ NA = w.NA;
  cu32* TAc = (cu32*)w.TA;
  cu32* NAc = (cu32*)w.NA;
  const int qN = P.q * P.n_normal;

  // this wave's rings and frames
  constexpr size_t kRingWords = (size_t)(W + kMaxH) * kDeepQ;
  constexpr size_t kFrameWords = (size_t)(W + kMaxH + 1) * kWave;
  uint32_t* __restrict__ area =
      w.deepq + (size_t)(blockIdx.x * kWib + wib) * (kLv * (kRingWords + kFrameWords));
  auto ring_y = [&](int l) { return area + (size_t)(l - 3) * kRingWords; };
  auto ring_ix = [&](int l) {
    return reinterpret_cast<int*>(area + (size_t)(l - 3) * kRingWords + (size_t)W * kDeepQ);
  };
  auto frame = [&](int l) { return area + kLv * kRingWords + (size_t)(l - 3) * kFrameWords; };
  auto counter = [&](const uint32_t* c, int l) { return (uint32_t)uniform((int)c[l - 3]); };
  auto queued = [&](int l) { return (int)(counter(q_queued, l) - counter(q_taken, l)); };

  int bs = -1, btp = 0, bfp = 0;
  int bidx[kMaxH];
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) bidx[i] = 0;

  // the expansion in registers: depth L, the lanes' prefixes of depth L-1
  // (intersection y, indices pix, last index), candidates d..hi-1
  int L = 3, d = 0, hi = 0;
  uint32_t y[W];
  int pix[kMaxH];
  int last = kNone;
#pragma unroll
  for (int k = 0; k < W; ++k) y[k] = 0u;
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) pix[i] = 0;

  auto wave_first = [&](int x) {   // smallest x over the wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
    return uniform(x);
  };
  // 1..64 entries of the depth-l ring into the registers (depth l+1 next)
  auto take = [&](int l, int n) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // written by other lanes
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t qh = counter(q_taken, l);
    const bool v = lane < n;
    const int e = (int)((qh + (uint32_t)lane) & (kDeepQ - 1));
    const uint32_t* __restrict__ ry = ring_y(l);
    const int* __restrict__ ri = ring_ix(l);
#pragma unroll
    for (int k = 0; k < W; ++k) y[k] = v ? ry[(size_t)k * kDeepQ + e] : 0u;
    last = kNone;
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) {
      pix[i] = (v && i < l) ? ri[i * kDeepQ + e] : 0;
      if (v && i == l - 1) last = pix[i];
    }
    q_taken[l - 3] = qh + (uint32_t)n;
    if (bound) inc = load_incumbent(st);
    L = l + 1;
    d = wave_first(last == kNone ? kNone : last + 1);
    hi = s_amax[L];
  };
  auto save = [&]() {   // the registers into the frame of depth L
    uint32_t* f = frame(L);
#pragma unroll
    for (int k = 0; k < W; ++k) f[(size_t)k * kWave + lane] = y[k];
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) f[(size_t)(W + i) * kWave + lane] = (uint32_t)pix[i];
    f[(size_t)(W + kMaxH) * kWave + lane] = (uint32_t)last;
    s_f[wib][0][L - 3] = d;
    s_f[wib][1][L - 3] = hi;
  };
  auto restore = [&]() {   // the frame of depth L into the registers
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t* f = frame(L);
#pragma unroll
    for (int k = 0; k < W; ++k) y[k] = f[(size_t)k * kWave + lane];
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) pix[i] = (int)f[(size_t)(W + i) * kWave + lane];
    last = (int)f[(size_t)(W + kMaxH) * kWave + lane];
    d = uniform(s_f[wib][0][L - 3]);
    hi = uniform(s_f[wib][1][L - 3]);
    if (bound) inc = load_incumbent(st);
  };

  // Inner depth L < h: candidates from d on until hi or until the depth-L
  // ring holds 64 entries.  Rows stream through two groups of KR rows, the
  // next in flight while the current one is tested (TA holds at least 128
  // rows past the last active one, so groups are read unclamped).
  auto run_inner = [&]() {
    const int l = L;
    uint32_t* __restrict__ ry = ring_y(l);
    int* __restrict__ ri = ring_ix(l);
    bool full = false;
    auto step = [&](int dd, const uint32_t (&row)[W]) {
      uint32_t yc[W];
      uint32_t any = 0;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        yc[k] = y[k] & row[k];
        any |= yc[k];
      }
      const unsigned long long mk = __ballot(dd > last);
      const unsigned long long mn = __ballot(any != 0) & mk;
      unsigned long long mx = all_pre ? mk : mn;   // extended
      if (bound && mx) {
        int t = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) t += __popc(yc[k]);
        const unsigned long long md =
            __ballot(((mx >> lane) & 1ull) && dominated(P.p * t + qN, pix[0], pix[1], inc));
        if (md) {
          mx &= ~md;
          if (lane == 0) cbp[l] += (unsigned long long)__popcll(md);
        }
      }
      if (lane == 0) {
        cne[l] += (unsigned long long)__popcll(mn);
        // children of an extended prefix: the sorted indices (idx(dd), G-h+l]
        cvis[l + 1] += (unsigned long long)__popcll(mx) *
                       (unsigned long long)(P.G - h + l - w.act[dd]);
      }
      if (mx) {
        const uint32_t qt = counter(q_queued, l);
        if ((mx >> lane) & 1ull) {
          const int rank = (int)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(mx >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mx, 0u));
          const int pos = (int)((qt + (uint32_t)rank) & (kDeepQ - 1));
#pragma unroll
          for (int k = 0; k < W; ++k) ry[(size_t)k * kDeepQ + pos] = yc[k];
          for (int i = 0; i < l - 1; ++i) ri[i * kDeepQ + pos] = pix[i];
          ri[(l - 1) * kDeepQ + pos] = dd;
        }
        const uint32_t qt2 = qt + (uint32_t)__popcll(mx);
        q_queued[l - 3] = qt2;
        full = (int)(qt2 - counter(q_taken, l)) >= kWave;
      }
    };
    auto group = [&](const uint32_t (&r)[KR][W]) {
#pragma unroll
      for (int j = 0; j < KR; ++j)
        if (d < hi && !full) {
          step(d, r[j]);
          ++d;
        }
    };
    if (d >= hi) return;
    cu32* ptr = TAc + (size_t)d * W;
    uint32_t ra[KR][W], rb[KR][W];
    load_group<W, KR>(ra, ptr);
    for (;;) {
      cu32* pn = ptr + KR * W;
      group_arrived<W, KR>(pn, ra);
      load_group<W, KR>(rb, pn);
      group(ra);
      if (d >= hi || full) break;
      ptr = pn;
      pn = ptr + KR * W;
      group_arrived<W, KR>(pn, rb);
      load_group<W, KR>(ra, pn);
      group(rb);
      if (d >= hi || full) break;
      ptr = pn;
    }
  };

  // Leaf depth: every candidate from d to hi, scored against the lane's best.
  auto run_leaves = [&]() {
    unsigned long long ne = 0;
    // leaves of this prefix win a tie against the lane's best exactly when
    // the prefix precedes the best's first h-1 indices
    auto prefix_first = [&]() {
      int cmp = 0;
#pragma unroll
      for (int i = 0; i < kMaxH - 1; ++i)
        if (cmp == 0 && i < h - 1) cmp = pix[i] < bidx[i] ? -1 : (pix[i] > bidx[i] ? 1 : 0);
      return cmp < 0;
    };
    int thr = min_tp_for(P, bs, bs < 0 || prefix_first());
    bool zr = false;
    uint32_t z[kMaxWN32];
#pragma unroll
    for (int k = 0; k < kMaxWN32; ++k) z[k] = 0u;
    auto offer = [&](int dd, int tp, unsigned long long m) {
      if (!((m >> lane) & 1ull)) return;
      if (!zr) {
#pragma unroll
        for (int k = 0; k < kMaxWN32; ++k) z[k] = lit ? 0u : ~0u;
#pragma unroll
        for (int i = 0; i < kMaxH - 1; ++i) {
          if (i < h - 1) {
#pragma unroll
            for (int k = 0; k < kMaxWN32; ++k)
              z[k] = nrm_join(z[k], NA[(size_t)pix[i] * kMaxWN32 + k], lit);
          }
        }
        zr = true;
      }
      const int fp = leaf_fp(z, NAc + (size_t)dd * kMaxWN32, lit);
      const int sc = P.p * tp + P.q * (P.n_normal - fp);
      // equal score: the smaller tuple (lexicographic, sorted indices),
      // compared only on a tie; the update of every field is a straight-line
      // select under one mask, as in the slot argmax
      int cmp = 0;
      if (sc == bs) {
#pragma unroll
        for (int i = 0; i < kMaxH; ++i) {
          const int x = i < h - 1 ? pix[i] : dd;
          const int ci = x < bidx[i] ? -1 : (x > bidx[i] ? 1 : 0);
          cmp = ((cmp == 0) & (i < h)) ? ci : cmp;
        }
      }
      const bool take_it = (sc > bs) | ((sc == bs) & (cmp < 0));
      bs = take_it ? sc : bs;
      btp = take_it ? tp : btp;
      bfp = take_it ? fp : bfp;
#pragma unroll
      for (int i = 0; i < kMaxH; ++i)
        bidx[i] = take_it ? (i < h - 1 ? pix[i] : (i == h - 1 ? dd : 0)) : bidx[i];
      if (take_it) {
        if (bound) {
          const unsigned long long key = leaf_key(sc, pix[0], pix[1]);
          if (key > inc) {
            const unsigned long long old = atomicMax(&st->incumbent, key);
            inc = old > key ? old : key;
          }
        }
      }
      // the best now comes from this prefix (or precedes it): later leaves
      // of the prefix lose ties
      thr = min_tp_for(P, bs, bs < 0 || prefix_first());
    };
    auto step = [&](int dd, const uint32_t (&row)[W]) {
      const int tp = popc_and_r<W>(y, row);
      const unsigned long long dm = __ballot(dd > last);
      ne += (unsigned long long)__popcll(__ballot(tp > 0) & dm);
      const unsigned long long m = __ballot(tp >= thr) & dm;
      if (m) offer(dd, tp, m);
    };
    auto group = [&](const uint32_t (&r)[KR][W]) {
#pragma unroll
      for (int j = 0; j < KR; ++j)
        if (d + j < hi) step(d + j, r[j]);
      d += KR;
    };
    if (d < hi) {
      cu32* ptr = TAc + (size_t)d * W;
      uint32_t ra[KR][W], rb[KR][W];
      load_group<W, KR>(ra, ptr);
      for (;;) {
        cu32* pn = ptr + KR * W;
        group_arrived<W, KR>(pn, ra);
        load_group<W, KR>(rb, pn);
        group(ra);
        if (d >= hi) break;
        ptr = pn;
        pn = ptr + KR * W;
        group_arrived<W, KR>(pn, rb);
        load_group<W, KR>(ra, pn);
        group(rb);
        if (d >= hi) break;
        ptr = pn;
      }
    }
    if (lane == 0) cne[h] += ne;
  };

  const uint32_t nwaves = gridDim.x * kWib;
  const uint32_t gw = blockIdx.x * kWib + wib;
  bool first = true, items_done = false, have = false;
  uint32_t susp = 0;   // bit l: the expansion of depth l is suspended in its frame
  int idle = 0;        // scheduling passes since the last expansion ran
  for (;;) {
    if (!have) {
      // every pass takes an item, readies an expansion or moves one depth
      // up: a long run of passes without the first two is a fault
      if (++idle > 4 * kMaxH + 16) {
        if (lane == 0) atomicOr(&st->overflow, 4);
        break;
      }
      if (L == 3) {
        if (!items_done) {
          // the next work item: 64 pairs x depth-3 candidates [c_lo, c_hi)
          uint32_t it = nitems;
          if (first) {
            it = gw;
            first = false;
          } else if (lane == 0) {
            const unsigned long long cur =
                __hip_atomic_load(&st->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur + nwaves < nitems) it = (uint32_t)(nwaves + atomicAdd(&st->cursor, 1ull));
          }
          it = (uint32_t)uniform((int)it);
          if (it >= nitems) {
            items_done = true;
          } else {
            idle = 0;
            const int c_lo = uniform((int)w.items[it].c_lo);
            const int c_hi = uniform((int)w.items[it].c_hi);
            const uint32_t batch = (uint32_t)uniform((int)w.items[it].batch);
            const uint32_t first_chunk = (uint32_t)uniform((int)w.items[it].pad) & 1u;
            const unsigned long long pi = (unsigned long long)batch * kPairBatch + lane;
            bool valid = pi < npairs;
            const unsigned long long e = valid ? plist[pi] : 0ull;
            const int a = (int)(e & 0xffff);
            const int b = (int)((e >> 16) & 0xffff);
            const int ct = (int)((e >> 32) & 0xffff);
            valid = valid && a < b && b < nA_all;   // list entries always satisfy this
            if (bound) {
              // the pair's own bound against the incumbent; its depth-3
              // visits (sorted indices (idx(b), G-h+2]) once per pair
              inc = load_incumbent(st);
              const bool drop = valid && dominated(P.p * ct + qN, a, b, inc);
              const unsigned long long md = __ballot(drop);
              if (first_chunk && lane == 0) cbp[2] += (unsigned long long)__popcll(md);
              unsigned long long v3 = (valid && !drop) ? (unsigned long long)(P.G - h + 2 - w.act[b]) : 0ull;
#pragma unroll
              for (int o = 32; o > 0; o >>= 1) v3 += __shfl_xor(v3, o, 64);
              if (first_chunk && lane == 0) cvis[3] += v3;
              valid = valid && !drop;
            }
            const int ra = valid ? a : 0, rb = valid ? b : 0;   // in-range rows for idle lanes
#pragma unroll
            for (int k = 0; k < W; ++k)
              y[k] = valid ? TA[(size_t)ra * W + k] & TA[(size_t)rb * W + k] : 0u;
#pragma unroll
            for (int i = 0; i < kMaxH; ++i) pix[i] = i == 0 ? ra : (i == 1 ? rb : 0);
            last = valid ? b : kNone;
            d = wave_first(valid ? (b + 1 > c_lo ? b + 1 : c_lo) : kNone);
            hi = c_hi;
            have = d < hi;
          }
        }
        if (items_done) {
          // flush: the shallowest ring that still holds entries
          int l = 3;
          while (l < h && queued(l) == 0) ++l;
          if (l >= h) break;
          const int n = queued(l);
          take(l, n < kWave ? n : kWave);
          have = true;
        }
        continue;
      }
      // depth L >= 4: a batch of the depth-(L-1) ring, the suspended parent
      // expansion, or back up
      const int n = queued(L - 1);
      const bool parent = (susp >> (L - 1)) & 1u;
      if (n >= kWave || (items_done && n > 0 && !parent)) {
        take(L - 1, n < kWave ? n : kWave);
        have = true;
      } else if (parent) {
        L = L - 1;
        susp &= ~(1u << L);
        restore();
        have = true;
      } else {
        L = L - 1;
      }
      continue;
    }
    idle = 0;
    if (L == h) {
      run_leaves();
      have = false;
      continue;
    }
    run_inner();
    have = false;
    if (d < hi) {
      // the depth-L ring is full: its batches first, this expansion later
      save();
      susp |= 1u << L;
      L = L + 1;
    } else if (queued(L) >= kWave) {
      L = L + 1;
    }
  }

  Slot sl = empty_slot();
  if (bs >= 0) {
    sl.s = bs;
    sl.tp = btp;
    sl.fp = bfp;
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) sl.idx[i] = bidx[i];
  }
  block_best_to(&w.slots[(size_t)phase * kSlotsPerPhase + blockIdx.x], sl);
  // counters: one atomic per wave and depth
  if (lane == 0) {
    for (int l = 2; l <= h; ++l) {
      if (l >= 3 && cne[l]) atomicAdd(&st->cnt.nonempty[l], cne[l]);
      if (l >= 3 && cvis[l]) atomicAdd(&st->cnt.visited[l], cvis[l]);
      if (cbp[l]) atomicAdd(&st->cnt.bound_pruned[l], cbp[l]);
    }
  }
  for (int vb = blockIdx.x + gridDim.x; vb < kPersistBlocks; vb += gridDim.x)
    if (threadIdx.x == 0) w.slots[(size_t)phase * kSlotsPerPhase + vb] = empty_slot();
}

template <typename K>
int resident_deep(K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel),
                                                   kBlock, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu;
}

template <int W64, bool kBound>
hipError_t launch_deep_b(const Problem& P, const Work& w, int phase, hipStream_t s) {
  static const int per_cu = resident_deep(&k_dfs_deep<W64, kBound>);
  int g = per_cu * (P.n_cu > 0 ? P.n_cu : 1);
  if (g > kPersistBlocks) g = kPersistBlocks;
  k_dfs_deep<W64, kBound><<<g, kBlock, 0, s>>>(P, w, phase);
  return hipGetLastError();
}

template <int W64>
hipError_t launch_deep_w(const Problem& P, const Work& w, int phase, hipStream_t s) {
  return P.mode == kPruneBound ? launch_deep_b<W64, true>(P, w, phase, s)
                               : launch_deep_b<W64, false>(P, w, phase, s);
}

// 32-bit words of the rings and frames a launch at row width w64 uses: one
// area per wave of its grid (resident blocks x compute units, at most
// kPersistBlocks blocks), the larger of the two instantiations.
template <int W64>
size_t deep_words_w(int n_cu) {
  static const int per_cu = std::max(resident_deep(&k_dfs_deep<W64, false>),
                                     resident_deep(&k_dfs_deep<W64, true>));
  size_t g = (size_t)per_cu * (size_t)(n_cu > 0 ? n_cu : 1);
  if (g > (size_t)kPersistBlocks) g = kPersistBlocks;
  const size_t W = 2 * (size_t)W64;
  return g * (kBlock / kWave) * (size_t)(kMaxH - 3) * ((W + kMaxH) * kDeepQ + (W + kMaxH + 1) * kWave);
}

}  // namespace

size_t deep_ring_words(int w64_max, int n_cu) {
  size_t m = 0;
#define PDFS_CASE(n) \
  if (n <= w64_max) m = std::max(m, deep_words_w<n>(n_cu));
  PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
  PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
  PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
  return m;
}

hipError_t launch_dfs_deep(const Problem& P, const Work& w, int phase, hipStream_t s) {
  if (!w.deepq || P.h < 5 || P.h > kMaxH || phase < 1 || phase > 2 ||
      (phase == 1 && P.mode != kPruneBound))
    return hipErrorInvalidValue;
  switch (w.w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_deep_w<n>(P, w, phase, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace pdfs
