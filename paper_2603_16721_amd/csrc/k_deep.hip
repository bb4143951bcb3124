// Depth-first expansion for h = 5..9 (Alg. 2 depths 3..h, Sec. III-C).
//
// Work unit as for h <= 4: 64 non-empty pairs (one per lane) x a range of
// depth-3 candidates.  Each lane walks its pair's subtree over depths
// 3..h-1 in Alg. 2's order with an explicit stack: the candidate index of
// every depth sits in LDS (one column per lane), the running intersection of
// the parent of the depth being enumerated in VGPRs.  A candidate's
// intersection is the parent's AND its row; a non-empty one (any one in
// exhaustive mode) becomes the parent of the next depth, and on the way back
// up the parent of the shallower depth is rebuilt from the stacked indices
// (y2 AND the rows of depths 3..l-2), so only one intersection per lane is
// ever held.
//
// The leaf depth is not walked per lane.  A non-empty depth-(h-1) prefix
// (its intersection and indices) goes into a ring of the wave in device
// memory; once 64 are queued the whole wave takes them, one per lane, and
// streams the leaf candidates c in (min last index, amax_h) through scalar
// row loads, each lane masking the c at or below its own last index -- the
// candidate row is loaded once per wave instead of once per lane.  Leaves
// whose TP reaches the lane's threshold (the least TP that can still replace
// its best, ties included when the prefix precedes the best's) are scored
// S = p*TP + q*(N_n - FP) and compared under (S desc, tuple asc); the normal
// join of a prefix is formed at its first such leaf.
//
// Counters: non-empty prefixes per depth, and for every extended depth-l
// prefix the depth-(l+1) visits of Alg. 2's loop bounds (sorted indices in
// (idx(g_l), G-h+l]), added to the round's counters by one atomic per wave
// and depth.  The depth-2 and depth-3 visit counts come from the pair
// kernel, as for h <= 4.  Bound pruning is not applied at these depths; the
// answers are the same (the bound is an exact pruning rule).
#include "dfs_core.h"
#include "pdfs_dev.h"
#include "slot_reduce.h"

namespace pdfs {

namespace {

template <int W64>
__global__ __launch_bounds__(256) void k_dfs_deep(Problem P, Work w) {
  constexpr int W = 2 * W64;
  __shared__ int stk[kBlock / kWave][kMaxH][kWave];   // candidate index per depth, per lane
  __shared__ int s_amax[kMaxH + 1];
  // per-lane counters (own column, no atomics): [0] non-empty, [1] visited
  __shared__ unsigned long long s_cnt[kBlock / kWave][2][kMaxH + 1][kWave];
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  if (threadIdx.x <= kMaxH) s_amax[threadIdx.x] = st->amax[threadIdx.x];
  int (*ix)[kWave] = stk[wib];
  unsigned long long (*cne)[kWave] = s_cnt[wib][0];
  unsigned long long (*cvis)[kWave] = s_cnt[wib][1];
  for (int d = 0; d <= kMaxH; ++d) cne[d][lane] = cvis[d][lane] = 0ull;
  __syncthreads();
  const int h = P.h;
  const bool all_pre = P.mode == kPruneNone;
  const bool lit = P.tn_literal != 0;
  const unsigned long long* __restrict__ plist = w.work_pairs;
  const unsigned long long npairs = st->n_work_pairs;
  const unsigned long long nit = st->n_items;
  const uint32_t nitems = (uint32_t)uniform((int)(nit < w.item_cap ? nit : w.item_cap));
  const int nA_all = uniform(st->nA);
  if (blockIdx.x == 0 && threadIdx.x == 0 && nit > w.item_cap) st->overflow |= 1;
  const uint32_t* __restrict__ TA = w.TA;
  const uint32_t* __restrict__ NA = w.NA;
  cu32* TAc = (cu32*)w.TA;
  cu32* NAc = (cu32*)w.NA;
  const int qN = P.q * P.n_normal;

  // this wave's leaf-prefix ring: [W][kDeepQ] intersections, [kMaxH][kDeepQ]
  // indices; qh / qt count entries taken / queued (wave-uniform)
  uint32_t* __restrict__ qy =
      w.deepq + (size_t)(blockIdx.x * (kBlock / kWave) + wib) * (size_t)(W + kMaxH) * kDeepQ;
  int* __restrict__ qix = reinterpret_cast<int*>(qy + (size_t)W * kDeepQ);
  int qh = 0, qt = 0;

  int bs = -1, btp = 0, bfp = 0;
  int bidx[kMaxH];
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) bidx[i] = 0;
  unsigned long long ne_w = 0;   // non-empty leaves (wave-uniform)

  // The wave takes `take` (1..64) queued prefixes, one per lane, and scores
  // their leaves.  Called with every lane of the wave active.
  auto drain = [&](int take) {
    // the entries were written by other lanes of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const bool v = lane < take;
    const int e = (qh + lane) & (kDeepQ - 1);
    uint32_t y[W];
#pragma unroll
    for (int k = 0; k < W; ++k) y[k] = v ? qy[(size_t)k * kDeepQ + e] : 0u;
    int pix[kMaxH];
    int last = 0x7fffffff;   // idle lanes mask every candidate
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) {
      pix[i] = (v && i < h - 1) ? qix[i * kDeepQ + e] : 0;
      if (v && i == h - 2) last = pix[i];
    }
    qh += take;
    int lo = last == 0x7fffffff ? last : last + 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lo = min(lo, __shfl_xor(lo, o, 64));
    lo = uniform(lo);
    const int hi = s_amax[h];
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
    // leaves of candidate d in lanes m (TP >= thr): score, compare, update
    auto offer = [&](int d, int tp, unsigned long long m) {
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
      const int fp = leaf_fp(z, NAc + (size_t)d * kMaxWN32, lit);
      const int sc = P.p * tp + P.q * (P.n_normal - fp);
      bool take_it = sc > bs;
      if (sc == bs) {
        // equal score: the smaller tuple (lexicographic, sorted indices)
        int cmp = 0;
#pragma unroll
        for (int i = 0; i < kMaxH; ++i) {
          if (cmp == 0 && i < h) {
            const int x = i < h - 1 ? pix[i] : d;
            cmp = x < bidx[i] ? -1 : (x > bidx[i] ? 1 : 0);
          }
        }
        take_it = cmp < 0;
      }
      if (take_it) {
        bs = sc;
        btp = tp;
        bfp = fp;
#pragma unroll
        for (int i = 0; i < kMaxH; ++i) bidx[i] = i < h - 1 ? pix[i] : (i == h - 1 ? d : 0);
      }
      // the best now comes from this prefix (or precedes it): later leaves
      // of the prefix lose ties
      thr = min_tp_for(P, bs, bs < 0 || prefix_first());
    };
    auto step = [&](int d, const uint32_t (&row)[W]) {
      const int tp = popc_and_r<W>(y, row);
      const unsigned long long dm = __ballot(d > last);
      ne_w += (unsigned long long)__popcll(__ballot(tp > 0) & dm);
      const unsigned long long m = __ballot(tp >= thr) & dm;
      if (m) offer(d, tp, m);
    };
    if (lo >= hi) return;
    // candidates stream through two register buffers of KR rows each, the
    // next group in flight while the current one is tested; TA holds at
    // least 128 rows past the last active one, so groups are read unclamped
    // and rows at or past hi are skipped
    constexpr int KR = W <= 4 ? 4 : (W <= 16 ? 2 : 1);
    int d = lo;
    auto group = [&](const uint32_t (&r)[KR][W]) {
#pragma unroll
      for (int j = 0; j < KR; ++j)
        if (d + j < hi) step(d + j, r[j]);
      d += KR;
    };
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
  };

  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  const uint32_t gw = blockIdx.x * (kBlock / kWave) + wib;
  bool first = true;
  for (;;) {
    uint32_t it = nitems;
    if (first) {
      it = gw;
      first = false;
    } else if (lane == 0) {
      const unsigned long long cur =
          __hip_atomic_load(&st->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur + nwaves < nitems)
        it = (uint32_t)(nwaves + atomicAdd(&st->cursor, 1ull));
    }
    it = (uint32_t)uniform((int)it);
    if (it >= nitems) break;
    const int c_lo = uniform((int)w.items[it].c_lo);
    const int c_hi = uniform((int)w.items[it].c_hi);
    const uint32_t batch = (uint32_t)uniform((int)w.items[it].batch);
    const unsigned long long pi = (unsigned long long)batch * kPairBatch + lane;
    bool valid = pi < npairs;
    const unsigned long long e = valid ? plist[pi] : 0ull;
    const int a = (int)(e & 0xffff);
    const int b = (int)((e >> 16) & 0xffff);
    valid = valid && a < b && b < nA_all;   // list entries always satisfy this
    const int lo3 = c_lo > b + 1 ? c_lo : b + 1;
    bool live = valid && lo3 < c_hi;
    if (!__any(live)) continue;
    const int ra = valid ? a : 0, rb = valid ? b : 0;   // in-range rows for idle lanes
    uint32_t y2[W], yp[W], yc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      y2[k] = TA[(size_t)ra * W + k] & TA[(size_t)rb * W + k];
      yp[k] = y2[k];
      yc[k] = 0u;
    }
    ix[0][lane] = a;
    ix[1][lane] = b;
    ix[2][lane] = lo3 - 1;
    int level = 3;   // the depth whose candidates the lane enumerates
    while (__any(live)) {
      bool push = false;   // a non-empty depth-(h-1) prefix in yc / ix
      do {
        if (!live) break;
        const int l = level;
        const int cand = ix[l - 1][lane] + 1;
        const int hi = l == 3 ? c_hi : s_amax[l];
        if (cand >= hi) {
          // this depth is exhausted: back to depth l-1, whose candidates'
          // parent is the intersection of depths 1..l-2
          if (l == 3) {
            live = false;
            break;
          }
          level = l - 1;
#pragma unroll
          for (int k = 0; k < W; ++k) yp[k] = y2[k];
          for (int d = 3; d <= l - 2; ++d) {
            const int r = ix[d - 1][lane];
#pragma unroll
            for (int k = 0; k < W; ++k) yp[k] &= TA[(size_t)r * W + k];
          }
          break;
        }
        ix[l - 1][lane] = cand;
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
          yc[k] = yp[k] & TA[(size_t)cand * W + k];
          any |= yc[k];
        }
        if (any) cne[l][lane] += 1ull;
        if (!(any || all_pre)) break;
        // extended: its children are the sorted indices (idx(cand), G-h+l]
        const int kids = P.G - h + l - w.act[cand];
        cvis[l + 1][lane] += (unsigned long long)kids;
        if (l == h - 1) {
          // the leaf depth is scored from the ring
          push = any != 0;
          break;
        }
        ix[l][lane] = cand;
        level = l + 1;
#pragma unroll
        for (int k = 0; k < W; ++k) yp[k] = yc[k];
      } while (false);
      // every lane of the wave is active again here
      const unsigned long long bal = __ballot(push);
      if (bal) {
        if (push) {
          const int rank = (int)__builtin_amdgcn_mbcnt_hi(
              (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          const int pos = (qt + rank) & (kDeepQ - 1);
#pragma unroll
          for (int k = 0; k < W; ++k) qy[(size_t)k * kDeepQ + pos] = yc[k];
          for (int i = 0; i < h - 1; ++i) qix[i * kDeepQ + pos] = ix[i][lane];
        }
        qt += __popcll(bal);
        if (qt - qh >= kWave) drain(kWave);
      }
    }
  }
  if (qt > qh) drain(qt - qh);

  Slot sl = empty_slot();
  if (bs >= 0) {
    sl.s = bs;
    sl.tp = btp;
    sl.fp = bfp;
#pragma unroll
    for (int i = 0; i < kMaxH; ++i) sl.idx[i] = bidx[i];
  }
  block_best_to(&w.slots[(size_t)2 * kSlotsPerPhase + blockIdx.x], sl);
  // counters: one atomic per wave and depth
  for (int d = 3; d <= h; ++d) {
    unsigned long long n = cne[d][lane] + (d == h && lane == 0 ? ne_w : 0ull), v = cvis[d][lane];
    for (int o = 32; o > 0; o >>= 1) {
      n += __shfl_xor(n, o, 64);
      v += __shfl_xor(v, o, 64);
    }
    if (lane == 0) {
      if (n) atomicAdd(&st->cnt.nonempty[d], n);
      if (d >= 4 && v) atomicAdd(&st->cnt.visited[d], v);
    }
  }
  for (int vb = blockIdx.x + gridDim.x; vb < kPersistBlocks; vb += gridDim.x)
    if (threadIdx.x == 0) w.slots[(size_t)2 * kSlotsPerPhase + vb] = empty_slot();
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

template <int W64>
hipError_t launch_deep_w(const Problem& P, const Work& w, hipStream_t s) {
  static const int per_cu = resident_deep(&k_dfs_deep<W64>);
  int g = per_cu * (P.n_cu > 0 ? P.n_cu : 1);
  if (g > kPersistBlocks) g = kPersistBlocks;
  k_dfs_deep<W64><<<g, kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dfs_deep(const Problem& P, const Work& w, hipStream_t s) {
  if (!w.deepq || P.h < 5 || P.h > kMaxH) return hipErrorInvalidValue;
  switch (w.w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_deep_w<n>(P, w, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace pdfs
