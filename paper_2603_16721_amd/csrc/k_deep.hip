// Depth-first expansion for h = 5..9 (Alg. 2 depths 3..h, Sec. III-C).
//
// Work unit as for h <= 4: 64 non-empty pairs (one per lane) x a range of
// depth-3 candidates.  Each lane walks its pair's subtree in Alg. 2's order
// with an explicit stack: the candidate index of every depth sits in LDS (one
// column per lane), the running intersection of the parent of the depth
// being enumerated in VGPRs.  A candidate's intersection is the parent's AND
// its row; a non-empty one (any one in exhaustive mode) becomes the parent of
// the next depth, and on the way back up the parent of the shallower depth is
// rebuilt from the stacked indices (y2 AND the rows of depths 3..l-2), so only
// one intersection per lane is ever held.  Leaves (depth h) with TP >= 1 are
// scored S = p*TP + q*(N_n - FP) and compared with the lane's best under
// (S desc, tuple asc); the normal intersection is formed only for a leaf
// whose best possible score (FP = 0) reaches the lane's best.
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
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  if (threadIdx.x <= kMaxH) s_amax[threadIdx.x] = st->amax[threadIdx.x];
  __syncthreads();
  int (*ix)[kWave] = stk[wib];
  const int h = P.h;
  const bool all_pre = P.mode == kPruneNone;
  const unsigned long long* __restrict__ plist = w.work_pairs;
  const unsigned long long npairs = st->n_work_pairs;
  const unsigned long long nit = st->n_items;
  const uint32_t nitems = (uint32_t)uniform((int)(nit < w.item_cap ? nit : w.item_cap));
  const int nA_all = uniform(st->nA);
  if (blockIdx.x == 0 && threadIdx.x == 0 && nit > w.item_cap) st->overflow |= 1;
  const uint32_t* __restrict__ TA = w.TA;
  const uint32_t* __restrict__ NA = w.NA;
  const int qN = P.q * P.n_normal;

  int bs = -1, btp = 0, bfp = 0;
  int bidx[kMaxH];
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) bidx[i] = 0;
  unsigned long long ne[kMaxH + 1], vis[kMaxH + 1];
#pragma unroll
  for (int d = 0; d <= kMaxH; ++d) ne[d] = vis[d] = 0;

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
    uint32_t y2[W], yp[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      y2[k] = TA[(size_t)ra * W + k] & TA[(size_t)rb * W + k];
      yp[k] = y2[k];
    }
    ix[0][lane] = a;
    ix[1][lane] = b;
    ix[2][lane] = lo3 - 1;
    int level = 3;   // the depth whose candidates the lane enumerates
    while (__any(live)) {
      if (!live) continue;
      const int l = level;
      const int cand = ix[l - 1][lane] + 1;
      const int hi = l == 3 ? c_hi : s_amax[l];
      if (cand >= hi) {
        // this depth is exhausted: back to depth l-1, whose candidates'
        // parent is the intersection of depths 1..l-2
        if (l == 3) {
          live = false;
          continue;
        }
        level = l - 1;
#pragma unroll
        for (int k = 0; k < W; ++k) yp[k] = y2[k];
        for (int d = 3; d <= l - 2; ++d) {
          const int r = ix[d - 1][lane];
#pragma unroll
          for (int k = 0; k < W; ++k) yp[k] &= TA[(size_t)r * W + k];
        }
        continue;
      }
      ix[l - 1][lane] = cand;
      uint32_t yc[W];
      uint32_t any = 0;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        yc[k] = yp[k] & TA[(size_t)cand * W + k];
        any |= yc[k];
      }
#pragma unroll
      for (int d = 3; d <= kMaxH; ++d)
        if (d == l && any) ne[d]++;
      if (l == h) {
        if (!any) continue;
        int tp = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) tp += __popc(yc[k]);
        if (P.p * tp + qN < bs) continue;   // cannot reach the lane's best
        uint32_t z[kMaxWN32];
#pragma unroll
        for (int k = 0; k < kMaxWN32; ++k) z[k] = P.tn_literal ? 0u : ~0u;
        for (int d = 1; d <= h; ++d) {
          const int r = ix[d - 1][lane];
#pragma unroll
          for (int k = 0; k < kMaxWN32; ++k)
            z[k] = nrm_join(z[k], NA[(size_t)r * kMaxWN32 + k], P.tn_literal);
        }
        int fp = 0;
#pragma unroll
        for (int k = 0; k < kMaxWN32; ++k) fp += __popc(z[k]);
        const int s = P.p * tp + P.q * (P.n_normal - fp);
        bool take = s > bs;
        if (s == bs) {
          // equal score: the smaller tuple (lexicographic, sorted indices)
          int cmp = 0;
#pragma unroll
          for (int i = 0; i < kMaxH; ++i) {
            if (cmp == 0 && i < h) {
              const int x = ix[i][lane];
              cmp = x < bidx[i] ? -1 : (x > bidx[i] ? 1 : 0);
            }
          }
          take = cmp < 0;
        }
        if (take) {
          bs = s;
          btp = tp;
          bfp = fp;
#pragma unroll
          for (int i = 0; i < kMaxH; ++i) bidx[i] = i < h ? ix[i][lane] : 0;
        }
        continue;
      }
      if (any || all_pre) {
        // extended: its children are the sorted indices (idx(cand), G-h+l]
        const int kids = P.G - h + l - w.act[cand];
#pragma unroll
        for (int d = 4; d <= kMaxH; ++d)
          if (d == l + 1) vis[d] += (unsigned long long)kids;
        ix[l][lane] = cand;
        level = l + 1;
#pragma unroll
        for (int k = 0; k < W; ++k) yp[k] = yc[k];
      }
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
  block_best_to(&w.slots[(size_t)2 * kSlotsPerPhase + blockIdx.x], sl);
  // counters: one atomic per wave and depth
#pragma unroll
  for (int d = 3; d <= kMaxH; ++d) {
    unsigned long long n = ne[d], v = vis[d];
    for (int o = 32; o > 0; o >>= 1) {
      n += __shfl_xor(n, o, 64);
      v += __shfl_xor(v, o, 64);
    }
    if (lane == 0 && d <= h) {
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
