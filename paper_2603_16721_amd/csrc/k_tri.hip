// Two-phase depth-4 expansion for h = 4 under empty-prefix pruning.
//
// The single-kernel DFS expands the depth-3 prefixes of one work item in
// passes of up to 64 (one per lane).  An item rarely yields a multiple of 64
// prefixes, so its last pass runs on a partly idle wave, and a pass streams
// the candidates d > min c, idling the lanes whose own c is larger.  Both
// costs scale with the length of the candidate stream, nA - 1 - c, which is
// long for the sparse genes early in the sparsest-first order and short for
// the dense ones at its end -- where most prefixes are.  So the level is
// split by stream length:
//
//   * prefixes with at least long_stream candidates (a per-context setting,
//     384 by default) are listed by the main
//     DFS kernel (and counted per c), bucketed by c with a counting sort and
//     expanded here in tiles of 64 consecutive entries: every lane busy, all
//     lanes of a tile with (nearly) the same c;
//   * the short ones stay in the main kernel's per-wave passes.
//
// The listed prefixes of a round are a subset of those of any earlier round
// of the run (the uncovered set and the active gene set only shrink), so a
// list sized for the first round holds every later one.  The depth-4 level
// and the leaf scoring are the single kernel's (expand4): results and
// counters are identical.
#include "dfs_core.h"
#include "pdfs_dev.h"
#include "slot_reduce.h"

namespace pdfs {

namespace {

// Slots and tally rows of blocks beyond a grid smaller than kPersistBlocks
// read as empty.
__device__ __forceinline__ void clear_absent_blocks(const Work& w, int phase, bool slots) {
  for (int vb = blockIdx.x + gridDim.x; vb < kPersistBlocks; vb += gridDim.x) {
    if (slots && threadIdx.x == 0) w.slots[(size_t)phase * kSlotsPerPhase + vb] = empty_slot();
    if (threadIdx.x < kTallyN)
      w.tallies[((size_t)phase * kPersistBlocks + vb) * kTallyN + threadIdx.x] = 0ull;
  }
}

// Per-round reset: empty list, zero per-c counts.
__device__ __forceinline__ void tri_begin_body(const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;
  const int nA = st->nA;
  if (w.tri_cap > 0)   // (a batched launch also reaches instances without lists)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nA; i += gridDim.x * blockDim.x)
      w.c_hist[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_tri = 0;
  }
}

__global__ void k_tri_begin(Work w) {
  tri_begin_body(w);
}

__global__ void k_tri_begin_m(const BatchDesc* __restrict__ bd) {
  tri_begin_body(bd[blockIdx.y].w);
}

// Sizing pass: counts the non-empty depth-3 prefixes with long candidate
// streams (the main kernel's listing test), writing nothing else.
template <int W64>
__global__ __launch_bounds__(256) void k_count_long(Problem P, Work w) {
  constexpr int W = 2 * W64;
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const unsigned long long* __restrict__ plist = w.work_pairs;
  const unsigned long long npairs = st->n_work_pairs;
  const unsigned long long nit = st->n_items;
  const uint32_t nitems = (uint32_t)uniform((int)(nit < w.item_cap ? nit : w.item_cap));
  const int nA_all = uniform(st->nA);
  const int c_long = nA_all - w.long_stream;
  const __attribute__((address_space(4))) Item* items =
      (const __attribute__((address_space(4))) Item*)w.items;
  cu32* TA = (cu32*)w.TA;
  unsigned long long n_long = 0;
  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  for (uint32_t it = blockIdx.x * (kBlock / kWave) + wib; it < nitems; it += nwaves) {
    const int c_lo = uniform((int)items[it].c_lo);
    const int c_hi = min(uniform((int)items[it].c_hi), c_long);
    if (c_lo >= c_hi) continue;
    const uint32_t batch = (uint32_t)uniform((int)items[it].batch);
    const unsigned long long pi = (unsigned long long)batch * kPairBatch + lane;
    bool valid = pi < npairs;
    const unsigned long long e = valid ? plist[pi] : 0ull;
    const int a = (int)(e & 0xffff);
    const int b = (int)((e >> 16) & 0xffff);
    valid = valid && a < b && b < nA_all;
    if (!__any(valid)) continue;
    uint32_t y2[W];
    const uint32_t vmask = valid ? ~0u : 0u;
    const int ra = valid ? a : 0, rb = valid ? b : 0;
#pragma unroll
    for (int k = 0; k < W; ++k) y2[k] = TA[(size_t)ra * W + k] & TA[(size_t)rb * W + k] & vmask;
    for (int c = c_lo; c < c_hi; ++c) {
      const uint32_t acc = fold_nonempty<W>(y2, TA + (size_t)c * W);
      n_long += (unsigned long long)__popcll(__ballot(valid && c > b && acc != 0));
    }
  }
  if (lane == 0 && n_long) atomicAdd(&st->n_tri, n_long);
}

// Exclusive prefix of the per-c counts, in place (one block).
__device__ __forceinline__ void scan_c_body(const Work& w) {
  __shared__ unsigned long long part[1024];
  RoundState* st = w.st;
  if (st->done || w.tri_cap == 0) return;
  const int nA = st->nA;
  const int tid = threadIdx.x;
  if (tid == 0 && st->n_tri > w.tri_cap) st->overflow |= 1;
  // the tile kernel's range cursors (the walk that used them has ended)
  if (tid < kSubQueues) w.cursors[tid * kCursorStride] = 0ull;
  const int per = (nA + 1023) / 1024;
  const int lo = tid * per;
  const int hi = lo + per < nA ? lo + per : nA;
  unsigned long long sum = 0;
  for (int i = lo; i < hi; ++i) sum += w.c_hist[i];
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned long long add = tid >= o ? part[tid - o] : 0ull;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  unsigned long long run = part[tid] - sum;
  for (int i = lo; i < hi; ++i) {
    const uint32_t x = w.c_hist[i];
    w.c_hist[i] = (uint32_t)run;
    run += x;
  }
}

__global__ __launch_bounds__(1024) void k_scan_c(Work w) {
  scan_c_body(w);
}

__global__ __launch_bounds__(1024) void k_scan_c_m(const BatchDesc* __restrict__ bd) {
  scan_c_body(bd[blockIdx.y].w);
}

// Scatter into c buckets: entry i goes to its bucket's offset plus the rank
// it was given when it was counted (no atomics; coalesced reads).
__device__ __forceinline__ void scatter_c_body(const Work& w) {
  RoundState* st = w.st;
  if (st->done || w.tri_cap == 0) return;
  const unsigned long long n = st->n_tri < w.tri_cap ? st->n_tri : w.tri_cap;
  for (unsigned long long i = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * kBlock) {
    const unsigned long long e = w.tri[i];
    const int c = (int)((e >> 32) & 0xffff);
    w.tri_s[(unsigned long long)w.c_hist[c] + w.tri_rank[i]] = e;
  }
}

__global__ __launch_bounds__(256) void k_scatter_c(Work w) {
  scatter_c_body(w);
}

__global__ __launch_bounds__(256) void k_scatter_c_m(const BatchDesc* __restrict__ bd) {
  scatter_c_body(bd[blockIdx.y].w);
}

// Depth-4 expansion of the sorted list, 64 consecutive prefixes per wave.
// Tiles go out in list order (ascending c: the longest streams first); a
// wave takes several consecutive tiles per cursor step when their streams
// are short, so that the cursor's atomic stays rare.
constexpr int kGrabIters = 2048;   // candidate rows worth one cursor step
constexpr int kMaxGrab = 16;

// Widest row at which the tile kernel is built for three waves per SIMD
// (wider: two, with the register room to hold its rows without spilling).
#ifndef PDFS_TILE3_MAX_W64
#define PDFS_TILE3_MAX_W64 16
#endif

// Depth-4 expansion of tile `it`: the listed prefixes it*64 .. it*64+63 (n
// listed in all), one per lane.
template <int W64>
__device__ __forceinline__ void tile_item(const Problem& P, const Work& w, RoundState* st,
                                          uint32_t it, unsigned long long n, int nA, uint32_t* zl,
                                          Best& best, Tally& tl, unsigned long long& inc,
                                          int lane) {
  constexpr int W = 2 * W64;
  constexpr bool kZL = W64 >= kZLdsMinW64;
  cu32* TA = (cu32*)w.TA;
  cu32* NA = (cu32*)w.NA;
  const unsigned long long t0 = (unsigned long long)it * kWave;
  bool valid = t0 + lane < n;
  const unsigned long long e = w.tri_s[valid ? t0 + lane : t0];
  int a3 = (int)(e & 0xffff);
  int b3 = (int)((e >> 16) & 0xffff);
  int c = (int)((e >> 32) & 0xffff);
  // listed entries always satisfy a < b < c < nA; anything else marks the
  // round corrupt and is never used as a row index
  if (valid && !(a3 < b3 && b3 < c && c < nA)) {
    st->overflow |= 2;
    valid = false;
  }
  if (!valid) a3 = b3 = c = 0;
  const uint32_t vmask = valid ? ~0u : 0u;
  uint32_t y3[W];
  NrmPre<kZL> z3;
  if constexpr (kZL) z3.s = zl;
#pragma unroll
  for (int k = 0; k < W; ++k)
    y3[k] = TA[(size_t)a3 * W + k] & TA[(size_t)b3 * W + k] & TA[(size_t)c * W + k] & vmask;
  uint32_t znz = 0;
#pragma unroll
  for (int k = 0; k < kMaxWN32; ++k) {
    const uint32_t z =
        nrm_join(nrm_join(NA[(size_t)a3 * kMaxWN32 + k], NA[(size_t)b3 * kMaxWN32 + k],
                          P.tn_literal),
                 NA[(size_t)c * kMaxWN32 + k], P.tn_literal) & vmask;
    z3.set(k, lane, z);
    znz |= z;
  }
  // visited at depth 4 below the prefix: sorted indices in (idx(c), G-1]
  if (valid) tl.vis4 += (unsigned long long)(P.G - 1 - w.act[c]);
  int cmin = valid ? c : 0x7fffffff;
  for (int o = 32; o > 0; o >>= 1) cmin = min(cmin, __shfl_xor(cmin, o, 64));
  expand4<W, false, kZL>(P, w, st, y3, z3, znz, valid, a3, b3, c, uniform(cmin), best, tl, inc);
}

template <int W64>
__global__ __launch_bounds__(256, (W64 <= PDFS_TILE3_MAX_W64 ? 3 : 2)) void k_dfs4_tiles(Problem P,
                                                                                        Work w) {
  constexpr bool kZL = W64 >= kZLdsMinW64;
  __shared__ uint32_t zbuf[kBlock / kWave][kZL ? kMaxWN32 * kWave : 1];
  RoundState* st = w.st;
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int wib = uniform(threadIdx.x >> 6);
  const unsigned long long n = st->n_tri < w.tri_cap ? st->n_tri : w.tri_cap;
  const uint32_t ntiles = (uint32_t)((n + kWave - 1) / kWave);
  const int nA = uniform(st->nA);

  Best best;
  best.init();
  Tally tl;
  tl.init();
  unsigned long long inc = 0;
  // Scheduling as in the depth-first walk: the tiles are split into
  // kSubQueues contiguous ranges with their own cursors; wave g takes its
  // first tile in range g % kSubQueues without an atomic, then grabs from
  // that range's cursor (as many tiles as make about kGrabIters candidate
  // rows: later tiles have shorter streams), then from the other ranges in
  // turn.
  const uint32_t nwaves = gridDim.x * (kBlock / kWave);
  const uint32_t gw = blockIdx.x * (kBlock / kWave) + wib;
  auto range_lo = [&](uint32_t r) {
    return (uint32_t)((unsigned long long)ntiles * r / kSubQueues);
  };
  auto range_waves = [&](uint32_t r) { return (nwaves + kSubQueues - 1 - r) / kSubQueues; };
  uint32_t qs = gw % kSubQueues;
  uint32_t q_left = kSubQueues;
  uint32_t t_next = range_lo(qs) + gw / kSubQueues;
  uint32_t t_end = t_next + 1;
  if (t_end > range_lo(qs + 1)) t_end = t_next;
  for (;;) {
    if (t_next >= t_end) {
      uint32_t start = 0, cnt = 0;
      while (q_left > 0) {
        const uint32_t hi = range_lo(qs + 1);
        const uint32_t base = range_lo(qs) + range_waves(qs);
        if (lane == 0) {
          unsigned long long* cur_p = w.cursors + (size_t)qs * kCursorStride;
          const unsigned long long cur =
              __hip_atomic_load(cur_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (base + cur < hi) {
            // stream length of the tile at the cursor: later tiles are shorter
            const int cp = (int)((w.tri_s[(base + cur) * kWave] >> 32) & 0xffff);
            const int len = nA - 1 - cp;
            int k = len > 0 ? kGrabIters / len : kMaxGrab;
            cnt = k < 1 ? 1u : (k > kMaxGrab ? (uint32_t)kMaxGrab : (uint32_t)k);
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
    const uint32_t it = t_next++;
    tile_item<W64>(P, w, st, it, n, nA, zbuf[wib], best, tl, inc, lane);
  }

  Slot sl = empty_slot();
  if (best.s >= 0) {
    sl.s = best.s; sl.tp = best.tp; sl.fp = best.fp;
    sl.idx[0] = best.idx(0); sl.idx[1] = best.idx(1); sl.idx[2] = best.idx(2); sl.idx[3] = best.idx(3);
  }
  block_best_to(&w.slots[(size_t)1 * kSlotsPerPhase + blockIdx.x], sl);
  unsigned long long v[kTallyN] = {0};
  if (lane == 0) {
    v[kTNe4] = tl.ne4;
    v[kTLeaves] = tl.ne4;
  }
  v[kTVis4] = tl.vis4;
  v[kTXv4] = tl.xv4;
  v[kTXfp] = tl.xfp;
  block_tally_to(w.tallies + ((size_t)1 * kPersistBlocks + blockIdx.x) * kTallyN, v);
  clear_absent_blocks(w, 1, true);
}

// The depth-4 tile step of a batched launch: one persistent grid drains the
// shared queue of every live instance's tiles, one tile per queue position
// (see k_dfs_multi for the per-instance hand-over).
template <int W64>
__global__ __launch_bounds__(256, (W64 <= PDFS_TILE3_MAX_W64 ? 3 : 2)) void k_dfs4_tiles_multi(
    const BatchDesc* __restrict__ bd, BatchQueue* __restrict__ bq) {
  constexpr bool kZL = W64 >= kZLdsMinW64;
  __shared__ uint32_t zbuf[kBlock / kWave][kZL ? kMaxWN32 * kWave : 1];
  const int lane = threadIdx.x & 63;
  const int wib = uniform(threadIdx.x >> 6);
  const uint32_t total = (uint32_t)uniform((int)bq->total);
  int cur = -1;
  uint32_t lo = 0, hi = 0;
  Problem P;
  Work w;
  RoundState* st = nullptr;
  unsigned long long n = 0;
  int nA = 0;
  Best best;
  Tally tl;
  unsigned long long inc = 0;
  auto flush = [&]() {
    Slot sl = empty_slot();
    if (best.s >= 0) {
      sl.s = best.s; sl.tp = best.tp; sl.fp = best.fp;
      sl.idx[0] = best.idx(0); sl.idx[1] = best.idx(1); sl.idx[2] = best.idx(2);
      sl.idx[3] = best.idx(3);
    }
    unsigned long long v[kTallyN] = {0};
    if (lane == 0) {
      v[kTNe4] = tl.ne4;
      v[kTLeaves] = tl.ne4;
    }
    v[kTVis4] = tl.vis4;
    v[kTXv4] = tl.xv4;
    v[kTXfp] = tl.xfp;
    wave_flush(w, st, 1, sl, v);
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
      int i = cur + 1;
      while ((uint32_t)uniform((int)bq->base[i + 1]) <= g) ++i;
      cur = i;
      lo = (uint32_t)uniform((int)bq->base[i]);
      hi = (uint32_t)uniform((int)bq->base[i + 1]);
      P = bd[i].P;
      w = bd[i].w;
      st = w.st;
      n = st->n_tri < w.tri_cap ? st->n_tri : w.tri_cap;
      nA = uniform(st->nA);
      best.init();
      tl.init();
      inc = 0;
    }
    tile_item<W64>(P, w, st, g - lo, n, nA, zbuf[wib], best, tl, inc, lane);
  }
  if (cur >= 0) flush();
}

// Blocks of a persistent kernel resident per compute unit, queried once.
template <typename K>
int resident(K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel),
                                                   kBlock, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu;
}

int grid_for(int per_cu, const Problem& P) {
  const int g = per_cu * (P.n_cu > 0 ? P.n_cu : 1);
  return g < kPersistBlocks ? g : kPersistBlocks;
}

template <int W64>
hipError_t launch_count_w(const Problem& P, const Work& w, hipStream_t s) {
  static const int per_cu = resident(&k_count_long<W64>);
  k_count_long<W64><<<grid_for(per_cu, P), kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

template <int W64>
hipError_t launch_tiles_w(const Problem& P, const Work& w, hipStream_t s) {
  static const int per_cu = resident(&k_dfs4_tiles<W64>);
  k_dfs4_tiles<W64><<<grid_for(per_cu, P), kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

template <int W64>
hipError_t launch_tiles_multi_w(const BatchDesc* bd, BatchQueue* bq, int n_cu, hipStream_t s) {
  static const int per_cu = resident(&k_dfs4_tiles_multi<W64>);
  int g = per_cu * (n_cu > 0 ? n_cu : 1);
  if (g > kPersistBlocks) g = kPersistBlocks;
  k_dfs4_tiles_multi<W64><<<g, kBlock, 0, s>>>(bd, bq);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tri_begin_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_tri_begin_m<<<dim3(64, n), kBlock, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_sort_triples_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_scan_c_m<<<dim3(1, n), 1024, 0, s>>>(bd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scatter_c_m<<<dim3(kPersistBlocks / 4, n), kBlock, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_dfs4_tiles_m(int w64, const BatchDesc* bd, BatchQueue* bq, int n_cu,
                               hipStream_t s) {
  switch (w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_tiles_multi_w<n>(bd, bq, n_cu, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_tri_begin(const Work& w, hipStream_t s) {
  k_tri_begin<<<64, kBlock, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_count_long(const Problem& P, const Work& w, hipStream_t s) {
  switch (w.w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_count_w<n>(P, w, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sort_triples(const Work& w, hipStream_t s) {
  k_scan_c<<<1, 1024, 0, s>>>(w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scatter_c<<<kPersistBlocks, kBlock, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_dfs4_tiles(const Problem& P, const Work& w, hipStream_t s) {
  switch (w.w64) {
#define PDFS_CASE(n) \
  case n:            \
    return launch_tiles_w<n>(P, w, s);
    PDFS_CASE(1) PDFS_CASE(2) PDFS_CASE(3) PDFS_CASE(4) PDFS_CASE(5) PDFS_CASE(6)
    PDFS_CASE(7) PDFS_CASE(8) PDFS_CASE(10) PDFS_CASE(12) PDFS_CASE(14) PDFS_CASE(16)
    PDFS_CASE(18) PDFS_CASE(20)
#undef PDFS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace pdfs
