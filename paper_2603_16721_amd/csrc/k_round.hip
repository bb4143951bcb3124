// Ingest and per-round kernels of the P-DFS / greedy-WSC path.
//
//  ingest (once per cohort, Sec. III-B): per-gene combined mutation counts,
//    stable counting sort -> sparsest-first order, gather of the sorted rows.
//  round begin / active / gather (Alg. 1 DelCols + Alg. 2 depth 1): the
//    uncovered sample list, the genes whose row meets it (a gene whose
//    depth-1 intersection is empty roots no combination with TP >= 1), and
//    the active rows re-packed over the uncovered columns only, so every
//    later intersection runs over ceil(|U|/64) words.
//  finish (Alg. 1 steps 4-7): exact (S desc, tuple asc) argmax over the
//    per-wave bests, the round record, and U <- U & ~cover(gamma*).
#include "pdfs_dev.h"
#include "slot_reduce.h"

namespace pdfs {

namespace {

// Argmax order of the round's slots: higher S first, then the smaller tuple
// over the first h indices.  Both the test and the update are written as
// straight-line selects over a fixed trip count: the index arrays stay in
// registers (a loop bounded by h indexes them at run time, which puts them in
// scratch memory), and no field of the slot is updated under a branch of its
// own (a short-circuit test with the copy under it was compiled into code
// that left the TP of the old slot beside the indices of the new one).
__device__ __forceinline__ bool slot_wins(const Slot& c, const Slot& b, int h) {
  bool lt = false, decided = false;
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) {
    const bool d = !decided & (i < h) & (c.idx[i] != b.idx[i]);
    lt = d ? (c.idx[i] < b.idx[i]) : lt;
    decided = decided | d;
  }
  return (c.s > b.s) | ((c.s == b.s) & (c.s >= 0) & lt);
}

__device__ __forceinline__ void take_if(Slot& b, const Slot& c, bool take) {
  b.s = take ? c.s : b.s;
  b.tp = take ? c.tp : b.tp;
  b.fp = take ? c.fp : b.fp;
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) b.idx[i] = take ? c.idx[i] : b.idx[i];
}

// ------------------------------------------------------------- ingest
__global__ void k_gene_counts(const uint64_t* __restrict__ T, int64_t ts,
                              const uint64_t* __restrict__ N, int64_t ns, int G, int wt, int wn,
                              uint32_t* __restrict__ counts) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  uint32_t c = 0;
  for (int w = 0; w < wt; ++w) c += __popcll(T[(size_t)g * ts + w]);
  if (N)
    for (int w = 0; w < wn; ++w) c += __popcll(N[(size_t)g * ns + w]);
  counts[g] = c;
}

// Sparsest-first order: a stable counting sort of the genes by their combined
// count (keys 0 .. n_tumor + n_normal), ties by caller index.  Gene g goes to
//   #{g' : key(g') < key(g)} + #{g' < g : key(g') = key(g)}.
// Genes are cut into tiles of kSortTile; a tile gives each of its genes the
// rank among the earlier genes of the tile with the same key, and its per-key
// counts; one exclusive scan over (key, tile) in key-major order then gives
// the first position of every (key, tile) group.
constexpr int kSortTile = 256;

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One block per tile.  tile_hist [ntiles][nkeys] must be zero.
__global__ __launch_bounds__(kSortTile) void k_sort_tile_ranks(const uint32_t* __restrict__ counts,
                                                               int G, int nkeys,
                                                               uint32_t* __restrict__ tile_hist,
                                                               uint32_t* __restrict__ rank) {
  __shared__ uint32_t key[kSortTile];
  const int i = threadIdx.x;
  const int g = blockIdx.x * kSortTile + i;
  const uint32_t k = g < G ? counts[g] : 0xffffffffu;
  key[i] = k;
  __syncthreads();
  if (g >= G) return;
  uint32_t r = 0;
  bool last = true;
  for (int j = 0; j < kSortTile; ++j) {
    const bool same = key[j] == k;
    r += (same && j < i) ? 1u : 0u;
    last = last && !(same && j > i);
  }
  rank[g] = r;
  if (last) tile_hist[(size_t)blockIdx.x * nkeys + k] = r + 1;
}

// One block: tile_hist[t][k] <- first position of the genes of tile t with
// key k (exclusive scan in the order k major, t minor).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ tile_hist, int nkeys,
                                                    int ntiles) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  const size_t n = (size_t)nkeys * ntiles;
  const size_t per = (n + 1023) / 1024;
  const size_t lo = (size_t)tid * per < n ? (size_t)tid * per : n;
  const size_t hi = lo + per < n ? lo + per : n;
  auto at = [&](size_t e) -> uint32_t& {
    return tile_hist[(e % (size_t)ntiles) * nkeys + e / (size_t)ntiles];
  };
  uint32_t sum = 0;
  for (size_t e = lo; e < hi; ++e) sum += at(e);
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t add = tid >= o ? part[tid - o] : 0u;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  uint32_t run = part[tid] - sum;
  for (size_t e = lo; e < hi; ++e) {
    const uint32_t x = at(e);
    at(e) = run;
    run += x;
  }
}

__global__ void k_sort_scatter(const uint32_t* __restrict__ counts,
                               const uint32_t* __restrict__ rank,
                               const uint32_t* __restrict__ tile_first, int G, int nkeys,
                               int32_t* __restrict__ perm) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const uint32_t pos = tile_first[(size_t)(g / kSortTile) * nkeys + counts[g]] + rank[g];
  perm[pos] = g;
}

__global__ void k_gather_sorted(const uint64_t* __restrict__ T, int64_t ts,
                                const uint64_t* __restrict__ N, int64_t ns,
                                const int32_t* __restrict__ perm, int G, int wt, int wn,
                                uint64_t* __restrict__ Ts, uint64_t* __restrict__ Ns) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G) return;
  int g = perm[i];
  for (int w = 0; w < wt; ++w) Ts[(size_t)i * wt + w] = T[(size_t)g * ts + w];
  for (int w = 0; w < wn; ++w) Ns[(size_t)i * wn + w] = N ? N[(size_t)g * ns + w] : 0ull;
}

// Normals carrying each sorted gene (rows are fixed for the cohort).
__global__ void k_normal_counts(const uint64_t* __restrict__ Ns, int G, int wn, int32_t* ncount) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int c = 0;
  for (int k = 0; k < wn; ++k) c += __popcll(Ns[(size_t)g * wn + k]);
  ncount[g] = c;
}

__global__ void k_check_pad(const uint64_t* __restrict__ T, int64_t ts, int G, int n,
                            int* __restrict__ bad) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G || (n & 63) == 0) return;
  int last = n >> 6;
  uint64_t pad = ~0ull << (n & 63);
  if (T[(size_t)g * ts + last] & pad) atomicOr(bad, 1);
}

__global__ void k_fill_u(uint64_t* U, int wt, int n) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= wt) return;
  int lo = w * 64;
  uint64_t v = 0;
  if (n - lo >= 64) v = ~0ull;
  else if (n > lo) v = (1ull << (n - lo)) - 1;
  U[w] = v;
}

// ------------------------------------------------------------- round begin
// One block of 64 threads: uncovered sample list and state reset.
__device__ __forceinline__ void round_begin_body(const Problem& P, const Work& w) {
  RoundState* st = w.st;
  if (st->done) return;   // rounds queued past the stop are no-ops
  const int lane = threadIdx.x;
  int base = 0;
  for (int w0 = 0; w0 < P.wt; w0 += 64) {
    int wi = w0 + lane;
    uint64_t word = wi < P.wt ? w.U[wi] : 0ull;
    int c = __popcll(word);
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    int off = base + incl - c;
    while (word) {
      int bit = __ffsll((unsigned long long)word) - 1;
      w.cols[off++] = wi * 64 + bit;
      word &= word - 1;
    }
    base += __shfl(incl, 63, 64);
  }
  if (lane == 0) {
    st->n_unc = base;
    st->nA = 0;
    st->found = 0;
    st->n_pairs = 0;
    st->n_work_pairs = 0;
    st->n_items = 0;
    st->cursor = 0;
    st->incumbent = 0;
    st->n_seed = 0;
    st->seed_t = 0;
    // overflow stays set for the rest of the run (cleared at run start)
    st->x_vis3 = st->x_vis4 = st->x_leaves = st->x_fp_leaves = 0;
  }
  for (int v = lane; v <= kMaxCount; v += 64) w.hist[v] = 0u;
  for (int l = lane; l <= kMaxH; l += 64) {
    st->amax[l] = 0;
    st->cnt.visited[l] = 0;
    st->cnt.nonempty[l] = 0;
    st->cnt.bound_pruned[l] = 0;
  }
}

__global__ void k_round_begin(Problem P, Work w) {
  round_begin_body(P, w);
}

__global__ void k_round_begin_m(const BatchDesc* __restrict__ bd) {
  round_begin_body(bd[blockIdx.y].P, bd[blockIdx.y].w);
}

// ------------------------------------------------------------- active genes
__device__ __forceinline__ void active_flags_body(const Problem& P, const Work& w) {
  if (w.st->done) return;
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P.G) return;
  uint64_t acc = 0;
  const uint64_t* row = w.Ts + (size_t)g * P.wt;
  for (int k = 0; k < P.wt; ++k) acc |= row[k] & w.U[k];
  // 1: the gene meets U; 2: it does not, but exhaustive mode walks it anyway
  w.flags[g] = acc != 0 ? 1 : (P.mode == kPruneNone ? 2 : 0);
}

__global__ void k_active_flags(Problem P, Work w) {
  active_flags_body(P, w);
}

__global__ void k_active_flags_m(const BatchDesc* __restrict__ bd) {
  active_flags_body(bd[blockIdx.y].P, bd[blockIdx.y].w);
}

// One block of 1024 threads: ordered compaction of the active flags, the
// per-depth limits amax[l] and the depth-1/2 counters (Alg. 2 loop bounds:
// depth l takes sorted indices up to G-h+l-1).  Thread t owns one contiguous
// range of genes, so one block-wide scan orders the whole list (a sweep of
// 1024-gene chunks would wait on a load and two barriers per chunk).
__device__ __forceinline__ void active_scan_body(const Problem& P, const Work& w) {
  __shared__ int wsum[16];
  __shared__ unsigned long long vsum[16];
  __shared__ int nsum[16];
  RoundState* st = w.st;
  if (st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int h = P.h;
  const int per = (P.G + 1023) >> 10;
  const int g_lo = min(tid * per, P.G), g_hi = min(g_lo + per, P.G);
  int mine = 0;
#pragma unroll 8
  for (int g = g_lo; g < g_hi; ++g) mine += w.flags[g] != 0;
  int incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(incl, o, 64);
    if (lane >= o) incl += x;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int off = 0, base = 0;   // genes before this wave's; all active genes
  for (int i = 0; i < 16; ++i) {
    off += (i < wid) ? wsum[i] : 0;
    base += wsum[i];
  }
  int pos = off + incl - mine;
  unsigned long long vis2 = 0;
  int ne1 = 0;   // genes meeting U within the depth-1 bound
#pragma unroll 8
  for (int g = g_lo; g < g_hi; ++g) {
    const int f = w.flags[g];
    if (f) {
      w.act[pos++] = g;
      if (h >= 2 && g <= P.G - h) vis2 += (unsigned long long)(P.G - h + 1 - g);
      if (f == 1 && g <= P.G - h) ++ne1;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    vis2 += __shfl_xor(vis2, o, 64);
    ne1 += __shfl_xor(ne1, o, 64);
  }
  if (lane == 0) {
    vsum[wid] = vis2;
    nsum[wid] = ne1;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long v = 0;
    int n1 = 0;
    for (int i = 0; i < 16; ++i) {
      v += vsum[i];
      n1 += nsum[i];
    }
    st->nA = base;
    st->cnt.visited[1] = (unsigned long long)(P.G - h + 1);
    st->cnt.nonempty[1] = (unsigned long long)n1;
    if (h >= 2) st->cnt.visited[2] = v;
  }
  // amax[l] = number of active genes with sorted index <= G-h+l-1: all of
  // them but those at the h-l highest indices
  if (tid >= 1 && tid <= h) {
    int above = 0;
    for (int g = max(P.G - h + tid, 0); g < P.G; ++g) above += w.flags[g] != 0;
    st->amax[tid] = base - above;
  }
}

__global__ __launch_bounds__(1024) void k_active_scan(Problem P, Work w) {
  active_scan_body(P, w);
}

__global__ __launch_bounds__(1024) void k_active_scan_m(const BatchDesc* __restrict__ bd) {
  active_scan_body(bd[blockIdx.y].P, bd[blockIdx.y].w);
}

// One wave per active gene: the row over the uncovered columns (the paper's
// DelCols done physically), the normal row, and optionally 0/1 bytes for the
// int8 MFMA pair table.
__device__ __forceinline__ void gather_active_body(const Problem& P, const Work& w, int unpack_t, int unpack_n) {
  const RoundState* st = w.st;
  if (st->done) return;
  const int nA = st->nA, n_unc = st->n_unc;
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (blockDim.x >> 6);
  const int W32 = 2 * w.w64;
  const int kpad = unpacked_row_bytes(w.w64);
  const int knpad = unpacked_row_bytes(P.wn);
  const uint32_t* Ns32 = reinterpret_cast<const uint32_t*>(w.Ns);
  for (int a = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); a < nA; a += waves) {
    const int g = w.act[a];
    const uint64_t* row = w.Ts + (size_t)g * P.wt;
    for (int k0 = 0; k0 < 64 * w.w64; k0 += 64) {
      int k = k0 + lane;
      int bit = 0;
      if (k < n_unc) {
        int s = w.cols[k];
        bit = (int)((row[s >> 6] >> (s & 63)) & 1ull);
      }
      unsigned long long word = __ballot(bit);
      if (lane < 2) w.TA[(size_t)a * W32 + (k0 >> 5) + lane] = (uint32_t)(word >> (32 * lane));
      if (unpack_t) w.A8[(size_t)a * kpad + k] = (int8_t)bit;
    }
    if (unpack_t)
      for (int k = 64 * w.w64 + lane; k < kpad; k += 64) w.A8[(size_t)a * kpad + k] = 0;
    if (lane < kMaxWN32)
      w.NA[(size_t)a * kMaxWN32 + lane] = lane < 2 * P.wn ? Ns32[(size_t)g * 2 * P.wn + lane] : 0u;
    if (unpack_n) {
      const uint64_t* nrow = w.Ns + (size_t)g * P.wn;
      for (int k = lane; k < knpad; k += 64)
        w.N8[(size_t)a * knpad + k] =
            k < 64 * P.wn ? (int8_t)((nrow[k >> 6] >> (k & 63)) & 1ull) : (int8_t)0;
    }
  }
}

__global__ __launch_bounds__(256) void k_gather_active(Problem P, Work w, int unpack_t,
                                                       int unpack_n) {
  gather_active_body(P, w, unpack_t, unpack_n);
}

__global__ __launch_bounds__(256) void k_gather_active_m(const BatchDesc* __restrict__ bd, int unpack_t, int unpack_n) {
  gather_active_body(bd[blockIdx.y].P, bd[blockIdx.y].w, unpack_t, unpack_n);
}

// ------------------------------------------------------------- h = 1
// Every active gene is a leaf: S = p*|T_g & U| + q*(N_n - |N_g|).
__global__ __launch_bounds__(256) void k_h1(Problem P, Work w) {
  const RoundState* st = w.st;
  if (st->done) return;
  const int nA = st->nA;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int W32 = 2 * w.w64;
  int bs = -1, btp = 0, bfp = 0, bi = 0;
  for (int a = gw * 64 + lane; a < nA; a += kWavesPerGrid * 64) {
    int tp = 0, fp = 0;
    for (int k = 0; k < W32; ++k) tp += __popc(w.TA[(size_t)a * W32 + k]);
    for (int k = 0; k < kMaxWN32; ++k) fp += __popc(w.NA[(size_t)a * kMaxWN32 + k]);
    int s = P.p * tp + P.q * (P.n_normal - fp);
    // one mask for every field (straight-line selects, as in the slot argmax)
    const bool take = (tp > 0) & ((s > bs) | ((s == bs) & (a < bi)));
    bs = take ? s : bs;
    btp = take ? tp : btp;
    bfp = take ? fp : bfp;
    bi = take ? a : bi;
  }
  Slot sl = empty_slot();
  if (bs >= 0) { sl.s = bs; sl.tp = btp; sl.fp = bfp; sl.idx[0] = bi; }
  block_best_to(&w.slots[blockIdx.x], sl);
  if (gw == 0 && lane == 0) w.st->cnt.visited[1] = (unsigned long long)P.G;
}

__global__ void k_clear_slots(Slot* slots, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  slots[i] = empty_slot();
}

// ------------------------------------------------------------- finish
// One block: argmax over the slots of the phases used this round, the round
// record, and the cover update U <- U & ~(U & T_g1 & ... & T_gh).
__device__ __forceinline__ void finish_round_body(const Problem& P, const Work& w, int phase_mask,
                                                  int tally_mask) {
  // batched launches (h >= 3) pass -1: the instance's own phases -- the seed
  // walk (bound mode) or the depth-4 tiles (two-phase) in phase 1, the main
  // walk in phase 2, the pair table's counts in row 0
  if (phase_mask < 0) {
    const bool two = P.mode == kPruneBound || (P.h == 4 && P.mode == kPruneEmpty && w.tri_cap > 0);
    phase_mask = two ? 6 : 4;
    tally_mask = two ? 7 : 5;
  }
  __shared__ Slot red[16];
  __shared__ int s_found;
  __shared__ Slot s_best;
  __shared__ int32_t s_sidx[kMaxH];
  __shared__ int32_t s_gene[kMaxH];
  __shared__ unsigned long long tsum[16][kTallyN];
  RoundState* st = w.st;
  if (st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int h = P.h;
  // a round whose lists overflowed is incomplete: it is not committed and the
  // run stops (the host reports the overflow)
  if (st->overflow) {
    if (tid == 0) st->done = 1;
    return;
  }
  {
    // per-block counter rows of the kernels that ran this round; thread t
    // always reads field t % kTallyN, so the reads are contiguous
    static_assert(1024 % kTallyN == 0, "tally rows must tile the block");
    constexpr int kIter = kPersistBlocks * kTallyN / 1024;
    unsigned long long v = 0;
    for (int ph = 0; ph < kSlotPhases; ++ph) {
      if (!((tally_mask >> ph) & 1)) continue;
      const unsigned long long* base = w.tallies + (size_t)ph * kPersistBlocks * kTallyN + tid;
      unsigned long long part[kIter];
#pragma unroll
      for (int i = 0; i < kIter; ++i) part[i] = base[(size_t)i * 1024];   // all loads in flight
#pragma unroll
      for (int i = 0; i < kIter; ++i) v += part[i];
    }
    // lanes l and l + 16, l + 32, l + 48 of a wave hold the same field
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < kTallyN) tsum[wid][lane] = v;
    __syncthreads();
    if (tid < kTallyN) {
      unsigned long long x = 0;
      for (int i = 0; i < 16; ++i) x += tsum[i][tid];
      switch (tid) {
        case kTNe2: st->cnt.nonempty[2] += x; break;
        case kTVis3: st->cnt.visited[3] += x; break;
        case kTNe3: st->cnt.nonempty[3] += x; break;
        case kTNe4: st->cnt.nonempty[4] += x; break;
        case kTVis4: st->cnt.visited[4] += x; break;
        case kTBp2: st->cnt.bound_pruned[2] += x; break;
        case kTBp3: st->cnt.bound_pruned[3] += x; break;
        case kTXv3: st->x_vis3 += x; break;
        case kTXv4: st->x_vis4 += x; break;
        case kTXfp: st->x_fp_leaves += x; break;
        case kTLeaves: st->x_leaves += x; break;
        default: break;
      }
    }
    __syncthreads();
  }
  Slot b;
  b.s = -1; b.tp = b.fp = 0;
  for (int i = 0; i < kMaxH; ++i) b.idx[i] = 0;
  for (int ph = 0; ph < kSlotPhases; ++ph) {
    if (!((phase_mask >> ph) & 1)) continue;
    // a context's own launches leave one slot per block; a batched launch
    // leaves the log of the waves that worked on this instance
    const Slot* src = w.slot_log ? w.slot_log + (size_t)ph * kLogCap
                                 : w.slots + (size_t)ph * kSlotsPerPhase;
    const int n = w.slot_log ? min((int)st->nlog[ph], kLogCap) : kSlotsPerPhase;
    for (int i = tid; i < n; i += 1024) {
      Slot c = src[i];
      take_if(b, c, slot_wins(c, b, h));
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    Slot c;
    c.s = __shfl_xor(b.s, o, 64);
    c.tp = __shfl_xor(b.tp, o, 64);
    c.fp = __shfl_xor(b.fp, o, 64);
    for (int i = 0; i < kMaxH; ++i) c.idx[i] = __shfl_xor(b.idx[i], o, 64);
    take_if(b, c, slot_wins(c, b, h));
  }
  if (lane == 0) red[wid] = b;
  __syncthreads();
  // The tail is a chain of small global reads and writes; they are spread
  // over threads (one per chosen gene, one per depth) instead of one thread.
  if (tid == 0) {
    for (int i = 1; i < 16; ++i) {
      Slot c = red[i];
      take_if(b, c, slot_wins(c, b, h));
    }
    int ok = b.s >= 0;
    if (ok) {
      // a slot index outside the active list would mean a corrupt slot
      const int nA = st->nA;
#pragma unroll
      for (int i = 0; i < kMaxH; ++i)
        if (i < h && (b.idx[i] < 0 || b.idx[i] >= nA || (i > 0 && b.idx[i] <= b.idx[i - 1])))
          ok = 0;
      if (b.tp <= 0) ok = 0;
      if (!ok) st->overflow |= 2;
    }
    s_best = b;
    s_found = ok;
  }
  __syncthreads();
  b = s_best;
  const int found = s_found;
  if (found && tid < h) {
    const int si = w.act[s_best.idx[tid]];
    s_sidx[tid] = si;
    s_gene[tid] = w.perm[si];
  }
  // whole-run totals per depth (this round's counters are final here)
  if (tid >= 64 && tid <= 64 + kMaxH) {
    const int l = tid - 64;
    st->tot.visited[l] += st->cnt.visited[l];
    st->tot.nonempty[l] += st->cnt.nonempty[l];
    st->tot.bound_pruned[l] += st->cnt.bound_pruned[l];
  }
  __syncthreads();
  if (tid == 0) {
    RoundRecord r;
    r.h = h;
    r.found = found;
    for (int i = 0; i < kMaxH; ++i) {
      r.sorted_idx[i] = (found && i < h) ? s_sidx[i] : -1;
      r.genes[i] = (found && i < h) ? s_gene[i] : -1;
    }
    r.tp = found ? b.tp : 0;
    r.fp = found ? b.fp : 0;
    r.tn = found ? P.n_normal - b.fp : 0;
    r.uncovered_before = st->n_unc;
    r.score_num = found ? (int64_t)P.p * b.tp + (int64_t)P.q * r.tn : 0;
    r.score_den = (int64_t)P.q * (int64_t)(st->n_unc + P.n_normal);
    st->found = found;
    if (found && st->rounds < w.rec_cap) w.recs[st->rounds] = r;
  }
  if (found && tid < P.wt) {
    uint64_t cov = w.U[tid];
    for (int i = 0; i < h; ++i) cov &= w.Ts[(size_t)s_sidx[i] * P.wt + tid];
    w.U[tid] &= ~cov;
  }
  if (tid == 0) {
    int cov = (P.n_tumor - st->n_unc) + (found ? b.tp : 0);
    st->covered = cov;
    st->rounds += found ? 1 : 0;
    st->executed += 1;
    const unsigned long long wu = (unsigned long long)((st->n_unc + 63) / 64);
    st->tx_vis3 += st->x_vis3;
    st->tx_vis4 += st->x_vis4;
    st->tx_vis_words3 += st->x_vis3 * wu;
    st->tx_vis_words4 += st->x_vis4 * wu;
    st->tx_leaves += st->x_leaves;
    st->tx_fp_leaves += st->x_fp_leaves;
    if (h >= 2) {
      // every active pair inside the depth-1/2 loop bounds, times |U|
      const unsigned long long a1 = (unsigned long long)st->amax[1];
      const unsigned long long a2 = (unsigned long long)st->amax[2];
      const unsigned long long pairs = a1 ? a1 * a2 - a1 * (a1 + 1) / 2 : 0;
      st->tx_pair_macs += pairs * (unsigned long long)st->n_unc;
    }
    st->done = (!s_found) || cov >= w.target || cov >= P.n_tumor ||
               (st->max_rounds > 0 && st->rounds >= st->max_rounds);
  }
}

__global__ __launch_bounds__(1024) void k_finish_round(Problem P, Work w, int phase_mask,
                                                      int tally_mask) {
  finish_round_body(P, w, phase_mask, tally_mask);
}

__global__ __launch_bounds__(1024) void k_finish_round_m(const BatchDesc* __restrict__ bd, int phase_mask, int tally_mask) {
  finish_round_body(bd[blockIdx.y].P, bd[blockIdx.y].w, phase_mask, tally_mask);
}

// Whole-run state: nothing done yet, totals cleared, the covered count of the
// starting mask.
__device__ __forceinline__ void run_begin_body(const Problem& P, const Work& w, int max_rounds) {
  RoundState* st = w.st;
  const int lane = threadIdx.x;
  int c = 0;
  for (int k = lane; k < P.wt; k += 64) c += __popcll(w.U[k]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) {
    st->done = (P.n_tumor - c) >= w.target || c == 0;
    st->rounds = 0;
    st->executed = 0;
    st->max_rounds = max_rounds;
    st->covered = P.n_tumor - c;
    st->n_unc = c;
    st->tx_vis3 = st->tx_vis4 = st->tx_leaves = st->tx_fp_leaves = st->tx_pair_macs = 0;
    st->tx_vis_words3 = st->tx_vis_words4 = 0;
    // nothing of an earlier run (a failed one included) carries over
    st->overflow = 0;
    st->found = 0;
    st->n_tri = 0;
  }
  for (int l = lane; l <= kMaxH; l += 64) {
    st->tot.visited[l] = 0;
    st->tot.nonempty[l] = 0;
    st->tot.bound_pruned[l] = 0;
  }
}

// After the host grew a list the stopped round overflowed: the run goes on
// from the same state (that round was not committed).
__global__ void k_run_resume(Work w) {
  if (threadIdx.x == 0) {
    w.st->overflow = 0;
    w.st->done = 0;
  }
}

__global__ void k_run_begin(Problem P, Work w, int max_rounds) {
  run_begin_body(P, w, max_rounds);
}

__global__ void k_run_begin_m(const BatchDesc* __restrict__ bd, int max_rounds) {
  run_begin_body(bd[blockIdx.y].P, bd[blockIdx.y].w, max_rounds);
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_gene_counts(const uint64_t* T, int64_t ts, const uint64_t* N, int64_t ns,
                              int G, int wt, int wn, uint32_t* counts, hipStream_t s) {
  k_gene_counts<<<(G + 255) / 256, 256, 0, s>>>(T, ts, N, ns, G, wt, wn, counts);
  return hipGetLastError();
}

size_t sort_tmp_words(int G, int max_key) {
  const size_t ntiles = (size_t)(G + kSortTile - 1) / kSortTile;
  return (size_t)G + ntiles * (size_t)(max_key + 1);
}

hipError_t sort_genes(const uint32_t* counts, int G, int max_key, uint32_t* tmp, int32_t* perm,
                      hipStream_t s) {
  const int ntiles = (G + kSortTile - 1) / kSortTile;
  const int nkeys = max_key + 1;
  uint32_t* rank = tmp;
  uint32_t* tile_hist = tmp + G;
  const size_t nh = (size_t)ntiles * nkeys;
  k_fill_u32<<<(int)((nh + 255) / 256 < 1024 ? (nh + 255) / 256 : 1024), 256, 0, s>>>(tile_hist,
                                                                                     nh, 0u);
  k_sort_tile_ranks<<<ntiles, kSortTile, 0, s>>>(counts, G, nkeys, tile_hist, rank);
  k_sort_scan<<<1, 1024, 0, s>>>(tile_hist, nkeys, ntiles);
  k_sort_scatter<<<(G + 255) / 256, 256, 0, s>>>(counts, rank, tile_hist, G, nkeys, perm);
  return hipGetLastError();
}

hipError_t launch_gather_sorted(const uint64_t* T, int64_t ts, const uint64_t* N, int64_t ns,
                                const int32_t* perm, int G, int wt, int wn, uint64_t* Ts,
                                uint64_t* Ns, hipStream_t s) {
  k_gather_sorted<<<(G + 255) / 256, 256, 0, s>>>(T, ts, N, ns, perm, G, wt, wn, Ts, Ns);
  return hipGetLastError();
}

hipError_t launch_normal_counts(const uint64_t* Ns, int G, int wn, int32_t* ncount,
                                hipStream_t s) {
  k_normal_counts<<<(G + 255) / 256, 256, 0, s>>>(Ns, G, wn, ncount);
  return hipGetLastError();
}

hipError_t launch_check_pad(const uint64_t* T, int64_t ts, int G, int n, int* bad,
                            hipStream_t s) {
  k_check_pad<<<(G + 255) / 256, 256, 0, s>>>(T, ts, G, n, bad);
  return hipGetLastError();
}

hipError_t launch_run_resume(const Work& w, hipStream_t s) {
  k_run_resume<<<1, 64, 0, s>>>(w);
  return hipGetLastError();
}

hipError_t launch_run_begin(const Problem& P, const Work& w, int max_rounds, hipStream_t s) {
  k_run_begin<<<1, 64, 0, s>>>(P, w, max_rounds);
  return hipGetLastError();
}

hipError_t launch_zero_u32(void* p, size_t n32, hipStream_t s) {
  if (n32 == 0) return hipSuccess;
  const size_t blocks = (n32 + 255) / 256;
  k_fill_u32<<<(int)(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(static_cast<uint32_t*>(p), n32,
                                                                  0u);
  return hipGetLastError();
}

hipError_t launch_fill_u(uint64_t* U, int wt, int n, hipStream_t s) {
  k_fill_u<<<(wt + 63) / 64, 64, 0, s>>>(U, wt, n);
  return hipGetLastError();
}

hipError_t launch_round_begin(const Problem& P, const Work& w, hipStream_t s) {
  k_round_begin<<<1, 64, 0, s>>>(P, w);
  return hipGetLastError();
}

hipError_t launch_active(const Problem& P, const Work& w, hipStream_t s) {
  k_active_flags<<<(P.G + 255) / 256, 256, 0, s>>>(P, w);
  k_active_scan<<<1, 1024, 0, s>>>(P, w);
  return hipGetLastError();
}

hipError_t launch_gather_active(const Problem& P, const Work& w, bool unpack_tumor,
                                bool unpack_normal, hipStream_t s) {
  int blocks = (P.G + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  k_gather_active<<<blocks, 256, 0, s>>>(P, w, unpack_tumor ? 1 : 0, unpack_normal ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_h1(const Problem& P, const Work& w, hipStream_t s) {
  k_h1<<<kPersistBlocks, kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

hipError_t launch_finish_round(const Problem& P, const Work& w, int phase_mask, int tally_mask,
                               hipStream_t s) {
  k_finish_round<<<1, 1024, 0, s>>>(P, w, phase_mask, tally_mask);
  return hipGetLastError();
}

// ---- batched launches: one block row per instance (blockIdx.y)
hipError_t launch_run_begin_m(const BatchDesc* bd, int n, int max_rounds, hipStream_t s) {
  k_run_begin_m<<<dim3(1, n), 64, 0, s>>>(bd, max_rounds);
  return hipGetLastError();
}

hipError_t launch_round_begin_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_round_begin_m<<<dim3(1, n), 64, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_active_m(const BatchDesc* bd, int n, int max_G, hipStream_t s) {
  k_active_flags_m<<<dim3((max_G + 255) / 256, n), 256, 0, s>>>(bd);
  k_active_scan_m<<<dim3(1, n), 1024, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_gather_active_m(const BatchDesc* bd, int n, int max_G, hipStream_t s) {
  int blocks = (max_G + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  k_gather_active_m<<<dim3(blocks, n), 256, 0, s>>>(bd, 1, 0);
  return hipGetLastError();
}

hipError_t launch_finish_round_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_finish_round_m<<<dim3(1, n), 1024, 0, s>>>(bd, -1, -1);
  return hipGetLastError();
}

hipError_t launch_clear_slots(Slot* slots, int n, hipStream_t s) {
  k_clear_slots<<<(n + 255) / 256, 256, 0, s>>>(slots, n);
  return hipGetLastError();
}

}  // namespace pdfs
