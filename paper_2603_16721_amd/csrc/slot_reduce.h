// Exact (S desc, tuple asc) argmax of per-lane candidates: wave shuffles,
// then one slot per block.  Device code only.
#pragma once
#include "pdfs_dev.h"

namespace pdfs {

// The test and the update are straight-line selects: no field of a slot is
// copied under a branch of its own, so every field of the winner moves
// together.
__device__ __forceinline__ bool slot_better(const Slot& c, const Slot& b) {
  bool lt = false, decided = false;
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) {
    const bool d = !decided & (c.idx[i] != b.idx[i]);
    lt = d ? (c.idx[i] < b.idx[i]) : lt;
    decided = decided | d;
  }
  return (c.s > b.s) | ((c.s == b.s) & (c.s >= 0) & lt);
}

__device__ __forceinline__ void slot_take_if(Slot& b, const Slot& c, bool take) {
  b.s = take ? c.s : b.s;
  b.tp = take ? c.tp : b.tp;
  b.fp = take ? c.fp : b.fp;
#pragma unroll
  for (int i = 0; i < kMaxH; ++i) b.idx[i] = take ? c.idx[i] : b.idx[i];
}

__device__ __forceinline__ Slot empty_slot() {
  Slot e;
  e.s = -1; e.tp = e.fp = 0;
  for (int i = 0; i < kMaxH; ++i) e.idx[i] = 0;
  return e;
}

__device__ __forceinline__ Slot wave_best(Slot b) {
  for (int o = 32; o > 0; o >>= 1) {
    Slot c;
    c.s = __shfl_xor(b.s, o, 64);
    c.tp = __shfl_xor(b.tp, o, 64);
    c.fp = __shfl_xor(b.fp, o, 64);
    for (int i = 0; i < kMaxH; ++i) c.idx[i] = __shfl_xor(b.idx[i], o, 64);
    slot_take_if(b, c, slot_better(c, b));
  }
  return b;
}

constexpr int kMaxBlockWaves = 16;   // blocks of up to 1024 threads

// Every thread of the block calls this once; thread 0 writes the block's best.
__device__ __forceinline__ void block_best_to(Slot* dst, Slot b) {
  __shared__ Slot red[kMaxBlockWaves];
  b = wave_best(b);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    Slot r = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
      slot_take_if(r, red[i], slot_better(red[i], r));
    *dst = r;
  }
}

// Sums per-lane counters over the block; thread 0 writes the block's row.
// vals: kTallyN values per thread (lanes may hold partial counts).
__device__ __forceinline__ void block_tally_to(unsigned long long* row,
                                               unsigned long long (&vals)[kTallyN]) {
  __shared__ unsigned long long red[kMaxBlockWaves][kTallyN];
  for (int f = 0; f < kTallyN; ++f) {
    unsigned long long v = vals[f];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    vals[f] = v;
  }
  if ((threadIdx.x & 63) == 0)
    for (int f = 0; f < kTallyN; ++f) red[threadIdx.x >> 6][f] = vals[f];
  __syncthreads();
  if (threadIdx.x < kTallyN) {
    unsigned long long v = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) v += red[i][threadIdx.x];
    row[threadIdx.x] = v;
  }
}

// Batched launches: a wave leaving an instance sends its best leaf (if any) to
// the instance's log of the phase and adds its counts to the instance's
// counter row of the phase (row 0; the other rows stay zero).  vals: as for
// block_tally_to.
__device__ __forceinline__ void wave_flush(const Work& w, RoundState* st, int phase, Slot b,
                                           unsigned long long (&vals)[kTallyN]) {
  b = wave_best(b);
  for (int f = 0; f < kTallyN; ++f) {
    unsigned long long v = vals[f];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    vals[f] = v;
  }
  if ((threadIdx.x & 63) == 0) {
    if (b.s >= 0) {
      const uint32_t pos = atomicAdd(&st->nlog[phase], 1u);
      if (pos < (uint32_t)kLogCap) w.slot_log[(size_t)phase * kLogCap + pos] = b;
      else atomicOr(&st->overflow, 1);
    }
    unsigned long long* row = w.tallies + (size_t)phase * kPersistBlocks * kTallyN;
    for (int f = 0; f < kTallyN; ++f)
      if (vals[f]) atomicAdd(&row[f], vals[f]);
  }
}

}  // namespace pdfs
