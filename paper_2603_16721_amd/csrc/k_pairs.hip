// Pairwise co-occurrence table on the int8 matrix cores.
//
// The depth-2 level of the search (the lambda level of Fig. 4 / Sec. III-D:
// every pair g1 < g2) needs |y2| = |U & x_g1 & x_g2| for all pairs of active
// genes.  Over 0/1 bytes that is the Gram matrix C = A * A^T with A the active
// tumour rows restricted to uncovered samples -- a genuinely dense
// contraction, so it runs on v_mfma_i32_32x32x32_i8 with int32 accumulation.
//
//  h = 2: the table is the answer.  With the normal Gram matrix FP = B * B^T
//         in the same pass, each pair with C > 0 is scored
//         S = p*C + q*(N_n - FP) and the wave keeps its best.
//  h > 2: the epilogue emits every pair with C > 0 inside Alg. 2's loop
//         bounds as a 64-bit record (a | b<<16 | C<<32); these are the
//         subtrees the depth-first kernels expand.
//
// Tiles: one wave computes one 32x32 block (ti <= tj, upper triangle only).
// Operand fragments are read straight from the unpacked rows (L2 resident);
// A and B use the same byte-to-k assignment, so the sum over k is the full
// dot product whatever that assignment is.  Output element r of lane l is
// row 8*(r/4) + 4*(l/32) + r%4, column l%32 of the block.
#include "pdfs_dev.h"

namespace pdfs {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void decode_tile(long long t, int T, int& ti, int& tj) {
  // t enumerates (ti, tj), ti <= tj, row by row: row ti holds T - ti tiles.
  // start(ti) = ti*T - ti*(ti-1)/2.
  double Td = (double)T + 0.5;
  int r = (int)(Td - sqrt(Td * Td - 2.0 * (double)t));
  if (r < 0) r = 0;
  if (r > T - 1) r = T - 1;
  auto start = [&](long long x) { return x * T - x * (x - 1) / 2; };
  while (r > 0 && start(r) > t) --r;
  while (r + 1 < T && start(r + 1) <= t) ++r;
  ti = r;
  tj = r + (int)(t - start(r));
}

template <bool kH2>
__global__ __launch_bounds__(256) void k_pairs(Problem P, Work w) {
  RoundState* st = w.st;
  const int nA = st->nA;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int T = (nA + 31) >> 5;
  const long long ntiles = (long long)T * (T + 1) / 2;
  const int kpad = 64 * w.w64;
  const int knpad = 64 * P.wn;
  const int amax1 = st->amax[1], amax2 = st->amax[2];
  const int half = lane >> 5, col = lane & 31;
  const int bound3 = P.G - P.h + 2;   // depth-3 loop bound (sorted index)

  int bs = -1, btp = 0, bfp = 0, bi = 0, bj = 0;
  unsigned long long ne2 = 0, vis3 = 0;

  for (long long t = gw; t < ntiles; t += kWavesPerGrid) {
    int ti, tj;
    decode_tile(t, T, ti, tj);
    if (ti * 32 >= amax1) continue;   // no valid g1 in this block row
    const int8_t* pa = w.A8 + (size_t)(ti * 32 + col) * kpad + 16 * half;
    const int8_t* pb = w.A8 + (size_t)(tj * 32 + col) * kpad + 16 * half;
    v16i acc = {0};
    for (int k0 = 0; k0 < kpad; k0 += 32) {
      v4i a = *reinterpret_cast<const v4i*>(pa + k0);
      v4i b = *reinterpret_cast<const v4i*>(pb + k0);
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
    }
    v16i accn = {0};
    if (kH2) {
      const int8_t* na = w.N8 + (size_t)(ti * 32 + col) * knpad + 16 * half;
      const int8_t* nb = w.N8 + (size_t)(tj * 32 + col) * knpad + 16 * half;
      for (int k0 = 0; k0 < knpad; k0 += 32) {
        v4i a = *reinterpret_cast<const v4i*>(na + k0);
        v4i b = *reinterpret_cast<const v4i*>(nb + k0);
        accn = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, accn, 0, 0, 0);
      }
    }
    const int j = tj * 32 + col;
    const bool jok = j < amax2;
    int sj = 0;
    if (!kH2 && jok) sj = w.act[j];
    unsigned long long mask[16];
    int nhit = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = ti * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      const bool ok = jok && i < j && i < amax1 && acc[r] > 0;
      if (kH2) {
        if (ok) {
          int s = P.p * acc[r] + P.q * (P.n_normal - accn[r]);
          if (s > bs || (s == bs && (i < bi || (i == bi && j < bj)))) {
            bs = s; btp = acc[r]; bfp = accn[r]; bi = i; bj = j;
          }
        }
        mask[r] = __ballot(ok);
        ne2 += __popcll(mask[r]);
      } else {
        mask[r] = __ballot(ok);
        nhit += __popcll(mask[r]);
        if (ok) vis3 += (unsigned long long)(bound3 - sj);
      }
    }
    if (!kH2 && nhit) {
      ne2 += nhit;
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&st->n_pairs, (unsigned long long)nhit);
      base = __shfl(base, 0, 64);
      const unsigned long long lt = (1ull << lane) - 1;
      unsigned long long off = base;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if ((mask[r] >> lane) & 1) {
          unsigned long long pos = off + __popcll(mask[r] & lt);
          const int i = ti * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          if (pos < w.pair_cap)
            w.pairs[pos] = (unsigned long long)i | ((unsigned long long)j << 16) |
                           ((unsigned long long)acc[r] << 32);
        }
        off += __popcll(mask[r]);
      }
    }
  }

  // counters: one atomic per wave
  for (int o = 32; o > 0; o >>= 1) vis3 += __shfl_xor(vis3, o, 64);
  if (lane == 0) {
    if (ne2) atomicAdd(&st->cnt.nonempty[2], ne2);
    if (!kH2 && vis3 && P.mode != kPruneBound) atomicAdd(&st->cnt.visited[3], vis3);
    if (!kH2 && st->n_pairs > w.pair_cap) st->overflow = 1;
  }
  if (kH2) {
    for (int o = 32; o > 0; o >>= 1) {
      int os = __shfl_xor(bs, o, 64), otp = __shfl_xor(btp, o, 64);
      int ofp = __shfl_xor(bfp, o, 64), oi = __shfl_xor(bi, o, 64), oj = __shfl_xor(bj, o, 64);
      if (os > bs || (os == bs && os >= 0 && (oi < bi || (oi == bi && oj < bj)))) {
        bs = os; btp = otp; bfp = ofp; bi = oi; bj = oj;
      }
    }
    if (lane == 0) {
      Slot sl;
      sl.s = bs; sl.tp = btp; sl.fp = bfp;
      sl.idx[0] = bi; sl.idx[1] = bj; sl.idx[2] = sl.idx[3] = 0; sl.pad = 0;
      w.slots[gw] = sl;
    }
  }
}

}  // namespace

hipError_t launch_pairs(const Problem& P, const Work& w, hipStream_t s) {
  if (P.h == 2)
    k_pairs<true><<<kPersistBlocks, kBlock, 0, s>>>(P, w);
  else
    k_pairs<false><<<kPersistBlocks, kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

}  // namespace pdfs
