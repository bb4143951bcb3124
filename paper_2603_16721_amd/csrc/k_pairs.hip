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
// Tiles: 128x128 block tiles of the upper triangle, staged through LDS.  A
// and B fragments use the same byte-to-k assignment, so the sum over k is the
// full dot product whatever that assignment is.  Output element r of lane l
// of a 32x32 MFMA block is row 8*(r/4) + 4*(l/32) + r%4, column l%32.
#include "pdfs_dev.h"
#include "slot_reduce.h"

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

// One 128x128 block tile (bi <= bj) per iteration of a persistent block; the
// four waves own 64x64 quadrants as 2x2 MFMA blocks.  K is staged through LDS
// 64 bytes at a time; the next chunk's global loads are issued before the
// current chunk's MFMAs.
constexpr int kBT = 128;          // block tile edge
constexpr int kKC = 128;          // K bytes per LDS chunk
constexpr int kLds = kKC + 16;    // padded LDS row stride (bytes)

__device__ __forceinline__ void mm_loop(const int8_t* __restrict__ M, int kpad, int rowA, int rowB,
                                        int8_t* sA, int8_t* sB, int tid, int wr, int wc,
                                        int half, int col, v16i (&acc)[2][2]) {
  // a panel chunk is 128 rows x kKC bytes = 8 (kKC/16) segments of 16 bytes
  // per row; thread tid stages segments v = tid + 256*u (u < kSeg) of each
  // panel: row v / kSegRow, segment v % kSegRow
  constexpr int kSegRow = kKC / 16;
  constexpr int kSeg = kBT * kSegRow / 256;
  const int8_t* pa[kSeg];
  const int8_t* pb[kSeg];
  int lo[kSeg];
  v4i ra[kSeg], rb[kSeg];
#pragma unroll
  for (int u = 0; u < kSeg; ++u) {
    const int v = tid + 256 * u, r = v / kSegRow, sg = v % kSegRow;
    pa[u] = M + (size_t)(rowA + r) * kpad + sg * 16;
    pb[u] = M + (size_t)(rowB + r) * kpad + sg * 16;
    lo[u] = r * kLds + sg * 16;
    ra[u] = *reinterpret_cast<const v4i*>(pa[u]);
    rb[u] = *reinterpret_cast<const v4i*>(pb[u]);
  }
  for (int k0 = 0; k0 < kpad; k0 += kKC) {
#pragma unroll
    for (int u = 0; u < kSeg; ++u) {
      *reinterpret_cast<v4i*>(sA + lo[u]) = ra[u];
      *reinterpret_cast<v4i*>(sB + lo[u]) = rb[u];
    }
    __syncthreads();
    if (k0 + kKC < kpad) {
      const int kn = k0 + kKC;
#pragma unroll
      for (int u = 0; u < kSeg; ++u) {
        ra[u] = *reinterpret_cast<const v4i*>(pa[u] + kn);
        rb[u] = *reinterpret_cast<const v4i*>(pb[u] + kn);
      }
    }
    {
#pragma unroll
      for (int kk = 0; kk < kKC; kk += 32) {
        v4i fa[2], fb[2];
#pragma unroll
        for (int m = 0; m < 2; ++m)
          fa[m] = *reinterpret_cast<const v4i*>(sA + (wr * 64 + m * 32 + col) * kLds + kk + 16 * half);
#pragma unroll
        for (int n = 0; n < 2; ++n)
          fb[n] = *reinterpret_cast<const v4i*>(sB + (wc * 64 + n * 32 + col) * kLds + kk + 16 * half);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[m], fb[n], acc[m][n], 0, 0, 0);
      }
    }
    __syncthreads();
  }
}

template <bool kH2>
__device__ __forceinline__ void pairs_body(const Problem& P, const Work& w) {
  __shared__ __attribute__((aligned(16))) int8_t sA[kBT * kLds];
  __shared__ __attribute__((aligned(16))) int8_t sB[kBT * kLds];
  __shared__ int wsum[4];
  __shared__ unsigned long long wbase;
  RoundState* st = w.st;
  if (st->done) return;
  const int nA = st->nA;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int T = (nA + kBT - 1) / kBT;
  const long long ntiles = (long long)T * (T + 1) / 2;
  const int kpad = unpacked_row_bytes(w.w64);
  const int knpad = unpacked_row_bytes(P.wn);
  const int amax1 = st->amax[1], amax2 = st->amax[2];
  const int half = lane >> 5, col = lane & 31;
  const int bound3 = P.G - P.h + 2;   // depth-3 loop bound (sorted index)

  int bs = -1, btp = 0, bfp = 0, bi_ = 0, bj_ = 0;
  unsigned long long ne2 = 0, vis3 = 0;

  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int bi, bj;
    decode_tile(t, T, bi, bj);
    if (bi * kBT >= amax1) continue;   // no valid g1 in this block row (uniform)
    // quadrant entirely below the diagonal of a diagonal tile: no pair i < j
    const bool active = !(bi == bj && wr > wc);
    v16i acc[2][2];
    v16i accn[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) { acc[m][n] = v16i{0}; accn[m][n] = v16i{0}; }
    // (a quadrant below the diagonal is computed too and masked below: it
    // keeps the accumulators in place across the K loop)
    mm_loop(w.A8, kpad, bi * kBT, bj * kBT, sA, sB, tid, wr, wc, half, col, acc);
    if (kH2) mm_loop(w.N8, knpad, bi * kBT, bj * kBT, sA, sB, tid, wr, wc, half, col, accn);

    // epilogue: pass 1 counts this wave's non-empty pairs (h > 2) or scores
    // them (h = 2); pass 2 writes the pairs at a block-reserved offset
    int nhit = 0;
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int j = bj * kBT + wc * 64 + n * 32 + col;
      const bool jok = active && j < amax2;
      int sj = 0;
      if (jok && (!kH2 || P.tn_literal)) sj = w.act[j];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = bi * kBT + wr * 64 + m * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          const int c = acc[m][n][r];
          const bool ok = jok && i < j && i < amax1 && c > 0;
          // exhaustive mode extends the empty pairs as well
          const bool emit = jok && i < j && i < amax1 && (c > 0 || P.mode == kPruneNone);
          if (kH2) {
            if (ok) {
              // literal reading: normals carrying either gene
              const int fp = P.tn_literal
                                 ? w.ncount[w.act[i]] + w.ncount[sj] - accn[m][n][r]
                                 : accn[m][n][r];
              const int s = P.p * c + P.q * (P.n_normal - fp);
              // one mask for every field (straight-line selects)
              const bool take =
                  (s > bs) | ((s == bs) & ((i < bi_) | ((i == bi_) & (j < bj_))));
              bs = take ? s : bs;
              btp = take ? c : btp;
              bfp = take ? fp : bfp;
              bi_ = take ? i : bi_;
              bj_ = take ? j : bj_;
            }
          } else if (emit) {
            ++nhit;
            vis3 += (unsigned long long)(bound3 - sj);
          }
          ne2 += ok ? 1 : 0;
        }
      }
    }
    if (!kH2) {
      // block-wide prefix of the per-lane counts, one atomic per tile
      int incl = nhit;
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane == 63) wsum[wave] = incl;
      __syncthreads();
      if (tid == 0) {
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        wbase = tot ? atomicAdd(&st->n_pairs, (unsigned long long)tot) : 0ull;
      }
      __syncthreads();
      unsigned long long pos = wbase + (unsigned long long)(incl - nhit);
      for (int q = 0; q < wave; ++q) pos += (unsigned long long)wsum[q];
      if (nhit) {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int j = bj * kBT + wc * 64 + n * 32 + col;
          const bool jok = active && j < amax2;
#pragma unroll
          for (int m = 0; m < 2; ++m) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int i = bi * kBT + wr * 64 + m * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
              const int c = acc[m][n][r];
              if (jok && i < j && i < amax1 && (c > 0 || P.mode == kPruneNone)) {
                if (pos < w.pair_cap)
                  w.pairs[pos] = (unsigned long long)i | ((unsigned long long)j << 16) |
                                 ((unsigned long long)c << 32);
                ++pos;
              }
            }
          }
        }
      }
      __syncthreads();   // wsum / wbase reused by the next tile
    }
  }

  // counters: one row per block
  unsigned long long v[kTallyN] = {0};
  v[kTNe2] = ne2;
  v[kTVis3] = (!kH2 && P.mode != kPruneBound) ? vis3 : 0;
  block_tally_to(w.tallies + (size_t)blockIdx.x * kTallyN, v);
  if (kH2) {
    Slot sl = empty_slot();
    if (bs >= 0) { sl.s = bs; sl.tp = btp; sl.fp = bfp; sl.idx[0] = bi_; sl.idx[1] = bj_; }
    block_best_to(&w.slots[blockIdx.x], sl);
  }
}

template <bool kH2>
__global__ __launch_bounds__(256) void k_pairs(Problem P, Work w) {
  pairs_body<kH2>(P, w);
}

template <bool kH2>
__global__ __launch_bounds__(256) void k_pairs_m(const BatchDesc* __restrict__ bd) {
  pairs_body<kH2>(bd[blockIdx.y].P, bd[blockIdx.y].w);
}

}  // namespace

// Batched launches (h >= 3): 256 blocks per instance; the counter rows of
// blocks 256.. stay as cleared at the start of the batched run.
hipError_t launch_pairs_m(const BatchDesc* bd, int n, hipStream_t s) {
  k_pairs_m<false><<<dim3(kPersistBlocks / 4, n), kBlock, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_pairs(const Problem& P, const Work& w, hipStream_t s) {
  if (P.h == 2)
    k_pairs<true><<<kPersistBlocks, kBlock, 0, s>>>(P, w);  // h = 2 writes one slot per block
  else
    k_pairs<false><<<kPersistBlocks, kBlock, 0, s>>>(P, w);
  return hipGetLastError();
}

}  // namespace pdfs
