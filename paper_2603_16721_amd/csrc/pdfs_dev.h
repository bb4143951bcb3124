// Internal declarations shared by the HIP kernels and the host orchestration
// of libpdfs.  Not part of the public ABI (that is include/pdfs.h).
//
// Device data layout of one cohort (all in HBM, library-owned):
//   Ts   uint64 [G][wt]   tumour rows in sorted (sparsest-first) order
//   Ns   uint64 [G][wn]   normal rows in sorted order (wn >= 1, zero-padded)
//   perm int32  [G]       sorted position -> caller gene id
//   U    uint64 [wt]      uncovered tumour samples of the current round
// Per-round workspace (DelCols done physically: only uncovered columns kept):
//   cols int32  [n_tumor]       uncovered sample ids, ascending
//   act  int32  [G]             active genes (sorted idx with T_g & U != 0)
//   TA   uint32 [G][w32]        active tumour rows over uncovered columns
//                               (w32 = 2*w64 words, zero padded)
//   NA   uint32 [G][16]         active normal rows (all normals, zero padded)
//   A8   int8   [G128][kpad]    active tumour rows unpacked to 0/1 bytes for
//                               the int8 MFMA pair table (kpad = 128*ceil(w64/2))
//   N8   int8   [G128][knpad]   same for normals (h = 2 only)
//   pairs uint64 [cap]          non-empty pairs (a | b<<16 | count<<32)
//   items  Item [cap]           DFS work items (pair batch x candidate range)
//   slots  Slot [nslot]         per-wave best candidates for the argmax
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdfs {

constexpr int kMaxH = 9;
constexpr int kWave = 64;
constexpr int kMaxW64 = 20;        // tumour words per row the DFS kernels take
constexpr int kMaxWN32 = 16;       // normal 32-bit words per row (n_normal <= 512)
constexpr int kPairBatch = 64;     // pairs per DFS batch (one per lane)
constexpr int kPersistBlocks = 1024;  // persistent grids: ~1.3 resident rounds of waves
constexpr int kBlock = 256;        // 4 waves per block
constexpr int kWavesPerGrid = kPersistBlocks * (kBlock / kWave);
constexpr int kSlotsPerPhase = kPersistBlocks;   // one argmax slot per block
constexpr int kDeepQ = 128;   // entries per prefix ring of the h >= 5 walk
constexpr int kSlotPhases = 3;     // pair kernel / seed DFS / main DFS
constexpr int kSeedPairs = 256;    // bound mode: pairs expanded first to set the incumbent
constexpr int kSeedCap = 1024;     // seed list capacity (ties at the threshold)
constexpr int kMaxCount = 1280;    // largest tumour count of a pair (n_tumor limit)
// two-phase depth 4: depth-3 prefixes with at least this many depth-4
// candidates left are listed and expanded in sorted tiles
#ifndef PDFS_LONG_STREAM
#define PDFS_LONG_STREAM 384
#endif
constexpr int kLongStream = PDFS_LONG_STREAM;

// The depth-first walk's work items are drained from kSubQueues contiguous
// ranges, each with its own cursor kCursorStride words (256 bytes) apart.
constexpr int kSubQueues = 32;
constexpr int kCursorStride = 32;

enum PruneMode { kPruneNone = 0, kPruneEmpty = 1, kPruneBound = 2 };

// RoundState::overflow: the pair list was too small for the round's pairs
constexpr int32_t kOverflowPairs = 1 | 8;

// Bytes per unpacked (one byte per sample) row for the MFMA pair table: the
// row's 64-bit words times 64, rounded up to the kernel's 128-byte K chunk.
__host__ __device__ constexpr int unpacked_row_bytes(int w64) { return 128 * ((w64 + 1) / 2); }

// Per-depth counters, index = depth.
struct Counters {
  unsigned long long visited[kMaxH + 1];
  unsigned long long nonempty[kMaxH + 1];
  unsigned long long bound_pruned[kMaxH + 1];
};

// One round's device-side state.  Written by the round kernels, read back by
// the host once per round.
struct RoundState {
  int32_t n_unc;        // |U| at round start
  int32_t nA;           // active genes
  int32_t amax[kMaxH + 1];  // depth l: active genes with sorted idx <= G-h+l-1
  int32_t found;        // 1 if the round found a combination
  int32_t done;         // stop flag after the update
  int32_t covered;      // tumour samples covered after this round
  int32_t rounds;       // rounds completed (device count)
  unsigned long long n_pairs;      // pairs emitted
  unsigned long long n_work_pairs; // pairs kept for the DFS
  unsigned long long n_items;      // DFS work items
  unsigned long long cursor;       // work-item cursor
  unsigned long long incumbent;    // bound key: (S+1)<<32 | (~a & 0xffff)<<16 | (~b & 0xffff)
  unsigned long long n_seed;       // pairs selected for the seed phase
  int32_t seed_t;                  // seed threshold on the pair count
  int32_t overflow;                // bit 0: a list hit its capacity; bit 1: corrupt slot;
                                   // bit 2: the h >= 5 walk's scheduler stalled; bit 3
                                   // (with bit 0): it was the pair list, and n_pairs
                                   // holds the count the round emitted
  Counters cnt;                    // this round's counters
  // work the DFS kernels had to do (active candidates only)
  unsigned long long x_vis3, x_vis4, x_leaves, x_fp_leaves;
  // ---- whole-run state (set by k_run_begin, advanced by k_finish_round)
  int32_t max_rounds;              // 0 = no cap
  int32_t executed;                // rounds whose kernels ran (incl. a final empty one)
  Counters tot;                    // counters summed over executed rounds
  unsigned long long tx_vis3, tx_vis4, tx_leaves, tx_fp_leaves, tx_pair_macs;
  unsigned long long tx_vis_words3, tx_vis_words4;   // visits x ceil(|U|/64)
  // ---- two-phase depth-4 (h = 4, empty-prefix pruning)
  unsigned long long n_tri;        // non-empty depth-3 prefixes listed this round
  // ---- batched launches: best-leaf log entries per slot phase this round
  uint32_t nlog[4];
};

// Per-block counter rows (summed by the round's finish kernel instead of
// thousands of same-address atomics).  Row layout:
enum TallyField {
  kTNe2 = 0,      // nonempty[2]
  kTVis3,         // visited[3]
  kTNe3,          // nonempty[3]
  kTNe4,          // nonempty[4]
  kTVis4,         // visited[4]
  kTBp2,          // bound_pruned[2]
  kTBp3,          // bound_pruned[3]
  kTXv3,          // active-candidate depth-3 visits
  kTXv4,          // active-candidate depth-4 visits
  kTXfp,          // leaves whose normal intersection was counted
  kTLeaves,       // scored leaves
  kTallyN = 16
};

// Result of one round (host-visible copy).
struct RoundRecord {
  int32_t found;
  int32_t h;
  int32_t sorted_idx[kMaxH];
  int32_t genes[kMaxH];
  int32_t tp, fp, tn, uncovered_before;
  int64_t score_num, score_den;
};

struct Slot {
  int32_t s;             // score, -1 = empty
  int32_t tp, fp;
  int32_t idx[kMaxH];    // active-list indices, ascending (zero past h)
};

struct Item {
  uint32_t batch;   // pair batch (kPairBatch consecutive work pairs)
  uint32_t c_lo;    // first depth-3 candidate (active index)
  uint32_t c_hi;    // one past the last
  uint32_t pad;
};

// Static problem description passed by value to kernels.
struct Problem {
  int32_t G, n_tumor, n_normal, wt, wn;
  int32_t h;
  int32_t p, q;
  int32_t mode;
  int32_t n_cu;   // compute units of the device (sizes the persistent DFS grid)
  int32_t tn_literal;   // FP = normals carrying any gene (else: carrying all)
};

// Round workspace pointers.
struct Work {
  const uint64_t* Ts;
  const uint64_t* Ns;
  const int32_t* perm;
  uint64_t* U;
  int32_t* cols;
  int32_t* act;
  const int32_t* ncount;            // [G] normals carrying each sorted gene
  uint8_t* flags;
  uint32_t* TA;
  uint32_t* NA;
  int8_t* A8;
  int8_t* N8;
  unsigned long long* pairs;
  unsigned long long* work_pairs;   // == pairs unless bound mode filters them
  unsigned long long* seed_pairs;   // [kSeedCap]
  uint32_t* hist;                   // [kMaxCount + 1] pair-count histogram
  Item* items;
  unsigned long long* cursors;      // [kSubQueues * kCursorStride] item cursors
  Slot* slots;
  unsigned long long* tallies;      // [kSlotPhases][kPersistBlocks][kTallyN]
  RoundState* st;
  RoundRecord* recs;                // one record per found round
  int32_t rec_cap;
  unsigned long long pair_cap;
  unsigned long long item_cap;
  int32_t w64;       // compacted tumour words per row used this round
  int32_t wn32;      // normal 32-bit words per row
  int32_t target;    // covered-count stop target
  int32_t chunk;     // depth-3 candidates per main-phase DFS item
  int32_t seed_n;    // bound mode: pairs expanded in the seed phase
  int32_t long_stream;   // two-phase depth 4: prefixes with at least this many
                         // depth-4 candidates are listed for the tile kernel
  // two-phase depth-4: listed triples a | b << 16 | c << 32, each entry's rank
  // among the listed entries of its c (taken when it is counted), the same
  // sorted by c, and per-c counts (then bucket offsets), nA entries
  unsigned long long* tri;
  uint32_t* tri_rank;
  unsigned long long* tri_s;
  uint32_t* c_hist;
  unsigned long long tri_cap;   // 0: count only
  // h >= 5: per wave of the deep walk and depth 3..kMaxH-1, a prefix ring of
  // kDeepQ entries ([tumour word][entry] intersections, then [depth][entry]
  // indices) and a frame for a suspended expansion ([word][lane])
  uint32_t* deepq;
  // batched launches: per slot phase, kLogCap best leaves appended by the
  // waves that worked on this instance (NULL for a context's own launches,
  // whose slots are one per block)
  Slot* slot_log;
};

// ---------------------------------------------------------------- batched
// Many cohorts' rounds in one launch per round step.  Light steps run one
// block row per instance (blockIdx.y); the depth-first steps drain one shared
// queue of (instance, item) work: instance i owns the queue positions
// [base[i], base[i+1]).  A wave's best leaf and counts for an instance go to
// that instance's log and counter row when the wave moves on (a wave's queue
// positions only grow, so it meets each instance at most once per launch).
constexpr int kMaxBatch = 64;
constexpr int kLogCap = kWavesPerGrid;

struct BatchDesc {
  Problem P;
  Work w;
};

struct BatchQueue {
  unsigned long long cursor;
  uint32_t n;       // instances
  uint32_t total;   // queue length (base[n])
  uint32_t base[kMaxBatch + 1];
};

// ---------------------------------------------------------------- launchers
// create time
hipError_t launch_gene_counts(const uint64_t* T, int64_t ts, const uint64_t* N, int64_t ns,
                              int G, int wt, int wn, uint32_t* counts, hipStream_t s);
// Stable counting sort by count (keys 0..max_key), ties by caller index:
// perm[i] = caller gene at sorted position i.  tmp: sort_tmp_words(G, max_key)
// words of device scratch.
size_t sort_tmp_words(int G, int max_key);
hipError_t sort_genes(const uint32_t* counts, int G, int max_key, uint32_t* tmp, int32_t* perm,
                      hipStream_t s);
hipError_t launch_gather_sorted(const uint64_t* T, int64_t ts, const uint64_t* N, int64_t ns,
                                const int32_t* perm, int G, int wt, int wn, uint64_t* Ts,
                                uint64_t* Ns, hipStream_t s);
hipError_t launch_normal_counts(const uint64_t* Ns, int G, int wn, int32_t* ncount,
                                hipStream_t s);
hipError_t launch_check_pad(const uint64_t* T, int64_t ts, int G, int n, int* bad, hipStream_t s);

// per round
hipError_t launch_round_begin(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_active(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_gather_active(const Problem& P, const Work& w, bool unpack_tumor,
                                bool unpack_normal, hipStream_t s);
hipError_t launch_h1(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_pairs(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_seed_select(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_make_items(const Problem& P, const Work& w, bool seed, hipStream_t s);
hipError_t launch_filter_pairs(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_use_all_pairs(const Work& w, hipStream_t s);
hipError_t launch_dfs(const Problem& P, const Work& w, int phase, hipStream_t s);
// h = 5..9: wave-wide expansion of every depth through per-depth prefix rings
hipError_t launch_dfs_deep(const Problem& P, const Work& w, int phase, hipStream_t s);
// two-phase depth-4 (h = 4, empty-prefix pruning): the main DFS lists the
// non-empty depth-3 prefixes with long candidate streams, they are bucketed
// by c and expanded in tiles of 64
hipError_t launch_tri_begin(const Work& w, hipStream_t s);
hipError_t launch_count_long(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_sort_triples(const Work& w, hipStream_t s);
hipError_t launch_dfs4_tiles(const Problem& P, const Work& w, hipStream_t s);
hipError_t launch_finish_round(const Problem& P, const Work& w, int phase_mask, int tally_mask,
                               hipStream_t s);
hipError_t launch_clear_slots(Slot* slots, int n, hipStream_t s);
// n32 32-bit words at p set to zero by a fill kernel (no memset node)
hipError_t launch_zero_u32(void* p, size_t n32, hipStream_t s);
hipError_t launch_fill_u(uint64_t* U, int wt, int n, hipStream_t s);
hipError_t launch_run_begin(const Problem& P, const Work& w, int max_rounds, hipStream_t s);
hipError_t launch_run_resume(const Work& w, hipStream_t s);
// 32-bit words of the h >= 5 walk's rings and frames for rows of up to
// w64_max words on a device of n_cu compute units (the launched grids' size).
size_t deep_ring_words(int w64_max, int n_cu);

// batched launches over n instances (descriptors bd in device memory; every
// instance at the same row width, h in {3, 4}); the depth-first steps take a
// queue built by launch_batch_queue over the instances they cover (kind 0:
// work items, 1: depth-4 tiles)
hipError_t launch_run_begin_m(const BatchDesc* bd, int n, int max_rounds, hipStream_t s);
hipError_t launch_round_begin_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_active_m(const BatchDesc* bd, int n, int max_G, hipStream_t s);
hipError_t launch_gather_active_m(const BatchDesc* bd, int n, int max_G, hipStream_t s);
hipError_t launch_pairs_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_seed_select_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_make_items_m(const BatchDesc* bd, int n, bool seed, hipStream_t s);
hipError_t launch_filter_pairs_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_use_all_pairs_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_batch_queue(const BatchDesc* bd, int n, BatchQueue* bq, int phase, int kind,
                              hipStream_t s);
hipError_t launch_dfs_m(int h, int w64, bool bound, const BatchDesc* bd, BatchQueue* bq,
                        int phase, int n_cu, hipStream_t s);
hipError_t launch_tri_begin_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_sort_triples_m(const BatchDesc* bd, int n, hipStream_t s);
hipError_t launch_dfs4_tiles_m(int w64, const BatchDesc* bd, BatchQueue* bq, int n_cu,
                               hipStream_t s);
hipError_t launch_finish_round_m(const BatchDesc* bd, int n, hipStream_t s);

}  // namespace pdfs
