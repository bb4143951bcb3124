// Host-side internals of libpdfs shared by the plain C ABI (pdfs_api.cpp) and
// the batched / served front ends (pdfs_batch.cpp).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pdfs.h"
#include "pdfs_dev.h"

namespace pdfs {

int dfs_row_words(int n);

// Rounds of one chunk (enqueued between two reads of the device state) are
// at most this many; rounds queued past the stop are no-ops on the device.
constexpr int kMaxChunk = 16;
// Chunks in flight at once: while the host reads the state after one chunk,
// the next is already queued, so the device does not wait for the host.
constexpr int kDepth = 2;

// Pinned host memory of a context: kDepth round states, then one round record
// (the allocation-free entry point's read-back).
constexpr size_t kPinnedBytes = kDepth * sizeof(RoundState) + sizeof(RoundRecord);

// Progress of one greedy run on a context, advanced without blocking.  The
// run's rounds go out in chunks; each chunk ends with a copy of the device
// state into its pinned slot and an event.  The row width of a chunk comes
// from the newest |U| the host has seen (any width >= ceil(|U|/64) gives the
// same results and |U| only shrinks), so with kDepth chunks in flight the
// width lags the device by at most the chunks still queued.
struct Run {
  bool active = false;      // started and not finished
  int h = 0;
  uint32_t p = 1, q = 1;
  int target = 0, max_rounds = 0;
  int n_unc = 0;            // |U| known to the host (only shrinks)
  int chunk = 1;            // rounds in the next chunk
  int enqueued = 0;         // rounds enqueued by this run
  int inflight = 0;         // chunks queued and not yet read
  int executed_before = 0;
  int32_t status = PDFS_OK;
  std::chrono::steady_clock::time_point t_prev;   // when the host last saw a chunk end
};

}  // namespace pdfs

struct pdfs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int prune_mode = PDFS_PRUNE_BOUND;
  int G = 0, n_tumor = 0, n_normal = 0, wt = 0, wn = 0;
  int nA_max = 0;
  int w64_max = 0;
  uint64_t* Ts = nullptr;
  uint64_t* Ns = nullptr;
  int32_t* perm = nullptr;
  int32_t* ncount = nullptr;           // normals carrying each sorted gene
  bool tn_literal = false;             // PDFS_OPT_TN_LITERAL
  uint64_t* U = nullptr;
  int32_t* cols = nullptr;
  int32_t* act = nullptr;
  uint8_t* flags = nullptr;
  uint32_t* TA = nullptr;
  uint32_t* NA = nullptr;
  int8_t* A8 = nullptr;
  int8_t* N8 = nullptr;
  unsigned long long* pairs = nullptr;
  unsigned long long* work_pairs = nullptr;   // bound mode only
  unsigned long long* seed_pairs = nullptr;
  uint32_t* hist = nullptr;
  unsigned long long* cursors = nullptr;
  unsigned long long pair_cap = 0;
  unsigned long long pair_cap_hint = 0;   // pdfs_options::pair_cap (0: default)
  pdfs::Item* items = nullptr;
  unsigned long long item_cap = 0;
  // two-phase depth-4 (h = 4, empty-prefix pruning): triple lists and per-c
  // counts, sized at run start for the run's first (largest) round
  unsigned long long* tri = nullptr;
  unsigned long long* tri_s = nullptr;
  uint32_t* tri_rank = nullptr;
  uint32_t* c_hist = nullptr;
  uint32_t* deepq = nullptr;   // h >= 5 leaf-prefix rings
  unsigned long long tri_cap = 0;
  bool two_phase = false;              // this run uses the two-phase path
  pdfs::Slot* slots = nullptr;
  unsigned long long* tallies = nullptr;
  pdfs::RoundState* st = nullptr;
  pdfs::RoundRecord* recs = nullptr;   // device, rec_cap records
  int rec_cap = 0;
  pdfs::RoundState* h_slots = nullptr; // pinned, kDepth states: one per chunk in flight
  pdfs::RoundState* h_st = nullptr;    // the newest state read (one of h_slots)
  pdfs::RoundRecord* h_rec = nullptr;  // pinned, after h_slots
  std::vector<int32_t> h_perm;
  std::string err;
  bool time_kernels = false;
  bool use_graphs = false;             // replay one captured round per row width
  int chunk_items = 256;               // depth-3 candidates per DFS work item
  int n_cu = 256;                      // compute units of the device
  int seed_pairs_n = 256;              // bound mode: pairs expanded first
  int long_stream = pdfs::kLongStream; // two-phase depth 4: listing threshold
  bool split3 = true;                  // h = 4, empty mode: long-stream prefixes as
                                       // depth-3 work units (the two-phase path)
  hipEvent_t ev[pdfs::kDepth][pdfs::kMaxChunk][5] = {};
  hipEvent_t chunk_done[pdfs::kDepth] = {};
  int chunk_rounds[pdfs::kDepth] = {};   // rounds of the chunk that uses each slot
  int next_slot = 0;                     // slot of the next chunk (rotates across runs)
  // per-call accumulation of the timed launches
  int64_t kernel_ns[3] = {0, 0, 0};
  int32_t kernel_launches[3] = {0, 0, 0};
  pdfs::Run run;
  // captured round graphs keyed by (h, w64, p, q, target, mode, chunk, seed,
  // two-phase, long-stream threshold)
  std::map<std::tuple<int, int, uint32_t, uint32_t, int, int, int, int, bool, int>, hipGraphExec_t>
      graphs;
  size_t bytes = 0;                    // device bytes held (admission accounting)
  bool async_alloc = false;            // stream-ordered allocation (batched / served)
  bool own_h_st = true;                // h_slots allocated by the context
};

namespace pdfs {

int32_t ctx_fail(pdfs_ctx* c, int32_t code, const std::string& msg);
// pdfs_create with two internal options: pinned_state (caller-owned pinned
// memory of kPinnedBytes, or NULL) and stream-ordered allocation on
// opt->stream.
int32_t create_ctx(const pdfs_matrix* m, const pdfs_options* opt, pdfs_ctx** out,
                   RoundState* pinned_state, bool async_alloc);
void begin_stats(pdfs_ctx* c, pdfs_stats* st);
void end_stats(pdfs_ctx* c, pdfs_stats* st, std::chrono::steady_clock::time_point t0);
const std::string& create_error();
// Row-indexed buffers (re-packed rows, unpacked bytes) regrown to hold rows of
// w64 words (batched launches run every instance at the widest width).
// Grows the pair list (and the item list) after a round emitted `emitted`
// pairs into it; the caller has drained every stream that uses the context.
int32_t grow_pair_list(pdfs_ctx* c, unsigned long long emitted);
int32_t grow_row_width(pdfs_ctx* c, int w64);
// Workspace of a run of depth h from |U| = n_unc: lists allocated, and for
// the two-phase path the prefix lists sized by a counting pass.
int32_t prepare_run(pdfs_ctx* c, int h, int n_unc);
// Starts a greedy run (U must already hold the starting mask on c->stream).
int32_t run_start(pdfs_ctx* c, int h, uint32_t p, uint32_t q, int target, int max_rounds,
                  int n_unc);
// Enqueues the next chunk of rounds and the state read-back; non-blocking.
int32_t run_enqueue(pdfs_ctx* c);
// Checks a pending chunk (waits for it when wait is true).  *done is set when
// the run has stopped; *ready when the chunk was processed.
int32_t run_poll(pdfs_ctx* c, bool wait, bool* ready, bool* done);
// Blocking run: start + chunks until done.
int32_t run_blocking(pdfs_ctx* c, int h, uint32_t p, uint32_t q, int target, int max_rounds,
                     int n_unc);
// One round record as the ABI's pdfs_combo.
void fill_combo(pdfs_combo* o, const RoundRecord& r, int h);
// Copies up to cap round records of the finished run into out; returns rounds.
int32_t run_records(pdfs_ctx* c, pdfs_combo* out, int32_t cap, int32_t* rounds);
int32_t check_call(pdfs_ctx* c, int h, uint32_t p, uint32_t q);
// Sets U from a host mask (NULL = all samples); returns |U| or -1.
int32_t set_uncovered(pdfs_ctx* c, const uint64_t* mask);
// Round workspace pointers and problem description of a context.
Work make_work(pdfs_ctx* c, int w64, int target);
Problem make_problem(const pdfs_ctx* c, int h, uint32_t p, uint32_t q);
// Enqueues one round on c->stream with workspace w (see pdfs_api.cpp).
int32_t enqueue_round(pdfs_ctx* c, const Problem& P, const Work& w, hipEvent_t* ev,
                      bool two_phase);
// Gets the static scratch array's device address on `device` once (the
// allocation-free entry point's workspace); called by create_ctx with the
// device current.
void scratch_init(int device);
// Device bytes a context of this shape will hold (admission control).
size_t footprint_bytes(int G, int n_tumor, int n_normal, int nA_max, int h, int prune_mode);

}  // namespace pdfs
