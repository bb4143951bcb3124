// C ABI of libpdfs: context setup (ingest + sparsest-first sort) and the
// per-round orchestration of the greedy weighted-set-cover loop.  All
// arithmetic of the search runs in the kernels of k_round.hip, k_pairs.hip
// and k_dfs.hip; this file moves buffers, picks kernel variants and reads the
// per-round record back.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pdfs.h"
#include "pdfs_dev.h"
#include "pdfs_host.h"

using namespace pdfs;

namespace {

thread_local std::string g_create_error;

int32_t fail(pdfs_ctx* c, int32_t code, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return code;
}

#define CK(ctx, expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, e_ == hipErrorOutOfMemory ? PDFS_ERR_OUT_OF_MEMORY : PDFS_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

// Device allocation of a context: stream-ordered on the context's stream when
// async_alloc is set (no device-wide synchronisation on free), plain otherwise.
hipError_t dmalloc(pdfs_ctx* c, void** p, size_t bytes) {
  bytes += 256;
  c->bytes += bytes;
  if (c->async_alloc) return hipMallocAsync(p, bytes, c->stream);
  return hipMalloc(p, bytes);
}

void dfree(pdfs_ctx* c, void* p) {
  if (!p) return;
  if (c->async_alloc) (void)hipFreeAsync(p, c->stream);
  else (void)hipFree(p);
}

template <typename T>
hipError_t dalloc(pdfs_ctx* c, T** p, size_t n) {
  return dmalloc(c, reinterpret_cast<void**>(p), n * sizeof(T));
}

void release(pdfs_ctx* c) {
  void* ptrs[] = {c->Ts, c->Ns, c->perm, c->ncount, c->U, c->cols, c->act, c->flags, c->TA, c->NA,
                  c->A8, c->N8, c->pairs, c->work_pairs, c->seed_pairs, c->hist, c->cursors,
                  c->items, c->slots, c->tallies, c->st, c->recs, c->tri, c->tri_s,
                  c->tri_rank, c->c_hist, c->deepq};
  for (void* p : ptrs) dfree(c, p);
  if (c->h_slots && c->own_h_st) (void)hipHostFree(c->h_slots);
  for (auto& set : c->ev)
    for (auto& row : set)
      for (hipEvent_t e : row)
        if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->chunk_done)
    if (e) (void)hipEventDestroy(e);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

int words(int n) { return (n + 63) / 64; }

// Exhaustive mode makes every gene a row of the round (its row over the
// uncovered samples may be empty), so the row-indexed buffers must hold G rows
// instead of the first round's active count.  Drops the buffers sized by the
// old count (they are re-made on demand) and the captured rounds that hold
// their addresses.
static int32_t grow_for_all_genes(pdfs_ctx* c) {
  if (c->nA_max >= c->G) return PDFS_OK;
  CK(c, hipStreamSynchronize(c->stream));
  void** bufs[] = {(void**)&c->TA, (void**)&c->NA, (void**)&c->A8, (void**)&c->N8,
                   (void**)&c->pairs, (void**)&c->work_pairs, (void**)&c->seed_pairs,
                   (void**)&c->items, (void**)&c->tri, (void**)&c->tri_s, (void**)&c->tri_rank,
                   (void**)&c->c_hist};
  for (void** b : bufs) {
    dfree(c, *b);
    *b = nullptr;
  }
  c->pair_cap = c->item_cap = c->tri_cap = 0;
  c->two_phase = false;
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->nA_max = c->G;
  const size_t rows = (size_t)((c->nA_max + 127) / 128 * 128 + 128);
  CK(c, dalloc(c, &c->TA, rows * 2 * (size_t)c->w64_max));
  CK(c, dalloc(c, &c->NA, rows * (size_t)kMaxWN32));
  CK(c, dalloc(c, &c->A8, rows * (size_t)unpacked_row_bytes(c->w64_max)));
  return PDFS_OK;
}

// Pair-list capacity: every pair of nA rows at most; the default start is
// max(2^21, 128 per active gene) (a G = 20000 cohort emits 1.5 M pairs in its
// densest round), and a round that emits more grows the list (regrow_pairs).
static unsigned long long pair_cap_for(int nA, unsigned long long hint) {
  const unsigned long long all = (unsigned long long)nA * (nA > 0 ? nA - 1 : 0) / 2;
  unsigned long long n = hint > 0 ? hint : 128ull * (unsigned long long)nA;
  if (hint == 0 && n < (1ull << 21)) n = 1ull << 21;
  if (n > all) n = all;
  return n < 64 ? 64 : n;
}

// Item-list capacity for a pair list of n pairs (two chunks per 64-pair batch,
// at least 2^20; the item builder lengthens chunks so that it never overflows).
static unsigned long long item_cap_for(unsigned long long n) {
  const unsigned long long ic = 2 * ((n + kPairBatch - 1) / kPairBatch);
  return ic < (1ull << 20) ? 1ull << 20 : ic;
}

// (Re)allocates the pair list (and its bound-mode work copy) and the item list
// for n pairs; the captured rounds holding the old addresses are dropped.
static int32_t alloc_pair_lists(pdfs_ctx* c, unsigned long long n) {
  void** bufs[] = {(void**)&c->pairs, (void**)&c->work_pairs, (void**)&c->items};
  for (void** b : bufs) {
    dfree(c, *b);
    *b = nullptr;
  }
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->pair_cap = c->item_cap = 0;
  CK(c, dalloc(c, &c->pairs, (size_t)n));
  if (c->prune_mode == PDFS_PRUNE_BOUND) CK(c, dalloc(c, &c->work_pairs, (size_t)n));
  const unsigned long long ic = item_cap_for(n);
  CK(c, dalloc(c, &c->items, (size_t)ic));
  c->pair_cap = n;
  c->item_cap = ic;
  return PDFS_OK;
}

// A round emitted `emitted` pairs into a shorter list: grows the list to that
// count + 1/4 (the caller has drained every stream that uses it).
static int32_t regrow_pairs_now(pdfs_ctx* c, unsigned long long emitted) {
  unsigned long long n = emitted + emitted / 4 + (1ull << 16);
  const unsigned long long all = pair_cap_for(c->nA_max, ~0ull);
  if (n > all) n = all;
  if (n <= c->pair_cap) return fail(c, PDFS_ERR_DEVICE, "pair count above every pair");
  return alloc_pair_lists(c, n);
}

// The same after the context's own stream has drained.
static int32_t regrow_pairs(pdfs_ctx* c, unsigned long long emitted) {
  CK(c, hipStreamSynchronize(c->stream));
  return regrow_pairs_now(c, emitted);
}

// Allocates the pair list, item list and normal bytes when a call first needs
// them.
int32_t ensure_workspace(pdfs_ctx* c, int h) {
  if (c->prune_mode == PDFS_PRUNE_NONE) {
    const int32_t rc = grow_for_all_genes(c);
    if (rc != PDFS_OK) return rc;
  }
  if (h >= 3 && !c->pairs) {
    const int32_t rc = alloc_pair_lists(c, pair_cap_for(c->nA_max, c->pair_cap_hint));
    if (rc != PDFS_OK) return rc;
  }
  if (h >= 3 && !c->seed_pairs) CK(c, dalloc(c, &c->seed_pairs, (size_t)kSeedCap));
  if (h >= 3 && c->prune_mode == PDFS_PRUNE_BOUND && !c->work_pairs)
    CK(c, dalloc(c, &c->work_pairs, (size_t)c->pair_cap));
  if (h >= 5 && !c->deepq)
    CK(c, dalloc(c, &c->deepq, deep_ring_words(c->w64_max, c->n_cu)));
  if (h == 2 && !c->N8) {
    size_t rows = (size_t)((c->nA_max + 127) / 128 * 128 + 128);
    CK(c, dalloc(c, &c->N8, rows * (size_t)unpacked_row_bytes(c->wn)));
  }
  return PDFS_OK;
}

}  // namespace

namespace pdfs {

Work make_work(pdfs_ctx* c, int w64, int target) {
  Work w;
  w.Ts = c->Ts; w.Ns = c->Ns; w.perm = c->perm; w.U = c->U; w.cols = c->cols; w.act = c->act;
  w.ncount = c->ncount;
  w.flags = c->flags; w.TA = c->TA; w.NA = c->NA; w.A8 = c->A8; w.N8 = c->N8;
  w.pairs = c->pairs;
  w.work_pairs = (c->prune_mode == PDFS_PRUNE_BOUND && c->work_pairs) ? c->work_pairs : c->pairs;
  w.seed_pairs = c->seed_pairs; w.hist = c->hist; w.items = c->items; w.slots = c->slots;
  w.cursors = c->cursors;
  w.tallies = c->tallies;
  w.st = c->st; w.recs = c->recs; w.rec_cap = c->rec_cap;
  w.pair_cap = c->pair_cap; w.item_cap = c->item_cap;
  w.w64 = w64; w.wn32 = 2 * c->wn; w.target = target;
  w.chunk = c->chunk_items; w.seed_n = c->seed_pairs_n; w.long_stream = c->long_stream;
  w.tri = c->tri; w.tri_s = c->tri_s; w.tri_rank = c->tri_rank; w.c_hist = c->c_hist;
  w.tri_cap = c->two_phase ? c->tri_cap : 0;
  w.deepq = c->deepq;
  w.slot_log = nullptr;
  return w;
}

Problem make_problem(const pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  Problem P;
  P.G = c->G; P.n_tumor = c->n_tumor; P.n_normal = c->n_normal; P.wt = c->wt; P.wn = c->wn;
  P.h = h; P.p = (int32_t)p; P.q = (int32_t)q; P.mode = c->prune_mode;
  P.n_cu = c->n_cu;
  P.tn_literal = c->tn_literal ? 1 : 0;
  return P;
}

// Enqueues one greedy round (every kernel returns at once if the run is
// already done).  ev = the round's five timing events (used when timing);
// two_phase: h = 4 under empty-prefix pruning lists long-stream prefixes for
// the tile kernel (the lists must be in w).
int32_t enqueue_round(pdfs_ctx* c, const Problem& P, const Work& w, hipEvent_t* ev,
                      bool two_phase) {
  const int h = P.h;
  hipStream_t s = c->stream;
  const bool tk = c->time_kernels;
  CK(c, launch_round_begin(P, w, s));
  CK(c, launch_active(P, w, s));
  CK(c, launch_gather_active(P, w, h >= 2, h == 2, s));
  if (h == 1) {
    CK(c, launch_h1(P, w, s));
  } else {
    if (tk) CK(c, hipEventRecord(ev[0], s));
    CK(c, launch_pairs(P, w, s));
    if (tk) CK(c, hipEventRecord(ev[1], s));
    if (h >= 5) {
      // depths 3..h expanded wave-wide through prefix rings
      if (c->prune_mode == PDFS_PRUNE_BOUND) {
        // as for h <= 4: the highest-count pairs first, then the pairs
        // whose bound can still reach the incumbent they set
        CK(c, launch_seed_select(P, w, s));
        CK(c, launch_make_items(P, w, true, s));
        if (tk) CK(c, hipEventRecord(ev[2], s));
        CK(c, launch_dfs_deep(P, w, 1, s));
        CK(c, launch_filter_pairs(P, w, s));
        CK(c, launch_make_items(P, w, false, s));
        CK(c, launch_dfs_deep(P, w, 2, s));
      } else {
        // every pair (the work list of the other modes is the pair list)
        Work wd = w;
        wd.work_pairs = wd.pairs;
        CK(c, launch_use_all_pairs(wd, s));
        CK(c, launch_make_items(P, wd, false, s));
        if (tk) CK(c, hipEventRecord(ev[2], s));
        CK(c, launch_dfs_deep(P, wd, 2, s));
      }
      if (tk) CK(c, hipEventRecord(ev[3], s));
    } else if (h >= 3) {
      if (c->prune_mode == PDFS_PRUNE_BOUND) {
        // seed phase: expand the highest-count pairs first so that the
        // incumbent is close to the round's answer, then keep only the pairs
        // whose bound can still reach it
        CK(c, launch_seed_select(P, w, s));
        CK(c, launch_make_items(P, w, true, s));
        if (tk) CK(c, hipEventRecord(ev[2], s));
        CK(c, launch_dfs(P, w, 1, s));
        CK(c, launch_filter_pairs(P, w, s));
        CK(c, launch_make_items(P, w, false, s));
      } else {
        CK(c, launch_use_all_pairs(w, s));
        CK(c, launch_make_items(P, w, false, s));
        if (tk) CK(c, hipEventRecord(ev[2], s));
      }
      if (two_phase) {
        // the main DFS lists the prefixes with long depth-4 streams; they are
        // bucketed by c and expanded in tiles
        CK(c, launch_tri_begin(w, s));
        CK(c, launch_dfs(P, w, 2, s));
        CK(c, launch_sort_triples(w, s));
        if (tk) CK(c, hipEventRecord(ev[4], s));
        CK(c, launch_dfs4_tiles(P, w, s));
      } else {
        CK(c, launch_dfs(P, w, 2, s));
      }
      if (tk) CK(c, hipEventRecord(ev[3], s));
    }
  }
  // slot phases written this round: 0 = h<=2 kernels, 1 = seed DFS or depth-4
  // tiles, 2 = main DFS
  const int phases = h <= 2 ? 1
                     : (h >= 5 ? (c->prune_mode == PDFS_PRUNE_BOUND ? 6 : 4)
                               : (c->prune_mode == PDFS_PRUNE_BOUND || two_phase ? 6 : 4));
  // counter rows: 0 = pair table (h >= 2), 1 = seed DFS or depth-4 tiles,
  // 2 = main DFS
  // (h >= 5: the deep walk adds its counters directly)
  const int tallies = h == 1 ? 0
                      : (h == 2 || h >= 5
                             ? 1
                             : (c->prune_mode == PDFS_PRUNE_BOUND || two_phase ? 7 : 5));
  CK(c, launch_finish_round(P, w, phases, tallies, s));
  return PDFS_OK;
}

}  // namespace pdfs

namespace pdfs {

int32_t ctx_fail(pdfs_ctx* c, int32_t code, const std::string& msg) { return fail(c, code, msg); }

// Enqueues `chunk` rounds at the run's current row width: replays of one
// captured round when graphs are on, direct launches otherwise.  slot = the
// chunk's event set when timing.
static int32_t enqueue_rounds(pdfs_ctx* c, const Problem& P, const Work& w, int chunk, int slot) {
  const Run& r = c->run;
  if (c->use_graphs && !c->time_kernels) {
    const auto key = std::make_tuple(P.h, w.w64, r.p, r.q, r.target, c->prune_mode,
                                     c->chunk_items, c->seed_pairs_n, c->two_phase,
                                     c->long_stream);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      hipGraph_t g = nullptr;
      hipGraphExec_t e = nullptr;
      CK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      const int32_t rc = enqueue_round(c, P, w, c->ev[slot][0], c->two_phase);
      hipGraph_t g2 = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->stream, &g2);
      if (rc != PDFS_OK) {
        if (g2) (void)hipGraphDestroy(g2);
        return rc;
      }
      CK(c, ec);
      g = g2;
      CK(c, hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      it = c->graphs.emplace(key, e).first;
    }
    for (int k = 0; k < chunk; ++k) CK(c, hipGraphLaunch(it->second, c->stream));
    return PDFS_OK;
  }
  for (int k = 0; k < chunk; ++k) {
    const int32_t rc = enqueue_round(c, P, w, c->ev[slot][k], c->two_phase);
    if (rc != PDFS_OK) return rc;
  }
  return PDFS_OK;
}

// Two-phase depth-4 path (h = 4, empty-prefix pruning): counts the non-empty
// depth-3 prefixes with long depth-4 streams in the run's first round (U as
// set for the run) with a depth-3 pass that writes nothing else, and grows
// the prefix lists to hold them.  Every later round of the run lists a
// subset.  When the lists would not fit comfortably in free device memory the
// run uses the single-kernel DFS alone.
static int32_t size_triples(pdfs_ctx* c, int h, int n_unc) {
  c->two_phase = false;
  if (h != 4 || c->prune_mode != PDFS_PRUNE_EMPTY || !c->split3) return PDFS_OK;
  const int w64 = dfs_row_words(words(n_unc > 0 ? n_unc : 1));
  if (w64 < 0 || w64 > c->w64_max) return PDFS_OK;   // reported when the run starts
  if (!c->c_hist) CK(c, dalloc(c, &c->c_hist, (size_t)c->nA_max + 1));
  hipStream_t s = c->stream;
  RoundState* hs = &c->h_slots[c->next_slot];
  for (int attempt = 0;; ++attempt) {
    const Problem P = make_problem(c, 4, 1, 1);
    Work w = make_work(c, w64, c->n_tumor + 1);
    w.tri_cap = 0;
    CK(c, launch_run_begin(P, w, 1, s));
    CK(c, launch_round_begin(P, w, s));
    CK(c, launch_active(P, w, s));
    CK(c, launch_gather_active(P, w, true, false, s));
    CK(c, launch_pairs(P, w, s));
    CK(c, launch_use_all_pairs(w, s));
    CK(c, launch_make_items(P, w, false, s));
    CK(c, launch_tri_begin(w, s));
    CK(c, launch_count_long(P, w, s));
    CK(c, hipMemcpyAsync(hs, c->st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    CK(c, hipStreamSynchronize(s));
    if (hs->overflow != kOverflowPairs || attempt > 0) break;
    const int32_t rc = regrow_pairs(c, hs->n_pairs);
    if (rc != PDFS_OK) return rc;
  }
  if (hs->overflow) return PDFS_OK;   // the run itself reports it
  const unsigned long long need = hs->n_tri;
  if (need > c->tri_cap) {
    const unsigned long long cap = need + need / 16 + 1024;
    size_t free_b = 0, total_b = 0;
    CK(c, hipMemGetInfo(&free_b, &total_b));
    const size_t per_entry = 2 * sizeof(unsigned long long) + sizeof(uint32_t);
    if (cap >= (1ull << 32) || cap * per_entry > free_b / 2) return PDFS_OK;
    dfree(c, c->tri);
    dfree(c, c->tri_s);
    dfree(c, c->tri_rank);
    c->tri = c->tri_s = nullptr;
    c->tri_rank = nullptr;
    c->tri_cap = 0;
    // captured rounds hold the old list addresses
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    CK(c, dalloc(c, &c->tri, (size_t)cap));
    CK(c, dalloc(c, &c->tri_s, (size_t)cap));
    CK(c, dalloc(c, &c->tri_rank, (size_t)cap));
    c->tri_cap = cap;
  }
  c->two_phase = true;
  return PDFS_OK;
}

int32_t grow_pair_list(pdfs_ctx* c, unsigned long long emitted) {
  return regrow_pairs_now(c, emitted);
}

int32_t grow_row_width(pdfs_ctx* c, int w64) {
  if (w64 <= c->w64_max) return PDFS_OK;
  // the row-indexed buffers are re-made at the wider stride; the deep walk's
  // rings (sized by the width) and the captured rounds holding the old
  // addresses are dropped and re-made on demand
  void** bufs[] = {(void**)&c->TA, (void**)&c->A8, (void**)&c->deepq};
  for (void** p : bufs) {
    dfree(c, *p);
    *p = nullptr;
  }
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->w64_max = w64;
  const size_t rows = (size_t)((c->nA_max + 127) / 128 * 128 + 128);
  CK(c, dalloc(c, &c->TA, rows * 2 * (size_t)c->w64_max));
  CK(c, dalloc(c, &c->A8, rows * (size_t)unpacked_row_bytes(c->w64_max)));
  return PDFS_OK;
}

int32_t prepare_run(pdfs_ctx* c, int h, int n_unc) {
  const int32_t rc = ensure_workspace(c, h);
  if (rc != PDFS_OK) return rc;
  return size_triples(c, h, n_unc);
}

int32_t run_start(pdfs_ctx* c, int h, uint32_t p, uint32_t q, int target, int max_rounds,
                  int n_unc) {
  int32_t rc = prepare_run(c, h, n_unc);
  if (rc != PDFS_OK) return rc;
  Run& r = c->run;
  // chunks of an earlier run still in flight are no-ops queued before
  // this run's work; their slots are simply reused in stream order
  r = Run();
  r.h = h; r.p = p; r.q = q; r.target = target; r.max_rounds = max_rounds; r.n_unc = n_unc;
  const Problem P = make_problem(c, h, p, q);
  Work w0 = make_work(c, 1, target);
  CK(c, launch_run_begin(P, w0, max_rounds, c->stream));
  r.active = true;
  r.t_prev = std::chrono::steady_clock::now();
  return PDFS_OK;
}

// The greedy loop on the device.  Chunks of rounds are queued until kDepth
// are in flight; each takes its row width from the newest |U| the host has
// read (any width >= ceil(|U|/64) gives the same results, and |U| only
// shrinks).  Rounds past a round cap are not queued at all.
int32_t run_enqueue(pdfs_ctx* c) {
  Run& r = c->run;
  while (r.active && r.inflight < kDepth) {
    if (r.max_rounds > 0 && r.enqueued >= r.max_rounds) break;
    const int w64 = dfs_row_words(words(r.n_unc > 0 ? r.n_unc : 1));
    if (w64 < 0 || w64 > c->w64_max) return fail(c, PDFS_ERR_UNSUPPORTED, "row too wide");
    int n = r.chunk;
    if (r.max_rounds > 0 && n > r.max_rounds - r.enqueued) n = r.max_rounds - r.enqueued;
    const int slot = c->next_slot;
    const Problem P = make_problem(c, r.h, r.p, r.q);
    const Work w = make_work(c, w64, r.target);
    const int32_t rc = enqueue_rounds(c, P, w, n, slot);
    if (rc != PDFS_OK) return rc;
    CK(c, hipMemcpyAsync(&c->h_slots[slot], c->st, sizeof(RoundState), hipMemcpyDeviceToHost,
                         c->stream));
    CK(c, hipEventRecord(c->chunk_done[slot], c->stream));
    c->chunk_rounds[slot] = n;
    c->next_slot = (slot + 1) % kDepth;
    r.enqueued += n;
    r.inflight += 1;
  }
  return PDFS_OK;
}

// Reads the oldest chunk in flight (waits for it when wait is true).
int32_t run_poll(pdfs_ctx* c, bool wait, bool* ready, bool* done) {
  Run& r = c->run;
  *ready = false;
  *done = !r.active;
  if (!r.active || r.inflight == 0) return PDFS_OK;
  const int slot = (c->next_slot - r.inflight + kDepth) % kDepth;
  if (wait) {
    CK(c, hipEventSynchronize(c->chunk_done[slot]));
  } else {
    const hipError_t q = hipEventQuery(c->chunk_done[slot]);
    if (q == hipErrorNotReady) return PDFS_OK;
    CK(c, q);
  }
  *ready = true;
  r.inflight -= 1;
  c->h_st = &c->h_slots[slot];
  const RoundState& st = *c->h_st;
  const int chunk = c->chunk_rounds[slot];
  const int ran = st.executed - r.executed_before;
  if (c->time_kernels) {
    for (int k = 0; k < ran && k < chunk; ++k) {
      hipEvent_t* ev = c->ev[slot][k];
      float ms = 0.f;
      if (r.h >= 2) {
        CK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
        c->kernel_ns[0] += (int64_t)(ms * 1e6);
        c->kernel_launches[0] += 1;
      }
      if (r.h >= 3) {
        CK(c, hipEventElapsedTime(&ms, ev[2], ev[3]));
        c->kernel_ns[1] += (int64_t)(ms * 1e6);
        c->kernel_launches[1] += 1;
      }
      if (r.h >= 3 && c->two_phase) {
        CK(c, hipEventElapsedTime(&ms, ev[4], ev[3]));
        c->kernel_ns[2] += (int64_t)(ms * 1e6);
        c->kernel_launches[2] += 1;
      }
    }
  }
  r.executed_before = st.executed;
  if (st.overflow & 2) {
    r.active = false;
    return fail(c, PDFS_ERR_DEVICE, "corrupt per-wave result slot or listed prefix");
  }
  if (st.overflow & 4) {
    r.active = false;
    return fail(c, PDFS_ERR_DEVICE, "deep walk scheduler made no progress");
  }
  if (st.overflow == kOverflowPairs) {
    // The round emitted more pairs than the list holds and was not
    // committed (nor anything after it: the run stopped there).  Grow the
    // list, clear the flags and go on from the same uncovered set.
    const unsigned long long emitted = st.n_pairs;
    const int executed = st.executed;
    int32_t rc = regrow_pairs(c, emitted);   // waits for the chunks in flight
    if (rc != PDFS_OK) {
      r.active = false;
      return rc;
    }
    Work w0 = make_work(c, 1, r.target);
    rc = launch_run_resume(w0, c->stream) == hipSuccess ? PDFS_OK : PDFS_ERR_DEVICE;
    if (rc != PDFS_OK) {
      r.active = false;
      return fail(c, rc, "resume after regrowing the pair list");
    }
    r.inflight = 0;
    r.enqueued = executed;
    r.executed_before = executed;
    r.chunk = 1;
    r.t_prev = std::chrono::steady_clock::now();
    return PDFS_OK;
  }
  if (st.overflow) {
    r.active = false;
    return fail(c, PDFS_ERR_OUT_OF_MEMORY, "item or prefix list capacity exceeded");
  }
  if (st.executed > c->n_tumor + 2) {
    r.active = false;
    return fail(c, PDFS_ERR_DEVICE, "greedy loop did not stop");
  }
  if (st.done || (r.max_rounds > 0 && r.enqueued >= r.max_rounds && r.inflight == 0)) {
    r.active = false;
    *done = true;
    return PDFS_OK;
  }
  r.n_unc = c->n_tumor - st.covered;
  // Chunk length: about kChunkNs of device work per chunk, from the time
  // between the last two chunk ends (the device had the next chunk queued,
  // so that interval is this chunk's device time when the host kept up).
  const auto now = std::chrono::steady_clock::now();
  const double ns = (double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - r.t_prev).count();
  r.t_prev = now;
  constexpr double kChunkNs = 1.0e6;
  if (ran > 0) {
    const double per_round = ns / ran;
    int n = per_round > 0 ? (int)(kChunkNs / per_round) : kMaxChunk;
    n = n < 1 ? 1 : (n > kMaxChunk ? kMaxChunk : n);
    // grow at most twofold per chunk so that one fast read does not jump far
    r.chunk = n > 2 * r.chunk ? 2 * r.chunk : n;
  }
  return PDFS_OK;
}

int32_t run_blocking(pdfs_ctx* c, int h, uint32_t p, uint32_t q, int target, int max_rounds,
                     int n_unc) {
  int32_t rc = run_start(c, h, p, q, target, max_rounds, n_unc);
  while (rc == PDFS_OK) {
    rc = run_enqueue(c);
    if (rc != PDFS_OK) break;
    bool ready = false, done = false;
    rc = run_poll(c, true, &ready, &done);
    if (done) break;
  }
  c->run.active = false;
  return rc;
}

}  // namespace pdfs

namespace pdfs {

void begin_stats(pdfs_ctx* c, pdfs_stats* st) {
  if (st) memset(st, 0, sizeof(*st));
  for (int i = 0; i < 3; ++i) {
    c->kernel_ns[i] = 0;
    c->kernel_launches[i] = 0;
  }
}

void end_stats(pdfs_ctx* c, pdfs_stats* st, std::chrono::steady_clock::time_point t0) {
  if (!st) return;
  const RoundState& r = *c->h_st;
  for (int l = 0; l <= PDFS_MAX_H; ++l) {
    st->visited[l] = r.tot.visited[l];
    st->nonempty[l] = r.tot.nonempty[l];
    st->bound_pruned[l] = r.tot.bound_pruned[l];
  }
  st->rounds = r.rounds;
  st->pair_macs = r.tx_pair_macs;
  st->dfs_visits[3] = r.tx_vis3;
  st->dfs_visits[4] = r.tx_vis4;
  st->dfs_visit_words3 = r.tx_vis_words3;
  st->dfs_visit_words4 = r.tx_vis_words4;
  st->dfs_leaves = r.tx_leaves;
  st->dfs_fp_leaves = r.tx_fp_leaves;
  for (int i = 0; i < 3; ++i) {
    st->kernel_ns[i] = c->kernel_ns[i];
    st->kernel_launches[i] = c->kernel_launches[i];
  }
  st->ns_total = std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now() - t0).count();
}

void fill_combo(pdfs_combo* o, const RoundRecord& r, int h) {
  memset(o, 0, sizeof(*o));
  o->h = h;
  for (int i = 0; i < PDFS_MAX_H; ++i) {
    o->genes[i] = i < h ? r.genes[i] : -1;
    o->sorted_idx[i] = i < h ? r.sorted_idx[i] : -1;
  }
  o->tp = r.tp; o->fp = r.fp; o->tn = r.tn;
  o->uncovered_before = r.uncovered_before;
  o->newly_covered = r.found ? r.tp : 0;
  o->score_num = r.score_num; o->score_den = r.score_den;
}

}  // namespace pdfs

namespace pdfs {

int32_t check_call(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (!c) return PDFS_ERR_INVALID_ARG;
  if (h < 1 || h > PDFS_MAX_H || h > c->G) return fail(c, PDFS_ERR_INVALID_ARG, "h out of range");
  if (q < 1) return fail(c, PDFS_ERR_INVALID_ARG, "alpha_q must be >= 1");
  double smax = (double)p * c->n_tumor + (double)q * c->n_normal;
  if (p > 65535u || q > 65535u || smax >= 1073741824.0)
    return fail(c, PDFS_ERR_INVALID_ARG, "p*n_tumor + q*n_normal must stay below 2^30");
  CK(c, hipSetDevice(c->device));
  return PDFS_OK;
}

int popcount_mask(const uint64_t* U, int wt) {
  int n = 0;
  for (int w = 0; w < wt; ++w) n += __builtin_popcountll(U[w]);
  return n;
}

bool mask_pad_ok(const uint64_t* U, int n, int wt) {
  if (n & 63) {
    if (U[n >> 6] & (~0ull << (n & 63))) return false;
  }
  for (int w = words(n); w < wt; ++w)
    if (U[w]) return false;
  return true;
}


int32_t set_uncovered(pdfs_ctx* c, const uint64_t* mask) {
  if (mask) {
    if (!mask_pad_ok(mask, c->n_tumor, c->wt))
      return fail(c, PDFS_ERR_INVALID_ARG, "uncovered mask has bits past n_tumor");
    CK(c, hipMemcpyAsync(c->U, mask, sizeof(uint64_t) * c->wt, hipMemcpyHostToDevice,
                         c->stream));
    return popcount_mask(mask, c->wt);
  }
  CK(c, launch_fill_u(c->U, c->wt, c->n_tumor, c->stream));
  return c->n_tumor;
}

int32_t run_records(pdfs_ctx* c, pdfs_combo* out, int32_t cap, int32_t* rounds) {
  *rounds = c->h_st->rounds;
  const int n = *rounds < cap ? *rounds : cap;
  if (n > 0 && out) {
    std::vector<RoundRecord> recs((size_t)n);
    CK(c, hipMemcpyAsync(recs.data(), c->recs, sizeof(RoundRecord) * recs.size(),
                         hipMemcpyDeviceToHost, c->stream));
    CK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i) fill_combo(&out[i], recs[i], c->run.h);
  }
  return PDFS_OK;
}

size_t footprint_bytes(int G, int n_tumor, int n_normal, int nA_max, int h, int prune_mode) {
  if (prune_mode == PDFS_PRUNE_NONE) nA_max = G;   // exhaustive mode: every gene is a row
  const size_t wt = (size_t)words(n_tumor), wn = (size_t)(n_normal > 0 ? words(n_normal) : 1);
  const size_t rows = (size_t)((nA_max + 127) / 128 * 128 + 128);
  const int w64max = dfs_row_words((int)wt);
  size_t b = (size_t)G * (wt + wn) * 8 + (size_t)G * 13 + (size_t)n_tumor * 8;
  b += rows * (2 * (size_t)w64max * 4 + kMaxWN32 * 4 + (size_t)unpacked_row_bytes(w64max));
  b += (size_t)kSlotPhases * kSlotsPerPhase * sizeof(Slot);
  b += (size_t)kSlotPhases * kPersistBlocks * kTallyN * 8;
  if (h >= 3) {
    const size_t pairs = (size_t)pair_cap_for(nA_max, 0);
    const size_t items = (size_t)item_cap_for(pairs);
    b += pairs * 8 * (prune_mode == PDFS_PRUNE_BOUND ? 2 : 1) + items * sizeof(Item) +
         (size_t)kSeedCap * 8;
  }
  if (h == 2) b += rows * (size_t)unpacked_row_bytes((int)wn);
  if (h >= 5) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n_cu = 256;
    b += deep_ring_words(w64max, n_cu) * 4;
  }
  return b + ((size_t)1 << 20);
}

}  // namespace pdfs

namespace {
}  // namespace

extern "C" {

const char* pdfs_strerror(int32_t s) {
  switch (s) {
    case PDFS_OK: return "ok";
    case PDFS_NO_COMBO: return "no combination covers an uncovered tumour sample";
    case PDFS_PENDING: return "pending";
    case PDFS_ERR_INVALID_ARG: return "invalid argument";
    case PDFS_ERR_UNSUPPORTED: return "unsupported";
    case PDFS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PDFS_ERR_DEVICE: return "device error";
    case PDFS_ERR_TRUNCATED: return "output truncated";
    default: return "unknown status";
  }
}

const char* pdfs_last_error(const pdfs_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

int32_t pdfs_set_prune_mode(pdfs_ctx* c, int32_t mode) {
  if (!c) return PDFS_ERR_INVALID_ARG;
  if (mode < PDFS_PRUNE_NONE || mode > PDFS_PRUNE_BOUND)
    return fail(c, PDFS_ERR_INVALID_ARG, "unknown prune mode");
  c->prune_mode = mode;
  return PDFS_OK;
}

int32_t pdfs_create(const pdfs_matrix* m, const pdfs_options* opt, pdfs_ctx** out) {
  return create_ctx(m, opt, out, nullptr, false);
}

void pdfs_destroy(pdfs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  // A context with stream-ordered memory frees in stream order; its own work
  // must be finished (callers destroy it once its run has stopped), but other
  // work sharing the stream need not be waited for.
  if (c->run.inflight > 0 || !c->async_alloc) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
  }
  release(c);
  delete c;
}

}  // extern "C"

namespace pdfs {

const std::string& create_error() { return g_create_error; }

int32_t create_ctx(const pdfs_matrix* m, const pdfs_options* opt, pdfs_ctx** out,
                   RoundState* pinned_state, bool async_alloc) {
  if (!out) return fail(nullptr, PDFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!m) return fail(nullptr, PDFS_ERR_INVALID_ARG, "matrix is NULL");
  if (m->G < 1 || m->n_tumor < 1 || m->n_normal < 0 || !m->tumor)
    return fail(nullptr, PDFS_ERR_INVALID_ARG, "need G >= 1, n_tumor >= 1, n_normal >= 0");
  const int wt = words(m->n_tumor);
  const int wn_in = m->n_normal > 0 ? words(m->n_normal) : 0;
  if (m->tumor_stride_words < wt)
    return fail(nullptr, PDFS_ERR_INVALID_ARG, "tumor_stride_words < ceil(n_tumor/64)");
  if (m->n_normal > 0 && (!m->normal || m->normal_stride_words < wn_in))
    return fail(nullptr, PDFS_ERR_INVALID_ARG, "normal matrix missing or stride too small");
  if (m->G > 65535) return fail(nullptr, PDFS_ERR_UNSUPPORTED, "G above 65535");
  if (pdfs::dfs_row_words(wt) < 0)
    return fail(nullptr, PDFS_ERR_UNSUPPORTED, "n_tumor above 1280");
  if (m->n_normal > 32 * kMaxWN32)
    return fail(nullptr, PDFS_ERR_UNSUPPORTED, "n_normal above 512");
  const int mode = opt ? opt->prune_mode : PDFS_PRUNE_BOUND;
  if (mode < PDFS_PRUNE_NONE || mode > PDFS_PRUNE_BOUND)
    return fail(nullptr, PDFS_ERR_INVALID_ARG, "unknown prune mode");

  pdfs_ctx* c = new pdfs_ctx();
  c->device = opt ? opt->device : 0;
  c->stream = opt ? static_cast<hipStream_t>(opt->stream) : nullptr;
  c->async_alloc = async_alloc && c->stream != nullptr;
  c->prune_mode = mode;
  c->time_kernels = opt && (opt->flags & PDFS_OPT_TIME_KERNELS);
  c->pair_cap_hint = opt && opt->pair_cap > 0 ? (unsigned long long)opt->pair_cap : 0ull;
  c->tn_literal = opt && (opt->flags & PDFS_OPT_TN_LITERAL);
  c->G = m->G; c->n_tumor = m->n_tumor; c->n_normal = m->n_normal;
  c->wt = wt; c->wn = wn_in > 0 ? wn_in : 1;
  c->w64_max = pdfs::dfs_row_words(wt);
  auto bail = [&](int32_t code) {
    g_create_error = c->err;
    release(c);
    delete c;
    return code;
  };
#define CKC(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                         \
      return bail(e_ == hipErrorOutOfMemory ? PDFS_ERR_OUT_OF_MEMORY : PDFS_ERR_DEVICE);  \
    }                                                                                      \
  } while (0)
  CKC(hipSetDevice(c->device));
  CKC(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  scratch_init(c->device);
  hipStream_t s = c->stream;
  const int G = m->G;
  if (c->time_kernels)
    for (auto& set : c->ev)
      for (auto& row : set)
        for (hipEvent_t& e : row) CKC(hipEventCreate(&e));
  for (hipEvent_t& e : c->chunk_done) CKC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  c->use_graphs = c->stream != nullptr && opt && (opt->flags & PDFS_OPT_GRAPHS);

  // Stage the caller's matrices on the device (strided as given).
  const uint64_t* dT = m->tumor;
  const uint64_t* dN = m->normal;
  uint64_t* stageT = nullptr;
  uint64_t* stageN = nullptr;
  if (!m->on_device) {
    CKC(dalloc(c, &stageT, (size_t)G * m->tumor_stride_words));
    CKC(hipMemcpyAsync(stageT, m->tumor, (size_t)G * m->tumor_stride_words * 8,
                       hipMemcpyHostToDevice, s));
    dT = stageT;
    if (m->n_normal > 0) {
      CKC(dalloc(c, &stageN, (size_t)G * m->normal_stride_words));
      CKC(hipMemcpyAsync(stageN, m->normal, (size_t)G * m->normal_stride_words * 8,
                         hipMemcpyHostToDevice, s));
      dN = stageN;
    }
  }
  if (m->n_normal == 0) dN = nullptr;
  auto free_stage = [&]() {
    dfree(c, stageT);
    dfree(c, stageN);
    stageT = stageN = nullptr;
  };

  // Pad bits must be zero.
  int* d_bad = nullptr;
  CKC(dalloc(c, &d_bad, 1));
  CKC(hipMemsetAsync(d_bad, 0, sizeof(int), s));
  CKC(launch_check_pad(dT, m->tumor_stride_words, G, m->n_tumor, d_bad, s));
  if (dN) CKC(launch_check_pad(dN, m->normal_stride_words, G, m->n_normal, d_bad, s));
  int bad = 0;
  CKC(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CKC(hipStreamSynchronize(s));
  dfree(c, d_bad);
  if (bad) {
    free_stage();
    c->err = "nonzero bits past the sample count";
    return bail(PDFS_ERR_INVALID_ARG);
  }

  // Sparsest-first order: stable counting sort of the combined counts.
  uint32_t* counts = nullptr;
  uint32_t* sort_tmp = nullptr;
  const int max_key = m->n_tumor + m->n_normal;
  CKC(dalloc(c, &counts, (size_t)G));
  CKC(dalloc(c, &sort_tmp, sort_tmp_words(G, max_key)));
  CKC(dalloc(c, &c->perm, (size_t)G));
  CKC(launch_gene_counts(dT, m->tumor_stride_words, dN, m->normal_stride_words, G, wt, wn_in,
                         counts, s));
  CKC(sort_genes(counts, G, max_key, sort_tmp, c->perm, s));
  CKC(dalloc(c, &c->Ts, (size_t)G * wt));
  CKC(dalloc(c, &c->Ns, (size_t)G * c->wn));
  CKC(launch_gather_sorted(dT, m->tumor_stride_words, dN, m->normal_stride_words, c->perm, G, wt,
                           c->wn, c->Ts, c->Ns, s));
  CKC(dalloc(c, &c->ncount, (size_t)G));
  CKC(launch_normal_counts(c->Ns, G, c->wn, c->ncount, s));
  c->h_perm.resize(G);
  CKC(hipMemcpyAsync(c->h_perm.data(), c->perm, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
  CKC(hipStreamSynchronize(s));
  dfree(c, sort_tmp);
  dfree(c, counts);
  free_stage();

  // Upper bound of the active list: genes with any tumour mutation.
  CKC(dalloc(c, &c->U, (size_t)wt));
  CKC(dalloc(c, &c->cols, (size_t)m->n_tumor));
  CKC(dalloc(c, &c->act, (size_t)G));
  CKC(dalloc(c, &c->flags, (size_t)G));
  CKC(dalloc(c, &c->st, 1));
  c->rec_cap = m->n_tumor + 1;   // every found round covers at least one sample
  CKC(dalloc(c, &c->recs, (size_t)c->rec_cap));
  CKC(dalloc(c, &c->slots, (size_t)kSlotPhases * kSlotsPerPhase));
  CKC(dalloc(c, &c->hist, (size_t)kMaxCount + 1));
  CKC(dalloc(c, &c->cursors, (size_t)kSubQueues * kCursorStride));
  CKC(dalloc(c, &c->tallies, (size_t)kSlotPhases * kPersistBlocks * kTallyN));
  if (pinned_state) {
    c->h_slots = pinned_state;
    c->own_h_st = false;
  } else {
    CKC(hipHostMalloc(reinterpret_cast<void**>(&c->h_slots), kPinnedBytes, hipHostMallocDefault));
  }
  c->h_st = &c->h_slots[0];
  c->h_rec = reinterpret_cast<RoundRecord*>(c->h_slots + kDepth);

  CKC(hipMemsetAsync(c->st, 0, sizeof(RoundState), s));
  CKC(launch_clear_slots(c->slots, kSlotPhases * kSlotsPerPhase, s));
  {
    Problem P;
    P.G = G; P.n_tumor = m->n_tumor; P.n_normal = m->n_normal; P.wt = wt; P.wn = c->wn;
    P.h = 1; P.p = 1; P.q = 1; P.mode = mode; P.n_cu = c->n_cu; P.tn_literal = 0;
    Work w = make_work(c, 1, 0);
    CKC(launch_fill_u(c->U, wt, m->n_tumor, s));
    CKC(launch_round_begin(P, w, s));
    CKC(launch_active(P, w, s));
    CKC(hipMemcpyAsync(c->h_st, c->st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    CKC(hipStreamSynchronize(s));
    c->nA_max = c->h_st->nA;
  }
  // row padding: whole 128-row MFMA block tiles
  const size_t rows = (size_t)((c->nA_max + 127) / 128 * 128 + 128);
  CKC(dalloc(c, &c->TA, rows * 2 * (size_t)c->w64_max));
  CKC(dalloc(c, &c->NA, rows * (size_t)kMaxWN32));
  CKC(dalloc(c, &c->A8, rows * (size_t)unpacked_row_bytes(c->w64_max)));
  *out = c;
  return PDFS_OK;
#undef CKC
}

}  // namespace pdfs

extern "C" {

int32_t pdfs_best_combo(pdfs_ctx* c, int32_t h, uint32_t p, uint32_t q, const uint64_t* uncovered,
                        pdfs_combo* out, pdfs_stats* stats) {
  int32_t rc = check_call(c, h, p, q);
  if (rc != PDFS_OK) return rc;
  if (!out) return fail(c, PDFS_ERR_INVALID_ARG, "out is NULL");
  auto t0 = std::chrono::steady_clock::now();
  begin_stats(c, stats);
  memset(out, 0, sizeof(*out));
  const int32_t n_unc = set_uncovered(c, uncovered);
  if (n_unc < 0) return n_unc;
  if (n_unc == 0) return PDFS_NO_COMBO;
  // one round: the target is out of reach, the round cap is 1
  rc = run_blocking(c, h, p, q, c->n_tumor + 1, 1, n_unc);
  if (rc != PDFS_OK) return rc;
  end_stats(c, stats, t0);
  int32_t rounds = 0;
  rc = run_records(c, out, 1, &rounds);
  if (rc != PDFS_OK) return rc;
  return rounds < 1 ? PDFS_NO_COMBO : PDFS_OK;
}

int32_t pdfs_wsc_run(pdfs_ctx* c, int32_t h, uint32_t p, uint32_t q, int32_t target_covered,
                     int32_t max_rounds, const uint64_t* initial_uncovered, pdfs_combo* out,
                     int32_t cap, int32_t* n_out, uint64_t* final_uncovered, pdfs_stats* stats) {
  int32_t rc = check_call(c, h, p, q);
  if (rc != PDFS_OK) return rc;
  if (!n_out || cap < 0 || (cap > 0 && !out))
    return fail(c, PDFS_ERR_INVALID_ARG, "bad output arguments");
  auto t0 = std::chrono::steady_clock::now();
  begin_stats(c, stats);
  *n_out = 0;
  const int K = target_covered > 0 ? target_covered : c->n_tumor;
  const int32_t n_unc = set_uncovered(c, initial_uncovered);
  if (n_unc < 0) return n_unc;
  rc = run_blocking(c, h, p, q, K, max_rounds > 0 ? max_rounds : 0, n_unc);
  if (rc != PDFS_OK) return rc;
  int32_t rounds = 0;
  rc = run_records(c, out, cap, &rounds);
  if (rc != PDFS_OK) return rc;
  *n_out = rounds;
  if (final_uncovered) {
    CK(c, hipMemcpyAsync(final_uncovered, c->U, sizeof(uint64_t) * c->wt, hipMemcpyDeviceToHost,
                         c->stream));
    CK(c, hipStreamSynchronize(c->stream));
  }
  end_stats(c, stats, t0);
  if (rounds > cap) return fail(c, PDFS_ERR_TRUNCATED, "more rounds than cap");
  return PDFS_OK;
}

}  // extern "C"
