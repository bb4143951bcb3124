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

namespace pdfs {
int dfs_row_words(int n);
}

using namespace pdfs;

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
  unsigned long long pair_cap = 0;
  Item* items = nullptr;
  unsigned long long item_cap = 0;
  Slot* slots = nullptr;
  unsigned long long* tallies = nullptr;
  RoundState* st = nullptr;
  RoundRecord* rec = nullptr;
  RoundState* h_st = nullptr;
  RoundRecord* h_rec = nullptr;
  std::vector<int32_t> h_perm;
  std::string err;
  bool time_kernels = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // per-call accumulation of the timed launches
  int64_t kernel_ns[2] = {0, 0};
  int32_t kernel_launches[2] = {0, 0};
};

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

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T) + 256);
}

void release(pdfs_ctx* c) {
  void* ptrs[] = {c->Ts, c->Ns, c->perm, c->U, c->cols, c->act, c->flags, c->TA, c->NA,
                  c->A8, c->N8, c->pairs, c->work_pairs, c->seed_pairs, c->hist,
                  c->items, c->slots, c->tallies, c->st, c->rec};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_rec) (void)hipHostFree(c->h_rec);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
}

int words(int n) { return (n + 63) / 64; }

// Allocates the pair list, item list and normal bytes when a call first needs
// them.
int32_t ensure_workspace(pdfs_ctx* c, int h) {
  if (h >= 3 && !c->pairs) {
    unsigned long long n = (unsigned long long)c->nA_max * (c->nA_max > 0 ? c->nA_max - 1 : 0) / 2;
    if (n < 64) n = 64;
    c->pair_cap = n;
    CK(c, dalloc(&c->pairs, (size_t)n));
    unsigned long long ic = 2 * ((n + kPairBatch - 1) / kPairBatch);
    if (ic < (1ull << 20)) ic = 1ull << 20;
    c->item_cap = ic;
    CK(c, dalloc(&c->items, (size_t)ic));
    CK(c, dalloc(&c->seed_pairs, (size_t)kSeedCap));
  }
  if (h >= 3 && c->prune_mode == PDFS_PRUNE_BOUND && !c->work_pairs)
    CK(c, dalloc(&c->work_pairs, (size_t)c->pair_cap));
  if (h == 2 && !c->N8) {
    size_t rows = (size_t)((c->nA_max + 127) / 128 * 128 + 128);
    CK(c, dalloc(&c->N8, rows * (size_t)unpacked_row_bytes(c->wn)));
  }
  return PDFS_OK;
}

Work make_work(pdfs_ctx* c, int w64, int target) {
  Work w;
  w.Ts = c->Ts; w.Ns = c->Ns; w.perm = c->perm; w.U = c->U; w.cols = c->cols; w.act = c->act;
  w.flags = c->flags; w.TA = c->TA; w.NA = c->NA; w.A8 = c->A8; w.N8 = c->N8;
  w.pairs = c->pairs;
  w.work_pairs = (c->prune_mode == PDFS_PRUNE_BOUND && c->work_pairs) ? c->work_pairs : c->pairs;
  w.seed_pairs = c->seed_pairs; w.hist = c->hist; w.items = c->items; w.slots = c->slots;
  w.tallies = c->tallies;
  w.st = c->st; w.rec = c->rec; w.pair_cap = c->pair_cap; w.item_cap = c->item_cap;
  w.w64 = w64; w.wn32 = 2 * c->wn; w.target = target;
  return w;
}

// One greedy round on the device; the round state and record land in the
// pinned host copies.
int32_t run_round(pdfs_ctx* c, int h, uint32_t p, uint32_t q, int target, int n_unc) {
  int w64 = dfs_row_words(words(n_unc > 0 ? n_unc : 1));
  if (w64 < 0 || w64 > c->w64_max) return fail(c, PDFS_ERR_UNSUPPORTED, "row too wide");
  int32_t rc = ensure_workspace(c, h);
  if (rc != PDFS_OK) return rc;
  Problem P;
  P.G = c->G; P.n_tumor = c->n_tumor; P.n_normal = c->n_normal; P.wt = c->wt; P.wn = c->wn;
  P.h = h; P.p = (int32_t)p; P.q = (int32_t)q; P.mode = c->prune_mode;
  Work w = make_work(c, w64, target);
  hipStream_t s = c->stream;
  CK(c, launch_round_begin(P, w, s));
  CK(c, launch_active(P, w, s));
  CK(c, launch_gather_active(P, w, h >= 2, h == 2, s));
  const bool tk = c->time_kernels;
  if (h == 1) {
    CK(c, launch_h1(P, w, s));
  } else {
    if (tk) CK(c, hipEventRecord(c->ev[0], s));
    CK(c, launch_pairs(P, w, s));
    if (tk) CK(c, hipEventRecord(c->ev[1], s));
    if (h >= 3) {
      if (c->prune_mode == PDFS_PRUNE_BOUND) {
        // seed phase: expand the highest-count pairs first so that the
        // incumbent is close to the round's answer, then keep only the pairs
        // whose bound can still reach it
        CK(c, launch_seed_select(P, w, s));
        CK(c, launch_make_items(P, w, true, s));
        if (tk) CK(c, hipEventRecord(c->ev[2], s));
        CK(c, launch_dfs(P, w, 1, s));
        CK(c, launch_filter_pairs(P, w, s));
        CK(c, launch_make_items(P, w, false, s));
      } else {
        CK(c, launch_use_all_pairs(w, s));
        CK(c, launch_make_items(P, w, false, s));
        if (tk) CK(c, hipEventRecord(c->ev[2], s));
      }
      CK(c, launch_dfs(P, w, 2, s));
      if (tk) CK(c, hipEventRecord(c->ev[3], s));
    }
  }
  // slot phases written this round: 0 = h<=2 kernels, 1 = seed DFS, 2 = main DFS
  const int phases = h <= 2 ? 1 : (c->prune_mode == PDFS_PRUNE_BOUND ? 6 : 4);
  // counter rows: 0 = pair table (h >= 2), 1 = seed DFS, 2 = main DFS
  const int tallies = h == 1 ? 0 : (h == 2 ? 1 : (c->prune_mode == PDFS_PRUNE_BOUND ? 7 : 5));
  CK(c, launch_finish_round(P, w, phases, tallies, s));
  CK(c, hipMemcpyAsync(c->h_st, c->st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
  CK(c, hipMemcpyAsync(c->h_rec, c->rec, sizeof(RoundRecord), hipMemcpyDeviceToHost, s));
  CK(c, hipStreamSynchronize(s));
  if (tk && h >= 2) {
    float ms = 0.f;
    CK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    c->kernel_ns[0] += (int64_t)(ms * 1e6);
    c->kernel_launches[0] += 1;
    if (h >= 3) {
      CK(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
      c->kernel_ns[1] += (int64_t)(ms * 1e6);
      c->kernel_launches[1] += 1;
    }
  }
  if (c->h_st->overflow & 2) return fail(c, PDFS_ERR_DEVICE, "corrupt per-wave result slot");
  if (c->h_st->overflow)
    return fail(c, PDFS_ERR_OUT_OF_MEMORY, "pair or item list capacity exceeded");
  return PDFS_OK;
}

void add_counters(pdfs_stats* st, const RoundState& r, int h) {
  if (!st) return;
  for (int l = 0; l <= PDFS_MAX_H; ++l) {
    st->visited[l] += r.cnt.visited[l];
    st->nonempty[l] += r.cnt.nonempty[l];
    st->bound_pruned[l] += r.cnt.bound_pruned[l];
  }
  const unsigned long long wu = (unsigned long long)words(r.n_unc);
  if (h >= 2) {
    // every active pair within the depth-1/2 loop bounds, times |U|
    const unsigned long long a1 = (unsigned long long)r.amax[1];
    const unsigned long long a2 = (unsigned long long)r.amax[2];
    unsigned long long pairs = 0;
    if (a1 > 0) pairs = a1 * a2 - a1 * (a1 + 1) / 2;   // sum over i < a1 of (a2 - 1 - i)
    st->pair_macs += pairs * (unsigned long long)r.n_unc;
  }
  st->dfs_visits[3] += r.x_vis3;
  st->dfs_visits[4] += r.x_vis4;
  st->dfs_visit_words3 += r.x_vis3 * wu;
  st->dfs_visit_words4 += r.x_vis4 * wu;
  st->dfs_leaves += r.x_leaves;
  st->dfs_fp_leaves += r.x_fp_leaves;
}

void begin_stats(pdfs_ctx* c, pdfs_stats* st) {
  if (st) memset(st, 0, sizeof(*st));
  c->kernel_ns[0] = c->kernel_ns[1] = 0;
  c->kernel_launches[0] = c->kernel_launches[1] = 0;
}

void end_stats(pdfs_ctx* c, pdfs_stats* st) {
  if (!st) return;
  for (int i = 0; i < 2; ++i) {
    st->kernel_ns[i] = c->kernel_ns[i];
    st->kernel_launches[i] = c->kernel_launches[i];
  }
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
  o->score_num = r.score_num; o->score_den = r.score_den;
}

int32_t check_call(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (!c) return PDFS_ERR_INVALID_ARG;
  if (h < 1 || h > PDFS_MAX_H || h > c->G) return fail(c, PDFS_ERR_INVALID_ARG, "h out of range");
  if (q < 1) return fail(c, PDFS_ERR_INVALID_ARG, "alpha_q must be >= 1");
  double smax = (double)p * c->n_tumor + (double)q * c->n_normal;
  if (p > 65535u || q > 65535u || smax >= 1073741824.0)
    return fail(c, PDFS_ERR_INVALID_ARG, "p*n_tumor + q*n_normal must stay below 2^30");
  if (h > 4) return fail(c, PDFS_ERR_UNSUPPORTED, "GPU path runs h = 1..4");
  if (c->prune_mode == PDFS_PRUNE_NONE)
    return fail(c, PDFS_ERR_UNSUPPORTED, "exhaustive mode is not run on the GPU");
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
  c->prune_mode = mode;
  c->time_kernels = opt && (opt->flags & PDFS_OPT_TIME_KERNELS);
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
  hipStream_t s = c->stream;
  const int G = m->G;
  if (c->time_kernels)
    for (hipEvent_t& e : c->ev) CKC(hipEventCreate(&e));

  // Stage the caller's matrices on the device (strided as given).
  const uint64_t* dT = m->tumor;
  const uint64_t* dN = m->normal;
  uint64_t* stageT = nullptr;
  uint64_t* stageN = nullptr;
  if (!m->on_device) {
    CKC(dalloc(&stageT, (size_t)G * m->tumor_stride_words));
    CKC(hipMemcpyAsync(stageT, m->tumor, (size_t)G * m->tumor_stride_words * 8,
                       hipMemcpyHostToDevice, s));
    dT = stageT;
    if (m->n_normal > 0) {
      CKC(dalloc(&stageN, (size_t)G * m->normal_stride_words));
      CKC(hipMemcpyAsync(stageN, m->normal, (size_t)G * m->normal_stride_words * 8,
                         hipMemcpyHostToDevice, s));
      dN = stageN;
    }
  }
  if (m->n_normal == 0) dN = nullptr;
  auto free_stage = [&]() {
    if (stageT) (void)hipFree(stageT);
    if (stageN) (void)hipFree(stageN);
  };

  // Pad bits must be zero.
  int* d_bad = nullptr;
  CKC(dalloc(&d_bad, 1));
  CKC(hipMemsetAsync(d_bad, 0, sizeof(int), s));
  CKC(launch_check_pad(dT, m->tumor_stride_words, G, m->n_tumor, d_bad, s));
  if (dN) CKC(launch_check_pad(dN, m->normal_stride_words, G, m->n_normal, d_bad, s));
  int bad = 0;
  CKC(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CKC(hipStreamSynchronize(s));
  (void)hipFree(d_bad);
  if (bad) {
    free_stage();
    c->err = "nonzero bits past the sample count";
    return bail(PDFS_ERR_INVALID_ARG);
  }

  // Sparsest-first order: stable radix sort of the combined counts.
  uint32_t* counts = nullptr;   // [G] counts, then [G] ids
  uint32_t* counts_sorted = nullptr;
  CKC(dalloc(&counts, 2 * (size_t)G));
  CKC(dalloc(&counts_sorted, (size_t)G));
  CKC(dalloc(&c->perm, (size_t)G));
  CKC(launch_gene_counts(dT, m->tumor_stride_words, dN, m->normal_stride_words, G, wt, wn_in,
                         counts, s));
  size_t tmp_bytes = 0;
  CKC(sort_genes(counts, counts_sorted, reinterpret_cast<int32_t*>(counts + G), c->perm, G,
                 nullptr, &tmp_bytes, s));
  void* tmp = nullptr;
  CKC(hipMalloc(&tmp, tmp_bytes + 256));
  CKC(sort_genes(counts, counts_sorted, reinterpret_cast<int32_t*>(counts + G), c->perm, G, tmp,
                 &tmp_bytes, s));
  CKC(dalloc(&c->Ts, (size_t)G * wt));
  CKC(dalloc(&c->Ns, (size_t)G * c->wn));
  CKC(launch_gather_sorted(dT, m->tumor_stride_words, dN, m->normal_stride_words, c->perm, G, wt,
                           c->wn, c->Ts, c->Ns, s));
  c->h_perm.resize(G);
  CKC(hipMemcpyAsync(c->h_perm.data(), c->perm, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
  std::vector<uint32_t> h_counts(G);
  CKC(hipMemcpyAsync(h_counts.data(), counts_sorted, sizeof(uint32_t) * G,
                     hipMemcpyDeviceToHost, s));
  CKC(hipStreamSynchronize(s));
  (void)hipFree(tmp);
  (void)hipFree(counts);
  (void)hipFree(counts_sorted);
  free_stage();

  // Upper bound of the active list: genes with any tumour mutation.
  CKC(dalloc(&c->U, (size_t)wt));
  CKC(dalloc(&c->cols, (size_t)m->n_tumor));
  CKC(dalloc(&c->act, (size_t)G));
  CKC(dalloc(&c->flags, (size_t)G));
  CKC(dalloc(&c->st, 1));
  CKC(dalloc(&c->rec, 1));
  CKC(dalloc(&c->slots, (size_t)kSlotPhases * kSlotsPerPhase));
  CKC(dalloc(&c->hist, (size_t)kMaxCount + 1));
  CKC(dalloc(&c->tallies, (size_t)kSlotPhases * kPersistBlocks * kTallyN));
  CKC(hipHostMalloc(reinterpret_cast<void**>(&c->h_st), sizeof(RoundState), hipHostMallocDefault));
  CKC(hipHostMalloc(reinterpret_cast<void**>(&c->h_rec), sizeof(RoundRecord), hipHostMallocDefault));
  CKC(hipMemsetAsync(c->st, 0, sizeof(RoundState), s));
  CKC(launch_clear_slots(c->slots, kSlotPhases * kSlotsPerPhase, s));
  {
    Problem P;
    P.G = G; P.n_tumor = m->n_tumor; P.n_normal = m->n_normal; P.wt = wt; P.wn = c->wn;
    P.h = 1; P.p = 1; P.q = 1; P.mode = mode;
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
  CKC(dalloc(&c->TA, rows * 2 * (size_t)c->w64_max));
  CKC(dalloc(&c->NA, rows * (size_t)kMaxWN32));
  CKC(dalloc(&c->A8, rows * (size_t)unpacked_row_bytes(c->w64_max)));
  *out = c;
  return PDFS_OK;
#undef CKC
}

void pdfs_destroy(pdfs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  release(c);
  delete c;
}

int32_t pdfs_best_combo(pdfs_ctx* c, int32_t h, uint32_t p, uint32_t q, const uint64_t* uncovered,
                        pdfs_combo* out, pdfs_stats* stats) {
  int32_t rc = check_call(c, h, p, q);
  if (rc != PDFS_OK) return rc;
  if (!out) return fail(c, PDFS_ERR_INVALID_ARG, "out is NULL");
  auto t0 = std::chrono::steady_clock::now();
  begin_stats(c, stats);
  int n_unc = c->n_tumor;
  if (uncovered) {
    if (!mask_pad_ok(uncovered, c->n_tumor, c->wt))
      return fail(c, PDFS_ERR_INVALID_ARG, "uncovered mask has bits past n_tumor");
    n_unc = popcount_mask(uncovered, c->wt);
    CK(c, hipMemcpyAsync(c->U, uncovered, sizeof(uint64_t) * c->wt, hipMemcpyHostToDevice,
                         c->stream));
  } else {
    CK(c, launch_fill_u(c->U, c->wt, c->n_tumor, c->stream));
  }
  memset(out, 0, sizeof(*out));
  if (n_unc == 0) return PDFS_NO_COMBO;
  rc = run_round(c, h, p, q, c->n_tumor + 1, n_unc);
  if (rc != PDFS_OK) return rc;
  add_counters(stats, *c->h_st, h);
  if (stats) {
    end_stats(c, stats);
    stats->rounds = c->h_rec->found ? 1 : 0;
    stats->ns_total = std::chrono::duration_cast<std::chrono::nanoseconds>(
                          std::chrono::steady_clock::now() - t0).count();
  }
  if (!c->h_rec->found) return PDFS_NO_COMBO;
  fill_combo(out, *c->h_rec, h);
  return PDFS_OK;
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
  int n_unc = c->n_tumor;
  if (initial_uncovered) {
    if (!mask_pad_ok(initial_uncovered, c->n_tumor, c->wt))
      return fail(c, PDFS_ERR_INVALID_ARG, "uncovered mask has bits past n_tumor");
    n_unc = popcount_mask(initial_uncovered, c->wt);
    CK(c, hipMemcpyAsync(c->U, initial_uncovered, sizeof(uint64_t) * c->wt,
                         hipMemcpyHostToDevice, c->stream));
  } else {
    CK(c, launch_fill_u(c->U, c->wt, c->n_tumor, c->stream));
  }
  int rounds = 0;
  while (c->n_tumor - n_unc < K && (max_rounds <= 0 || rounds < max_rounds) && n_unc > 0) {
    rc = run_round(c, h, p, q, K, n_unc);
    if (rc != PDFS_OK) return rc;
    add_counters(stats, *c->h_st, h);
    const RoundRecord& r = *c->h_rec;
    if (!r.found) break;
    if (r.tp <= 0 || r.tp > n_unc) return fail(c, PDFS_ERR_DEVICE, "round made no progress");
    if (rounds < cap) fill_combo(&out[rounds], r, h);
    ++rounds;
    n_unc -= r.tp;
  }
  *n_out = rounds;
  if (final_uncovered) {
    CK(c, hipMemcpyAsync(final_uncovered, c->U, sizeof(uint64_t) * c->wt, hipMemcpyDeviceToHost,
                         c->stream));
    CK(c, hipStreamSynchronize(c->stream));
  }
  if (stats) {
    end_stats(c, stats);
    stats->rounds = rounds;
    stats->ns_total = std::chrono::duration_cast<std::chrono::nanoseconds>(
                          std::chrono::steady_clock::now() - t0).count();
  }
  if (rounds > cap) return fail(c, PDFS_ERR_TRUNCATED, "more rounds than cap");
  return PDFS_OK;
}

}  // extern "C"
