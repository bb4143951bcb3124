// Allocation-free variant of pdfs_best_combo (one argmax round, Alg. 1 step 4
// done as Alg. 2) for callers that cannot allocate device memory: code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// Every per-round buffer the round's kernels use (uncovered-sample list,
// active list, re-packed rows, unpacked bytes for the pair table, pair and
// work lists, work items, argmax slots, counter rows, round state, round
// record) is carved from one file-scope device array, `scratch`, instead of
// the context's own lazily allocated workspace.  The cohort itself (sorted
// rows, permutation, uncovered mask) is the context's, made by pdfs_create.
//
// The array's device address is taken once per device with
// hipGetSymbolAddress when a context is first created there (the device is
// current then), and only that address is passed to kernels and fill
// launches.  Every call on a device shares that device's array and leaves its
// contents behind; a call clears what must start at zero (round state, slots,
// counter rows) itself.  Calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/pdfs.h"
#include "pdfs_dev.h"
#include "pdfs_host.h"

namespace pdfs {

namespace {

// Size of the static scratch array: held on every device the library sets up
// a context on, until the process ends.
#ifndef PDFS_NOALLOC_SCRATCH_MIB
#define PDFS_NOALLOC_SCRATCH_MIB 64
#endif
constexpr size_t kScratchBytes = (size_t)PDFS_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the round workspace inside the scratch array.
struct Layout {
  size_t st, recs, slots, tallies, zero_end;   // [st, zero_end) is cleared per call
  size_t cols, act, flags, TA, NA, A8, N8, hist, cursors, seed, pairs, work, items;
  size_t total;
  unsigned long long pair_cap = 0, item_cap = 0;
};

// Plans the workspace of one round at row width w64max.  The fixed part is
// sized exactly; the pair list (and its bound-mode copy) and the item list
// take what is left, up to the exact bound of nA(nA-1)/2 pairs.  Returns
// false (with the bytes the fixed part needs) when it does not fit.
bool plan(const pdfs_ctx* c, int h, Layout& L, size_t* need) {
  const int nA = c->prune_mode == PDFS_PRUNE_NONE ? c->G : c->nA_max;
  const size_t rows = (size_t)((nA + 127) / 128 * 128 + 128);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.st = take(sizeof(RoundState));
  L.recs = take(sizeof(RoundRecord));
  L.tallies = take((size_t)kSlotPhases * kPersistBlocks * kTallyN * 8);
  L.zero_end = o;
  L.slots = take((size_t)kSlotPhases * kSlotsPerPhase * sizeof(Slot));
  L.cols = take((size_t)c->n_tumor * 4);
  L.act = take((size_t)c->G * 4);
  L.flags = take((size_t)c->G);
  L.TA = take(rows * 2 * (size_t)c->w64_max * 4);
  L.NA = take(rows * (size_t)kMaxWN32 * 4);
  L.A8 = take(rows * (size_t)unpacked_row_bytes(c->w64_max));
  L.N8 = take(h == 2 ? rows * (size_t)unpacked_row_bytes(c->wn) : 0);
  L.hist = take((size_t)(kMaxCount + 1) * 4);
  L.cursors = take((size_t)kSubQueues * kCursorStride * 8);
  L.seed = take((size_t)kSeedCap * 8);
  *need = o;
  if (o >= kScratchBytes) return false;
  L.pairs = L.work = L.items = o;
  if (h >= 3) {
    // The rest holds the pair list (and its bound-mode work copy) and the
    // item list: 8 (16) bytes per pair, plus two 16-byte items per 64-pair
    // batch and 2048 spare items.
    const bool bound = c->prune_mode == PDFS_PRUNE_BOUND;
    const size_t fixed = (size_t)2048 * sizeof(Item) + 3 * 256;
    const size_t avail = kScratchBytes - o;
    if (avail <= fixed + 64 * 17) return false;
    const double per_pair = (bound ? 16.0 : 8.0) + 2.0 * sizeof(Item) / kPairBatch;
    unsigned long long cap = (unsigned long long)((double)(avail - fixed) / per_pair);
    const unsigned long long exact = (unsigned long long)nA * (nA > 0 ? nA - 1 : 0) / 2;
    if (cap > exact) cap = exact;
    if (cap < 64) cap = 64;
    L.pair_cap = cap;
    L.pairs = take(cap * 8);
    L.work = bound ? take(cap * 8) : L.pairs;
    L.item_cap = 2 * ((cap + kPairBatch - 1) / kPairBatch) + 2048;
    L.items = take(L.item_cap * sizeof(Item));
  }
  L.total = o;
  *need = o;
  return o <= kScratchBytes;
}

int32_t nfail(pdfs_ctx* c, int32_t code, const std::string& msg) {
  return ctx_fail(c, code, msg);
}

#define NCK(expr)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return nfail(c, PDFS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

void scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_rc[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
  g_scratch_done[device] = true;
}

}  // namespace pdfs

using namespace pdfs;

extern "C" {

int32_t pdfs_best_combo_noalloc(pdfs_ctx* c, int32_t h, uint32_t p, uint32_t q,
                                const uint64_t* uncovered, pdfs_combo* out, pdfs_stats* stats) {
  int32_t rc = check_call(c, h, p, q);
  if (rc != PDFS_OK) return rc;
  if (!out) return nfail(c, PDFS_ERR_INVALID_ARG, "out is NULL");
  if (h > 4) return nfail(c, PDFS_ERR_UNSUPPORTED, "the allocation-free round takes h <= 4");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices && g_scratch_done[c->device]) {
      if (!g_scratch_ptr[c->device])
        return nfail(c, PDFS_ERR_DEVICE,
                     std::string("static scratch address: ") +
                         hipGetErrorString(g_scratch_rc[c->device]));
      base = static_cast<unsigned char*>(g_scratch_ptr[c->device]);
    }
  }
  if (!base) return nfail(c, PDFS_ERR_DEVICE, "static scratch not set up on this device");
  Layout L;
  size_t need = 0;
  if (!plan(c, h, L, &need))
    return nfail(c, PDFS_ERR_UNSUPPORTED,
                 "round workspace of " + std::to_string(need) + " bytes exceeds the " +
                     std::to_string(kScratchBytes) + "-byte static scratch");
  const auto t0 = std::chrono::steady_clock::now();
  begin_stats(c, stats);
  memset(out, 0, sizeof(*out));
  const int32_t n_unc = set_uncovered(c, uncovered);
  if (n_unc < 0) return n_unc;
  if (n_unc == 0) return PDFS_NO_COMBO;
  const int w64 = dfs_row_words((n_unc + 63) / 64);
  if (w64 < 0 || w64 > c->w64_max) return nfail(c, PDFS_ERR_UNSUPPORTED, "row too wide");

  const Problem P = make_problem(c, h, p, q);
  Work w = make_work(c, w64, c->n_tumor + 1);
  w.st = reinterpret_cast<RoundState*>(base + L.st);
  w.recs = reinterpret_cast<RoundRecord*>(base + L.recs);
  w.rec_cap = 1;
  w.tallies = reinterpret_cast<unsigned long long*>(base + L.tallies);
  w.slots = reinterpret_cast<Slot*>(base + L.slots);
  w.cols = reinterpret_cast<int32_t*>(base + L.cols);
  w.act = reinterpret_cast<int32_t*>(base + L.act);
  w.flags = base + L.flags;
  w.TA = reinterpret_cast<uint32_t*>(base + L.TA);
  w.NA = reinterpret_cast<uint32_t*>(base + L.NA);
  w.A8 = reinterpret_cast<int8_t*>(base + L.A8);
  w.N8 = reinterpret_cast<int8_t*>(base + L.N8);
  w.hist = reinterpret_cast<uint32_t*>(base + L.hist);
  w.cursors = reinterpret_cast<unsigned long long*>(base + L.cursors);
  w.seed_pairs = reinterpret_cast<unsigned long long*>(base + L.seed);
  w.pairs = reinterpret_cast<unsigned long long*>(base + L.pairs);
  w.work_pairs = reinterpret_cast<unsigned long long*>(base + L.work);
  w.items = reinterpret_cast<Item*>(base + L.items);
  w.pair_cap = L.pair_cap;
  w.item_cap = L.item_cap;
  // single-kernel depth 4 (no prefix lists), no deep-walk rings
  w.tri = w.tri_s = nullptr;
  w.tri_rank = nullptr;
  w.c_hist = nullptr;
  w.tri_cap = 0;
  w.deepq = nullptr;

  hipStream_t s = c->stream;
  // what a round expects to start from zero; the rest is written before use
  NCK(launch_zero_u32(base + L.st, (L.zero_end - L.st) / 4, s));
  NCK(launch_clear_slots(w.slots, kSlotPhases * kSlotsPerPhase, s));
  NCK(launch_run_begin(P, w, 1, s));
  const int slot = c->next_slot;
  rc = enqueue_round(c, P, w, c->ev[slot][0], false);
  if (rc != PDFS_OK) return rc;
  RoundState* hs = &c->h_slots[slot];
  NCK(hipMemcpyAsync(hs, w.st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
  NCK(hipMemcpyAsync(c->h_rec, w.recs, sizeof(RoundRecord), hipMemcpyDeviceToHost, s));
  NCK(hipStreamSynchronize(s));
  c->h_st = hs;
  if (c->time_kernels && hs->executed > 0) {
    hipEvent_t* ev = c->ev[slot][0];
    float ms = 0.f;
    if (h >= 2) {
      NCK(hipEventElapsedTime(&ms, ev[0], ev[1]));
      c->kernel_ns[0] += (int64_t)(ms * 1e6);
      c->kernel_launches[0] += 1;
    }
    if (h >= 3) {
      NCK(hipEventElapsedTime(&ms, ev[2], ev[3]));
      c->kernel_ns[1] += (int64_t)(ms * 1e6);
      c->kernel_launches[1] += 1;
    }
  }
  if (hs->overflow & 2) return nfail(c, PDFS_ERR_DEVICE, "corrupt per-wave result slot");
  if (hs->overflow)
    return nfail(c, PDFS_ERR_OUT_OF_MEMORY,
                 "the round's " + std::to_string(hs->n_pairs) +
                     " pairs exceed the static scratch's pair list of " +
                     std::to_string(L.pair_cap));
  end_stats(c, stats, t0);
  if (hs->rounds < 1 || !c->h_rec->found) return PDFS_NO_COMBO;
  fill_combo(out, *c->h_rec, h);
  return PDFS_OK;
}

}  // extern "C"
