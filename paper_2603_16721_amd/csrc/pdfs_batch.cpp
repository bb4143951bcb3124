// Batched and served front ends of libpdfs (see include/pdfs.h).
//
// Both keep one context per cohort (device-resident bit matrices, uncovered
// mask and round state) and drive many greedy runs from one host thread
// without blocking: each run advances by chunks of rounds (one captured HIP
// graph per row width, replayed), and a chunk's completion is observed with
// an event query.  Runs are spread over one stream per hardware queue, so the
// rounds of different cohorts overlap on the device.  The arithmetic is the
// plain path's: every result equals pdfs_wsc_run on that cohort alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <sys/stat.h>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/pdfs.h"
#include "pdfs_dev.h"
#include "pdfs_host.h"

using namespace pdfs;

namespace {

constexpr int kStreams = 4;   // one per hardware queue of the device

using Clock = std::chrono::steady_clock;

void add_stats(pdfs_stats* dst, const pdfs_stats& s) {
  for (int l = 0; l <= PDFS_MAX_H; ++l) {
    dst->visited[l] += s.visited[l];
    dst->nonempty[l] += s.nonempty[l];
    dst->bound_pruned[l] += s.bound_pruned[l];
    dst->dfs_visits[l] += s.dfs_visits[l];
  }
  dst->rounds += s.rounds;
  for (int i = 0; i < 3; ++i) {
    dst->kernel_ns[i] += s.kernel_ns[i];
    dst->kernel_launches[i] += s.kernel_launches[i];
  }
  dst->pair_macs += s.pair_macs;
  dst->dfs_leaves += s.dfs_leaves;
  dst->dfs_fp_leaves += s.dfs_fp_leaves;
  dst->dfs_visit_words3 += s.dfs_visit_words3;
  dst->dfs_visit_words4 += s.dfs_visit_words4;
}

// ------------------------------------------------------------------ tuner
// How the depth-first search is cut into work changes only scheduling,
// never results.  The tuner times the first round of a representative
// instance for each candidate and keeps the fastest per instance class (h,
// row width, active-gene bucket, pruning mode, device):
//   * split depth: for h = 4 under empty-prefix pruning, depth-3 prefixes
//     with long depth-4 streams become work units of their own (listed,
//     bucketed and expanded in 64-prefix tiles; split depth 3) or stay in
//     their pair's work item (split depth 2), and the stream length from
//     which a prefix is listed;
//   * tile shape of a work item: 64 pairs x `chunk` depth-3 candidates;
//   * bound mode: the number of highest-count pairs expanded first.
// Choices are kept for the process and in a JSON file (PDFS_TUNE_CACHE, else
// $XDG_CACHE_HOME/pdfs/tune.json or ~/.cache/pdfs/tune.json) read when the
// first batch is tuned and rewritten after every new entry.
struct TuneChoice {
  int chunk = 256, seed = 256, split = 3, long_stream = kLongStream;
  double ms = 0.0;
};
using TuneKey = std::tuple<int, int, int, int, std::string>;

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tuned;
bool g_tune_loaded = false;

int bucket_of(int n) {
  int b = 0;
  while ((1 << (b + 1)) <= n) ++b;
  return b;
}

std::string tune_cache_path() {
  if (const char* p = std::getenv("PDFS_TUNE_CACHE")) return p;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/pdfs/tune.json";
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/pdfs/tune.json";
  return std::string();
}

std::string device_tag(int device) {
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

// One entry per line: {"h":4,"w":16,"g":13,"mode":1,"device":"gfx950...","chunk":256,
// "seed":256,"split":3,"long_stream":384,"ms":1.23}
void load_tune_cache() {
  g_tune_loaded = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    int h = 0, w = 0, g = 0, mode = 0;
    TuneChoice c;
    char dev[128] = {0};
    if (std::sscanf(line,
                    " {\"h\":%d,\"w\":%d,\"g\":%d,\"mode\":%d,\"device\":\"%127[^\"]\","
                    "\"chunk\":%d,\"seed\":%d,\"split\":%d,\"long_stream\":%d,\"ms\":%lf",
                    &h, &w, &g, &mode, dev, &c.chunk, &c.seed, &c.split, &c.long_stream,
                    &c.ms) == 10)
      g_tuned[std::make_tuple(h, w, g, mode, std::string(dev))] = c;
  }
  std::fclose(f);
}

void save_tune_cache() {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  // the directory chain, one level at a time (existing levels are kept)
  const size_t slash = path.rfind('/');
  for (size_t i = path.find('/', 1); slash != std::string::npos && i != std::string::npos && i <= slash;
       i = path.find('/', i + 1))
    (void)mkdir(path.substr(0, i).c_str(), 0755);
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "[\n");
  size_t k = 0;
  for (const auto& kv : g_tuned) {
    const TuneChoice& c = kv.second;
    std::fprintf(f,
                 "{\"h\":%d,\"w\":%d,\"g\":%d,\"mode\":%d,\"device\":\"%s\",\"chunk\":%d,"
                 "\"seed\":%d,\"split\":%d,\"long_stream\":%d,\"ms\":%.4f}%s\n",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 std::get<3>(kv.first), std::get<4>(kv.first).c_str(), c.chunk, c.seed, c.split,
                 c.long_stream, c.ms, ++k < g_tuned.size() ? "," : "");
  }
  std::fprintf(f, "]\n");
  std::fclose(f);
  (void)std::rename(tmp.c_str(), path.c_str());
}

double time_first_round(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (set_uncovered(c, nullptr) <= 0) return 1e30;
  (void)hipStreamSynchronize(c->stream);
  const auto t0 = Clock::now();
  if (run_blocking(c, h, p, q, c->n_tumor + 1, 1, c->n_tumor) != PDFS_OK) return 1e30;
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

void apply(pdfs_ctx* c, const TuneChoice& t) {
  c->chunk_items = t.chunk;
  c->seed_pairs_n = t.seed;
  c->split3 = t.split == 3;
  c->long_stream = t.long_stream;
}

void autotune(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (h < 3) return;
  const TuneKey key = std::make_tuple(h, dfs_row_words((c->n_tumor + 63) / 64),
                                      bucket_of(c->nA_max), c->prune_mode, device_tag(c->device));
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      apply(c, it->second);
      return;
    }
  }
  std::vector<TuneChoice> cand;
  static const int chunks[] = {64, 128, 256, 512, 1024};
  static const int seeds[] = {128, 256, 1024};
  static const int streams[] = {256, 384, 768};
  const bool bound = c->prune_mode == PDFS_PRUNE_BOUND;
  const bool split_choice = h == 4 && c->prune_mode == PDFS_PRUNE_EMPTY;
  for (int ci : chunks) {
    TuneChoice t;
    t.chunk = ci;
    if (bound) {
      for (int sd : seeds) {
        t.seed = sd;
        cand.push_back(t);
      }
    } else if (split_choice) {
      t.split = 2;
      cand.push_back(t);
      t.split = 3;
      for (int ls : streams) {
        t.long_stream = ls;
        cand.push_back(t);
      }
    } else {
      cand.push_back(t);
    }
  }
  TuneChoice best;
  best.ms = 1e30;
  apply(c, TuneChoice());
  (void)time_first_round(c, h, p, q);   // warm-up (allocations, graph capture)
  for (const TuneChoice& t : cand) {
    apply(c, t);
    double s = time_first_round(c, h, p, q);
    s = std::min(s, time_first_round(c, h, p, q));
    if (s * 1e3 < best.ms) {
      best = t;
      best.ms = s * 1e3;
    }
  }
  apply(c, best);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tuned[key] = best;
  save_tune_cache();
}

}  // namespace

// ===================================================================== batch
struct pdfs_batch {
  int device = 0;
  bool autotune = false;
  std::vector<hipStream_t> streams;
  std::vector<pdfs_ctx*> ctx;
  std::string err;
  // ---- one launch per round step over every instance (h in {3, 4})
  hipStream_t ms = nullptr;                  // stream of the batched launches
  RoundState* st_all = nullptr;              // device: round state of each instance
  RoundState* h_st_all = nullptr;            // pinned: kDepth copies of st_all
  Slot* logs = nullptr;                      // device: per instance, phase: kLogCap leaves
  BatchQueue* queues = nullptr;              // device: one per h group and kind
  // per grouping of the instances into row-width ranges: the descriptor
  // array (every instance at its range's width) and the captured round
  std::map<std::vector<int>, BatchDesc*> descs;
  std::map<std::vector<int>, bool> desc_fresh;   // uploaded for the current run
  std::map<std::pair<std::vector<int>, int>, hipGraphExec_t> graphs;
  int max_ranges = 0;                        // ranges per h (0: 1 bound, 4 empty)
  hipEvent_t done_ev[kDepth] = {};
  hipEvent_t fork_ev = nullptr;              // ranges' depth-first launches run side by side
  std::vector<hipEvent_t> join_ev;
  int n_alloc = 0;                           // instances the batched buffers hold
  bool streams_only = false;                 // PDFS_OPT_BATCH_STREAMS: no batched launches
  bool one_launch = false;                   // PDFS_OPT_BATCH_ONE_LAUNCH: batched launches in every mode
};

namespace {

int32_t batch_fail(pdfs_batch* b, int32_t code, const std::string& msg) {
  b->err = msg;
  return code;
}

// The failing instance's own detail.
int32_t batch_fail(pdfs_batch* b, int32_t code, int inst) {
  b->err = "instance " + std::to_string(inst) + ": " +
           (inst >= 0 && inst < (int)b->ctx.size() ? b->ctx[inst]->err : std::string());
  return code;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Batched runs as one launch per round step.  Instances are ordered h = 3
// first, then h = 4 (the depth-first kernels are built per h); every light
// step covers all of them with one block row per instance, each depth-first
// step drains one shared queue per h group.  The row width of a chunk of
// rounds is the largest any live instance needs (narrower instances run at
// it: any width >= ceil(|U|/64) gives the same results).
constexpr int kMaxRanges = 8;   // row-width ranges per h

struct MultiRun {
  int n = 0;
  std::vector<int> order;    // position -> instance index (h = 3 first, widest first)
  int max_G = 0;
  int n_cu = 256;
  bool bound = false;
  bool tiles = false;        // some instance uses the two-phase depth 4
  int max_ranges = 1;        // row-width ranges per h
  uint32_t p = 1, q = 1;
  std::vector<int> target;   // per position
  std::vector<int> h;        // per position
};

// A grouping: consecutive ranges of positions with one row width each,
// flattened as (h, first position, count, w64) quadruples.
using Grouping = std::vector<int>;

// Ranges of equal h over the fixed position order, each at the widest width
// its live members need (done instances need nothing); adjacent ranges merge
// (the wider width wins) until each h has at most max_ranges, the pair whose
// widths are closest first.
Grouping make_grouping(const MultiRun& m, const std::vector<int>& need) {
  Grouping g;
  for (int hh = 3; hh <= 4; ++hh) {
    std::vector<std::array<int, 3>> r;   // first, count, width
    for (int k = 0; k < m.n; ++k) {
      if (m.h[k] != hh) continue;
      const int wk = need[k];
      if (!r.empty() && (r.back()[2] == wk || wk == 0)) {
        r.back()[1] += 1;
      } else if (!r.empty() && r.back()[2] == 0) {
        r.back()[1] += 1;
        r.back()[2] = wk;
      } else {
        r.push_back({k, 1, wk});
      }
    }
    while ((int)r.size() > m.max_ranges) {
      size_t best = 0;
      double ratio = 1e30;
      for (size_t j = 0; j + 1 < r.size(); ++j) {
        const double a = std::max(1, r[j][2]), c = std::max(1, r[j + 1][2]);
        const double x = std::max(a, c) / std::min(a, c);
        if (x < ratio) { ratio = x; best = j; }
      }
      r[best][1] += r[best + 1][1];
      r[best][2] = std::max(r[best][2], r[best + 1][2]);
      r.erase(r.begin() + (long)best + 1);
    }
    for (const auto& x : r) {
      g.push_back(hh);
      g.push_back(x[0]);
      g.push_back(x[1]);
      g.push_back(std::max(1, x[2]));
    }
  }
  return g;
}

#define BCK(expr)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return batch_fail(b, e_ == hipErrorOutOfMemory ? PDFS_ERR_OUT_OF_MEMORY : PDFS_ERR_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

int32_t ensure_multi_buffers(pdfs_batch* b, int n) {
  if (b->n_alloc >= n) return PDFS_OK;
  if (b->st_all) (void)hipFree(b->st_all);
  if (b->h_st_all) (void)hipHostFree(b->h_st_all);
  if (b->logs) (void)hipFree(b->logs);
  b->st_all = nullptr;
  b->h_st_all = nullptr;
  b->logs = nullptr;
  BCK(hipMalloc(reinterpret_cast<void**>(&b->st_all), sizeof(RoundState) * n));
  BCK(hipHostMalloc(reinterpret_cast<void**>(&b->h_st_all), sizeof(RoundState) * n * kDepth,
                    hipHostMallocDefault));
  BCK(hipMalloc(reinterpret_cast<void**>(&b->logs),
                sizeof(Slot) * (size_t)n * kSlotPhases * kLogCap));
  if (!b->queues)
    BCK(hipMalloc(reinterpret_cast<void**>(&b->queues), sizeof(BatchQueue) * 2 * kMaxRanges * 2));
  for (hipEvent_t& e : b->done_ev)
    if (!e) BCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (!b->fork_ev) BCK(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  while ((int)b->join_ev.size() < 2 * kMaxRanges) {
    hipEvent_t e = nullptr;
    BCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->join_ev.push_back(e);
  }
  // descriptor arrays and graphs hold the old addresses
  for (auto& kv : b->descs) (void)hipFree(kv.second);
  b->descs.clear();
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  b->n_alloc = n;
  return PDFS_OK;
}

// The descriptor array of a grouping for this run (uploaded on first use;
// never rewritten while the run may still read it).
int32_t descs_for(pdfs_batch* b, const MultiRun& m, const Grouping& g, BatchDesc** out) {
  auto it = b->descs.find(g);
  if (it == b->descs.end()) {
    BatchDesc* d = nullptr;
    BCK(hipMalloc(reinterpret_cast<void**>(&d), sizeof(BatchDesc) * m.n));
    it = b->descs.emplace(g, d).first;
    b->desc_fresh[g] = false;
  }
  if (!b->desc_fresh[g]) {
    std::vector<BatchDesc> h((size_t)m.n);
    for (size_t r = 0; r < g.size(); r += 4) {
      const int w64 = g[r + 3];
      for (int k = g[r + 1]; k < g[r + 1] + g[r + 2]; ++k) {
        pdfs_ctx* c = b->ctx[m.order[k]];
        // the instance's row buffers must hold rows of this width
        if (w64 > c->w64_max)
          return batch_fail(b, PDFS_ERR_DEVICE, "instance " + std::to_string(m.order[k]) +
                                                    ": row buffers narrower than its range");
        h[k].P = make_problem(c, m.h[k], m.p, m.q);
        Work w = make_work(c, w64, m.target[k]);
        w.st = b->st_all + k;
        w.slot_log = b->logs + (size_t)k * kSlotPhases * kLogCap;
        h[k].w = w;
      }
    }
    BCK(hipMemcpy(it->second, h.data(), sizeof(BatchDesc) * m.n, hipMemcpyHostToDevice));
    b->desc_fresh[g] = true;
  }
  *out = it->second;
  return PDFS_OK;
}

// One round of every instance: light steps over all, depth-first steps per
// range (one shared queue and one launch at the range's width each).
int32_t enqueue_multi_round(pdfs_batch* b, const MultiRun& m, BatchDesc* bd, const Grouping& g) {
  hipStream_t s = b->ms;
  const int n = m.n;
  BCK(launch_round_begin_m(bd, n, s));
  BCK(launch_active_m(bd, n, m.max_G, s));
  BCK(launch_gather_active_m(bd, n, m.max_G, s));
  BCK(launch_pairs_m(bd, n, s));
  // The ranges of a depth-first step go out side by side on the batch's
  // streams (fork from and join back into the round's stream), so that one
  // range's tail overlaps the next range's work.
  const int nr = (int)g.size() / 4;
  auto range_stream = [&](int r) { return b->streams[(size_t)r % b->streams.size()]; };
  auto fork = [&]() -> int32_t {
    if (nr < 2) return PDFS_OK;
    BCK(hipEventRecord(b->fork_ev, s));
    for (int r = 1; r < nr && r < (int)b->streams.size(); ++r)
      BCK(hipStreamWaitEvent(range_stream(r), b->fork_ev, 0));
    return PDFS_OK;
  };
  auto join = [&]() -> int32_t {
    if (nr < 2) return PDFS_OK;
    for (int r = 1; r < nr && r < (int)b->streams.size(); ++r) {
      BCK(hipEventRecord(b->join_ev[r], range_stream(r)));
      BCK(hipStreamWaitEvent(s, b->join_ev[r], 0));
    }
    return PDFS_OK;
  };
  auto dfs_step = [&](int phase) -> int32_t {
    int32_t e = fork();
    if (e != PDFS_OK) return e;
    for (int r = 0; r < nr; ++r) {
      const int* x = &g[(size_t)r * 4];
      BatchQueue* q = b->queues + r;
      BCK(launch_batch_queue(bd + x[1], x[2], q, phase, 0, range_stream(r)));
      BCK(launch_dfs_m(x[0], x[3], m.bound, bd + x[1], q, phase, m.n_cu, range_stream(r)));
    }
    return join();
  };
  int32_t rc = PDFS_OK;
  if (m.bound) {
    BCK(launch_seed_select_m(bd, n, s));
    BCK(launch_make_items_m(bd, n, true, s));
    if ((rc = dfs_step(1)) != PDFS_OK) return rc;
    BCK(launch_filter_pairs_m(bd, n, s));
    BCK(launch_make_items_m(bd, n, false, s));
    if ((rc = dfs_step(2)) != PDFS_OK) return rc;
  } else {
    BCK(launch_use_all_pairs_m(bd, n, s));
    BCK(launch_make_items_m(bd, n, false, s));
    if (m.tiles) BCK(launch_tri_begin_m(bd, n, s));
    if ((rc = dfs_step(2)) != PDFS_OK) return rc;
    if (m.tiles) {
      BCK(launch_sort_triples_m(bd, n, s));
      if ((rc = fork()) != PDFS_OK) return rc;
      for (int r = 0; r < nr; ++r) {
        const int* x = &g[(size_t)r * 4];
        if (x[0] != 4) continue;
        BatchQueue* q = b->queues + 2 * kMaxRanges + r;
        BCK(launch_batch_queue(bd + x[1], x[2], q, 1, 1, range_stream(r)));
        BCK(launch_dfs4_tiles_m(x[3], bd + x[1], q, m.n_cu, range_stream(r)));
      }
      if ((rc = join()) != PDFS_OK) return rc;
    }
  }
  BCK(launch_finish_round_m(bd, n, s));
  return PDFS_OK;
}

// `rounds` batched rounds of a grouping: replays of one captured round.
int32_t enqueue_multi_rounds(pdfs_batch* b, const MultiRun& m, const Grouping& g, int rounds) {
  BatchDesc* bd = nullptr;
  int32_t rc = descs_for(b, m, g, &bd);
  if (rc != PDFS_OK) return rc;
  const auto key = std::make_pair(g, (m.bound ? 1 : 0) | (m.tiles ? 2 : 0));
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    BCK(hipStreamBeginCapture(b->ms, hipStreamCaptureModeThreadLocal));
    rc = enqueue_multi_round(b, m, bd, g);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->ms, &gr);
    if (rc != PDFS_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    BCK(ec);
    hipGraphExec_t e = nullptr;
    const hipError_t ei = hipGraphInstantiate(&e, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    BCK(ei);
    it = b->graphs.emplace(key, e).first;
  }
  for (int k = 0; k < rounds; ++k) BCK(hipGraphLaunch(it->second, b->ms));
  return PDFS_OK;
}

int words64(int n) { return (n + 63) / 64; }

// The greedy loop of every instance through batched launches.
int32_t run_multi(pdfs_batch* b, const int32_t* h, uint32_t p, uint32_t q, const int32_t* target,
                  pdfs_combo* const* outs, const int32_t* caps, int32_t* n_outs, pdfs_stats* stats,
                  std::chrono::steady_clock::time_point t0) {
  const int n = (int)b->ctx.size();
  MultiRun m;
  m.n = n;
  m.p = p;
  m.q = q;
  m.bound = b->ctx[0]->prune_mode == PDFS_PRUNE_BOUND;
  m.n_cu = b->ctx[0]->n_cu;
  m.max_ranges = b->max_ranges > 0 ? std::min(b->max_ranges, kMaxRanges) : (m.bound ? 1 : 4);
  int32_t rc = ensure_multi_buffers(b, n);
  if (rc != PDFS_OK) return rc;
  // earlier work of the instances (creation, tuning) may sit on any of the
  // batch's streams; everything below runs on one
  for (hipStream_t s : b->streams) BCK(hipStreamSynchronize(s));
  b->ms = b->streams[0];
  for (auto& kv : b->desc_fresh) kv.second = false;
  std::vector<int> w0((size_t)n);   // first-round width of each instance
  for (int i = 0; i < n; ++i) {
    pdfs_ctx* c = b->ctx[i];
    c->stream = b->ms;
    const int32_t u = set_uncovered(c, nullptr);
    if (u < 0) return batch_fail(b, u, i);
    rc = prepare_run(c, h[i], u);
    if (rc != PDFS_OK) return batch_fail(b, rc, i);
    m.tiles = m.tiles || c->two_phase;
    // counter rows: the batched kernels write row 0 of a phase (and the pair
    // table its first rows); the rest must read zero
    BCK(launch_zero_u32(c->tallies, (size_t)kSlotPhases * kPersistBlocks * kTallyN * 2, b->ms));
    w0[i] = dfs_row_words(words64(u > 0 ? u : 1));
    if (w0[i] < 0) return batch_fail(b, PDFS_ERR_UNSUPPORTED, "row too wide");
    m.max_G = std::max(m.max_G, c->G);
  }
  // positions: h = 3 first, then h = 4, each widest first, so that instances
  // of close widths sit in one range
  for (int hh = 3; hh <= 4; ++hh) {
    std::vector<int> idx;
    for (int i = 0; i < n; ++i)
      if (h[i] == hh) idx.push_back(i);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return w0[a] > w0[c]; });
    m.order.insert(m.order.end(), idx.begin(), idx.end());
  }
  std::vector<int> need((size_t)n);
  for (int k = 0; k < n; ++k) {
    const int i = m.order[k];
    m.h.push_back(h[i]);
    m.target.push_back(target && target[i] > 0 ? target[i] : b->ctx[i]->n_tumor);
    need[k] = w0[i];
  }
  Grouping g = make_grouping(m, need);
  // an instance's rows are packed at its range's width; ranges merge and
  // split as the run goes on, but no width exceeds the widest first-round
  // one, to which every instance's row buffers are regrown
  const int w_all = *std::max_element(w0.begin(), w0.end());
  for (int i = 0; i < n; ++i) {
    rc = grow_row_width(b->ctx[i], w_all);
    if (rc != PDFS_OK) return batch_fail(b, rc, i);
  }
  {
    BatchDesc* bd = nullptr;
    if ((rc = descs_for(b, m, g, &bd)) != PDFS_OK) return rc;
    BCK(launch_run_begin_m(bd, n, 0, b->ms));
  }
  // chunks of batched rounds, kDepth in flight, each ending with a copy of
  // every instance's state; the grouping of a chunk comes from the newest
  // states read
  int inflight = 0, slot = 0, chunk = 1;
  int executed_before = 0;
  auto t_prev = Clock::now();
  const RoundState* hs = nullptr;
  bool finished = false;
  while (!finished) {
    while (inflight < kDepth) {
      const int sl = (slot + inflight) % kDepth;
      if ((rc = enqueue_multi_rounds(b, m, g, chunk)) != PDFS_OK) return rc;
      BCK(hipMemcpyAsync(b->h_st_all + (size_t)sl * n, b->st_all, sizeof(RoundState) * n,
                         hipMemcpyDeviceToHost, b->ms));
      BCK(hipEventRecord(b->done_ev[sl], b->ms));
      ++inflight;
    }
    BCK(hipEventSynchronize(b->done_ev[slot]));
    hs = b->h_st_all + (size_t)slot * n;
    --inflight;
    slot = (slot + 1) % kDepth;
    finished = true;
    int executed = 0;
    // instances whose pair list was too small: their round stopped uncommitted;
    // once everything queued has drained, grow their lists and go on
    bool regrown = false;
    for (int k = 0; k < n; ++k) {
      if (hs[k].overflow != kOverflowPairs) continue;
      if (!regrown) {
        BCK(hipStreamSynchronize(b->ms));
        regrown = true;
      }
      pdfs_ctx* c = b->ctx[m.order[k]];
      rc = grow_pair_list(c, hs[k].n_pairs);
      if (rc != PDFS_OK) return batch_fail(b, rc, m.order[k]);
      Work w = make_work(c, 1, m.target[k]);
      w.st = b->st_all + k;
      BCK(launch_run_resume(w, b->ms));
    }
    if (regrown) {
      // the descriptors and captured rounds hold the old list addresses; the
      // chunk still in flight was a no-op for the regrown instances
      for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
      b->graphs.clear();
      for (auto& kv : b->desc_fresh) kv.second = false;
      inflight = 0;
      finished = false;
      continue;
    }
    for (int k = 0; k < n; ++k) {
      const RoundState& st = hs[k];
      if (st.overflow & 2) return batch_fail(b, PDFS_ERR_DEVICE, "instance " +
                                             std::to_string(m.order[k]) + ": corrupt result slot");
      if (st.overflow)
        return batch_fail(b, PDFS_ERR_OUT_OF_MEMORY, "instance " + std::to_string(m.order[k]) +
                                                     ": list capacity exceeded");
      if (st.executed > b->ctx[m.order[k]]->n_tumor + 2)
        return batch_fail(b, PDFS_ERR_DEVICE, "greedy loop did not stop");
      executed = std::max(executed, st.executed);
      if (st.done) {
        need[k] = 0;
        continue;
      }
      finished = false;
      const int unc = b->ctx[m.order[k]]->n_tumor - st.covered;
      need[k] = std::min(need[k], dfs_row_words(words64(unc > 0 ? unc : 1)));
    }
    g = make_grouping(m, need);
    const auto now = Clock::now();
    const double ns = (double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - t_prev).count();
    t_prev = now;
    const int ran = executed - executed_before;
    executed_before = executed;
    if (ran > 0) {
      int c = (int)(1.0e6 / (ns / ran));
      c = c < 1 ? 1 : (c > kMaxChunk ? kMaxChunk : c);
      chunk = c > 2 * chunk ? 2 * chunk : c;
    }
  }
  // the chunks still in flight are no-ops; wait for them before reading
  BCK(hipStreamSynchronize(b->ms));
  int32_t result = PDFS_OK;
  for (int k = 0; k < n; ++k) {
    const int i = m.order[k];
    pdfs_ctx* c = b->ctx[i];
    const RoundState& st = hs[k];
    const int rounds = st.rounds;
    n_outs[i] = rounds;
    const int cap = caps ? caps[i] : 0;
    const int nc = std::min(rounds, cap);
    if (nc > 0 && outs && outs[i]) {
      std::vector<RoundRecord> recs((size_t)nc);
      BCK(hipMemcpy(recs.data(), c->recs, sizeof(RoundRecord) * nc, hipMemcpyDeviceToHost));
      for (int r = 0; r < nc; ++r) fill_combo(&outs[i][r], recs[r], h[i]);
    }
    if (rounds > cap) {
      result = PDFS_ERR_TRUNCATED;
      b->err = "instance " + std::to_string(i) + ": more rounds than its cap";
    }
    if (stats) {
      for (int l = 0; l <= PDFS_MAX_H; ++l) {
        stats->visited[l] += st.tot.visited[l];
        stats->nonempty[l] += st.tot.nonempty[l];
        stats->bound_pruned[l] += st.tot.bound_pruned[l];
      }
      stats->rounds += st.rounds;
      stats->pair_macs += st.tx_pair_macs;
      stats->dfs_visits[3] += st.tx_vis3;
      stats->dfs_visits[4] += st.tx_vis4;
      stats->dfs_leaves += st.tx_leaves;
      stats->dfs_fp_leaves += st.tx_fp_leaves;
      stats->dfs_visit_words3 += st.tx_vis_words3;
      stats->dfs_visit_words4 += st.tx_vis_words4;
    }
  }
  if (stats)
    stats->ns_total = std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
  return result;
}

}  // namespace

extern "C" {

const char* pdfs_batch_last_error(const pdfs_batch* b) {
  return b ? b->err.c_str() : create_error().c_str();
}

int32_t pdfs_batch_create(const pdfs_matrix* inst, int32_t n, const pdfs_options* opt,
                          pdfs_batch** out) {
  if (!out || !inst || n < 1)
    return ctx_fail(nullptr, PDFS_ERR_INVALID_ARG, "need out, inst and n >= 1");
  *out = nullptr;
  pdfs_batch* b = new pdfs_batch();
  b->device = opt ? opt->device : 0;
  b->autotune = opt && (opt->flags & PDFS_OPT_AUTOTUNE);
  b->streams_only = opt && (opt->flags & PDFS_OPT_BATCH_STREAMS);
  b->one_launch = opt && (opt->flags & PDFS_OPT_BATCH_ONE_LAUNCH);
  if (b->streams_only && b->one_launch) {
    delete b;
    return ctx_fail(nullptr, PDFS_ERR_INVALID_ARG,
                    "PDFS_OPT_BATCH_STREAMS and PDFS_OPT_BATCH_ONE_LAUNCH exclude each other");
  }
  if (hipSetDevice(b->device) != hipSuccess) {
    delete b;
    return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipSetDevice failed");
  }
  for (int k = 0; k < kStreams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      pdfs_batch_destroy(b);
      return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
    b->streams.push_back(s);
  }
  for (int i = 0; i < n; ++i) {
    pdfs_options o{};
    if (opt) o = *opt;
    o.stream = b->streams[i % kStreams];
    if (!(o.flags & PDFS_OPT_TIME_KERNELS)) o.flags |= PDFS_OPT_GRAPHS;
    pdfs_ctx* c = nullptr;
    const int32_t rc = create_ctx(&inst[i], &o, &c, nullptr, true);
    if (rc != PDFS_OK) {
      const std::string why = "instance " + std::to_string(i) + ": " + create_error();
      pdfs_batch_destroy(b);
      return ctx_fail(nullptr, rc, why);
    }
    b->ctx.push_back(c);
  }
  *out = b;
  return PDFS_OK;
}

int32_t pdfs_batch_run(pdfs_batch* b, const int32_t* h, uint32_t p, uint32_t q,
                       const int32_t* target, pdfs_combo* const* outs, const int32_t* caps,
                       int32_t* n_outs, pdfs_stats* stats) {
  if (!b) return PDFS_ERR_INVALID_ARG;
  b->err.clear();
  if (!h || !n_outs) return batch_fail(b, PDFS_ERR_INVALID_ARG, "h and n_outs must not be NULL");
  const int n = (int)b->ctx.size();
  const auto t0 = Clock::now();
  if (stats) memset(stats, 0, sizeof(*stats));
  for (int i = 0; i < n; ++i) {
    const int32_t rc = check_call(b->ctx[i], h[i], p, q);
    if (rc != PDFS_OK) return batch_fail(b, rc, i);
    n_outs[i] = 0;
  }
  if (b->autotune)
    for (int i = 0; i < n; ++i) autotune(b->ctx[i], h[i], p, q);
  // one launch per round step over every instance when all take it (h = 3, 4
  // with empty or bound pruning) and it is the faster way for the mode (bound
  // pruning) or asked for; the stream-parallel runs below otherwise
  const int pm = b->ctx[0]->prune_mode;
  bool multi = n <= kMaxBatch && pm != PDFS_PRUNE_NONE && !b->streams_only &&
               (b->one_launch || pm == PDFS_PRUNE_BOUND);
  for (int i = 0; i < n; ++i)
    multi = multi && (h[i] == 3 || h[i] == 4) && b->ctx[i]->tn_literal == b->ctx[0]->tn_literal;
  if (multi) return run_multi(b, h, p, q, target, outs, caps, n_outs, stats, t0);
  for (int i = 0; i < n; ++i) {
    pdfs_ctx* c = b->ctx[i];
    begin_stats(c, nullptr);
    const int32_t n_unc = set_uncovered(c, nullptr);
    if (n_unc < 0) return batch_fail(b, n_unc, i);
    const int K = (target && target[i] > 0) ? target[i] : c->n_tumor;
    const int32_t rc = run_start(c, h[i], p, q, K, 0, n_unc);
    if (rc != PDFS_OK) return batch_fail(b, rc, i);
  }
  // feed every run without blocking until all have stopped
  int32_t first_err = PDFS_OK;
  int err_inst = -1;
  int remaining = n;
  std::vector<bool> live(n, true);
  while (remaining > 0) {
    for (int i = 0; i < n; ++i) {
      if (!live[i]) continue;
      const int32_t rc = run_enqueue(b->ctx[i]);
      if (rc != PDFS_OK) {
        if (first_err == PDFS_OK) { first_err = rc; err_inst = i; }
        live[i] = false;
        --remaining;
      }
    }
    bool progressed = false;
    for (int i = 0; i < n; ++i) {
      if (!live[i]) continue;
      bool ready = false, done = false;
      const int32_t rc = run_poll(b->ctx[i], false, &ready, &done);
      progressed |= ready;
      if (rc != PDFS_OK || done) {
        if (rc != PDFS_OK && first_err == PDFS_OK) { first_err = rc; err_inst = i; }
        live[i] = false;
        --remaining;
      }
    }
    if (!progressed && remaining > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (first_err != PDFS_OK) return batch_fail(b, first_err, err_inst);
  int32_t result = PDFS_OK;
  for (int i = 0; i < n; ++i) {
    pdfs_ctx* c = b->ctx[i];
    int32_t rounds = 0;
    const int cap = caps ? caps[i] : 0;
    const int32_t rc = run_records(c, outs ? outs[i] : nullptr, cap, &rounds);
    if (rc != PDFS_OK) return batch_fail(b, rc, i);
    n_outs[i] = rounds;
    if (rounds > cap) {
      result = PDFS_ERR_TRUNCATED;
      b->err = "instance " + std::to_string(i) + ": more rounds than its cap";
    }
    if (stats) {
      pdfs_stats s;
      memset(&s, 0, sizeof(s));
      end_stats(c, &s, t0);
      add_stats(stats, s);
    }
  }
  if (stats)
    stats->ns_total = std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
  return result;
}

void pdfs_batch_destroy(pdfs_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : b->descs) (void)hipFree(kv.second);
  if (b->st_all) (void)hipFree(b->st_all);
  if (b->h_st_all) (void)hipHostFree(b->h_st_all);
  if (b->logs) (void)hipFree(b->logs);
  if (b->queues) (void)hipFree(b->queues);
  for (hipEvent_t e : b->done_ev)
    if (e) (void)hipEventDestroy(e);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (hipEvent_t e : b->join_ev) (void)hipEventDestroy(e);
  for (pdfs_ctx* c : b->ctx) pdfs_destroy(c);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // extern "C"

// ==================================================================== server
namespace {

struct Request {
  uint64_t ticket = 0;
  int h = 0;
  uint32_t p = 1, q = 1;
  int target = 0;
  pdfs_matrix m{};
  std::vector<uint64_t> T, N;   // copies, row stride = words
  size_t bytes = 0;              // estimated device footprint
  Clock::time_point t_submit, t_done;
  pdfs_ctx* ctx = nullptr;
  RoundState* pinned = nullptr;
  int32_t status = PDFS_PENDING;
  std::string err;               // detail of a failed solve
  std::vector<pdfs_combo> result;
  int32_t rounds = 0;
};

}  // namespace

struct pdfs_server {
  int device = 0;
  int prune_mode = PDFS_PRUNE_BOUND;
  std::vector<hipStream_t> streams;
  std::vector<RoundState*> pinned_pool;   // kPinnedBytes of pinned state per active slot
  size_t budget = 0, used = 0;
  int max_active = 8;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::vector<std::shared_ptr<Request>> active;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  int next_stream = 0;
  hipStream_t admit_stream = nullptr;   // ingest of admitted requests
  std::string err;   // detail of the last failing call (guarded by mu)
};

namespace {

int32_t server_fail(pdfs_server* s, int32_t code, const std::string& msg) {
  std::lock_guard<std::mutex> g(s->mu);
  s->err = msg;
  return code;
}

// Finishes a run: records copied to the request, device memory released.
void complete(pdfs_server* s, const std::shared_ptr<Request>& r, int32_t status) {
  if (status == PDFS_OK && r->ctx) {
    r->result.resize((size_t)r->ctx->n_tumor + 1);
    int32_t rounds = 0;
    status = run_records(r->ctx, r->result.data(), (int32_t)r->result.size(), &rounds);
    r->rounds = rounds;
    r->result.resize((size_t)std::min<int32_t>(rounds, (int32_t)r->result.size()));
  }
  if (status != PDFS_OK && status != PDFS_ERR_TRUNCATED)
    r->err = r->ctx ? r->ctx->err : create_error();
  if (r->ctx) {
    pdfs_destroy(r->ctx);
    r->ctx = nullptr;
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (r->pinned) s->pinned_pool.push_back(r->pinned);
  r->pinned = nullptr;
  s->used -= r->bytes;
  r->t_done = Clock::now();
  r->status = status;
  r->T.clear();
  r->T.shrink_to_fit();
  r->N.clear();
  r->N.shrink_to_fit();
  s->cv.notify_all();
}

// Admission: FIFO; the head request waits until a slot is free and its
// footprint fits both the budget and the device's free memory.
bool admit_one(pdfs_server* s) {
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->queue.empty() || (int)s->active.size() >= s->max_active || s->pinned_pool.empty())
      return false;
    r = s->queue.front();
    if (s->used + r->bytes > s->budget) return false;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && r->bytes + (64ull << 20) > free_b)
      return false;
    s->queue.pop_front();
    s->used += r->bytes;
    r->pinned = s->pinned_pool.back();
    s->pinned_pool.pop_back();
  }
  // Ingest (copy, pad check, sort, first active count) runs on the server's
  // own admission stream, so its synchronisations never wait for the rounds
  // that running requests have queued; the run then joins a shared stream.
  pdfs_options o{};
  o.prune_mode = s->prune_mode;
  o.device = s->device;
  o.stream = s->admit_stream;
  o.flags = PDFS_OPT_GRAPHS;
  int32_t rc = create_ctx(&r->m, &o, &r->ctx, r->pinned, true);
  if (rc == PDFS_OK) {
    r->ctx->stream = s->streams[s->next_stream++ % (int)s->streams.size()];
    rc = check_call(r->ctx, r->h, r->p, r->q);
  }
  int32_t n_unc = 0;
  if (rc == PDFS_OK) {
    n_unc = set_uncovered(r->ctx, nullptr);
    if (n_unc < 0) rc = n_unc;
  }
  if (rc == PDFS_OK) {
    const int K = r->target > 0 ? r->target : r->ctx->n_tumor;
    rc = run_start(r->ctx, r->h, r->p, r->q, K, 0, n_unc);
  }
  if (rc != PDFS_OK) {
    complete(s, r, rc);
    return true;
  }
  std::lock_guard<std::mutex> g(s->mu);
  s->active.push_back(r);
  return true;
}

void worker_loop(pdfs_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->stop && s->queue.empty() && s->active.empty()) return;
      if (s->queue.empty() && s->active.empty())
        s->cv.wait_for(g, std::chrono::milliseconds(5));
    }
    while (admit_one(s)) {
    }
    std::vector<std::shared_ptr<Request>> act;
    {
      std::lock_guard<std::mutex> g(s->mu);
      act = s->active;
    }
    bool progressed = false;
    for (auto& r : act) {
      int32_t rc = run_enqueue(r->ctx);
      bool ready = false, done = false;
      if (rc == PDFS_OK) rc = run_poll(r->ctx, false, &ready, &done);
      progressed |= ready;
      if (rc != PDFS_OK || done) {
        {
          std::lock_guard<std::mutex> g(s->mu);
          s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        }
        complete(s, r, rc);
        progressed = true;
      }
    }
    if (!progressed && !act.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

const char* pdfs_server_last_error(const pdfs_server* s) {
  thread_local std::string copy;
  if (!s) return create_error().c_str();
  pdfs_server* m = const_cast<pdfs_server*>(s);
  std::lock_guard<std::mutex> g(m->mu);
  copy = s->err;
  return copy.c_str();
}

int32_t pdfs_server_create(const pdfs_options* opt, uint64_t hbm_budget_bytes, int32_t max_active,
                           pdfs_server** out) {
  if (!out) return ctx_fail(nullptr, PDFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  const int mode = opt ? opt->prune_mode : PDFS_PRUNE_BOUND;
  if (mode < PDFS_PRUNE_NONE || mode > PDFS_PRUNE_BOUND)
    return ctx_fail(nullptr, PDFS_ERR_INVALID_ARG, "unknown prune mode");
  pdfs_server* s = new pdfs_server();
  s->device = opt ? opt->device : 0;
  s->prune_mode = mode;
  s->max_active = max_active > 0 ? max_active : 8;
  if (hipSetDevice(s->device) != hipSuccess) {
    delete s;
    return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipSetDevice failed");
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete s;
    return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipMemGetInfo failed");
  }
  s->budget = hbm_budget_bytes ? (size_t)hbm_budget_bytes : free_b / 10 * 9;
  for (int k = 0; k < kStreams; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      pdfs_server_destroy(s);
      return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(st);
  }
  if (hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking) != hipSuccess) {
    pdfs_server_destroy(s);
    return ctx_fail(nullptr, PDFS_ERR_DEVICE, "hipStreamCreateWithFlags failed");
  }
  for (int k = 0; k < s->max_active; ++k) {
    RoundState* p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), kPinnedBytes, hipHostMallocDefault) !=
        hipSuccess) {
      pdfs_server_destroy(s);
      return ctx_fail(nullptr, PDFS_ERR_OUT_OF_MEMORY, "pinned round-state pool");
    }
    s->pinned_pool.push_back(p);
  }
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return PDFS_OK;
}

int32_t pdfs_server_submit(pdfs_server* s, const pdfs_matrix* m, int32_t h, uint32_t p,
                           uint32_t q, int32_t target, uint64_t* ticket) {
  if (!s) return PDFS_ERR_INVALID_ARG;
  if (!m || !ticket || m->on_device)
    return server_fail(s, PDFS_ERR_INVALID_ARG, "need a host matrix and a ticket pointer");
  if (m->G < 1 || m->n_tumor < 1 || m->n_normal < 0 || !m->tumor)
    return server_fail(s, PDFS_ERR_INVALID_ARG, "need G >= 1, n_tumor >= 1, n_normal >= 0");
  const int wt = (m->n_tumor + 63) / 64;
  const int wn = m->n_normal > 0 ? (m->n_normal + 63) / 64 : 0;
  if (m->tumor_stride_words < wt || (wn && (!m->normal || m->normal_stride_words < wn)))
    return server_fail(s, PDFS_ERR_INVALID_ARG, "matrix stride below the row length");
  if (h < 1 || h > PDFS_MAX_H || h > m->G || q < 1)
    return server_fail(s, PDFS_ERR_INVALID_ARG, "h out of range or alpha_q < 1");
  auto r = std::make_shared<Request>();
  r->t_submit = Clock::now();
  r->h = h; r->p = p; r->q = q; r->target = target;
  r->T.resize((size_t)m->G * wt);
  int nA = 0;
  for (int g = 0; g < m->G; ++g) {
    uint64_t any = 0;
    for (int k = 0; k < wt; ++k) {
      const uint64_t v = m->tumor[(size_t)g * m->tumor_stride_words + k];
      r->T[(size_t)g * wt + k] = v;
      any |= v;
    }
    nA += any != 0;
  }
  if (wn) {
    r->N.resize((size_t)m->G * wn);
    for (int g = 0; g < m->G; ++g)
      for (int k = 0; k < wn; ++k)
        r->N[(size_t)g * wn + k] = m->normal[(size_t)g * m->normal_stride_words + k];
  }
  r->m = *m;
  r->m.on_device = 0;
  r->m.tumor = r->T.data();
  r->m.tumor_stride_words = wt;
  r->m.normal = wn ? r->N.data() : nullptr;
  r->m.normal_stride_words = wn;
  r->bytes = footprint_bytes(m->G, m->n_tumor, m->n_normal, nA, h, s->prune_mode);
  std::lock_guard<std::mutex> g(s->mu);
  if (r->bytes > s->budget) {
    s->err = "request footprint " + std::to_string(r->bytes) + " B above the server budget " +
             std::to_string(s->budget) + " B";
    return PDFS_ERR_OUT_OF_MEMORY;
  }
  r->ticket = s->next_ticket++;
  s->queue.push_back(r);
  s->tickets[r->ticket] = r;
  *ticket = r->ticket;
  s->cv.notify_all();
  return PDFS_OK;
}

int32_t pdfs_server_poll(pdfs_server* s, uint64_t ticket, pdfs_combo* out, int32_t cap,
                         int32_t* n_out, int64_t* latency_ns) {
  if (!s) return PDFS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) {
    s->err = "unknown ticket " + std::to_string(ticket);
    return PDFS_ERR_INVALID_ARG;
  }
  auto r = it->second;
  if (r->status == PDFS_PENDING) return PDFS_PENDING;
  const int32_t status = r->status;
  if (status != PDFS_OK) s->err = "ticket " + std::to_string(ticket) + ": " + r->err;
  if (status == PDFS_OK) {
    const int n = std::min<int32_t>(cap, (int32_t)r->result.size());
    for (int i = 0; i < n && out; ++i) out[i] = r->result[(size_t)i];
    if (n_out) *n_out = r->rounds;
  }
  if (latency_ns)
    *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(r->t_done - r->t_submit).count();
  s->tickets.erase(it);
  if (status == PDFS_OK && r->rounds > cap) {
    s->err = "ticket " + std::to_string(ticket) + ": more rounds than cap";
    return PDFS_ERR_TRUNCATED;
  }
  return status;
}

int32_t pdfs_server_drain(pdfs_server* s) {
  if (!s) return PDFS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> g(s->mu);
  s->cv.wait(g, [&] { return s->queue.empty() && s->active.empty(); });
  return PDFS_OK;
}

void pdfs_server_destroy(pdfs_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
  for (RoundState* p : s->pinned_pool) (void)hipHostFree(p);
  delete s;
}

}  // extern "C"
