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
#include <atomic>
#include <chrono>
#include <condition_variable>
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
// The split granularity of the depth-first search -- depth-3 candidates per
// work item, and in bound mode the number of highest-count pairs expanded
// before the rest -- changes only scheduling, never results.  The tuner times
// the first round of a representative instance for each candidate setting
// and keeps the fastest per instance class (h, row width, active-gene
// bucket, pruning mode) for the life of the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tuned;

int bucket_of(int n) {
  int b = 0;
  while ((1 << (b + 1)) <= n) ++b;
  return b;
}

double time_first_round(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (set_uncovered(c, nullptr) <= 0) return 1e30;
  (void)hipStreamSynchronize(c->stream);
  const auto t0 = Clock::now();
  if (run_blocking(c, h, p, q, c->n_tumor + 1, 1, c->n_tumor) != PDFS_OK) return 1e30;
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

void autotune(pdfs_ctx* c, int h, uint32_t p, uint32_t q) {
  if (h < 3) return;
  const auto key = std::make_tuple(h, dfs_row_words((c->n_tumor + 63) / 64), bucket_of(c->nA_max),
                                   c->prune_mode);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      c->chunk_items = it->second.first;
      c->seed_pairs_n = it->second.second;
      return;
    }
  }
  static const int chunks[] = {64, 128, 256, 512, 1024};
  static const int seeds[] = {128, 256, 1024};
  const int nseed = c->prune_mode == PDFS_PRUNE_BOUND ? 3 : 1;
  double best = 1e30;
  int bc = c->chunk_items, bs = c->seed_pairs_n;
  c->chunk_items = 256;
  c->seed_pairs_n = 256;
  (void)time_first_round(c, h, p, q);   // warm-up (allocations, graph capture)
  for (int ci : chunks) {
    for (int si = 0; si < nseed; ++si) {
      c->chunk_items = ci;
      c->seed_pairs_n = nseed == 1 ? 256 : seeds[si];
      double t = time_first_round(c, h, p, q);
      t = std::min(t, time_first_round(c, h, p, q));
      if (t < best) { best = t; bc = c->chunk_items; bs = c->seed_pairs_n; }
    }
  }
  c->chunk_items = bc;
  c->seed_pairs_n = bs;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tuned[key] = {bc, bs};
}

}  // namespace

// ===================================================================== batch
struct pdfs_batch {
  int device = 0;
  bool autotune = false;
  std::vector<hipStream_t> streams;
  std::vector<pdfs_ctx*> ctx;
  std::string err;
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
