// Serving: tables, synchronous multi-query scans, and a continuous-batching
// query server.
//
// The server owns a host thread and `n_streams` HIP streams (default
// priority).  Submitted queries wait in a FIFO; admission refuses a query
// (SCAN_EBUSY) when max_inflight queries are admitted and unfinished, or when
// one more would take the device workspace of admitted queries past the HBM
// budget.  A free stream launches the oldest pending queries (at most
// max_batch) as one batch when the batch is full, when the oldest has waited
// batch_window_us, when no stream is busy (nothing to overlap with), or when a
// stream has just finished (continuous batching).  A batch is one launch of
// the conjunctive query kernel over its queries; its 32-byte result slots come
// back with one copy on the same stream, and the thread polls the stream's
// completion event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "scan_internal.h"
#include "serve_kernels.h"

using namespace scan_dev;

struct scan_table {
  int device = 0;
  uint64_t n = 0, nb = 0;
  uint32_t n_cols = 0;
  uint32_t stage_words = 0;  // LDS words holding one block of every column (shared-decode kernel)
  std::vector<QCol> cols;
  QCol* cols_dev = nullptr;
};

namespace {

// Default launch shape of the query kernel: 64-block windows, and as many
// work-groups per CU as fit (the kernel is bound by dependent-load latency,
// so every resident wavefront helps).
constexpr uint32_t kDefaultWindow = 64;

uint32_t default_wgs_per_cu(const scan_table* t, bool shared) {
  int occ = 0;
  const hipError_t e = shared ? query_shared_occupancy(&occ, t->stage_words) : query_scan_occupancy(&occ);
  if (e != hipSuccess || occ < 1) return 2u;
  return (uint32_t)std::min(occ, 16);
}

// The shared-decode kernel keeps a bit per table column and one block of
// every column in LDS: tables of at most 64 columns whose blocks fit 64 KiB.
bool use_shared(const scan_table* t, uint32_t kernel) {
  return kernel == SCAN_QUERY_SHARED && t->n_cols <= kSharedMaxCols && t->stage_words <= kSharedMaxStageWords;
}

double now_us() {
  using namespace std::chrono;
  return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// Device bytes one admitted query holds: its descriptor and result slot in
// a stream's batch buffers and its pinned result staging.
constexpr uint64_t kQueryBytes = sizeof(QDesc) + 2 * sizeof(QOut);

struct Policy {
  scan_server_config cfg;

  bool admit(uint32_t inflight) const {
    if (inflight >= cfg.max_inflight) return false;
    return (uint64_t)(inflight + 1) * kQueryBytes <= cfg.hbm_budget_bytes;
  }
  // Queries a free stream launches now (0: keep waiting).
  uint32_t launch_count(size_t pending, double oldest_wait_us, uint32_t busy, bool freed) const {
    if (pending == 0) return 0;
    const uint32_t n = (uint32_t)std::min<size_t>(pending, cfg.max_batch);
    if (pending >= cfg.max_batch || oldest_wait_us >= (double)cfg.batch_window_us || busy == 0 || freed) return n;
    return 0;
  }
};

scan_status check_config(scan_ctx* ctx, const scan_server_config* c) {
  if (!c) return fail(ctx, SCAN_EINVAL, "config is NULL");
  if (c->max_inflight == 0 || c->n_streams == 0 || c->n_streams > 16 || c->max_batch == 0)
    return fail(ctx, SCAN_EINVAL, "max_inflight, max_batch must be positive and n_streams in 1..16");
  if (c->max_batch > (1u << 20)) return fail(ctx, SCAN_EINVAL, "max_batch is at most 2^20");
  if (c->window_blocks > 64) return fail(ctx, SCAN_EINVAL, "window_blocks is at most 64");
  if (c->wgs_per_cu > 16) return fail(ctx, SCAN_EINVAL, "wgs_per_cu is at most 16");
  if (c->kernel != SCAN_QUERY_SHARED && c->kernel != SCAN_QUERY_PER_QUERY)
    return fail(ctx, SCAN_EINVAL, "kernel must be SCAN_QUERY_SHARED or SCAN_QUERY_PER_QUERY");
  return SCAN_OK;
}

scan_status check_query(scan_ctx* ctx, const scan_table* t, const scan_query& q) {
  if (q.n_filters < 1 || q.n_filters > (uint32_t)kQueryMaxFilters)
    return fail(ctx, SCAN_EINVAL, "a query has 1..%d filters", kQueryMaxFilters);
  for (uint32_t f = 0; f < q.n_filters; ++f)
    if (q.filter_col[f] >= t->n_cols) return fail(ctx, SCAN_EINVAL, "filter column %u out of range", q.filter_col[f]);
  if (q.sum_col >= t->n_cols) return fail(ctx, SCAN_EINVAL, "sum column %u out of range", q.sum_col);
  return SCAN_OK;
}

QDesc make_desc(const scan_query& q) {
  QDesc d;
  std::memset(&d, 0, sizeof d);
  d.nf = q.n_filters;
  d.sum_col = q.sum_col;
  for (uint32_t f = 0; f < q.n_filters; ++f) {
    d.col[f] = q.filter_col[f];
    d.lo[f] = q.filter[f].lo;
    d.hi[f] = q.filter[f].hi;
  }
  return d;
}

// Device buffers of one batch of up to `cap` queries.
struct BatchSlot {
  uint32_t cap = 0;
  QDesc* q_dev = nullptr;
  QOut* out_dev = nullptr;
  uint32_t* cursor = nullptr;
  QDesc* q_host = nullptr;   // pinned
  QOut* out_host = nullptr;  // pinned

  hipError_t allocate(uint32_t n) {
    cap = std::max(1u, n);
    hipError_t e;
    if ((e = hipMalloc(&q_dev, sizeof(QDesc) * cap)) != hipSuccess) return e;
    if ((e = hipMalloc(&out_dev, sizeof(QOut) * cap)) != hipSuccess) return e;
    if ((e = hipMalloc(&cursor, 256)) != hipSuccess) return e;
    if ((e = hipHostMalloc(&q_host, sizeof(QDesc) * cap, hipHostMallocDefault)) != hipSuccess) return e;
    return hipHostMalloc(&out_host, sizeof(QOut) * cap, hipHostMallocDefault);
  }
  void release() {
    for (void* p : {(void*)q_dev, (void*)out_dev, (void*)cursor})
      if (p) (void)hipFree(p);
    for (void* p : {(void*)q_host, (void*)out_host})
      if (p) (void)hipHostFree(p);
    *this = BatchSlot();
  }
};

// Enqueue setup + scan + result copy of slot.q_host[0..nq) on `st`.  The
// shared-decode kernel runs the queries in launches of at most 64; its grid
// is capped by the number of windows.
hipError_t enqueue_queries(const scan_table* t, BatchSlot& s, uint32_t nq, uint32_t G, uint32_t grid, bool shared,
                           hipStream_t st) {
  hipError_t e = hipMemcpyAsync(s.q_dev, s.q_host, sizeof(QDesc) * nq, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  QArgs a;
  a.cols = t->cols_dev;
  a.q = s.q_dev;
  a.out = s.out_dev;
  a.cursor = s.cursor;
  a.nq = nq;
  a.G = G;
  a.n = t->n;
  a.nb = t->nb;
  a.items = ((t->nb + G - 1) / G) * (uint64_t)nq;
  a.stage_words = t->stage_words;
  a.pad = 0;
  if ((e = launch_query_setup(a, st)) != hipSuccess) return e;
  if (shared) {
    const uint64_t windows = (t->nb + G - 1) / G;
    const uint32_t g = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(grid, windows));
    for (uint32_t off = 0; off < nq && e == hipSuccess; off += kSharedMaxQueries) {
      QArgs c = a;
      c.q = s.q_dev + off;
      c.out = s.out_dev + off;
      c.nq = std::min(kSharedMaxQueries, nq - off);
      c.items = windows;
      e = launch_query_shared(c, g, st);
    }
  } else {
    e = launch_query_scan(a, grid, st);
  }
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(s.out_host, s.out_dev, sizeof(QOut) * nq, hipMemcpyDeviceToHost, st);
}

}  // namespace

// ------------------------------------------------------------------ server

struct Pending {
  uint64_t ticket;
  scan_query q;
  double submit_us;
};

struct scan_server {
  scan_ctx* ctx = nullptr;  // device and compute-unit count only; the server uses its own streams
  const scan_table* table = nullptr;
  Policy pol;
  uint32_t grid = 0, G = 16;
  bool shared = true;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done_ev;
  std::vector<BatchSlot> slots;
  std::vector<std::vector<Pending>> running;  // per stream
  std::deque<Pending> pending;
  std::deque<scan_query_result> done;
  uint32_t inflight = 0;
  uint64_t next_ticket = 1;
  uint64_t batches = 0, launched_queries = 0;
  std::mutex mu;
  std::condition_variable cv_done;
  std::atomic<bool> stop{false};
  std::thread worker;
  hipError_t dev_err = hipSuccess;

  void loop();
};

void scan_server::loop() {
  (void)hipSetDevice(ctx->device);
  while (!stop.load()) {
    bool worked = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      bool freed = false;
      const double t = now_us();
      for (size_t s = 0; s < streams.size(); ++s) {
        if (running[s].empty()) continue;
        const hipError_t q = hipEventQuery(done_ev[s]);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess && dev_err == hipSuccess) dev_err = q;
        for (size_t i = 0; i < running[s].size(); ++i) {
          const Pending& p = running[s][i];
          scan_query_result r;
          std::memset(&r, 0, sizeof r);
          r.ticket = p.ticket;
          r.submit_us = p.submit_us;
          r.done_us = t;
          if (q == hipSuccess) {
            r.count = slots[s].out_host[i].count;
            r.sum = (int64_t)slots[s].out_host[i].sum;
            r.blocks_read = slots[s].out_host[i].blocks;
            r.status = SCAN_OK;
          } else {
            r.status = SCAN_EDEVICE;
          }
          done.push_back(r);
        }
        inflight -= (uint32_t)running[s].size();
        running[s].clear();
        freed = worked = true;
      }
      for (size_t s = 0; s < streams.size() && !pending.empty(); ++s) {
        if (!running[s].empty()) continue;
        uint32_t busy = 0;
        for (auto& r : running) busy += r.empty() ? 0u : 1u;
        const uint32_t n = pol.launch_count(pending.size(), t - pending.front().submit_us, busy, freed);
        if (n == 0) break;
        BatchSlot& sl = slots[s];
        for (uint32_t i = 0; i < n; ++i) {
          running[s].push_back(pending.front());
          pending.pop_front();
          sl.q_host[i] = make_desc(running[s].back().q);
        }
        hipError_t e = enqueue_queries(table, sl, n, G, grid, shared, streams[s]);
        if (e == hipSuccess) e = hipEventRecord(done_ev[s], streams[s]);
        if (e != hipSuccess && dev_err == hipSuccess) dev_err = e;
        ++batches;
        launched_queries += n;
        worked = true;
      }
      if (worked) cv_done.notify_all();
    }
    if (!worked) std::this_thread::sleep_for(std::chrono::microseconds(10));
  }
}

extern "C" {

scan_status scan_table_create(scan_ctx* ctx, const scan_table_column* cols, uint32_t n_cols, scan_table** out) {
  if (!ctx) return SCAN_EINVAL;
  if (!out || !cols || n_cols == 0) return fail(ctx, SCAN_EINVAL, "columns and out must not be NULL/empty");
  *out = nullptr;
  const uint64_t n = cols[0].col.n;
  if (n == 0) return fail(ctx, SCAN_EINVAL, "a table needs rows");
  std::vector<QCol> qc(n_cols);
  for (uint32_t i = 0; i < n_cols; ++i) {
    const scan_table_column& c = cols[i];
    scan_status st = validate_column(ctx, &c.col, c.enc, c.b);
    if (st != SCAN_OK) return st;
    if (c.enc != SCAN_ENC_FOR && c.enc != SCAN_ENC_DICT)
      return fail(ctx, SCAN_EUNSUPPORTED, "table column %u: frame-of-reference or dictionary only", i);
    if (c.col.layout != SCAN_LAYOUT_RM) return fail(ctx, SCAN_EUNSUPPORTED, "table column %u: row-major only", i);
    if (!c.col.zone_min) return fail(ctx, SCAN_EINVAL, "table column %u: zone maps are required", i);
    if (c.col.n != n) return fail(ctx, SCAN_EINVAL, "table column %u: %llu rows, column 0 has %llu", i,
                                  (unsigned long long)c.col.n, (unsigned long long)n);
    QCol& q = qc[i];
    std::memset(&q, 0, sizeof q);
    q.payload = c.col.payload;
    q.refs = c.enc == SCAN_ENC_FOR ? c.col.block_ref : nullptr;
    q.dict = c.col.dict;
    q.zmin = static_cast<const uint32_t*>(c.col.zone_min);
    q.zmax = static_cast<const uint32_t*>(c.col.zone_max);
    q.b = c.b;
    q.enc = (uint32_t)c.enc;
    q.dict_len = c.col.dict_len;
  }
  // staging slots of the shared-decode kernel: 32 b words then a spill word,
  // rounded to 16 bytes, one slot per column
  uint64_t off = 0;
  for (uint32_t i = 0; i < n_cols; ++i) {
    qc[i].stage_off = (uint32_t)std::min<uint64_t>(off, 0xFFFFFFFFu);
    off += 32u * (uint64_t)qc[i].b + 4u;
  }
  scan_table* t = new scan_table();
  t->stage_words = (uint32_t)std::min<uint64_t>(off, 0xFFFFFFFFu);
  t->device = ctx->device;
  t->n = n;
  t->nb = (n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  t->n_cols = n_cols;
  t->cols = qc;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc(&t->cols_dev, sizeof(QCol) * n_cols);
  if (e == hipSuccess) e = hipMemcpy(t->cols_dev, qc.data(), sizeof(QCol) * n_cols, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (t->cols_dev) (void)hipFree(t->cols_dev);
    delete t;
    return hip_fail(ctx, e, "table upload");
  }
  *out = t;
  return SCAN_OK;
}

void scan_table_destroy(scan_table* t) {
  if (!t) return;
  if (t->cols_dev) (void)hipFree(t->cols_dev);
  delete t;
}

scan_status scan_query_run(scan_ctx* ctx, const scan_table* t, const scan_query* queries, size_t n,
                           scan_query_result* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!t || (n && (!queries || !out))) return fail(ctx, SCAN_EINVAL, "table, queries and out must not be NULL");
  if (n == 0) return SCAN_OK;
  if (n > (1u << 20)) return fail(ctx, SCAN_EINVAL, "at most 2^20 queries per call");
  for (size_t i = 0; i < n; ++i) {
    scan_status st = check_query(ctx, t, queries[i]);
    if (st != SCAN_OK) return st;
  }
  const auto tit = ctx->tunes.find(std::make_tuple((int32_t)-2, 0u, (int32_t)-1));
  const scan_tune tn = tit != ctx->tunes.end() ? tit->second : scan_tune{0, 0, 0, 0};
  const bool shared = use_shared(t, (uint32_t)ctx->query_kernel);
  const uint32_t G = tn.window_blocks > 0 ? (uint32_t)std::min(tn.window_blocks, shared ? 32 : 64)
                                          : (shared ? kSharedWindow : kDefaultWindow);
  if (((t->nb + G - 1) / G) * (uint64_t)n >= (1ull << 31)) return fail(ctx, SCAN_EINVAL, "too many work items");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  BatchSlot s;
  e = s.allocate((uint32_t)n);
  if (e != hipSuccess) {
    s.release();
    return fail(ctx, SCAN_ENOMEM, "query buffers: %s", hipGetErrorString(e));
  }
  for (size_t i = 0; i < n; ++i) s.q_host[i] = make_desc(queries[i]);
  const double t0 = now_us();
  const uint32_t grid = (uint32_t)ctx->cus * (tn.wgs_per_cu > 0 ? (uint32_t)std::min(tn.wgs_per_cu, 16)
                                                                   : default_wgs_per_cu(t, shared));
  e = enqueue_queries(t, s, (uint32_t)n, G, grid, shared, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  const double t1 = now_us();
  if (e == hipSuccess)
    for (size_t i = 0; i < n; ++i) {
      scan_query_result r;
      std::memset(&r, 0, sizeof r);
      r.ticket = i;
      r.count = s.out_host[i].count;
      r.sum = (int64_t)s.out_host[i].sum;
      r.blocks_read = s.out_host[i].blocks;
      r.submit_us = t0;
      r.done_us = t1;
      r.status = SCAN_OK;
      out[i] = r;
    }
  s.release();
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "query scan");
}

// The query kernel's tuning is kept under (enc -2, b 0, strategy -1).
scan_status scan_query_set_tune(scan_ctx* ctx, int32_t wgs_per_cu, int32_t window_blocks) {
  if (!ctx) return SCAN_EINVAL;
  if (wgs_per_cu < 0 || wgs_per_cu > 16 || window_blocks < 0 || window_blocks > 64)
    return fail(ctx, SCAN_EINVAL, "wgs_per_cu in 0..16, window_blocks in 0..64");
  scan_tune& t = ctx->tunes[std::make_tuple((int32_t)-2, 0u, (int32_t)-1)];
  t.wg_size = 0;
  t.wgs_per_cu = wgs_per_cu;
  t.window_blocks = window_blocks;
  return SCAN_OK;
}

scan_status scan_query_set_kernel(scan_ctx* ctx, int32_t kernel) {
  if (!ctx) return SCAN_EINVAL;
  if (kernel != SCAN_QUERY_SHARED && kernel != SCAN_QUERY_PER_QUERY)
    return fail(ctx, SCAN_EINVAL, "kernel must be SCAN_QUERY_SHARED or SCAN_QUERY_PER_QUERY");
  ctx->query_kernel = kernel;
  return SCAN_OK;
}

scan_status scan_server_create(scan_ctx* ctx, const scan_table* t, const scan_server_config* cfg,
                               scan_server** out) {
  if (!ctx) return SCAN_EINVAL;
  if (!t || !out) return fail(ctx, SCAN_EINVAL, "table and out must not be NULL");
  scan_status st = check_config(ctx, cfg);
  if (st != SCAN_OK) return st;
  const bool shared = use_shared(t, cfg->kernel);
  const uint32_t G = cfg->window_blocks ? std::min(cfg->window_blocks, shared ? 32u : 64u)
                                        : (shared ? kSharedWindow : kDefaultWindow);
  if (((t->nb + G - 1) / G) * (uint64_t)cfg->max_batch >= (1ull << 31))
    return fail(ctx, SCAN_EINVAL, "max_batch x windows exceeds 2^31 work items");
  *out = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  scan_server* s = new scan_server();
  s->ctx = ctx;
  s->table = t;
  s->pol.cfg = *cfg;
  s->G = G;
  s->shared = shared;
  s->grid = (uint32_t)ctx->cus * (cfg->wgs_per_cu ? cfg->wgs_per_cu : default_wgs_per_cu(t, shared));
  const uint32_t ns = cfg->n_streams;
  s->streams.assign(ns, nullptr);
  s->done_ev.assign(ns, nullptr);
  s->slots.resize(ns);
  s->running.resize(ns);
  for (uint32_t i = 0; i < ns && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = s->slots[i].allocate(cfg->max_batch);
  }
  if (e != hipSuccess) {
    for (uint32_t i = 0; i < ns; ++i) {
      s->slots[i].release();
      if (s->done_ev[i]) (void)hipEventDestroy(s->done_ev[i]);
      if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
    }
    delete s;
    return hip_fail(ctx, e, "server resources");
  }
  s->worker = std::thread([s] { s->loop(); });
  *out = s;
  return SCAN_OK;
}

scan_status scan_server_submit(scan_server* s, const scan_query* q, uint64_t* ticket) {
  if (!s) return SCAN_EINVAL;
  if (!q) return SCAN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->dev_err != hipSuccess) return SCAN_EDEVICE;
  if (q->n_filters < 1 || q->n_filters > (uint32_t)kQueryMaxFilters || q->sum_col >= s->table->n_cols)
    return SCAN_EINVAL;
  for (uint32_t f = 0; f < q->n_filters; ++f)
    if (q->filter_col[f] >= s->table->n_cols) return SCAN_EINVAL;
  if (!s->pol.admit(s->inflight)) return SCAN_EBUSY;
  const uint64_t tk = s->next_ticket++;
  s->pending.push_back(Pending{tk, *q, now_us()});
  ++s->inflight;
  if (ticket) *ticket = tk;
  return SCAN_OK;
}

scan_status scan_server_poll(scan_server* s, scan_query_result* out, size_t max, size_t* n_out, uint32_t wait_us) {
  if (!s || !n_out || (max && !out)) return SCAN_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
  size_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return s->dev_err == hipSuccess ? SCAN_OK : SCAN_EDEVICE;
}

scan_status scan_server_stats(scan_server* s, uint64_t* stats4) {
  if (!s || !stats4) return SCAN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  stats4[0] = s->batches;
  stats4[1] = s->launched_queries;
  stats4[2] = s->inflight;
  stats4[3] = s->pending.size();
  return SCAN_OK;
}

double scan_server_clock_us(void) { return now_us(); }

void scan_server_destroy(scan_server* s) {
  if (!s) return;
  s->stop.store(true);
  if (s->worker.joinable()) s->worker.join();
  for (size_t i = 0; i < s->streams.size(); ++i) {
    (void)hipStreamSynchronize(s->streams[i]);
    s->slots[i].release();
    (void)hipEventDestroy(s->done_ev[i]);
    (void)hipStreamDestroy(s->streams[i]);
  }
  delete s;
}

// Discrete-event run of the server's admission and batching policy on the
// host: arrivals at arrival_us[i] (non-decreasing), a batch of q queries
// occupying its stream for batch_fixed_us + q * per_query_us.  Writes each
// query's launch and completion times (-1 and status SCAN_EBUSY when refused
// at arrival).  Uses the same Policy code as the live server.
scan_status scan_serve_simulate(const scan_server_config* cfg, const double* arrival_us, size_t n,
                                double batch_fixed_us, double per_query_us, double* launch_us, double* done_us,
                                int32_t* status, uint64_t* n_batches) {
  if (!cfg || (n && (!arrival_us || !launch_us || !done_us || !status))) return SCAN_EINVAL;
  if (cfg->max_inflight == 0 || cfg->n_streams == 0 || cfg->n_streams > 16 || cfg->max_batch == 0)
    return SCAN_EINVAL;
  for (size_t i = 1; i < n; ++i)
    if (arrival_us[i] < arrival_us[i - 1]) return SCAN_EINVAL;
  Policy pol;
  pol.cfg = *cfg;
  const uint32_t ns = cfg->n_streams;
  std::vector<double> free_at(ns, -1.0);       // busy until (negative: idle)
  std::vector<std::vector<size_t>> run(ns);
  std::deque<size_t> pend;
  uint32_t inflight = 0;
  uint64_t batches = 0;
  size_t next = 0;
  double t = n ? arrival_us[0] : 0.0;
  while (next < n || !pend.empty() || inflight) {
    // completions at time t
    bool freed = false;
    for (uint32_t s = 0; s < ns; ++s)
      if (!run[s].empty() && free_at[s] <= t) {
        for (size_t i : run[s]) done_us[i] = free_at[s];
        inflight -= (uint32_t)run[s].size();
        run[s].clear();
        free_at[s] = -1.0;
        freed = true;
      }
    // arrivals at time t
    while (next < n && arrival_us[next] <= t) {
      if (pol.admit(inflight)) {
        pend.push_back(next);
        ++inflight;
        status[next] = SCAN_OK;
      } else {
        status[next] = SCAN_EBUSY;
        launch_us[next] = -1.0;
        done_us[next] = -1.0;
      }
      ++next;
    }
    // launches
    for (uint32_t s = 0; s < ns && !pend.empty(); ++s) {
      if (!run[s].empty()) continue;
      uint32_t busy = 0;
      for (auto& r : run) busy += r.empty() ? 0u : 1u;
      const uint32_t k = pol.launch_count(pend.size(), t - arrival_us[pend.front()], busy, freed);
      if (k == 0) break;
      for (uint32_t i = 0; i < k; ++i) {
        run[s].push_back(pend.front());
        launch_us[pend.front()] = t;
        pend.pop_front();
      }
      free_at[s] = t + batch_fixed_us + per_query_us * k;
      ++batches;
    }
    // next event
    double tn = 1e300;
    if (next < n) tn = std::min(tn, arrival_us[next]);
    for (uint32_t s = 0; s < ns; ++s)
      if (!run[s].empty()) tn = std::min(tn, free_at[s]);
    // a window still to expire (one that already expired waits for a stream)
    if (!pend.empty() && arrival_us[pend.front()] + (double)cfg->batch_window_us > t)
      tn = std::min(tn, arrival_us[pend.front()] + (double)cfg->batch_window_us);
    if (tn >= 1e299) break;
    t = tn;
  }
  if (n_batches) *n_batches = batches;
  return SCAN_OK;
}

}  // extern "C"
