// Batched scans: host side.  A batch is planned once: validation, column
// descriptors, work items, zone-map segments and device buffers, then one
// planning pass on the device
//   setup (class counts, dictionary code ranges)
//   -> [zone-map features -> selector MLP]  (when a selector is loaded)
//   -> select (strategy per column, written on the device)
//   -> [class pruning on the host, see prune_classes]
// then the class lists, built on the host in item order (so that a plan, and
// the static schedule the class scans follow over it, is the same however
// the device ran), whose strategies and lists every replay reuses (the items, the
// selector and the zone maps are fixed for the life of the batch).  The
// replay sequence
//   reset (result slots) -> the class scans that have items (persistent,
//   static schedule over each list), in sequence (forking them over graph
//   branches is an option; running concurrently they contend and measured
//   slower)
// is captured into a HIP graph, so a replay is one hipGraphLaunch whatever
// the number of columns; the 32-byte result slots come back with one copy.
// If capture or instantiation fails the same sequence is enqueued launch by
// launch.  The same column descriptors serve the single-column selector
// (scan_run with SCAN_STRAT_AUTO) and the feature export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch_kernels.h"
#include "scan_internal.h"

using namespace scan_dev;

namespace scan_dev {
hipError_t launch_batch_setup(const BatchArgs& a, hipStream_t st);
hipError_t launch_batch_features(const BatchCol* cols, uint32_t n_cols, const BatchWork* segs, uint32_t n_segs,
                                 FeatPart* parts, float* X, hipStream_t st);
hipError_t launch_batch_select(BatchCol* cols, uint32_t n_cols, const float* scores, int32_t k, float margin,
                               BatchOut* out, hipStream_t st);
hipError_t launch_batch_reset(const BatchCol* cols, uint32_t n_cols, BatchOut* out, hipStream_t st);
hipError_t launch_mlp_forward(const float* theta, const float* X, uint32_t rows, float* out, hipStream_t st);
}  // namespace scan_dev

namespace {

constexpr uint32_t kMaxWindow = 64;  // a wavefront's block-survivor list holds 64 entries
constexpr int kMaxBranches = 4;      // graph branches the class scans are forked over

// Device buffers of a batch (or of the one-column selector scratch).
struct BatchBuffers {
  BatchCol* cols = nullptr;
  BatchWork* work = nullptr;
  uint32_t* lists = nullptr;
  uint32_t* counters = nullptr;  // per-class item counts [12]
  BatchOut* out = nullptr;
  BatchOut* out_host = nullptr;  // pinned
  float* feats = nullptr;
  float* scores = nullptr;
  BatchWork* segs = nullptr;     // zone-map segments (selector features)
  FeatPart* fparts = nullptr;    // their sums
  uint32_t n_segs = 0;

  void release() {
    for (void* p : {(void*)cols, (void*)work, (void*)lists, (void*)counters, (void*)out, (void*)feats, (void*)scores,
                    (void*)segs, (void*)fparts})
      if (p) (void)hipFree(p);
    if (out_host) (void)hipHostFree(out_host);
    *this = BatchBuffers();
  }

  hipError_t allocate(size_t n_cols, size_t n_work, size_t n_seg) {
    const size_t nc = std::max<size_t>(1, n_cols), nw = std::max<size_t>(1, n_work), ns = std::max<size_t>(1, n_seg);
    hipError_t e;
    if ((e = hipMalloc(&cols, sizeof(BatchCol) * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&work, sizeof(BatchWork) * nw)) != hipSuccess) return e;
    if ((e = hipMalloc(&lists, sizeof(uint32_t) * nw * kBatchClasses)) != hipSuccess) return e;
    if ((e = hipMalloc(&counters, sizeof(uint32_t) * kBatchClasses)) != hipSuccess) return e;
    if ((e = hipMalloc(&out, sizeof(BatchOut) * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&feats, sizeof(float) * 6 * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&scores, sizeof(float) * 8 * nc)) != hipSuccess) return e;
    if ((e = hipMalloc(&segs, sizeof(BatchWork) * ns)) != hipSuccess) return e;
    if ((e = hipMalloc(&fparts, sizeof(FeatPart) * ns)) != hipSuccess) return e;
    n_segs = (uint32_t)n_seg;
    return hipHostMalloc(&out_host, sizeof(BatchOut) * nc, hipHostMallocDefault);
  }
};

BatchArgs make_args(const BatchBuffers& m, uint32_t n_cols, uint32_t n_work, int cls) {
  BatchArgs a;
  a.cols = m.cols;
  a.work = m.work;
  a.lists = m.lists;
  a.counts = m.counters;
  a.out = m.out;
  a.n_cols = n_cols;
  a.n_work = n_work;
  a.cls = cls;
  a.pad = 0;
  return a;
}

// Host descriptors of the columns, their validation status and the work
// items (windows of up to `window` blocks of every non-empty valid column).
void plan_cols(scan_ctx* ctx, const scan_item* items, size_t n, uint32_t window, std::vector<BatchCol>& cols,
               std::vector<int32_t>& status, std::vector<BatchWork>* work, std::vector<BatchWork>& segs) {
  segs.clear();
  cols.resize(n);
  status.assign(n, SCAN_OK);
  for (size_t i = 0; i < n; ++i) {
    const scan_item& it = items[i];
    BatchCol c;
    std::memset(&c, 0, sizeof c);
    c.requested = it.strategy;
    c.enc = it.enc;
    c.b = it.b;
    scan_status st = validate_column(ctx, &it.col, it.enc, it.b);
    if (st == SCAN_OK && it.col.layout != SCAN_LAYOUT_RM)
      st = fail(ctx, SCAN_EUNSUPPORTED, "batched scans read row-major columns");
    if (st == SCAN_OK && it.strategy >= 0 && (it.strategy & SCAN_ALL_MATCH))
      st = fail(ctx, SCAN_EUNSUPPORTED, "batched scans do not take the all-match shortcut");
    if (st == SCAN_OK && it.strategy >= 0) {
      st = check_strategy(ctx, &it.col, it.enc, it.b, it.strategy);
      const int dec = it.strategy & 3;
      if (st == SCAN_OK && dec != SCAN_DEC_RM_LDS && dec != SCAN_DEC_RM_DIRECT)
        st = fail(ctx, SCAN_EUNSUPPORTED, "batched scans use the RM-LDS or RM-direct decoder");
    }
    if (st != SCAN_OK) {
      status[i] = st;
      c.flags = kColSkip;
      c.strategy = it.strategy;
      cols[i] = c;
      continue;
    }
    c.payload = it.col.payload;
    c.refs = it.col.block_ref;
    c.bases = it.col.block_base;
    c.dict = it.col.dict;
    c.dict_len = it.col.dict_len;
    c.zmin = it.col.zone_min;
    c.zmax = it.col.zone_max;
    c.n = it.col.n;
    c.nb = (it.col.n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
    c.tail = c.nb ? (uint32_t)(it.col.n - (c.nb - 1) * SCAN_BLOCK_VALUES) : 0u;
    c.lo = it.pred.lo;
    c.hi = it.pred.hi;
    bool empty = it.col.n == 0 || it.pred.lo >= it.pred.hi;
    if (it.enc == SCAN_ENC_FOR && !empty) {
      const int64_t lo = std::max<int64_t>(it.pred.lo, 0), hi = std::min<int64_t>(it.pred.hi, (int64_t)1 << 32);
      if (lo >= hi) empty = true;
      else {
        c.lo32 = (uint32_t)lo;
        c.hi32m1 = (uint32_t)(hi - 1);
      }
    }
    const bool zm = it.col.zone_min != nullptr;
    c.flags = (empty ? kColEmpty : 0u) | (zm ? kColHasZm : 0u);
    uint32_t mask = 0;
    for (int q = 0; q < 8; ++q)
      if (zm || !((q >> 2) & 1)) mask |= 1u << q;
    c.valid_mask = mask;
    int32_t h = heuristic_strategy(&it.col, it.enc, it.b) & ~SCAN_ALL_MATCH;
    if ((h & 3) != SCAN_DEC_RM_LDS && (h & 3) != SCAN_DEC_RM_DIRECT) h = (h & ~3) | SCAN_DEC_RM_DIRECT;
    c.heuristic = h;
    c.strategy = it.strategy >= 0 ? it.strategy : h;
    // zone-map segments of every column with zone maps (the selector's
    // features read them, also for an empty predicate)
    c.fseg0 = (uint32_t)segs.size();
    if (zm)
      for (uint64_t k = 0; k < c.nb; k += kFeatSegBlocks)
        segs.push_back(BatchWork{(uint32_t)i, (uint32_t)std::min<uint64_t>(kFeatSegBlocks, c.nb - k), k});
    c.fsegs = (uint32_t)segs.size() - c.fseg0;
    cols[i] = c;
    // items of four windows, one per wavefront of the work-group that takes
    // the item: fewer items (each costs its descriptor loads, pipeline start
    // and result atomics) and no wavefront alone on a dense item
    const uint64_t span = 4u * (uint64_t)window;
    if (work && !empty)
      for (uint64_t k = 0; k < c.nb; k += span)
        work->push_back(BatchWork{(uint32_t)i, (uint32_t)std::min<uint64_t>(span, c.nb - k), k});
  }
}

// Setup, then (with selector parameters) features and network scores, then
// selection: enqueued on `st`.
hipError_t enqueue_select(const BatchBuffers& m, uint32_t n_cols, const float* theta, float margin, hipStream_t st) {
  hipError_t e = launch_batch_setup(make_args(m, n_cols, 0, 0), st);
  if (e != hipSuccess || n_cols == 0) return e;
  if (theta) {
    e = launch_batch_features(m.cols, n_cols, m.segs, m.n_segs, m.fparts, m.feats, st);
    if (e != hipSuccess) return e;
    e = launch_mlp_forward(theta, m.feats, n_cols, m.scores, st);
    if (e != hipSuccess) return e;
  }
  return launch_batch_select(m.cols, n_cols, theta ? m.scores : nullptr, 8, margin, m.out, st);
}

// Selector class of a row-major strategy: decoder bit, mode, zone maps.
int selector_class(int32_t s) { return (s & 1) | (((s >> 2) & 1) << 1) | (((s >> 3) & 1) << 2); }

// The network predicts each column's time alone; a class scan costs a launch
// and a drain on top of its columns' times (scan_batch_set_class_cost).
// Columns the network moves away from their heuristic strategy into a class
// that no heuristic or explicit column uses are moved back when the
// predicted gains (exp of the predicted log-times, microseconds) of all the
// class's columns add up to less than `class_us`.
void prune_classes(std::vector<BatchCol>& cols, const std::vector<float>& scores, double class_us) {
  uint32_t base = 0;
  double gain[kBatchClasses] = {};
  auto learned = [](const BatchCol& c) {
    return !(c.flags & (kColEmpty | kColSkip)) && c.requested < 0 && c.strategy != c.heuristic;
  };
  for (size_t i = 0; i < cols.size(); ++i) {
    const BatchCol& c = cols[i];
    if (c.flags & (kColEmpty | kColSkip)) continue;
    const int k = batch_class(c.enc, c.strategy);
    if (!learned(c)) {
      base |= 1u << k;
      continue;
    }
    const float* sc = &scores[i * 8];
    gain[k] += std::exp((double)sc[selector_class(c.heuristic)]) - std::exp((double)sc[selector_class(c.strategy)]);
  }
  for (BatchCol& c : cols) {
    if (!learned(c)) continue;
    const int k = batch_class(c.enc, c.strategy);
    if (!((base >> k) & 1u) && gain[k] < class_us) c.strategy = c.heuristic;
  }
}

// Class scans with items, from the planned strategies.
uint32_t used_classes(const std::vector<BatchCol>& cols) {
  uint32_t mask = 0;
  for (const BatchCol& c : cols)
    if (!(c.flags & (kColEmpty | kColSkip))) mask |= 1u << batch_class(c.enc, c.strategy);
  return mask;
}

}  // namespace

struct BatchPlan {
  size_t n_items = 0;
  uint32_t n_work = 0;
  std::vector<BatchCol> cols;
  std::vector<int32_t> status;
  BatchBuffers mem;
  bool selector = false;
  uint32_t grid = 0;
  uint32_t grid_cls[kBatchClasses] = {};  // grid clamped to the work-groups that fit at once
  uint32_t cls_mask = 0;                  // class scans a replay launches
  uint32_t kernels = 0;                   // kernels per replay
  hipGraphExec_t exec = nullptr;          // the captured replay (null: direct launches)
  bool forked = false;                    // class scans on parallel graph branches
  float margin = 0.0f;                    // the selector's margin when prepared
  uint32_t pruned = 0;                    // columns moved back to the heuristic (prune_classes)
  int order = 0;                          // class-list order (scan_batch_set_order)
};

static void free_plan(BatchPlan* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->mem.release();
  delete b;
}

// One-column scratch of the selector path of scan_run, per context.
struct PickScratch {
  BatchBuffers mem;
};
static std::map<const scan_ctx*, PickScratch*>& pick_scratch() {
  static std::map<const scan_ctx*, PickScratch*> m;
  return m;
}

void destroy_batches(scan_ctx* ctx) {
  for (auto& kv : ctx->batches) free_plan(kv.second);
  ctx->batches.clear();
  auto& ps = pick_scratch();
  auto it = ps.find(ctx);
  if (it != ps.end()) {
    it->second->mem.release();
    delete it->second;
    ps.erase(it);
  }
}

// The replay sequence on `st`.  With nbr > 0 branch streams (graph capture)
// the class scans are forked over them after the reset kernel (ev[0]) and
// joined back (ev[1..nbr]): class scans touch disjoint columns, so they may
// run concurrently.
static hipError_t enqueue_batch(BatchPlan* b, hipStream_t st, const hipStream_t* br, int nbr, const hipEvent_t* ev) {
  if (b->n_items == 0) return hipSuccess;
  hipError_t e = launch_batch_reset(b->mem.cols, (uint32_t)b->n_items, b->mem.out, st);
  if (e != hipSuccess || b->n_work == 0 || b->cls_mask == 0) return e;
  if (nbr > 0) {
    e = hipEventRecord(ev[0], st);
    for (int i = 0; i < nbr && e == hipSuccess; ++i) e = hipStreamWaitEvent(br[i], ev[0], 0);
    if (e != hipSuccess) return e;
  }
  int k = 0;
  for (int cls = 0; cls < kBatchClasses; ++cls) {
    if (!((b->cls_mask >> cls) & 1u)) continue;
    const hipStream_t s = nbr > 0 ? br[k++ % nbr] : st;
    e = batch_class_fn(cls)(make_args(b->mem, (uint32_t)b->n_items, b->n_work, cls), b->grid_cls[cls], 256, s,
                            nullptr);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < nbr && e == hipSuccess; ++i) {
    e = hipEventRecord(ev[1 + i], br[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[1 + i], 0);
  }
  return e;
}

// Capture the replay sequence into b->exec.  Any failure leaves b->exec null
// (replays then enqueue the launches directly) and clears the error state.
static void capture_batch(scan_ctx* ctx, BatchPlan* b, bool forked) {
  const int ncls = __builtin_popcount(b->cls_mask);
  const int nbr = forked ? std::min(kMaxBranches, ncls) : 0;
  hipStream_t cs = nullptr;
  hipStream_t br[kMaxBranches] = {};
  hipEvent_t ev[kMaxBranches + 1] = {};
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < nbr && ok; ++i) ok = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i <= nbr && ok; ++i) ok = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
  if (ok && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    const hipError_t le = enqueue_batch(b, cs, br, nbr, ev);
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    ok = le == hipSuccess && ee == hipSuccess && g != nullptr;
    if (ok) ok = hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
  } else {
    ok = false;
  }
  if (g) (void)hipGraphDestroy(g);
  for (int i = 0; i <= nbr; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  for (int i = 0; i < nbr; ++i)
    if (br[i]) (void)hipStreamDestroy(br[i]);
  if (cs) (void)hipStreamDestroy(cs);
  if (!ok && x) {
    (void)hipGraphExecDestroy(x);
    x = nullptr;
  }
  (void)hipGetLastError();
  (void)ctx;
  b->exec = ok ? x : nullptr;
  b->forked = ok && nbr > 0;
}

static void fill_results(const BatchPlan* b, scan_result* out) {
  for (size_t i = 0; i < b->n_items; ++i) {
    scan_result r;
    std::memset(&r, 0, sizeof r);
    const BatchCol& c = b->cols[i];
    r.status = b->status[i];
    if (r.status == SCAN_OK) {
      const BatchOut& o = b->mem.out_host[i];
      const int32_t s = (int32_t)o.pad;
      r.count = o.count;
      r.sum = (int64_t)o.sum;
      r.blocks_total = c.nb;
      r.strategy_used = s;
      // An empty predicate reads nothing; without zone maps the scan still
      // accounts every block, as a single-column scan does.
      if (c.flags & kColEmpty) r.blocks_read = (c.lo < c.hi && !((s >> 3) & 1)) ? c.nb : 0;
      else r.blocks_read = o.blocks;
    } else {
      r.strategy_used = c.requested;
    }
    out[i] = r;
  }
}

// Strategy for one column from the loaded selector (synchronous).
scan_status selector_pick(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                          int32_t* out) {
  if (!ctx->selector_ready) return fail(ctx, SCAN_EUNSUPPORTED, "no selector loaded");
  if (col->layout != SCAN_LAYOUT_RM) return fail(ctx, SCAN_EUNSUPPORTED, "the selector covers row-major columns");
  scan_item it;
  std::memset(&it, 0, sizeof it);
  it.col = *col;
  it.enc = enc;
  it.b = b;
  it.pred = *pred;
  it.agg = SCAN_AGG_COUNT | SCAN_AGG_SUM;
  it.strategy = SCAN_STRAT_AUTO;
  std::vector<BatchCol> cols;
  std::vector<int32_t> status;
  std::vector<BatchWork> segs;
  plan_cols(ctx, &it, 1, kMaxWindow, cols, status, nullptr, segs);
  if (status[0] != SCAN_OK) return (scan_status)status[0];
  auto& ps = pick_scratch();
  PickScratch*& sc = ps[ctx];
  if (sc && sc->mem.n_segs < segs.size()) {  // grown for a longer column
    sc->mem.release();
    delete sc;
    sc = nullptr;
  }
  if (!sc) {
    sc = new PickScratch();
    const hipError_t e = sc->mem.allocate(1, 1, std::max<size_t>(segs.size(), 64));
    if (e != hipSuccess) {
      sc->mem.release();
      delete sc;
      ps.erase(ctx);
      return fail(ctx, SCAN_ENOMEM, "selector scratch: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemcpyAsync(sc->mem.cols, cols.data(), sizeof(BatchCol), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !segs.empty())
    e = hipMemcpyAsync(sc->mem.segs, segs.data(), sizeof(BatchWork) * segs.size(), hipMemcpyHostToDevice,
                       ctx->stream);
  if (e == hipSuccess) {
    BatchBuffers m = sc->mem;
    m.n_segs = (uint32_t)segs.size();
    e = enqueue_select(m, 1, selector_theta(ctx), ctx->selector_margin, ctx->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sc->mem.out_host, sc->mem.out, sizeof(BatchOut), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "selector");
  *out = (int32_t)sc->mem.out_host[0].pad;
  // the all-match shortcut only saves work: add it wherever zone maps are used and block sums exist
  if (((*out >> 3) & 1) && col->block_sum) *out |= SCAN_ALL_MATCH;
  return SCAN_OK;
}

extern "C" {

scan_status scan_batch_prepare(scan_ctx* ctx, const scan_item* items, size_t n_items, uint64_t* handle) {
  if (!ctx) return SCAN_EINVAL;
  if (!handle || (n_items && !items)) return fail(ctx, SCAN_EINVAL, "items and handle must not be NULL");
  if (n_items > (1u << 24)) return fail(ctx, SCAN_EINVAL, "at most 2^24 items per batch");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const scan_tune t = effective_tune(ctx, -1, 0, -1);
  const uint32_t window = (uint32_t)std::clamp(t.window_blocks, 1, (int)kMaxWindow);
  BatchPlan* b = new BatchPlan();
  b->n_items = n_items;
  b->selector = ctx->selector_ready;
  b->margin = ctx->selector_margin;
  b->order = ctx->batch_order;
  b->grid = (uint32_t)ctx->cus * (uint32_t)std::clamp(t.wgs_per_cu, 1, 16);
  // dictionary classes hold the dictionary in LDS: fewer of their work-groups
  // fit on a compute unit, and their static shares are sized by the grid
  for (int cls = 0; cls < kBatchClasses; ++cls) {
    int occ = 0;
    b->grid_cls[cls] = b->grid;
    if (batch_class_fn(cls)(make_args(b->mem, 0, 0, cls), 0, 256, ctx->stream, &occ) == hipSuccess && occ > 0)
      b->grid_cls[cls] = std::min<uint32_t>(b->grid, (uint32_t)ctx->cus * (uint32_t)occ);
  }
  std::vector<BatchWork> work, segs;
  plan_cols(ctx, items, n_items, window, b->cols, b->status, &work, segs);
  if (work.size() > 0xFFFFFFFFull || segs.size() > 0xFFFFFFFFull) {
    free_plan(b);
    return fail(ctx, SCAN_EINVAL, "too many work items");
  }
  b->n_work = (uint32_t)work.size();
  e = b->mem.allocate(n_items, work.size(), b->selector ? segs.size() : 0);
  if (e != hipSuccess) {
    free_plan(b);
    return fail(ctx, SCAN_ENOMEM, "batch buffers: %s", hipGetErrorString(e));
  }
  if (n_items) e = hipMemcpy(b->mem.cols, b->cols.data(), sizeof(BatchCol) * n_items, hipMemcpyHostToDevice);
  if (e == hipSuccess && !work.empty())
    e = hipMemcpy(b->mem.work, work.data(), sizeof(BatchWork) * work.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && b->selector && !segs.empty())
    e = hipMemcpy(b->mem.segs, segs.data(), sizeof(BatchWork) * segs.size(), hipMemcpyHostToDevice);
  // The planning pass.  The selector as it is now decides the strategies:
  // a later change of the context's selector does not reach this batch.
  const uint32_t n = (uint32_t)n_items;
  if (e == hipSuccess && n)
    e = enqueue_select(b->mem, n, b->selector ? selector_theta(ctx) : nullptr, b->margin, ctx->stream);
  if (e == hipSuccess && n)
    e = hipMemcpyAsync(b->cols.data(), b->mem.cols, sizeof(BatchCol) * n, hipMemcpyDeviceToHost, ctx->stream);
  std::vector<float> scores;
  if (e == hipSuccess && n && b->selector) {
    scores.resize((size_t)n * 8);
    e = hipMemcpyAsync(scores.data(), b->mem.scores, sizeof(float) * scores.size(), hipMemcpyDeviceToHost,
                       ctx->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && n && b->selector) {
    std::vector<int32_t> before(n);
    for (uint32_t i = 0; i < n; ++i) before[i] = b->cols[i].strategy;
    prune_classes(b->cols, scores, ctx->class_scan_us);
    for (uint32_t i = 0; i < n; ++i) b->pruned += b->cols[i].strategy != before[i] ? 1u : 0u;
    e = hipMemcpy(b->mem.cols, b->cols.data(), sizeof(BatchCol) * n, hipMemcpyHostToDevice);
  }
  // class lists: in item order (items are in column order, then block
  // order), or that order walked with a stride (scan_batch_set_order)
  if (e == hipSuccess && b->n_work) {
    std::vector<uint32_t> lists((size_t)b->n_work * kBatchClasses);
    uint32_t counts[kBatchClasses] = {};
    for (uint32_t i = 0; i < b->n_work; ++i) {
      const BatchCol& c = b->cols[work[i].col];
      if (c.flags & (kColEmpty | kColSkip)) continue;
      const int k = batch_class(c.enc, c.strategy);
      lists[(size_t)k * b->n_work + counts[k]++] = i;
    }
    if (b->order == 1) {
      // position j takes item (j * P) mod L, P = 2^31 - 1 (a prime above any
      // list length L, so the walk is a permutation)
      std::vector<uint32_t> tmp;
      for (int k = 0; k < kBatchClasses; ++k) {
        const uint64_t L = counts[k];
        if (L < 2) continue;
        uint32_t* l = &lists[(size_t)k * b->n_work];
        tmp.assign(l, l + L);
        for (uint64_t j = 0; j < L; ++j) l[j] = tmp[(j * 2147483647ull) % L];
      }
    }
    e = hipMemcpyAsync(b->mem.lists, lists.data(), sizeof(uint32_t) * lists.size(), hipMemcpyHostToDevice,
                       ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->mem.counters, counts, sizeof(counts), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);  // the host arrays outlive the copies
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    free_plan(b);
    return hip_fail(ctx, e, "batch planning");
  }
  b->cls_mask = b->n_work ? used_classes(b->cols) : 0u;
  b->kernels = n == 0 ? 0u : 1u + (uint32_t)__builtin_popcount(b->cls_mask);
  if (ctx->batch_graph && b->kernels) capture_batch(ctx, b, ctx->batch_graph == 2);
  const uint64_t h = ctx->next_batch++;
  ctx->batches[h] = b;
  *handle = h;
  return SCAN_OK;
}

scan_status scan_batch_replay(scan_ctx* ctx, uint64_t handle, scan_result* out) {
  if (!ctx) return SCAN_EINVAL;
  auto it = ctx->batches.find(handle);
  if (it == ctx->batches.end()) return fail(ctx, SCAN_EINVAL, "unknown batch handle %llu", (unsigned long long)handle);
  BatchPlan* b = it->second;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = b->exec ? hipGraphLaunch(b->exec, ctx->stream) : enqueue_batch(b, ctx->stream, nullptr, 0, nullptr);
  if (e == hipSuccess && out && b->n_items)
    e = hipMemcpyAsync(b->mem.out_host, b->mem.out, sizeof(BatchOut) * b->n_items, hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess && out) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch replay");
  if (out) fill_results(b, out);
  return SCAN_OK;
}

scan_status scan_batch_release(scan_ctx* ctx, uint64_t handle) {
  if (!ctx) return SCAN_EINVAL;
  auto it = ctx->batches.find(handle);
  if (it == ctx->batches.end()) return fail(ctx, SCAN_EINVAL, "unknown batch handle %llu", (unsigned long long)handle);
  (void)hipStreamSynchronize(ctx->stream);
  free_plan(it->second);
  ctx->batches.erase(it);
  return SCAN_OK;
}

scan_status scan_batch_run(scan_ctx* ctx, const scan_item* items, size_t n_items, scan_result* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!out && n_items) return fail(ctx, SCAN_EINVAL, "out must not be NULL");
  uint64_t h = 0;
  scan_status st = scan_batch_prepare(ctx, items, n_items, &h);
  if (st != SCAN_OK) return st;
  st = scan_batch_replay(ctx, h, out);
  const scan_status st2 = scan_batch_release(ctx, h);
  return st != SCAN_OK ? st : st2;
}

scan_status scan_batch_set_tune(scan_ctx* ctx, const scan_tune* t) {
  if (!ctx) return SCAN_EINVAL;
  if (!t) return fail(ctx, SCAN_EINVAL, "tune is NULL");
  if (t->wgs_per_cu < 0 || t->wgs_per_cu > 16) return fail(ctx, SCAN_EINVAL, "wgs_per_cu must be in 0..16");
  if (t->window_blocks < 0 || t->window_blocks > (int)kMaxWindow)
    return fail(ctx, SCAN_EINVAL, "window_blocks must be in 0..%u", kMaxWindow);
  ctx->tunes[std::make_tuple((int32_t)-1, 0u, (int32_t)-1)] = *t;
  return SCAN_OK;
}

scan_status scan_batch_autotune(scan_ctx* ctx, const scan_item* items, size_t n_items, int32_t reps, scan_tune* out,
                               float* ms_out) {
  if (!ctx) return SCAN_EINVAL;
  if (n_items == 0 || !items) return fail(ctx, SCAN_EINVAL, "the autotuner needs a non-empty batch");
  if (reps < 1) reps = 3;
  reps = std::min(reps, 16);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  scan_status st = ensure_evict_buffer(ctx);
  if (st != SCAN_OK) return st;
  const auto key = std::make_tuple((int32_t)-1, 0u, (int32_t)-1);
  const bool had = ctx->tunes.count(key) > 0;
  const scan_tune saved = had ? ctx->tunes[key] : scan_tune{0, 0, 0, 0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(ctx, SCAN_EDEVICE, "events");
  }
  static const int kPerCu[] = {1, 2, 4, 8};
  static const int kWin[] = {16, 32, 64};
  const int saved_order = ctx->batch_order;
  float best_ms = 1e30f;
  scan_tune best = saved;
  int best_order = saved_order;
  for (int order = 0; order < 2 && st == SCAN_OK; ++order)
  for (int pc : kPerCu) {
    for (int win : kWin) {
      ctx->tunes[key] = scan_tune{0, pc, win, 0};
      ctx->batch_order = order;
      uint64_t h = 0;
      st = scan_batch_prepare(ctx, items, n_items, &h);
      if (st != SCAN_OK) break;
      float ts[16];
      st = scan_batch_replay(ctx, h, nullptr);  // warm: code objects, graph upload
      for (int i = 0; i < reps && st == SCAN_OK; ++i) {
        evict_caches(ctx);
        hipEventRecord(e0, ctx->stream);
        st = scan_batch_replay(ctx, h, nullptr);
        hipEventRecord(e1, ctx->stream);
        if (st == SCAN_OK && hipEventSynchronize(e1) == hipSuccess) hipEventElapsedTime(&ts[i], e0, e1);
      }
      const scan_status st2 = scan_batch_release(ctx, h);
      if (st == SCAN_OK) st = st2;
      if (st != SCAN_OK) break;
      std::sort(ts, ts + reps);
      if (ts[reps / 2] < best_ms) {
        best_ms = ts[reps / 2];
        best = scan_tune{0, pc, win, 0};
        best_order = order;
      }
    }
    if (st != SCAN_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SCAN_OK) {
    if (had) ctx->tunes[key] = saved;
    else ctx->tunes.erase(key);
    ctx->batch_order = saved_order;
    return st;
  }
  ctx->tunes[key] = best;
  ctx->batch_order = best_order;
  if (out) {
    *out = best;
    out->depth = best_order;  // for batches: the class-list order chosen
  }
  if (ms_out) *ms_out = best_ms;
  return SCAN_OK;
}

scan_status scan_batch_set_order(scan_ctx* ctx, int32_t order) {
  if (!ctx) return SCAN_EINVAL;
  if (order != 0 && order != 1) return fail(ctx, SCAN_EINVAL, "order must be 0 or 1");
  ctx->batch_order = order;
  return SCAN_OK;
}

scan_status scan_batch_set_class_cost(scan_ctx* ctx, float us) {
  if (!ctx) return SCAN_EINVAL;
  if (!(us >= 0.0f) || !std::isfinite(us)) return fail(ctx, SCAN_EINVAL, "class cost must be finite and >= 0");
  ctx->class_scan_us = us;
  return SCAN_OK;
}

scan_status scan_batch_set_graph(scan_ctx* ctx, int32_t mode) {
  if (!ctx) return SCAN_EINVAL;
  if (mode < 0 || mode > 2) return fail(ctx, SCAN_EINVAL, "graph mode must be 0, 1 or 2");
  ctx->batch_graph = mode;
  return SCAN_OK;
}

scan_status scan_batch_info(scan_ctx* ctx, uint64_t handle, scan_batch_stats* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!out) return fail(ctx, SCAN_EINVAL, "out is NULL");
  auto it = ctx->batches.find(handle);
  if (it == ctx->batches.end()) return fail(ctx, SCAN_EINVAL, "unknown batch handle %llu", (unsigned long long)handle);
  const BatchPlan* b = it->second;
  out->captured = b->exec ? (b->forked ? 2 : 1) : 0;
  out->kernels = b->kernels;
  out->class_mask = b->cls_mask;
  out->work_items = b->n_work;
  out->pruned = b->pruned;
  out->reserved = 0;
  return SCAN_OK;
}

scan_status scan_features(scan_ctx* ctx, const scan_item* items, size_t n_items, float* X_dev) {
  if (!ctx) return SCAN_EINVAL;
  if (n_items == 0) return SCAN_OK;
  if (!items || !X_dev) return fail(ctx, SCAN_EINVAL, "items and X must not be NULL");
  if (n_items > (1u << 24)) return fail(ctx, SCAN_EINVAL, "at most 2^24 items");
  std::vector<BatchCol> cols;
  std::vector<int32_t> status;
  std::vector<BatchWork> segs;
  plan_cols(ctx, items, n_items, kMaxWindow, cols, status, nullptr, segs);
  for (size_t i = 0; i < n_items; ++i)
    if (status[i] != SCAN_OK) return (scan_status)status[i];
  BatchBuffers m;
  hipError_t e = m.allocate(n_items, 1, segs.size());
  if (e == hipSuccess)
    e = hipMemcpyAsync(m.cols, cols.data(), sizeof(BatchCol) * n_items, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !segs.empty())
    e = hipMemcpyAsync(m.segs, segs.data(), sizeof(BatchWork) * segs.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = launch_batch_setup(make_args(m, (uint32_t)n_items, 0, 0), ctx->stream);
  if (e == hipSuccess)
    e = launch_batch_features(m.cols, (uint32_t)n_items, m.segs, (uint32_t)segs.size(), m.fparts, X_dev,
                              ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  m.release();
  if (e != hipSuccess) return hip_fail(ctx, e, "features");
  return SCAN_OK;
}

}  // extern "C"
