// Host runtime of the C ABI: context, argument validation, strategy
// resolution, launch geometry and the single-column scan entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/scan.h"
#include "launch_tables.h"
#include "scan_internal.h"

using namespace scan_dev;

namespace scan_dev {
hipError_t launch_beta_read(const void* buf, uint64_t bytes, uint32_t grid, uint32_t block, int unroll,
                            uint64_t* sink, hipStream_t st);
hipError_t launch_beta_triad(float* a, const float* b, const float* c, float s, uint64_t n, uint32_t grid,
                             hipStream_t st);
hipError_t launch_cache_flush(void* buf, uint64_t bytes, uint32_t grid, uint32_t salt, hipStream_t st);
}  // namespace scan_dev

scan_status fail(scan_ctx* ctx, scan_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

scan_status hip_fail(scan_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, SCAN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

namespace {

// Width group of the instantiation units: 1-4, 5-8, 9-16, 17-32.
int width_group(uint32_t b) { return b <= 4 ? 0 : b <= 8 ? 1 : b <= 16 ? 2 : 3; }

// The alternative step depth's kernel, or nullptr where it does not exist.
LaunchFn code_fn_alt(int enc, int dec, int mode, int pf, uint32_t b) {
  static LaunchFn (*const direct[4])(int, int, int, int) = {code_fn_alt_rm_direct_a, code_fn_alt_rm_direct_b,
                                                            code_fn_alt_rm_direct_c, code_fn_alt_rm_direct_d};
  static LaunchFn (*const li[4])(int, int, int, int) = {code_fn_alt_li_a, code_fn_alt_li_b, code_fn_alt_li_c,
                                                        code_fn_alt_li_d};
  const int g = width_group(b);
  if (dec == DEC_RM_DIRECT) return direct[g](enc, mode, pf, (int)b);
  if (dec == DEC_LI) return li[g](enc, mode, pf, (int)b);
  return nullptr;
}

LaunchFn code_fn(int enc, int dec, int mode, int pf, uint32_t b) {
  static LaunchFn (*const lds[4])(int, int, int, int) = {code_fn_rm_lds_a, code_fn_rm_lds_b, code_fn_rm_lds_c,
                                                         code_fn_rm_lds_d};
  static LaunchFn (*const direct[4])(int, int, int, int) = {code_fn_rm_direct_a, code_fn_rm_direct_b,
                                                            code_fn_rm_direct_c, code_fn_rm_direct_d};
  static LaunchFn (*const li[4])(int, int, int, int) = {code_fn_li_a, code_fn_li_b, code_fn_li_c, code_fn_li_d};
  const int g = width_group(b);
  switch (dec) {
    case DEC_RM_LDS: return lds[g](enc, mode, pf, (int)b);
    case DEC_RM_DIRECT: return direct[g](enc, mode, pf, (int)b);
    case DEC_LI: return li[g](enc, mode, pf, (int)b);
    case DEC_BYTES: return code_fn_bytes(enc, mode, pf, (int)b);
  }
  return nullptr;
}

LaunchFn delta_fn(int dec, int mode, uint32_t b) {
  static LaunchFn (*const lds[4])(int, int) = {delta_fn_rm_lds_a, delta_fn_rm_lds_b, delta_fn_rm_lds_c,
                                               delta_fn_rm_lds_d};
  static LaunchFn (*const direct[4])(int, int) = {delta_fn_rm_direct_a, delta_fn_rm_direct_b, delta_fn_rm_direct_c,
                                                  delta_fn_rm_direct_d};
  const int g = width_group(b);
  switch (dec) {
    case DEC_RM_LDS: return lds[g](mode, (int)b);
    case DEC_RM_DIRECT: return direct[g](mode, (int)b);
  }
  return nullptr;
}

}  // namespace

// ------------------------------------------------------------ validation

scan_status validate_column(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b) {
  if (!col) return fail(ctx, SCAN_EINVAL, "column is NULL");
  if (b < 1 || b > 32) return fail(ctx, SCAN_EINVAL, "bit width %u outside 1..32", b);
  if (enc < SCAN_ENC_FOR || enc > SCAN_ENC_DICT) return fail(ctx, SCAN_EINVAL, "unknown encoding %d", enc);
  if (col->layout > SCAN_LAYOUT_LI) return fail(ctx, SCAN_EINVAL, "unknown layout %u", col->layout);
  if (col->n == 0) return SCAN_OK;
  if (!col->payload) return fail(ctx, SCAN_EINVAL, "payload is NULL");
  if (reinterpret_cast<uintptr_t>(col->payload) % 16u)
    return fail(ctx, SCAN_EINVAL, "payload must be 16-byte aligned");
  if (enc == SCAN_ENC_DELTA_FOR && !col->block_base) return fail(ctx, SCAN_EINVAL, "delta column without bases");
  if (enc == SCAN_ENC_DICT) {
    if (!col->dict || col->dict_len == 0) return fail(ctx, SCAN_EINVAL, "dictionary column without entries");
    const uint64_t cap = std::min<uint64_t>(SCAN_MAX_DICT, b >= 13 ? SCAN_MAX_DICT : (1ull << b));
    if (col->dict_len > cap) return fail(ctx, SCAN_EINVAL, "dict_len %u exceeds min(2^b, 4096)", col->dict_len);
  }
  if (enc != SCAN_ENC_FOR && col->layout != SCAN_LAYOUT_RM)
    return fail(ctx, SCAN_EINVAL, "delta and dictionary columns are row-major");
  if ((col->zone_min == nullptr) != (col->zone_max == nullptr))
    return fail(ctx, SCAN_EINVAL, "zone_min and zone_max must both be set or both NULL");
  return SCAN_OK;
}

int32_t heuristic_strategy(const scan_column* col, int32_t enc, uint32_t b) {
  const int zm = col->zone_min ? 1 : 0;
  // the all-match shortcut only ever saves work: on whenever it can be
  const int32_t am = (zm && col->block_sum) ? SCAN_ALL_MATCH : 0;
  if (enc == SCAN_ENC_FOR && col->layout == SCAN_LAYOUT_LI) return SCAN_STRATEGY(SCAN_DEC_LI, SCAN_PRED_BF, zm) | am;
  (void)b;
  return SCAN_STRATEGY(SCAN_DEC_RM_DIRECT, SCAN_PRED_BF, zm) | am;
}

scan_status check_strategy(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, int32_t s) {
  if (s < 0 || s > 31) return fail(ctx, SCAN_EINVAL, "strategy %d out of range", s);
  const int dec = s & 3, zm = (s >> 3) & 1, am = (s >> 4) & 1;
  if (zm && !col->zone_min) return fail(ctx, SCAN_EUNSUPPORTED, "zone-map strategy on a column without zone maps");
  if (am && (!zm || !col->block_sum))
    return fail(ctx, SCAN_EUNSUPPORTED, "the all-match shortcut needs zone maps and block sums");
  if (dec == SCAN_DEC_LI) {
    if (enc != SCAN_ENC_FOR || col->layout != SCAN_LAYOUT_LI)
      return fail(ctx, SCAN_EUNSUPPORTED, "lane-interleaved decoder needs a FOR column in the LI layout");
  } else {
    if (col->layout != SCAN_LAYOUT_RM) return fail(ctx, SCAN_EUNSUPPORTED, "decoder %d needs the row-major layout", dec);
    if (dec == SCAN_DEC_BYTES && (enc != SCAN_ENC_FOR || (b != 8 && b != 16 && b != 32)))
      return fail(ctx, SCAN_EUNSUPPORTED, "byte-aligned decoder needs a FOR column with b in {8,16,32}");
  }
  return SCAN_OK;
}

// ------------------------------------------------------------ tuning

scan_tune default_tune(int32_t enc, uint32_t b, int32_t s) {
  scan_tune t;
  if (enc < 0) {
    // batches (every width in one class kernel): four work-groups per CU
    // (the class kernels are latency-bound; one per CU measured 1.3x slower)
    // and 64-block windows
    t.wg_size = 256;
    t.wgs_per_cu = 4;
    t.window_blocks = 64;
    t.depth = 0;
    return t;
  }
  // From the autotuner on MI355X (2^28-value columns, cold, branch-free):
  // few resident wavefronts, each streaming its own windows, beat full
  // occupancy from b = 8 on (fewer concurrent streams into HBM); narrower,
  // compute-bound widths want more work-groups (four up to b = 3, two up to
  // b = 7) and long windows; the transposed decoder wants longer windows than
  // the row-major ones at high widths.
  t.wg_size = 256;
  t.wgs_per_cu = b <= 3 ? 4 : b <= 7 ? 2 : 1;
  if (b <= 12) t.window_blocks = 64;
  else if (b <= 16 || (s >= 0 && (s & 3) == SCAN_DEC_LI)) t.window_blocks = 16;
  else t.window_blocks = 4;
  // Delta scans wait on their per-block prefix sums: the autotuner on MI355X
  // picks 4-8 work-groups per CU and short windows (2-16 blocks), with zone
  // maps too.
  if (enc == SCAN_ENC_DELTA_FOR) {
    const bool zm = s >= 0 && ((s >> 3) & 1);
    t.wgs_per_cu = zm || b <= 12 ? 8 : 4;
    t.window_blocks = zm || b <= 8 ? 16 : b <= 12 ? 8 : 4;
    t.depth = 0;
    return t;
  }
  // Dictionary scans wait on LDS gathers: the autotuner on MI355X (2^28
  // codes, 10 % selected, cold, branch-free) picks as many work-groups per CU
  // as the LDS dictionary lets fit up to b = 8 and two above, and 64-, 16-
  // and 4-block windows at b = 4, 8 and 12.
  if (enc == SCAN_ENC_DICT) {
    t.wgs_per_cu = b <= 8 ? 8 : 2;
    t.window_blocks = b <= 4 ? 64 : b <= 8 ? 16 : 4;
  }
  // With zone maps every window costs one dependent zone-map load and ballot
  // per wavefront: 64-block windows test 64 blocks per step.
  if (s >= 0 && ((s >> 3) & 1)) t.window_blocks = 64;
  t.depth = 0;
  return t;
}

scan_tune effective_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t s) {
  scan_tune t = default_tune(enc, b, s);
  auto it = ctx->tunes.find(std::make_tuple(enc, b, s));
  if (it != ctx->tunes.end()) {
    if (it->second.wg_size) t.wg_size = it->second.wg_size;
    if (it->second.wgs_per_cu) t.wgs_per_cu = it->second.wgs_per_cu;
    if (it->second.window_blocks) t.window_blocks = it->second.window_blocks;
    if (it->second.depth) t.depth = it->second.depth;
  }
  return t;
}

// ------------------------------------------------------------ launch

// Blocks one wavefront decodes per pipelined step (the kernels' Geo<B>).
uint32_t step_blocks(int dec, uint32_t b) {
  if (dec == DEC_RM_LDS) return b >= 32 ? 1u : std::min(8u, 32u / b);
  if (dec == DEC_BYTES) return b >= 32 ? 1u : 32u / b;
  return 2u * (b >= 16 ? 1u : std::min(4u, 16u / b));
}

// Resident work-groups per compute unit of one kernel instance (cached).
scan_status occupancy(scan_ctx* ctx, LaunchFn fn, uint32_t block, int* occ) {
  auto key = std::make_pair(reinterpret_cast<const void*>(fn), block);
  auto it = ctx->occupancy.find(key);
  if (it != ctx->occupancy.end()) {
    *occ = it->second;
    return SCAN_OK;
  }
  Params dummy;
  std::memset(&dummy, 0, sizeof dummy);
  hipError_t e = fn(dummy, 0, block, ctx->stream, occ);
  if (e != hipSuccess) return hip_fail(ctx, e, "occupancy query");
  if (*occ < 1) *occ = 1;
  ctx->occupancy[key] = *occ;
  return SCAN_OK;
}

// Kernel parameters of one (column, strategy) scan writing its work-group
// partials to `partials` and its result to `out_dev`: fills p and the
// launcher, or sets trivially_empty (n = 0, lo >= hi, or a predicate outside
// a FOR column's u32 domain).  ctx may be null (messages are then dropped).
scan_status scan_params(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        int32_t s, int32_t depth, Partial* partials, Result* out_dev, Params& p, LaunchFn& fn,
                        bool& trivially_empty) {
  const int dec = s & 3, mode = (s >> 2) & 1, zm = (s >> 3) & 1;
  std::memset(&p, 0, sizeof p);
  fn = nullptr;
  p.payload = col->payload;
  p.refs = col->block_ref;
  p.bases = col->block_base;
  p.dict = col->dict;
  p.dict_len = col->dict_len;
  p.zmin = col->zone_min;
  p.zmax = col->zone_max;
  p.n = col->n;
  p.nb = (col->n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  p.lo = pred->lo;
  p.hi = pred->hi;
  p.use_zm = (uint32_t)zm;
  p.use_am = (uint32_t)((s >> 4) & 1);
  p.bsum = col->block_sum;
  p.tail = (uint32_t)(col->n - (p.nb ? (p.nb - 1) : 0) * SCAN_BLOCK_VALUES);
  p.strategy = s;
  p.partials = partials;
  p.out = out_dev;
  trivially_empty = (col->n == 0 || pred->lo >= pred->hi);
  int pf = PF_RANGE;
  if (enc == SCAN_ENC_FOR) {
    // Clamp the predicate to the u32 value domain of FOR columns.
    const int64_t lo = std::max<int64_t>(pred->lo, 0);
    const int64_t hi = std::min<int64_t>(pred->hi, (int64_t)1 << 32);
    if (lo >= hi) trivially_empty = true;
    else {
      p.lo32 = (uint32_t)lo;
      p.hi32m1 = (uint32_t)(hi - 1);
      pf = col->block_ref ? PF_REFS : (p.lo32 == 0 ? PF_LO0 : PF_RANGE);
    }
  }
  if (trivially_empty) return SCAN_OK;
  fn = nullptr;
  if (depth == 1 && enc != SCAN_ENC_DELTA_FOR) fn = code_fn_alt(enc, dec, mode, pf, b);
  if (!fn) fn = enc == SCAN_ENC_DELTA_FOR ? delta_fn(dec, mode, b) : code_fn(enc, dec, mode, pf, b);
  if (!fn) return fail(ctx, SCAN_EUNSUPPORTED, "no kernel for enc %d b %u strategy %d", enc, b, s);
  return SCAN_OK;
}

// Whether the alternative step depth exists for this scan (its predicate
// form included).
bool has_alt_depth(const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred, int32_t s) {
  if (enc == SCAN_ENC_DELTA_FOR || (enc == SCAN_ENC_FOR && col->block_ref)) return false;
  const int64_t lo = std::max<int64_t>(pred->lo, 0);
  const int pf = enc == SCAN_ENC_FOR && lo == 0 ? PF_LO0 : PF_RANGE;
  return code_fn_alt(enc, s & 3, (s >> 2) & 1, pf, b) != nullptr;
}

// Launch geometry: p.G, p.units and the grid, from the tuning, the resident
// work-groups per CU of the kernel (`occ`) and a cap on the grid (the number
// of partials the caller's buffer holds).
void scan_geometry(Params& p, const scan_tune& t, int occ, int cus, uint32_t max_grid, int dec, uint32_t b,
                   uint32_t& grid) {
  const uint32_t block = (uint32_t)t.wg_size;
  const uint64_t per_cu = t.wgs_per_cu > 0 ? std::min<uint64_t>((uint64_t)t.wgs_per_cu, (uint64_t)occ) : (uint64_t)occ;
  const uint64_t waves = block / 64u;
  const uint32_t win = t.window_blocks > 0 ? (uint32_t)t.window_blocks : step_blocks(dec, b);
  p.G = std::min<uint32_t>(win, 64u);
  p.units = (p.nb + p.G - 1) / p.G;
  const uint64_t need = (p.units + waves - 1) / waves;
  const uint64_t cap = std::min<uint64_t>((uint64_t)cus * std::max<uint64_t>(1, per_cu), max_grid);
  grid = (uint32_t)std::max<uint64_t>(1, std::min(need, cap));
}

// Fills p and the launch geometry for one (column, strategy) on a context.
scan_status prepare_scan(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                         int32_t s, Result* out_dev, Params& p, LaunchFn& fn, uint32_t& grid, uint32_t& block,
                         bool& trivially_empty) {
  const scan_tune t = effective_tune(ctx, enc, b, s);
  scan_status st = scan_params(ctx, col, enc, b, pred, s, t.depth, ctx->partials, out_dev, p, fn, trivially_empty);
  if (st != SCAN_OK || trivially_empty) return st;
  block = (uint32_t)t.wg_size;
  if (block < 64 || block > 256 || block % 64) return fail(ctx, SCAN_EINVAL, "wg_size %u invalid (64..256)", block);
  int occ = 0;
  st = occupancy(ctx, fn, block, &occ);
  if (st != SCAN_OK) return st;
  scan_geometry(p, t, occ, ctx->cus, ctx->max_grid, s & 3, b, grid);
  return SCAN_OK;
}

scan_status enqueue_scan(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                         int32_t strategy, Result* out_dev, Result* host_empty_out) {
  Params p;
  LaunchFn fn = nullptr;
  uint32_t grid = 0, block = 0;
  bool empty = false;
  scan_status st = prepare_scan(ctx, col, enc, b, pred, strategy, out_dev, p, fn, grid, block, empty);
  if (st != SCAN_OK) return st;
  if (empty) {
    Result r{};
    r.blocks_total = p.nb;
    r.blocks_read = (pred->lo < pred->hi && !((strategy >> 3) & 1)) ? p.nb : 0;
    r.strategy_used = strategy;
    if (host_empty_out) {
      *host_empty_out = r;
      return SCAN_OK;
    }
    hipError_t e = hipMemcpyAsync(out_dev, &r, sizeof r, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(ctx->stream);  // r lives on this host stack frame
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    return SCAN_OK;
  }
  hipError_t e = fn(p, grid, block, ctx->stream, nullptr);
  if (e == hipSuccess) e = launch_fold(p.partials, grid, p.out, p.nb, p.strategy, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "scan kernel launch");
  return SCAN_OK;
}

// The autotuners' cache-evicting read: a 512 MiB buffer of the context,
// allocated on first use, read in full before each timed run.
constexpr uint64_t kEvictBytes = 512ull << 20;

scan_status ensure_evict_buffer(scan_ctx* ctx) {
  if (ctx->evict_buf) return SCAN_OK;
  hipError_t e = hipMalloc(&ctx->evict_buf, kEvictBytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(evict)");
  e = hipMemsetAsync(ctx->evict_buf, 1, kEvictBytes, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemsetAsync(evict)");
  return SCAN_OK;
}

void evict_caches(scan_ctx* ctx) {
  (void)scan_dev::launch_beta_read(ctx->evict_buf, kEvictBytes, (uint32_t)ctx->cus * 8u, 1024u, 1,
                                   reinterpret_cast<uint64_t*>(ctx->ticket) + 8, ctx->stream);
}

scan_status resolve_strategy(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b,
                             const scan_predicate* pred, int32_t strategy, bool allow_sync, int32_t* out) {
  if (strategy == SCAN_STRAT_AUTO) {
    if (allow_sync && ctx->selector_ready) {
      scan_status st = selector_pick(ctx, col, enc, b, pred, out);
      if (st == SCAN_OK) return SCAN_OK;
    }
    *out = heuristic_strategy(col, enc, b);
    return SCAN_OK;
  }
  *out = strategy;
  return SCAN_OK;
}

// ------------------------------------------------------------ C ABI

extern "C" {

scan_status scan_create(scan_ctx** out, int device, void* hip_stream) {
  if (!out) return SCAN_EINVAL;
  *out = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return SCAN_EDEVICE;
  scan_ctx* ctx = new scan_ctx();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete ctx;
    return SCAN_EDEVICE;
  }
  ctx->cus = prop.multiProcessorCount;
  ctx->max_grid = 16384;
  if (hipMalloc(&ctx->partials, sizeof(Partial) * ctx->max_grid) != hipSuccess ||
      hipMalloc(&ctx->ticket, 256) != hipSuccess || hipMalloc(&ctx->out_dev, sizeof(Result) * 2) != hipSuccess ||
      hipHostMalloc(&ctx->out_host, sizeof(Result) * 2, hipHostMallocDefault) != hipSuccess) {
    scan_destroy(ctx);
    return SCAN_ENOMEM;
  }
  if (hipEventCreateWithFlags(&ctx->order_event, hipEventDisableTiming) != hipSuccess) {
    ctx->order_event = nullptr;
    scan_destroy(ctx);
    return SCAN_EDEVICE;
  }
  if (hipMemset(ctx->ticket, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    scan_destroy(ctx);
    return SCAN_EDEVICE;
  }
  *out = ctx;
  return SCAN_OK;
}

scan_status scan_set_stream(scan_ctx* ctx, void* hip_stream) {
  if (!ctx) return SCAN_EINVAL;
  hipStream_t next = static_cast<hipStream_t>(hip_stream);
  if (next == ctx->stream) return SCAN_OK;
  // Every scan writes the context's partials and result slot: work enqueued
  // on the new stream must not start before what the old stream still holds.
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipEventRecord(ctx->order_event, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(next, ctx->order_event, 0);
  if (e != hipSuccess) return hip_fail(ctx, e, "ordering the new stream after the old one");
  ctx->stream = next;
  return SCAN_OK;
}

void scan_destroy(scan_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  destroy_batches(ctx);
  destroy_selector(ctx);
  destroy_select(ctx);
  if (ctx->partials) (void)hipFree(ctx->partials);
  if (ctx->ticket) (void)hipFree(ctx->ticket);
  if (ctx->out_dev) (void)hipFree(ctx->out_dev);
  if (ctx->out_host) (void)hipHostFree(ctx->out_host);
  if (ctx->evict_buf) (void)hipFree(ctx->evict_buf);
  if (ctx->order_event) (void)hipEventDestroy(ctx->order_event);
  delete ctx;
}

const char* scan_last_error(const scan_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int scan_device_cus(const scan_ctx* ctx) { return ctx ? ctx->cus : 0; }

scan_status scan_run(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                     uint32_t agg, int32_t strategy, scan_result* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!pred || !out) return fail(ctx, SCAN_EINVAL, "predicate and result must not be NULL");
  (void)agg;
  scan_status st = validate_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  int32_t s = 0;
  st = resolve_strategy(ctx, col, enc, b, pred, strategy, true, &s);
  if (st != SCAN_OK) return st;
  st = check_strategy(ctx, col, enc, b, s);
  if (st != SCAN_OK) return st;
  Result host_r{};
  bool host_done = false;
  {
    Params p;
    LaunchFn fn = nullptr;
    uint32_t grid = 0, block = 0;
    bool empty = false;
    st = prepare_scan(ctx, col, enc, b, pred, s, ctx->out_dev, p, fn, grid, block, empty);
    if (st != SCAN_OK) return st;
    if (empty) {
      host_r.blocks_total = p.nb;
      host_r.blocks_read = (pred->lo < pred->hi && !((s >> 3) & 1)) ? p.nb : 0;
      host_r.strategy_used = s;
      host_done = true;
    } else {
      e = fn(p, grid, block, ctx->stream, nullptr);
      if (e == hipSuccess) e = launch_fold(p.partials, grid, p.out, p.nb, p.strategy, ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "scan kernel launch");
    }
  }
  if (!host_done) {
    e = hipMemcpyAsync(ctx->out_host, ctx->out_dev, sizeof(Result), hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    host_r = *ctx->out_host;
  }
  static_assert(sizeof(Result) == sizeof(scan_result), "result layout");
  std::memcpy(out, &host_r, sizeof host_r);
  return SCAN_OK;
}

scan_status scan_run_async(scan_ctx* ctx, const scan_item* item, scan_result* out_dev) {
  if (!ctx) return SCAN_EINVAL;
  if (!item || !out_dev) return fail(ctx, SCAN_EINVAL, "item and out_dev must not be NULL");
  scan_status st = validate_column(ctx, &item->col, item->enc, item->b);
  if (st != SCAN_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  int32_t s = 0;
  st = resolve_strategy(ctx, &item->col, item->enc, item->b, &item->pred, item->strategy, false, &s);
  if (st != SCAN_OK) return st;
  st = check_strategy(ctx, &item->col, item->enc, item->b, s);
  if (st != SCAN_OK) return st;
  return enqueue_scan(ctx, &item->col, item->enc, item->b, &item->pred, s, reinterpret_cast<Result*>(out_dev),
                      nullptr);
}

scan_status scan_sync(scan_ctx* ctx) {
  if (!ctx) return SCAN_EINVAL;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "hipStreamSynchronize");
}

scan_status scan_set_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t strategy, const scan_tune* t) {
  if (!ctx) return SCAN_EINVAL;
  if (!t) return fail(ctx, SCAN_EINVAL, "tune is NULL");
  if (t->wg_size && (t->wg_size < 64 || t->wg_size > 1024 || t->wg_size % 64))
    return fail(ctx, SCAN_EINVAL, "wg_size must be a multiple of 64 in 64..1024");
  if (t->wgs_per_cu < 0 || t->wgs_per_cu > 64) return fail(ctx, SCAN_EINVAL, "wgs_per_cu must be in 0..64");
  if (t->wg_size > 256) return fail(ctx, SCAN_EINVAL, "wg_size above 256 is not supported");
  if (t->window_blocks < 0 || t->window_blocks > 64) return fail(ctx, SCAN_EINVAL, "window_blocks must be in 0..64");
  if (t->depth < 0 || t->depth > 1) return fail(ctx, SCAN_EINVAL, "depth must be 0 or 1");
  ctx->tunes[std::make_tuple(enc, b, strategy)] = *t;
  return SCAN_OK;
}

scan_status scan_get_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t strategy, scan_tune* t) {
  if (!ctx) return SCAN_EINVAL;
  if (!t) return fail(ctx, SCAN_EINVAL, "tune is NULL");
  *t = effective_tune(ctx, enc, b, strategy);
  return SCAN_OK;
}

scan_status scan_autotune(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b,
                          const scan_predicate* pred, int32_t strategy, int32_t reps, scan_tune* out, float* ms_out) {
  if (!ctx) return SCAN_EINVAL;
  if (!pred) return fail(ctx, SCAN_EINVAL, "predicate is NULL");
  scan_status st = validate_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  st = check_strategy(ctx, col, enc, b, strategy);
  if (st != SCAN_OK) return st;
  if (reps < 1) reps = 3;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  // A read of twice the 256 MB last-level cache between timed runs keeps the
  // column cold, as it is when a scan streams it once.
  st = ensure_evict_buffer(ctx);
  if (st != SCAN_OK) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(ctx, SCAN_EDEVICE, "events");
  const scan_tune saved = effective_tune(ctx, enc, b, strategy);
  const bool had = ctx->tunes.count(std::make_tuple(enc, b, strategy)) > 0;
  static const int kWg[] = {64, 128, 256};
  static const int kPerCu[] = {1, 2, 4, 8};
  static const int kWin[] = {2, 4, 8, 16, 64};
  const int depths = has_alt_depth(col, enc, b, pred, strategy) ? 2 : 1;
  float best_ms = 1e30f;
  scan_tune best = saved;
  constexpr int kShapes = 3 * 4 * 5;
  for (int k = 0; k < depths * kShapes && st == SCAN_OK; ++k) {
    const int shape = k % kShapes;
    const scan_tune t{kWg[shape / 20], kPerCu[(shape / 5) % 4], kWin[shape % 5], k / kShapes};
    ctx->tunes[std::make_tuple(enc, b, strategy)] = t;
    float ts[16];
    const int r = std::min(reps, 16);
    for (int i = 0; i < r && st == SCAN_OK; ++i) {
      evict_caches(ctx);
      hipEventRecord(e0, ctx->stream);
      st = enqueue_scan(ctx, col, enc, b, pred, strategy, ctx->out_dev, nullptr);
      hipEventRecord(e1, ctx->stream);
      if (st != SCAN_OK) break;
      hipEventSynchronize(e1);
      hipEventElapsedTime(&ts[i], e0, e1);
    }
    if (st != SCAN_OK) break;
    std::sort(ts, ts + r);
    if (ts[r / 2] < best_ms) {
      best_ms = ts[r / 2];
      best = t;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != SCAN_OK) {
    if (had) ctx->tunes[std::make_tuple(enc, b, strategy)] = saved;
    else ctx->tunes.erase(std::make_tuple(enc, b, strategy));
    return st;
  }
  ctx->tunes[std::make_tuple(enc, b, strategy)] = best;
  if (out) *out = best;
  if (ms_out) *ms_out = best_ms;
  return SCAN_OK;
}

scan_status scan_tune_save(scan_ctx* ctx, const char* path) {
  if (!ctx) return SCAN_EINVAL;
  if (!path) return fail(ctx, SCAN_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(ctx, SCAN_EINVAL, "cannot write %s", path);
  std::fprintf(f, "{\"format\": \"scan-autotune-1\", \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : ctx->tunes) {
    std::fprintf(f, "  {\"enc\": %d, \"b\": %u, \"strategy\": %d, \"wg_size\": %d, \"wgs_per_cu\": %d, "
                    "\"window_blocks\": %d, \"depth\": %d}%s\n",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second.wg_size,
                 kv.second.wgs_per_cu, kv.second.window_blocks, kv.second.depth, ++i < ctx->tunes.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return SCAN_OK;
}

scan_status scan_tune_load(scan_ctx* ctx, const char* path) {
  if (!ctx) return SCAN_EINVAL;
  if (!path) return fail(ctx, SCAN_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, SCAN_EINVAL, "cannot read %s", path);
  // Entries are parsed first and installed only if the whole file is valid:
  // a line naming an entry that does not parse or holds an invalid tuning,
  // or a file without any entry, is an error and changes nothing.
  char line[512];
  std::vector<std::pair<std::tuple<int32_t, uint32_t, int32_t>, scan_tune>> got;
  int lineno = 0, bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    if (!std::strstr(line, "\"enc\"")) continue;  // the header and the closing bracket
    int enc, strat, wg, pc, win, depth = 0;
    unsigned b;
    const int fields = std::sscanf(line,
                                   " {\"enc\": %d, \"b\": %u, \"strategy\": %d, \"wg_size\": %d, \"wgs_per_cu\": %d, "
                                   "\"window_blocks\": %d, \"depth\": %d}",
                                   &enc, &b, &strat, &wg, &pc, &win, &depth);
    if (fields != 7 && !(fields == 6 && std::strstr(line, "\"depth\"") == nullptr)) {  // no depth field: 0
      if (!bad) bad = lineno;
      continue;
    }
    const scan_tune t{wg, pc, win, depth};
    const bool ok = (wg == 0 || (wg >= 64 && wg <= 256 && wg % 64 == 0)) && pc >= 0 && pc <= 64 && win >= 0 &&
                    win <= 64 && depth >= 0 && depth <= 1;
    if (!ok) {
      if (!bad) bad = lineno;
      continue;
    }
    got.emplace_back(std::make_tuple((int32_t)enc, (uint32_t)b, (int32_t)strat), t);
  }
  std::fclose(f);
  if (bad) return fail(ctx, SCAN_EINVAL, "%s: line %d is not a valid tuning entry", path, bad);
  if (got.empty()) return fail(ctx, SCAN_EINVAL, "%s holds no tuning entry", path);
  for (const auto& kv : got) ctx->tunes[kv.first] = kv.second;
  return SCAN_OK;
}

scan_status scan_beta_read(scan_ctx* ctx, const void* buf, uint64_t bytes, int32_t wgs, int32_t wg_size,
                           int32_t unroll, uint64_t* sink) {
  if (!ctx) return SCAN_EINVAL;
  if (!buf || !sink || bytes % 16u) return fail(ctx, SCAN_EINVAL, "beta_read needs a buffer, a sink and bytes % 16 == 0");
  if (wg_size == 0) wg_size = 256;
  if (wgs == 0) wgs = ctx->cus * 8;
  if (unroll == 0) unroll = 4;
  if (wg_size < 64 || wg_size > 1024 || wg_size % 64 || wgs < 1)
    return fail(ctx, SCAN_EINVAL, "bad beta_read geometry");
  hipError_t e = launch_beta_read(buf, bytes, (uint32_t)wgs, (uint32_t)wg_size, unroll, sink, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "beta_read launch");
}

scan_status scan_beta_triad(scan_ctx* ctx, float* a, const float* b, const float* c, float s, uint64_t n) {
  if (!ctx) return SCAN_EINVAL;
  if (!a || !b || !c || n % 4u) return fail(ctx, SCAN_EINVAL, "triad needs three buffers and n % 4 == 0");
  hipError_t e = launch_beta_triad(a, b, c, s, n, (uint32_t)ctx->cus * 8u, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "triad launch");
}

scan_status scan_cache_flush(scan_ctx* ctx, void* buf, uint64_t bytes) {
  if (!ctx) return SCAN_EINVAL;
  if (!buf || bytes % 16u) return fail(ctx, SCAN_EINVAL, "flush needs a buffer and bytes % 16 == 0");
  hipError_t e = launch_cache_flush(buf, bytes, (uint32_t)ctx->cus * 8u, ++ctx->flush_salt, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "flush launch");
}

}  // extern "C"
