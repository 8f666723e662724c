// Materializing select, refinement and gather: host side.  Each call is
// synchronous on the context stream; work space (per-block counts and
// offsets, tile sums, refinement ballots) is owned by the context and grows
// on demand.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "scan_internal.h"
#include "select_kernels.h"

using namespace scan_dev;

struct SelectWork {
  void* buf = nullptr;
  size_t bytes = 0;
  uint32_t* host_total = nullptr;  // pinned
};

namespace {

// Work-space layout for `m` counted units (blocks or chunks of positions):
// [zrange 2 x i64][total u32 + pad][counts m][offsets m][tile sums][ballots 16 per unit]
struct WsLayout {
  int64_t* zrange;
  uint32_t* total;
  uint32_t* counts;
  uint32_t* offsets;
  uint32_t* tiles;
  uint64_t* ballots;
};

size_t ws_bytes(uint64_t m, bool ballots) {
  const uint64_t tiles = (m + kScanTile - 1) / kScanTile + 1;
  size_t b = 64 + 2 * ((m * 4 + 255) & ~255ull) + ((tiles * 4 + 255) & ~255ull);
  if (ballots) b += m * 16 * 8;
  return b;
}

scan_status get_ws(scan_ctx* ctx, uint64_t m, bool ballots, WsLayout& L) {
  if (!ctx->select) ctx->select = new SelectWork();
  SelectWork* w = ctx->select;
  const size_t need = ws_bytes(m, ballots);
  hipError_t e = hipSuccess;
  if (need > w->bytes) {
    e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && w->buf) e = hipFree(w->buf);
    w->buf = nullptr;
    w->bytes = 0;
    if (e == hipSuccess) e = hipMalloc(&w->buf, need);
    if (e != hipSuccess) return fail(ctx, SCAN_ENOMEM, "select work space: %s", hipGetErrorString(e));
    w->bytes = need;
  }
  if (!w->host_total) {
    e = hipHostMalloc(&w->host_total, 64, hipHostMallocDefault);
    if (e != hipSuccess) return fail(ctx, SCAN_ENOMEM, "select staging: %s", hipGetErrorString(e));
  }
  char* p = static_cast<char*>(w->buf);
  const uint64_t tiles = (m + kScanTile - 1) / kScanTile + 1;
  L.zrange = reinterpret_cast<int64_t*>(p);
  L.total = reinterpret_cast<uint32_t*>(p + 16);
  p += 64;
  L.counts = reinterpret_cast<uint32_t*>(p);
  p += (m * 4 + 255) & ~255ull;
  L.offsets = reinterpret_cast<uint32_t*>(p);
  p += (m * 4 + 255) & ~255ull;
  L.tiles = reinterpret_cast<uint32_t*>(p);
  p += (tiles * 4 + 255) & ~255ull;
  L.ballots = ballots ? reinterpret_cast<uint64_t*>(p) : nullptr;
  return SCAN_OK;
}

scan_status check_select_column(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b) {
  scan_status st = validate_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  if (enc != SCAN_ENC_FOR && enc != SCAN_ENC_DICT)
    return fail(ctx, SCAN_EUNSUPPORTED, "select, refine and gather take frame-of-reference or dictionary columns");
  if (col->layout != SCAN_LAYOUT_RM) return fail(ctx, SCAN_EUNSUPPORTED, "select, refine and gather read row-major");
  if (col->n > 0xFFFFFFFFull) return fail(ctx, SCAN_EINVAL, "positions are u32: at most 2^32 - 1 rows");
  return SCAN_OK;
}

SelParams make_params(const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred, bool zm, bool am,
                      const WsLayout& L) {
  SelParams p;
  std::memset(&p, 0, sizeof p);
  p.payload = col->payload;
  p.refs = enc == SCAN_ENC_FOR ? col->block_ref : nullptr;
  p.dict = col->dict;
  p.zmin = static_cast<const uint32_t*>(col->zone_min);
  p.zmax = static_cast<const uint32_t*>(col->zone_max);
  p.zrange = L.zrange;
  p.marks = L.ballots;
  p.counts = L.counts;
  p.offsets = L.offsets;
  p.n = col->n;
  p.nb = (col->n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  p.lo = pred ? pred->lo : 0;
  p.hi = pred ? pred->hi : 0;
  p.b = b;
  p.enc = (uint32_t)enc;
  p.dict_len = col->dict_len;
  p.use_zm = zm ? 1u : 0u;
  p.use_am = am ? 1u : 0u;
  return p;
}

}  // namespace

void destroy_select(scan_ctx* ctx) {
  if (!ctx->select) return;
  if (ctx->select->buf) (void)hipFree(ctx->select->buf);
  if (ctx->select->host_total) (void)hipHostFree(ctx->select->host_total);
  delete ctx->select;
  ctx->select = nullptr;
}

extern "C" {

scan_status scan_select(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        uint32_t flags, uint32_t* positions, uint64_t capacity, uint64_t* n_selected) {
  if (!ctx) return SCAN_EINVAL;
  if (!col || !pred || !n_selected) return fail(ctx, SCAN_EINVAL, "column, predicate and n_selected must not be NULL");
  scan_status st = check_select_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  const bool zm = flags & 1u, am = (flags & 3u) == 3u;
  if (flags & ~3u) return fail(ctx, SCAN_EINVAL, "flags: bit 0 zone maps, bit 1 all-match");
  if (zm && !col->zone_min) return fail(ctx, SCAN_EUNSUPPORTED, "zone maps requested on a column without them");
  *n_selected = 0;
  if (col->n == 0 || pred->lo >= pred->hi) return SCAN_OK;
  const uint64_t nb = (col->n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  WsLayout L;
  st = get_ws(ctx, nb, true, L);  // 16 pass ballots per block
  if (st != SCAN_OK) return st;
  const SelParams p = make_params(col, enc, b, pred, zm, am, L);
  const uint32_t grid = (uint32_t)ctx->cus * 8u;
  hipError_t e = launch_select_setup(p, L.zrange, ctx->stream);
  if (e == hipSuccess) e = launch_select_mark(p, grid, ctx->stream);
  if (e == hipSuccess) e = launch_exclusive_scan(L.counts, nb, L.offsets, L.tiles, L.total, ctx->stream);
  if (positions && capacity >= col->n) {
    // every outcome fits: write without waiting for the count
    if (e == hipSuccess) e = launch_select_write(p, positions, grid, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ctx->select->host_total, L.total, 4, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "select");
    *n_selected = *ctx->select->host_total;
    return SCAN_OK;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->select->host_total, L.total, 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "select count");
  const uint64_t total = *ctx->select->host_total;
  *n_selected = total;
  if (total == 0) return SCAN_OK;
  if (total > capacity)
    return fail(ctx, SCAN_ENOMEM, "%llu positions selected, capacity %llu", (unsigned long long)total,
                (unsigned long long)capacity);
  if (!positions) return fail(ctx, SCAN_EINVAL, "positions must not be NULL");
  e = launch_select_write(p, positions, grid, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "select write");
}

scan_status scan_refine(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        const uint32_t* positions_in, uint64_t n_in, uint32_t* positions_out, uint64_t* n_out) {
  if (!ctx) return SCAN_EINVAL;
  if (!col || !pred || !n_out) return fail(ctx, SCAN_EINVAL, "column, predicate and n_out must not be NULL");
  scan_status st = check_select_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  *n_out = 0;
  if (n_in == 0 || pred->lo >= pred->hi) return SCAN_OK;
  if (!positions_in || !positions_out) return fail(ctx, SCAN_EINVAL, "position arrays must not be NULL");
  if (n_in > 0xFFFFFFFFull) return fail(ctx, SCAN_EINVAL, "at most 2^32 - 1 positions");
  const uint64_t chunks = (n_in + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  WsLayout L;
  st = get_ws(ctx, chunks, true, L);
  if (st != SCAN_OK) return st;
  const SelParams p = make_params(col, enc, b, pred, false, false, L);
  const uint32_t grid = (uint32_t)ctx->cus * 8u;
  hipError_t e = launch_select_setup(p, L.zrange, ctx->stream);
  if (e == hipSuccess) e = launch_refine_mark(p, positions_in, n_in, L.ballots, L.counts, grid, ctx->stream);
  if (e == hipSuccess) e = launch_exclusive_scan(L.counts, chunks, L.offsets, L.tiles, L.total, ctx->stream);
  if (e == hipSuccess)
    e = launch_refine_write(positions_in, n_in, L.ballots, L.offsets, positions_out, grid, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->select->host_total, L.total, 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "refine");
  *n_out = *ctx->select->host_total;
  return SCAN_OK;
}

scan_status scan_gather(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const uint32_t* positions,
                        uint64_t n, int64_t* values) {
  if (!ctx) return SCAN_EINVAL;
  if (!col) return fail(ctx, SCAN_EINVAL, "column must not be NULL");
  scan_status st = check_select_column(ctx, col, enc, b);
  if (st != SCAN_OK) return st;
  if (n == 0) return SCAN_OK;
  if (!positions || !values) return fail(ctx, SCAN_EINVAL, "positions and values must not be NULL");
  WsLayout L;
  std::memset(&L, 0, sizeof L);
  const SelParams p = make_params(col, enc, b, nullptr, false, false, L);
  hipError_t e = launch_gather(p, positions, n, values, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "gather");
}

}  // extern "C"
