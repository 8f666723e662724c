// Run-length encoded columns: host side of the fused scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "rle_kernels.h"
#include "scan_internal.h"

using namespace scan_dev;

namespace {

// Validates the call and enqueues the clear + scan launches; the result lands
// in `out` (device memory).
scan_status enqueue_rle(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred, uint32_t flags,
                        Result* out) {
  if (flags & ~3u) return fail(ctx, SCAN_EINVAL, "flags: bit 0 zone maps, bit 1 all-match");
  const bool zm = flags & 1u, am = (flags & 3u) == 3u;
  if (col->n && (!col->run_value || !col->run_len || !col->block_run))
    return fail(ctx, SCAN_EINVAL, "run values, lengths and block starts must not be NULL");
  if (col->n && ((reinterpret_cast<uintptr_t>(col->run_value) & 15u) ||
                 (reinterpret_cast<uintptr_t>(col->run_len) & 7u)))
    return fail(ctx, SCAN_EINVAL, "run values must be 16-byte and run lengths 8-byte aligned");
  if (zm && (!col->zone_min || !col->zone_max))
    return fail(ctx, SCAN_EUNSUPPORTED, "zone maps requested on a column without them");
  RleParams p;
  std::memset(&p, 0, sizeof p);
  p.run_value = col->run_value;
  p.run_len = col->run_len;
  p.block_run = col->block_run;
  p.zmin = col->zone_min;
  p.zmax = col->zone_max;
  p.out = out;
  p.partials = ctx->partials;
  p.nb = (col->n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  p.lo = pred->lo;
  p.hi = pred->hi;
  p.use_zm = zm ? 1u : 0u;
  p.use_am = am ? 1u : 0u;
  p.strategy_used = (int32_t)flags;
  p.empty = (col->n == 0 || pred->lo >= pred->hi) ? 1u : 0u;
  hipError_t e = hipSetDevice(ctx->device);
  // 512-thread work-groups, one partial each (folded by the fold kernel
  // launched after it): eight per CU for the flat pass without zone maps
  // (6.9 against 6.3-6.4 TB/s with two), two for the chunked pass with them
  // (its per-chunk ballots measured no faster with more)
  const uint32_t grid = std::min<uint32_t>((uint32_t)ctx->cus * (zm ? 2u : 8u), ctx->max_grid);
  if (e == hipSuccess) e = launch_rle_scan(p, grid, ctx->stream);
  return e == hipSuccess ? SCAN_OK : hip_fail(ctx, e, "rle scan");
}

}  // namespace

extern "C" {

scan_status scan_run_rle(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred, uint32_t flags,
                         scan_result* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!col || !pred || !out) return fail(ctx, SCAN_EINVAL, "column, predicate and out must not be NULL");
  scan_status st = enqueue_rle(ctx, col, pred, flags, ctx->out_dev);
  if (st != SCAN_OK) return st;
  hipError_t e = hipMemcpyAsync(ctx->out_host, ctx->out_dev, sizeof(Result), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "rle scan");
  std::memcpy(out, ctx->out_host, sizeof *out);
  return SCAN_OK;
}

scan_status scan_run_rle_async(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred,
                               uint32_t flags, scan_result* out_dev) {
  if (!ctx) return SCAN_EINVAL;
  if (!col || !pred || !out_dev) return fail(ctx, SCAN_EINVAL, "column, predicate and out_dev must not be NULL");
  return enqueue_rle(ctx, col, pred, flags, reinterpret_cast<Result*>(out_dev));
}

}  // extern "C"
