// Run-length encoded columns: host side of the fused scan.
#include <hip/hip_runtime.h>

#include <cstring>

#include "rle_kernels.h"
#include "scan_internal.h"

using namespace scan_dev;

extern "C" {

scan_status scan_run_rle(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred, uint32_t flags,
                         scan_result* out) {
  if (!ctx) return SCAN_EINVAL;
  if (!col || !pred || !out) return fail(ctx, SCAN_EINVAL, "column, predicate and out must not be NULL");
  if (flags & ~3u) return fail(ctx, SCAN_EINVAL, "flags: bit 0 zone maps, bit 1 all-match");
  const bool zm = flags & 1u, am = (flags & 3u) == 3u;
  if (col->n && (!col->run_value || !col->run_len || !col->block_run))
    return fail(ctx, SCAN_EINVAL, "run values, lengths and block starts must not be NULL");
  if (zm && (!col->zone_min || !col->zone_max))
    return fail(ctx, SCAN_EUNSUPPORTED, "zone maps requested on a column without them");
  const uint64_t nb = (col->n + SCAN_BLOCK_VALUES - 1) / SCAN_BLOCK_VALUES;
  std::memset(out, 0, sizeof *out);
  out->blocks_total = nb;
  out->strategy_used = (int32_t)flags;
  if (col->n == 0 || pred->lo >= pred->hi) return SCAN_OK;
  hipError_t e = hipSetDevice(ctx->device);
  RleParams p;
  std::memset(&p, 0, sizeof p);
  p.run_value = col->run_value;
  p.run_len = col->run_len;
  p.block_run = col->block_run;
  p.zmin = col->zone_min;
  p.zmax = col->zone_max;
  p.out = ctx->out_dev;
  p.nb = nb;
  p.lo = pred->lo;
  p.hi = pred->hi;
  p.use_zm = zm ? 1u : 0u;
  p.use_am = am ? 1u : 0u;
  if (e == hipSuccess) e = launch_rle_scan(p, (uint32_t)ctx->cus * 8u, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->out_host, ctx->out_dev, sizeof(Result), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "rle scan");
  out->count = ctx->out_host->count;
  out->sum = ctx->out_host->sum;
  out->blocks_read = ctx->out_host->blocks_read;
  return SCAN_OK;
}

}  // extern "C"
