// Learned strategy selector: host side.
#include "scan_internal.h"

scan_status selector_pick(scan_ctx* ctx, const scan_column*, int32_t, uint32_t, const scan_predicate*, int32_t*) {
  return fail(ctx, SCAN_EUNSUPPORTED, "no selector loaded");
}

void destroy_selector(scan_ctx* ctx) { ctx->selector_ready = false; }
