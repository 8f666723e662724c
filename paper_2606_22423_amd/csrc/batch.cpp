// Batched scans: host side.
#include "scan_internal.h"

void destroy_batches(scan_ctx* ctx) { ctx->batches.clear(); }
