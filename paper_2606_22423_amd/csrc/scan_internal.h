// Host-side internals shared by the runtime's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>

#include "../../include/scan.h"
#include "device_common.h"

namespace scan_dev {
using LaunchFn = hipError_t (*)(const Params&, uint32_t grid, uint32_t block, hipStream_t stream, int* occ);
hipError_t launch_write_result(Result* out, const Result& r, hipStream_t st);
}  // namespace scan_dev

struct SelectorState;
struct BatchPlan;
struct SelectWork;

struct scan_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cus = 0;
  uint32_t max_grid = 0;
  scan_dev::Partial* partials = nullptr;  // per-work-group partial results (device)
  uint32_t* ticket = nullptr;             // 256 bytes of device scratch (the autotuner's read-probe sink)
  scan_dev::Result* out_dev = nullptr;    // result slot of synchronous scans (device)
  scan_dev::Result* out_host = nullptr;   // pinned staging for it
  uint32_t flush_salt = 0;
  void* evict_buf = nullptr;              // autotuner's cache-evicting read buffer
  hipEvent_t order_event = nullptr;       // orders a new stream after the old one (scan_set_stream)
  std::string err;
  std::map<std::tuple<int32_t, uint32_t, int32_t>, scan_tune> tunes;
  std::map<std::pair<const void*, uint32_t>, int> occupancy;
  bool selector_ready = false;
  float selector_margin = 0.0f;       // keep the heuristic unless the network predicts a gain above this (log time)
  SelectorState* selector = nullptr;
  std::map<uint64_t, BatchPlan*> batches;
  SelectWork* select = nullptr;       // materializing select work space
  uint64_t next_batch = 1;
  int32_t query_kernel = 0;           // SCAN_QUERY_PER_QUERY or SCAN_QUERY_SHARED (scan_query_run)
  int batch_graph = 1;                // prepared batches: 0 direct launches, 1 graph, 2 graph with forked class scans
  float class_scan_us = 10.0f;        // cost of one more class scan in a batch replay (scan_batch_set_class_cost)
  int batch_order = 1;                // class-list order of prepared batches (scan_batch_set_order)
};

scan_status fail(scan_ctx* ctx, scan_status st, const char* fmt, ...);
scan_status hip_fail(scan_ctx* ctx, hipError_t e, const char* what);
scan_status validate_column(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b);
scan_status check_strategy(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, int32_t s);
int32_t heuristic_strategy(const scan_column* col, int32_t enc, uint32_t b);
scan_tune effective_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t s);
scan_tune default_tune(int32_t enc, uint32_t b, int32_t s);
scan_status ensure_evict_buffer(scan_ctx* ctx);
void evict_caches(scan_ctx* ctx);
scan_status scan_params(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        int32_t s, int32_t depth, scan_dev::Partial* partials, scan_dev::Result* out_dev,
                        scan_dev::Params& p, scan_dev::LaunchFn& fn, bool& trivially_empty);
void scan_geometry(scan_dev::Params& p, const scan_tune& t, int occ, int cus, uint32_t max_grid, int dec, uint32_t b,
                   uint32_t& grid);
scan_status enqueue_scan(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                         int32_t strategy, scan_dev::Result* out_dev, scan_dev::Result* host_empty_out);
namespace scan_dev {
hipError_t launch_beta_read(const void* buf, uint64_t bytes, uint32_t grid, uint32_t block, int unroll,
                            uint64_t* sink, hipStream_t st);
}

// Learned selector (selector.cpp; the one-column pick lives in batch.cpp).
scan_status selector_pick(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b,
                          const scan_predicate* pred, int32_t* out);
const float* selector_theta(scan_ctx* ctx);
void destroy_selector(scan_ctx* ctx);

// Batched scans (batch.cpp).
void destroy_batches(scan_ctx* ctx);

// Materializing select (select.cpp).
void destroy_select(scan_ctx* ctx);
