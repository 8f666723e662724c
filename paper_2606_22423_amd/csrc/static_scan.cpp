// scan_run_static: the single-column scan for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).  Same kernels and results as scan_run_async; the work-group
// partials, which a context keeps in its own allocation, live here in a
// file-scope device array instead, and no context is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/scan.h"
#include "scan_internal.h"

using namespace scan_dev;

namespace {

// One partial (32 bytes) per work-group of a launch: 4096 of them, 128 KiB
// per device, held until the process ends.  The launch is capped to this many
// work-groups (the default shapes use at most four per compute unit).
constexpr uint32_t kStaticPartials = SCAN_STATIC_MAX_WORKGROUPS;
constexpr int kMaxDevices = 64;

__device__ __align__(256) Partial scratch[kStaticPartials];

// Per device: the address of `scratch` there (each device holds its own copy
// of the array) and its compute-unit count, set up once with that device
// current.
struct DeviceSlot {
  Partial* scratch = nullptr;
  int cus = 0;
  bool ready = false;
};
DeviceSlot g_slots[kMaxDevices];
std::mutex g_setup;

scan_status setup_device(int dev, DeviceSlot** out) {
  std::lock_guard<std::mutex> lock(g_setup);
  DeviceSlot& s = g_slots[dev];
  if (!s.ready) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return SCAN_EDEVICE;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
      (void)hipGetLastError();
      return SCAN_EDEVICE;
    }
    s.scratch = static_cast<Partial*>(ptr);
    s.cus = cus;
    s.ready = true;
  }
  *out = &s;
  return SCAN_OK;
}

}  // namespace

extern "C" scan_status scan_run_static(const scan_item* item, void* hip_stream, scan_result* out_dev) {
  if (!item || !out_dev) return SCAN_EINVAL;
  scan_status st = validate_column(nullptr, &item->col, item->enc, item->b);
  if (st != SCAN_OK) return st;
  const int32_t s = item->strategy == SCAN_STRAT_AUTO ? heuristic_strategy(&item->col, item->enc, item->b)
                                                       : item->strategy;
  st = check_strategy(nullptr, &item->col, item->enc, item->b, s);
  if (st != SCAN_OK) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SCAN_EDEVICE;
  DeviceSlot* slot = nullptr;
  st = setup_device(dev, &slot);
  if (st != SCAN_OK) return st;
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  Result* out = reinterpret_cast<Result*>(out_dev);
  Params p;
  LaunchFn fn = nullptr;
  bool empty = false;
  const scan_tune t = default_tune(item->enc, item->b, s);
  st = scan_params(nullptr, &item->col, item->enc, item->b, &item->pred, s, t.depth, slot->scratch, out, p, fn, empty);
  if (st != SCAN_OK) return st;
  if (empty) {
    Result r;
    std::memset(&r, 0, sizeof r);
    r.blocks_total = p.nb;
    r.blocks_read = (item->pred.lo < item->pred.hi && !((s >> 3) & 1)) ? p.nb : 0;
    r.strategy_used = s;
    return launch_write_result(out, r, stream) == hipSuccess ? SCAN_OK : SCAN_EDEVICE;
  }
  int occ = 0;
  if (fn(p, 0, (uint32_t)t.wg_size, stream, &occ) != hipSuccess) return SCAN_EDEVICE;
  uint32_t grid = 0;
  scan_geometry(p, t, std::max(occ, 1), slot->cus, kStaticPartials, s & 3, item->b, grid);
  if (grid > kStaticPartials) return SCAN_EINVAL;  // the scratch holds one partial per work-group
  hipError_t e = fn(p, grid, (uint32_t)t.wg_size, stream, nullptr);
  if (e == hipSuccess) e = launch_fold(p.partials, grid, p.out, p.nb, p.strategy, stream);
  return e == hipSuccess ? SCAN_OK : SCAN_EDEVICE;
}
