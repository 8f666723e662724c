// Batch kernels around the class scans: per-column setup, zone-map
// features for the selector, strategy selection and item binning.
#include "batch_kernels.h"

namespace scan_dev {

hipError_t launch_batch_for_lds_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_for_lds_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_for_direct_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_for_direct_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_delta_lds_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_delta_lds_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_delta_direct_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_delta_direct_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_dict_lds_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_dict_lds_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_dict_direct_bf(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);
hipError_t launch_batch_dict_direct_sv(const BatchArgs&, uint32_t, uint32_t, hipStream_t, int*);

BatchLaunchFn batch_class_fn(int cls) {
  static const BatchLaunchFn table[kBatchClasses] = {launch_batch_for_lds_bf, launch_batch_for_lds_sv, launch_batch_for_direct_bf, launch_batch_for_direct_sv, launch_batch_delta_lds_bf, launch_batch_delta_lds_sv, launch_batch_delta_direct_bf, launch_batch_delta_direct_sv, launch_batch_dict_lds_bf, launch_batch_dict_lds_sv, launch_batch_dict_direct_bf, launch_batch_dict_direct_sv};
  return (cls >= 0 && cls < kBatchClasses) ? table[cls] : nullptr;
}

// Per column: clear the result slot, find a dictionary's code range
// [lower_bound(D, lo), lower_bound(D, hi)) by binary search in global memory.
// Thread 0 also clears the per-class item counters.
__global__ __launch_bounds__(256) void batch_setup_kernel(BatchArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    for (int c = 0; c < kBatchClasses; ++c) a.counts[c] = 0;
  }
  if (i >= a.n_cols) return;
  a.out[i] = BatchOut{0, 0, 0, 0};
  BatchCol& c = a.cols[i];
  if (c.enc == ENC_DICT && c.dict_len) {
    uint32_t lo = 0, e = c.dict_len;
    while (lo < e) {
      const uint32_t m = (lo + e) >> 1;
      if (c.dict[m] < c.lo) lo = m + 1u;
      else e = m;
    }
    uint32_t lo2 = 0, e2 = c.dict_len;
    while (lo2 < e2) {
      const uint32_t m = (lo2 + e2) >> 1;
      if (c.dict[m] < c.hi) lo2 = m + 1u;
      else e2 = m;
    }
    c.clo = lo;
    c.chi = lo2;
  }
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_min_f64(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ double wave_max_f64(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Selector features of each column from its zone maps only (fp64 sums):
//   f0 = b/32, f1 = log2(n)/24,
//   f2 = log10(max(s, 1e-6))/6 with s = sum_k c_k overlap_k / n, overlap_k the
//        share of block k's [min, max] covered by [lo, hi) (values spread evenly),
//   f3 = fraction of blocks whose [min, max] meets [lo, hi),
//   f4 = 1 - mean_k(max_k - min_k) / (max(max) - min(min) + 1) (clustering),
//   f5 = encoding / 2.
// Dictionary columns use codes and the code range; columns without zone maps
// get s = 1, f3 = 1, f4 = 0.
// Two launches: every segment of up to 256 blocks of a column is summed by
// one wavefront (four zone-map pairs per lane, all loaded before any is used:
// one memory latency per segment, so a 2^24-value column costs no more than
// a short one), then one wavefront per column adds its segments' sums in a
// fixed order (lane j takes segments j, j + 64, ..., then a fixed butterfly),
// so the features are the same bits on every run.
__device__ __forceinline__ void feat_bounds(const BatchCol& c, double& lo, double& hi) {
  if (c.enc == ENC_DICT) {
    lo = (double)c.clo;
    hi = (double)c.chi;
  } else {
    lo = (double)c.lo;
    hi = (double)c.hi;
  }
}

__global__ __launch_bounds__(256) void batch_feat_seg_kernel(const BatchCol* cols, const BatchWork* segs,
                                                             uint32_t n_segs, FeatPart* parts) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t seg = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (seg >= n_segs) return;  // wave-uniform
  const BatchWork w = segs[seg];
  const BatchCol& c = cols[w.col];
  double lo, hi;
  feat_bounds(c, lo, hi);
  constexpr int kU = kFeatSegBlocks / 64;
  double mn[kU], mx[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const uint32_t j = lane + 64u * u;
    const uint64_t k = w.k0 + (j < w.nblk ? j : 0u);
    if (c.enc == ENC_DELTA) {
      mn[u] = (double)static_cast<const int64_t*>(c.zmin)[k];
      mx[u] = (double)static_cast<const int64_t*>(c.zmax)[k];
    } else {
      mn[u] = (double)static_cast<const uint32_t*>(c.zmin)[k];
      mx[u] = (double)static_cast<const uint32_t*>(c.zmax)[k];
    }
  }
  double acc = 0.0, meet = 0.0, spread = 0.0, gmin = 1e300, gmax = -1e300;
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const uint32_t j = lane + 64u * u;
    if (j >= w.nblk) break;
    const uint64_t k = w.k0 + j;
    const double cnt = (k == c.nb - 1) ? (double)c.tail : 1024.0;
    if (lo < hi) {
      const double ov = fmax(fmin(hi, mx[u] + 1.0) - fmax(lo, mn[u]), 0.0) / (mx[u] - mn[u] + 1.0);
      acc += cnt * ov;
      meet += (mx[u] < lo || mn[u] >= hi) ? 0.0 : 1.0;
    }
    spread += mx[u] - mn[u];
    gmin = fmin(gmin, mn[u]);
    gmax = fmax(gmax, mx[u]);
  }
  acc = wave_sum_f64(acc);
  meet = wave_sum_f64(meet);
  spread = wave_sum_f64(spread);
  gmin = wave_min_f64(gmin);
  gmax = wave_max_f64(gmax);
  if (lane == 0) parts[seg] = FeatPart{acc, meet, spread, gmin, gmax};
}

__global__ __launch_bounds__(256) void batch_feat_col_kernel(const BatchCol* cols, uint32_t n_cols,
                                                             const FeatPart* parts, float* X) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t col = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (col >= n_cols) return;  // wave-uniform
  const BatchCol c = cols[col];
  double lo, hi;
  feat_bounds(c, lo, hi);
  double s = 1.0, frac = 1.0, clust = 0.0;
  if ((c.flags & kColHasZm) && c.nb && c.fsegs) {
    double acc = 0.0, meet = 0.0, spread = 0.0, gmin = 1e300, gmax = -1e300;
    for (uint32_t j = lane; j < c.fsegs; j += 64u) {
      const FeatPart q = parts[c.fseg0 + j];
      acc += q.acc;
      meet += q.meet;
      spread += q.spread;
      gmin = fmin(gmin, q.gmin);
      gmax = fmax(gmax, q.gmax);
    }
    acc = wave_sum_f64(acc);
    meet = wave_sum_f64(meet);
    spread = wave_sum_f64(spread);
    gmin = wave_min_f64(gmin);
    gmax = wave_max_f64(gmax);
    s = acc / (double)c.n;
    frac = meet / (double)c.nb;
    clust = 1.0 - (spread / (double)c.nb) / (gmax - gmin + 1.0);
  }
  if (!(lo < hi)) s = 0.0;
  if (lane == 0) {
    float* x = X + (size_t)col * 6u;
    x[0] = (float)((double)c.b / 32.0);
    x[1] = (float)(log2((double)c.n) / 24.0);
    x[2] = (float)(log10(fmax(s, 1e-6)) / 6.0);
    x[3] = (float)frac;
    x[4] = (float)clust;
    x[5] = (float)((double)c.enc / 2.0);
  }
}

// Strategy per column: the requested one, else the selector's choice, else
// the heuristic when no selector scores are given.  The selector's choice is
// the argmin over the column's allowed classes (ties to the lowest class;
// class c = decoder c&1, SV (c>>1)&1, zone maps (c>>2)&1), except that the
// heuristic's class is kept unless its predicted log-time exceeds the
// argmin's by at least `margin` (margin 0: the plain argmin).
// The choice is also recorded in the column's result slot.
__global__ __launch_bounds__(256) void batch_select_kernel(BatchCol* cols, uint32_t n_cols, const float* scores,
                                                           int32_t k, float margin, BatchOut* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cols) return;
  BatchCol& c = cols[i];
  int32_t s = c.requested;
  if (s < 0) {
    s = c.heuristic;
    if (scores) {
      float best = 0.0f;
      int bc = -1;
      for (int q = 0; q < k; ++q) {
        if (!((c.valid_mask >> q) & 1u)) continue;
        const float v = scores[(size_t)i * k + q];
        if (bc < 0 || v < best) {
          best = v;
          bc = q;
        }
      }
      const int hc = (s & 1) | (((s >> 2) & 1) << 1) | (((s >> 3) & 1) << 2);
      const bool keep = ((c.valid_mask >> hc) & 1u) && scores[(size_t)i * k + hc] - best < margin;
      if (bc >= 0 && !keep) s = (bc & 1) | (((bc >> 1) & 1) << 2) | (((bc >> 2) & 1) << 3);
    }
  }
  c.strategy = s;
  out[i].pad = (uint64_t)(uint32_t)s;
}

hipError_t launch_batch_setup(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(batch_setup_kernel, dim3((a.n_cols + 255) / 256 + 1), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_batch_features(const BatchCol* cols, uint32_t n_cols, const BatchWork* segs, uint32_t n_segs,
                                 FeatPart* parts, float* X, hipStream_t st) {
  if (n_segs) {
    hipLaunchKernelGGL(batch_feat_seg_kernel, dim3((n_segs + 3) / 4), dim3(256), 0, st, cols, segs, n_segs, parts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_cols == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_feat_col_kernel, dim3((n_cols + 3) / 4), dim3(256), 0, st, cols, n_cols, parts, X);
  return hipGetLastError();
}

hipError_t launch_batch_select(BatchCol* cols, uint32_t n_cols, const float* scores, int32_t k, float margin,
                               BatchOut* out, hipStream_t st) {
  hipLaunchKernelGGL(batch_select_kernel, dim3((n_cols + 255) / 256), dim3(256), 0, st, cols, n_cols, scores, k,
                     margin, out);
  return hipGetLastError();
}

// Start of a replay of a planned batch: every result slot cleared, carrying
// the strategy its column uses (fixed when the batch was planned).
__global__ __launch_bounds__(256) void batch_reset_kernel(const BatchCol* cols, uint32_t n_cols, BatchOut* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cols) out[i] = BatchOut{0, 0, 0, (uint64_t)(uint32_t)cols[i].strategy};
}

hipError_t launch_batch_reset(const BatchCol* cols, uint32_t n_cols, BatchOut* out, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((n_cols + 255) / 256), dim3(256), 0, st, cols, n_cols, out);
  return hipGetLastError();
}


}  // namespace scan_dev
