// Batched scans: thousands of columns of mixed length, width, encoding and
// strategy in one sequence of launches.
//
// Each column is cut into work items of up to four windows of G blocks, which
// the four wavefronts of a work-group share.  A binning kernel
// sorts the items into twelve classes (encoding x decoder x predicate mode),
// reading each column's strategy from device memory (so a selector kernel that
// ran earlier on the same stream decides it), and one persistent kernel per
// class walks its item list on a static schedule: work-group g of G takes
// items g, g + G, ... below the class count, its four wavefronts one window
// each (no shared cursor, every loop bounded by counts fixed before the
// launch; dictionary classes give each work-group a contiguous share of the
// list instead, see batch_dict_share).  For an item it switches
// (wave-uniformly) on the column's width to the same templated range
// decoders the single-column kernels use, and each wavefront adds its exact
// partial (count, sum mod 2^64, blocks read) to the column's slot with three
// 64-bit atomics.
// Zone maps on/off is a per-column run-time flag.
#pragma once

#include "scan_kernels.h"

namespace scan_dev {

constexpr int kBatchClasses = 12;  // enc (3) x decoder {RM-LDS, RM-direct} x mode {BF, SV}

// One batch column (device).
struct BatchCol {
  const uint32_t* payload;
  const uint32_t* refs;
  const int64_t* bases;
  const int64_t* dict;
  const void* zmin;
  const void* zmax;
  uint64_t n, nb;
  int64_t lo, hi;
  uint32_t lo32, hi32m1;  // FOR: predicate clamped to the u32 domain
  uint32_t dict_len, tail;
  uint32_t b;
  int32_t enc;
  int32_t requested;      // strategy asked for, or -1 (choose on device)
  int32_t strategy;       // strategy used (written on device)
  uint32_t clo, chi;      // dictionary code range (written on device)
  uint32_t valid_mask;    // selector classes allowed for this column (bit c)
  uint32_t flags;         // kColEmpty | kColHasZm | kColSkip
  int32_t heuristic;      // strategy used when no selector is loaded
  uint32_t fseg0;         // first zone-map segment of the column (selector features)
  uint32_t fsegs;         // number of its segments (0: no zone maps or no blocks)
  uint32_t pad;
};

enum : uint32_t { kColEmpty = 1u, kColHasZm = 2u, kColSkip = 4u };

struct BatchWork {
  uint32_t col;
  uint32_t nblk;
  uint64_t k0;
};

// Zone-map sums of one segment of a column's blocks (selector features; see
// batch_feat_seg_kernel).
struct FeatPart {
  double acc, meet, spread, gmin, gmax;
};

// Blocks per zone-map segment: one wavefront reads four zone-map pairs per
// lane at once.
constexpr uint32_t kFeatSegBlocks = 256;

struct BatchOut {
  uint64_t count, sum, blocks;
  uint64_t pad;  // strategy used (written by the selection kernel)
};

struct BatchArgs {
  BatchCol* cols;
  const BatchWork* work;
  uint32_t* lists;     // kBatchClasses lists of n_work item indices
  uint32_t* counts;    // kBatchClasses item counts (appended to by the binning kernel)
  BatchOut* out;       // per column
  uint32_t n_cols, n_work;
  int32_t cls;         // class handled by this launch
  uint32_t pad;
};

__host__ __device__ inline int batch_class(int enc, int strategy) {
  return enc * 4 + (strategy & 1) * 2 + ((strategy >> 2) & 1);
}

__device__ __forceinline__ Params batch_params(const BatchCol& c) {
  Params p;
  p.payload = c.payload;
  p.refs = c.refs;
  p.bases = c.bases;
  p.dict = c.dict;
  p.zmin = c.zmin;
  p.zmax = c.zmax;
  p.bsum = nullptr;  // batches do not take the all-match shortcut
  p.n = c.n;
  p.nb = c.nb;
  p.units = 0;
  p.lo = c.lo;
  p.hi = c.hi;
  p.lo32 = c.lo32;
  p.hi32m1 = c.hi32m1;
  p.dict_len = c.dict_len;
  p.G = 0;
  p.use_zm = (c.strategy >> 3) & 1;
  p.tail = c.tail;
  p.strategy = c.strategy;
  p.use_am = 0;
  p.partials = nullptr;
  p.out = nullptr;
  return p;
}

constexpr uint32_t kBatchWaveWords = kListWords + 32u * 32u + 4u + 2u * kRingEntries;

template <int B, int ENC, int DEC, int MODE>
__device__ __forceinline__ void batch_item(const Params& p, const BatchCol& c, uint64_t k0, uint64_t k1,
                                           uint32_t lane, uint32_t* list, uint32_t* st, BatchOut* out) {
  uint64_t count, blocks, lsum;
  if constexpr (ENC == ENC_DELTA) {
    WaveState<RelT<B>> s;
    s.ring = reinterpret_cast<RelT<B>*>(st + 32u * 32u + 4u);
    delta_range<B, DEC, MODE, true>(p, s, lane, list, st, k0, k1, 64, 64);
    if constexpr (MODE == MODE_SV) sv_drain_rest<ENC_DELTA, RelT<B>>(s, lane, nullptr, 0);
    count = s.count + wave_sum_u64(s.lcount);
    blocks = s.blocks;
    lsum = s.lsum + (lane == 0 ? s.refsum : 0ull);
  } else {
    WaveState<uint32_t> s;
    s.ring = st + 32u * 32u + 4u;
    const uint32_t dlast = c.dict_len ? c.dict_len - 1u : 0u;
    if (ENC == ENC_FOR && c.refs)
      scan_range<B, DEC, MODE, ENC, PF_REFS, STEP_SMALL>(p, s, lane, list, st, k0, k1, 64, 64, c.dict, dlast, c.clo, c.chi);
    else
      scan_range<B, DEC, MODE, ENC, PF_RANGE, STEP_SMALL>(p, s, lane, list, st, k0, k1, 64, 64, c.dict, dlast, c.clo,
                                                    c.chi);
    if constexpr (MODE == MODE_SV) sv_drain_rest<ENC, uint32_t>(s, lane, c.dict, dlast);
    count = s.count + wave_sum_u64(s.lcount);
    blocks = s.blocks;
    lsum = s.lsum + (lane == 0 ? s.refsum : 0ull);
  }
  const uint64_t sum = wave_sum_u64(lsum);
  if (lane == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->count), (unsigned long long)count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->sum), (unsigned long long)sum);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->blocks), (unsigned long long)blocks);
  }
}

// Dictionary classes.  A per-value gather of dictionary entries from global
// memory is bound by the vector memory unit's per-lane address processing, so
// the dictionary (at most kMaxDict int64 entries) is staged in LDS; one copy
// per wavefront does not fit, so the wavefronts of a work-group take items
// together: the work-group walks its contiguous share of the class list, its
// wavefronts split each item's blocks, and the dictionary is staged again only
// when the column changes.  A wavefront keeps its partial across the items of
// one column and adds it to the column's slot when the column changes.
template <int MODE>
__device__ __forceinline__ void dict_flush(WaveState<uint32_t>& s, uint32_t lane, const int64_t* dict_lds,
                                           uint32_t dlast, BatchOut* out) {
  if constexpr (MODE == MODE_SV) sv_drain_rest<ENC_DICT, uint32_t>(s, lane, dict_lds, dlast);
  const uint64_t count = s.count + wave_sum_u64(s.lcount);
  const uint64_t sum = wave_sum_u64(s.lsum + (lane == 0 ? s.refsum : 0ull));
  if (lane == 0 && (count | sum | s.blocks)) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->count), (unsigned long long)count);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->sum), (unsigned long long)sum);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out->blocks), (unsigned long long)s.blocks);
  }
  s.count = s.blocks = s.refsum = s.lsum = s.lcount = 0;
  s.head = s.tail = 0;
}

#define SCAN_WIDTHS_ALL(F)                                                                                \
  F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16) F(17) F(18) F(19) F(20) \
      F(21) F(22) F(23) F(24) F(25) F(26) F(27) F(28) F(29) F(30) F(31) F(32)

#define BATCH_SHARE_CASE(B)                                                                 \
  case B:                                                                                   \
    batch_item<B, ENC, DEC, MODE>(p, c, w.k0 + b0, w.k0 + b1, lane, list, st, out);         \
    break;

#define BATCH_DICT_CASE(B)                                                                                    \
  case B:                                                                                                     \
    scan_range<B, DEC, MODE, ENC_DICT, PF_RANGE, STEP_SMALL>(p, s, lane, list, st, w.k0 + b0, w.k0 + b1, 64, 64, dict, \
                                                       dlast, c.clo, c.chi);                                  \
    break;

constexpr uint32_t kBatchDictBytes = kDictLdsBytes;

template <int DEC, int MODE>
__device__ __forceinline__ void batch_dict_share(const BatchArgs& a, const uint32_t* items, uint32_t n,
                                                 int64_t* dict, uint32_t* list, uint32_t* st, uint32_t lane,
                                                 uint32_t wave) {
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t per = n / gridDim.x + (n % gridDim.x ? 1u : 0u);
  const uint64_t i0 = (uint64_t)blockIdx.x * per;
  const uint64_t i1 = i0 + per < (uint64_t)n ? i0 + per : (uint64_t)n;
  WaveState<uint32_t> s;
  s.ring = st + 32u * 32u + 4u;
  uint32_t cur = 0xFFFFFFFFu, dlast = 0;
  for (uint64_t idx = i0; idx < i1; ++idx) {
    const BatchWork w = a.work[items[idx]];
    const uint32_t col = __builtin_amdgcn_readfirstlane(w.col);
    if (col != cur) {
      if (cur != 0xFFFFFFFFu) dict_flush<MODE>(s, lane, dict, dlast, a.out + cur);
      __syncthreads();  // every wavefront is done with the previous dictionary
      const int64_t* src = a.cols[col].dict;
      const uint32_t len = a.cols[col].dict_len < kMaxDict ? a.cols[col].dict_len : kMaxDict;
      const uint32_t clo = a.cols[col].clo, chi = a.cols[col].chi;
      // the form stage_dictionary writes: packed (branch-free classes, when the
      // window's range allows) or masked, 0 outside [clo, chi) up to the zero slot
      uint64_t base = clo < chi ? (uint64_t)src[clo] : 0ull;
      const bool packed = MODE == MODE_BF && (clo >= chi || (uint64_t)src[chi - 1u] - base < kDictMaxRange);
      // slots a code can reach: the entries, and up to 2^b (at most kMaxDict)
      const uint32_t b = a.cols[col].b;
      const uint32_t reach = b <= 12u ? (1u << b) : kMaxDict;
      const uint32_t top = len > reach ? len : reach;
      // eight loads in flight per thread, then their slots
      for (uint32_t c0 = 0; c0 < top; c0 += blockDim.x * 8u) {
        int64_t e[8];
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j) {
          const uint32_t i = c0 + threadIdx.x + j * blockDim.x;
          e[j] = (i >= clo && i < chi) ? src[i] : 0;
        }
#pragma unroll
        for (uint32_t j = 0; j < 8u; ++j) {
          const uint32_t i = c0 + threadIdx.x + j * blockDim.x;
          if (i < top)
            dict[i] = (packed && i >= clo && i < chi)
                          ? (int64_t)(((uint64_t)e[j] - base) | (1ull << kDictCountShift)) : e[j];
        }
      }
      if (threadIdx.x == 0) dict[kDictZeroSlot] = 0;
      s.dict_packed = packed;
      s.dict_base = base;
      __syncthreads();
      cur = col;
      dlast = len ? len - 1u : 0u;
    }
    const BatchCol c = a.cols[col];
    const Params p = batch_params(c);
    // this wavefront's share of the item's blocks
    const uint32_t q = (w.nblk + nw - 1u) / nw;
    const uint32_t b0 = wave * q < w.nblk ? wave * q : w.nblk;
    const uint32_t b1 = b0 + q < w.nblk ? b0 + q : w.nblk;
    if (b0 < b1) {
      switch (c.b) {
        SCAN_WIDTHS_ALL(BATCH_DICT_CASE)
        default: break;
      }
    }
  }
  if (cur != 0xFFFFFFFFu) dict_flush<MODE>(s, lane, dict, dlast, a.out + cur);
}

template <int ENC, int DEC, int MODE>
// At least two wavefronts per SIMD (two work-groups per CU): at most 256 VGPRs.
__global__ __launch_bounds__(256, 2) void batch_scan(const BatchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  constexpr uint32_t kDictBytes = ENC == ENC_DICT ? kBatchDictBytes : 0u;
  uint32_t* list = reinterpret_cast<uint32_t*>(smem + kDictBytes) + wave * kBatchWaveWords;
  uint32_t* st = list + kListWords;
  const uint32_t cnt = __builtin_amdgcn_readfirstlane(a.counts[a.cls]);
  const uint32_t n = cnt < a.n_work ? cnt : a.n_work;
  const uint32_t* items = a.lists + (size_t)a.cls * a.n_work;
  if constexpr (ENC == ENC_DICT) {
    batch_dict_share<DEC, MODE>(a, items, n, reinterpret_cast<int64_t*>(smem), list, st, lane, wave);
  } else {
    // The four wavefronts of a work-group split every item: the items whose
    // blocks survive the zone maps are dense (a sorted delta column's
    // survivors are one contiguous range), and no wavefront decodes a whole
    // dense item alone.
    const uint32_t nw = blockDim.x >> 6;
    for (uint32_t idx = blockIdx.x; idx < n; idx += gridDim.x) {
      const BatchWork w = a.work[items[idx]];
      const BatchCol c = a.cols[w.col];
      const Params p = batch_params(c);
      BatchOut* out = a.out + w.col;
      const uint32_t q = (w.nblk + nw - 1u) / nw;
      const uint32_t b0 = wave * q < w.nblk ? wave * q : w.nblk;
      const uint32_t b1 = b0 + q < w.nblk ? b0 + q : w.nblk;
      if (b0 < b1) {
        switch (c.b) {
          SCAN_WIDTHS_ALL(BATCH_SHARE_CASE)
          default: break;
        }
      }
    }
  }
}

using BatchLaunchFn = hipError_t (*)(const BatchArgs&, uint32_t grid, uint32_t block, hipStream_t st, int* occ);

template <int ENC, int DEC, int MODE>
hipError_t launch_batch_class(const BatchArgs& a, uint32_t grid, uint32_t block, hipStream_t st, int* occ) {
  if constexpr (ENC == ENC_DICT) {
    // the dictionary is addressed from LDS address 0 (see dict_at)
    static const hipError_t lds0 = [] {
      hipFuncAttributes fa;
      const hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(batch_scan<ENC, DEC, MODE>));
      if (e != hipSuccess) return e;
      return fa.sharedSizeBytes == 0 ? hipSuccess : hipErrorInvalidConfiguration;
    }();
    if (lds0 != hipSuccess) return lds0;
  }
  const uint32_t lds = (ENC == ENC_DICT ? kBatchDictBytes : 0u) + (block / 64u) * kBatchWaveWords * 4u;
  if (occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, batch_scan<ENC, DEC, MODE>, (int)block, lds);
  hipLaunchKernelGGL((batch_scan<ENC, DEC, MODE>), dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

// Defined in the k_batch_*.hip instantiation units; indexed by batch_class().
BatchLaunchFn batch_class_fn(int cls);

}  // namespace scan_dev
