// Materializing select: the ascending positions of the rows that pass a
// range predicate, written to HBM, and late materialization on a position
// list (refine by another column's predicate, gather values).
//
// Select runs in three steps so that the output order is the row order:
//  1. count: every wavefront takes blocks k = w, w + W, ... (W wavefronts),
//     tests the zone map, stages and decodes the block (values j = lane + 64 t)
//     and stores the block's match count;
//  2. an exclusive scan of the counts gives each block its output offset
//     (tiles of 1024 counts per work-group, one work-group over the tile
//     totals, then the tile offsets added back);
//  3. write: blocks with matches are decoded again and the matches of step t
//     are compacted with ballot + mbcnt at offset + (matches of steps < t),
//     so positions leave in ascending order.  A block entirely inside the
//     predicate (all-match, with zone maps) writes its position range without
//     being read.
// Work loops use a wave-uniform block index (readfirstlane), so their
// control flow is the same in every lane.
#include "device_common.h"
#include "runtime_decode.h"
#include "select_kernels.h"

namespace scan_dev {

namespace {

constexpr int kSelWaves = 4;

// Code-space window [clo, chi) of block k (FOR: minus the block reference,
// clipped to [0, 2^b); dictionary: the code range itself).
struct ZRange {
  int64_t lo, hi;  // the predicate in the zone-map / code domain
};

__device__ __forceinline__ ZRange load_range(const SelParams& p) {
  return ZRange{p.zrange[0], p.zrange[1]};
}

__device__ __forceinline__ void block_code_range(const SelParams& p, const ZRange& zr, uint64_t k, int64_t& clo,
                                                 int64_t& chi) {
  clo = zr.lo;
  chi = zr.hi;
  if (p.enc != ENC_DICT) {
    const int64_t ref = p.refs ? (int64_t)p.refs[k] : 0;
    const int64_t top = int64_t(1) << p.b;
    clo = clo - ref > 0 ? clo - ref : 0;
    chi = chi - ref < top ? chi - ref : top;
  }
}

// 0: skip the block, 1: decode it, 2: every valid value matches (all-match).
__device__ __forceinline__ int block_class(const SelParams& p, const ZRange& zr, uint64_t k) {
  if (zr.lo >= zr.hi) return 0;
  if (!p.use_zm) return 1;
  const int64_t mn = p.zmin[k], mx = p.zmax[k];
  if (mx < zr.lo || mn >= zr.hi) return 0;
  if (p.use_am && mn >= zr.lo && mx < zr.hi) return 2;
  return 1;
}

__device__ __forceinline__ uint32_t block_valid(const SelParams& p, uint64_t k) {
  return k == p.nb - 1 ? (uint32_t)(p.n - k * kBlockValues) : kBlockValues;
}

// Pass bits of the staged block: bit t of the result is value lane + 64 t.
__device__ __forceinline__ uint32_t block_pass_bits(const SelParams& p, const ZRange& zr, const uint32_t* st,
                                                    uint64_t k, uint32_t lane) {
  int64_t clo, chi;
  block_code_range(p, zr, k, clo, chi);
  if (clo >= chi) return 0u;
  const uint32_t valid = block_valid(p, k);
  const Extract ex(st, lane, p.b);
  const uint32_t lo32 = (uint32_t)clo, wm1 = (uint32_t)(chi - clo - 1);
  uint32_t bits = 0;
#pragma unroll
  for (uint32_t t = 0; t < 16u; ++t) {
    const bool ok = ((ex(t) - lo32) <= wm1) && (lane + 64u * t < valid);
    bits |= ok ? (1u << t) : 0u;
  }
  return bits;
}

}  // namespace

__global__ __launch_bounds__(256) void select_count_kernel(const SelParams p) {
  __shared__ __align__(16) uint32_t lds[kSelWaves][kRtStageWords];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* st = lds[wave];
  const ZRange zr = load_range(p);
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  for (uint64_t k = (uint64_t)blockIdx.x * kSelWaves + wave; k < p.nb; k += tw) {
    const int cls = block_class(p, zr, k);
    uint32_t cnt = 0;
    if (cls == 2) {
      cnt = block_valid(p, k);
    } else if (cls == 1) {
      stage_rt_block(st, p.payload, p.b, k, lane);
      const uint32_t bits = block_pass_bits(p, zr, st, k, lane);
      cnt = (uint32_t)wave_sum_u64(__builtin_popcount(bits));
    }
    p.counts[k] = cnt;  // every lane stores the same value
  }
}

// Exclusive scan of tiles of kScanTile counts (256 threads, 4 per thread).
__global__ __launch_bounds__(256) void scan_tiles_kernel(const uint32_t* in, uint64_t m, uint32_t* out,
                                                         uint32_t* tile_sums) {
  __shared__ uint32_t wsum[4];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)tid * 4u;
  uint32_t v[4], run = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = base + i < m ? in[base + i] : 0u;
    run += v[i];
  }
  // inclusive scan of the per-thread totals within the wavefront
  uint32_t incl = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= (uint32_t)d) incl += y;
  }
  if (lane == 63u) wsum[wave] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (uint32_t q = 0; q < wave; ++q) woff += wsum[q];
  uint32_t acc = woff + incl - run;  // exclusive prefix of this thread
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (base + i < m) out[base + i] = acc;
    acc += v[i];
  }
  if (tid == 255u) tile_sums[blockIdx.x] = woff + incl;
}

// Exclusive scan of the tile totals in place (one work-group of 1024
// threads, up to kScanTile * 4 tiles); the grand total goes to *total.
__global__ __launch_bounds__(1024) void scan_top_kernel(uint32_t* tile_sums, uint32_t ntiles, uint32_t* total) {
  __shared__ uint32_t wsum[16];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  uint32_t v[4], run = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t j = tid * 4u + i;
    v[i] = j < ntiles ? tile_sums[j] : 0u;
    run += v[i];
  }
  uint32_t incl = run;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= (uint32_t)d) incl += y;
  }
  if (lane == 63u) wsum[wave] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (uint32_t q = 0; q < wave; ++q) woff += wsum[q];
  uint32_t acc = woff + incl - run;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t j = tid * 4u + i;
    if (j < ntiles) tile_sums[j] = acc;
    acc += v[i];
  }
  if (tid == 1023u) *total = woff + incl;
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint32_t* out, uint64_t m, const uint32_t* tile_sums) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] += tile_sums[i / kScanTile];
}

__global__ __launch_bounds__(256) void select_write_kernel(const SelParams p, uint32_t* positions) {
  __shared__ __align__(16) uint32_t lds[kSelWaves][kRtStageWords];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* st = lds[wave];
  const ZRange zr = load_range(p);
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  for (uint64_t k = (uint64_t)blockIdx.x * kSelWaves + wave; k < p.nb; k += tw) {
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(p.counts[k]);
    if (cnt == 0u) continue;
    const uint32_t base = __builtin_amdgcn_readfirstlane(p.offsets[k]);
    const uint32_t first = (uint32_t)(k * kBlockValues);
    if (block_class(p, zr, k) == 2) {
      for (uint32_t j = lane; j < cnt; j += 64u) positions[base + j] = first + j;
      continue;
    }
    stage_rt_block(st, p.payload, p.b, k, lane);
    const uint32_t bits = block_pass_bits(p, zr, st, k, lane);
    uint32_t off = base;
#pragma unroll
    for (uint32_t t = 0; t < 16u; ++t) {
      const bool ok = (bits >> t) & 1u;
      const uint64_t m = ballot(ok);
      if (ok) positions[off + mbcnt(m)] = first + lane + 64u * t;
      off += (uint32_t)__builtin_popcountll(m);
    }
  }
}

// Refine, pass 1: chunk c holds input positions c*1024 + lane + 64 t; each
// chunk stores its 16 ballots and its pass count.
__global__ __launch_bounds__(256) void refine_mark_kernel(const SelParams p, const uint32_t* pos, uint64_t m,
                                                          uint64_t* ballots, uint32_t* counts) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t nchunks = (m + kBlockValues - 1) / kBlockValues;
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  const ZRange zr = load_range(p);
  for (uint64_t c = (uint64_t)blockIdx.x * kSelWaves + wave; c < nchunks; c += tw) {
    uint32_t cnt = 0;
#pragma unroll 4
    for (uint32_t t = 0; t < 16u; ++t) {
      const uint64_t q = c * kBlockValues + lane + 64u * t;
      bool ok = false;
      const uint32_t i = q < m ? pos[q] : 0u;
      if (q < m && i < p.n) {  // a position past the column never passes
        const uint32_t code = code_at(p.payload, p.b, i);
        if (p.enc == ENC_DICT) {
          ok = (int64_t)code >= zr.lo && (int64_t)code < zr.hi;
        } else {
          const int64_t v = (int64_t)(uint32_t)((p.refs ? p.refs[i >> 10] : 0u) + code);
          ok = v >= zr.lo && v < zr.hi;
        }
      }
      const uint64_t bl = ballot(ok);
      ballots[c * 16u + t] = bl;  // every lane stores the same value
      cnt += (uint32_t)__builtin_popcountll(bl);
    }
    counts[c] = cnt;  // every lane stores the same value
  }
}

// Refine, pass 2: the kept positions at the chunk offsets, in input order.
__global__ __launch_bounds__(256) void refine_write_kernel(const uint32_t* pos, uint64_t m, const uint64_t* ballots,
                                                           const uint32_t* offsets, uint32_t* out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t nchunks = (m + kBlockValues - 1) / kBlockValues;
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  for (uint64_t c = (uint64_t)blockIdx.x * kSelWaves + wave; c < nchunks; c += tw) {
    uint32_t off = __builtin_amdgcn_readfirstlane(offsets[c]);
    for (uint32_t t = 0; t < 16u; ++t) {
      const uint64_t bl = ballots[c * 16u + t];
      const bool ok = (bl >> lane) & 1ull;
      if (ok) out[off + mbcnt(bl)] = pos[c * kBlockValues + lane + 64u * t];
      off += (uint32_t)__builtin_popcountll(bl);
    }
  }
}

__global__ __launch_bounds__(256) void gather_kernel(const SelParams p, const uint32_t* pos, uint64_t m,
                                                     int64_t* values) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint32_t i = pos[q];
  if (i >= p.n) {  // a position past the column reads nothing
    values[q] = 0;
    return;
  }
  const uint32_t code = code_at(p.payload, p.b, i);
  if (p.enc == ENC_DICT) {
    const uint32_t last = p.dict_len - 1u;
    values[q] = p.dict[code < last ? code : last];
  } else {
    values[q] = (int64_t)(uint32_t)((p.refs ? p.refs[i >> 10] : 0u) + code);
  }
}

// The predicate in the zone-map / code domain, into p.zrange[0..1]:
// frame of reference [lo, hi) clamped to [0, 2^32]; dictionary
// [lower_bound(lo), lower_bound(hi)) over the entries.
__global__ void select_setup_kernel(const SelParams p, int64_t* zrange) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t zl, zh;
  if (p.enc == ENC_DICT) {
    zl = lower_bound_global(p.dict, p.dict_len, p.lo);
    zh = lower_bound_global(p.dict, p.dict_len, p.hi);
  } else {
    zl = p.lo > 0 ? p.lo : 0;
    zh = p.hi < (int64_t(1) << 32) ? p.hi : (int64_t(1) << 32);
  }
  if (p.lo >= p.hi) zh = zl;
  zrange[0] = zl;
  zrange[1] = zh;
}

// ------------------------------------------------------------ launchers

hipError_t launch_select_count(const SelParams& p, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(select_count_kernel, dim3(grid), dim3(64 * kSelWaves), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint64_t m, uint32_t* out, uint32_t* tile_sums,
                                 uint32_t* total, hipStream_t st) {
  const uint64_t ntiles = (m + kScanTile - 1) / kScanTile;
  if (ntiles == 0 || ntiles > 4096) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((uint32_t)ntiles), dim3(256), 0, st, in, m, out, tile_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, st, tile_sums, (uint32_t)ntiles, total);
  hipLaunchKernelGGL(scan_add_kernel, dim3((uint32_t)((m + 255) / 256)), dim3(256), 0, st, out, m, tile_sums);
  return hipGetLastError();
}

hipError_t launch_select_write(const SelParams& p, uint32_t* positions, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(select_write_kernel, dim3(grid), dim3(64 * kSelWaves), 0, st, p, positions);
  return hipGetLastError();
}

hipError_t launch_refine_mark(const SelParams& p, const uint32_t* pos, uint64_t m, uint64_t* ballots,
                              uint32_t* counts, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(refine_mark_kernel, dim3(grid), dim3(64 * kSelWaves), 0, st, p, pos, m, ballots, counts);
  return hipGetLastError();
}

hipError_t launch_refine_write(const uint32_t* pos, uint64_t m, const uint64_t* ballots, const uint32_t* offsets,
                               uint32_t* out, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(refine_write_kernel, dim3(grid), dim3(64 * kSelWaves), 0, st, pos, m, ballots, offsets, out);
  return hipGetLastError();
}

hipError_t launch_gather(const SelParams& p, const uint32_t* pos, uint64_t m, int64_t* values, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((uint32_t)((m + 255) / 256)), dim3(256), 0, st, p, pos, m, values);
  return hipGetLastError();
}

hipError_t launch_select_setup(const SelParams& p, int64_t* zrange, hipStream_t st) {
  hipLaunchKernelGGL(select_setup_kernel, dim3(1), dim3(64), 0, st, p, zrange);
  return hipGetLastError();
}

}  // namespace scan_dev
