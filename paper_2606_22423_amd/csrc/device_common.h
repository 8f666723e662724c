// Device-side building blocks shared by every scan kernel (gfx950, wave64).
//
// A scan kernel turns a column into one exact (count, sum, blocks_read)
// triple.  Integer addition mod 2^64 is associative and commutative, so every
// reduction order below gives the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scan_dev {

constexpr uint32_t kBlockValues = 1024;  // values per block (zone map / layout unit)
constexpr uint32_t kMaxDict = 4096;      // dictionary entries staged in LDS
// The LDS dictionary area: kMaxDict entries, then one zero entry (read for a
// partial last block's padding slots and for codes past the area), padded to
// 16 bytes.  Branch-free scans of dictionaries of b <= 5 also keep a table of
// code pairs in it, between the entries and the zero slot.
constexpr uint32_t kDictZeroSlot = kMaxDict;
constexpr uint32_t kDictLdsBytes = kMaxDict * 8u + 16u;
constexpr uint32_t kRingEntries = 128;   // per-wavefront selection-vector ring (u32 or u64 entries)

enum Dec { DEC_RM_LDS = 0, DEC_RM_DIRECT = 1, DEC_LI = 2, DEC_BYTES = 3 };
enum Mode { MODE_BF = 0, MODE_SV = 1 };
enum Enc { ENC_FOR = 0, ENC_DELTA = 1, ENC_DICT = 2 };

// Same memory layout as scan_result in include/scan.h.
struct Result {
  uint64_t count;
  int64_t sum;
  uint64_t blocks_read;
  uint64_t blocks_total;
  int32_t strategy_used;
  int32_t status;
};

struct Partial {
  uint64_t count, sum, blocks, pad;
};

struct Params {
  const uint32_t* payload;
  const uint32_t* refs;    // FOR block references, or null
  const int64_t* bases;    // DELTA block bases
  const int64_t* dict;     // DICT entries
  const void* zmin;        // per-block zone maps (u32 or int64), or null
  const void* zmax;
  const uint64_t* bsum;    // per-block sums of decoded values (all-match shortcut), or null
  uint64_t n;              // values
  uint64_t nb;             // blocks
  uint64_t units;          // work units of G blocks
  int64_t lo, hi;          // predicate [lo, hi) on decoded values (lo < hi)
  uint32_t lo32, hi32m1;   // FOR: the predicate clamped to the u32 domain, [lo32, hi32m1]
  uint32_t dict_len;
  uint32_t G;              // blocks per wavefront work unit, 1..64
  uint32_t use_zm;
  uint32_t tail;           // valid values in the last block, 1..1024
  int32_t strategy;
  uint32_t use_am;         // all-match shortcut (needs use_zm and bsum)
  Partial* partials;       // one per work-group
  Result* out;
};

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Position of this lane among the set lanes of m below it.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  return (uint64_t)readlane((uint32_t)x, l) | ((uint64_t)readlane((uint32_t)(x >> 32), l) << 32);
}

// Next work item of a wavefront from a shared counter.  Every lane takes
// part in the atomic (lane 0 adds 1, the others 0; the compiler folds it into
// one atomic per wavefront) and the first lane's old value is read into a
// scalar register.  The item is thus wave-uniform by construction and the
// work loop's control flow stays uniform.  (Fetching with `if (lane == 0)`
// and broadcasting with a lane shuffle let the optimizer route lanes 1-63
// back to the broadcast without passing the fetch; with lane 0 held outside
// that path they re-read item 0 forever.)
__device__ __forceinline__ uint32_t wave_next_item(uint32_t* cursor, uint32_t lane) {
  const uint32_t old = atomicAdd(cursor, lane == 0 ? 1u : 0u);
  return __builtin_amdgcn_readfirstlane(old);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint32_t lo = __shfl_xor((uint32_t)x, o, 64);
    uint32_t hi = __shfl_xor((uint32_t)(x >> 32), o, 64);
    x += ((uint64_t)hi << 32) | lo;
  }
  return x;
}

// Funnel shift: bits [s, s+32) of the 64-bit value hi:lo.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbit(hi, lo, s);
}

template <int B>
__device__ __forceinline__ constexpr uint32_t width_mask() {
  return B == 32 ? 0xFFFFFFFFu : ((1u << B) - 1u);
}

// Code t of a 32-code slice held in registers w[0..B): bits [t*B, t*B+B).
// Every shift is a compile-time constant (one v_bfe_u32, or alignbit + and).
template <int B>
__device__ __forceinline__ uint32_t slice_code(const uint32_t (&w)[B], int t) {
  const int bit = t * B;
  const int wi = bit >> 5, sh = bit & 31;
  if (B == 32) return w[t];
  if (sh + B <= 32) return (w[wi] >> sh) & width_mask<B>();
  return funnel(w[wi + 1], w[wi], sh) & width_mask<B>();
}

// FOR block predicate: values [lo32, hi32m1] mapped to codes c = v - ref in
// [0, 2^B): pass iff (c - loc) <= wm1 (u32), when nonempty.
template <int B>
__device__ __forceinline__ bool for_code_range(uint32_t ref, uint32_t lo32, uint32_t hi32m1,
                                               uint32_t& loc, uint32_t& wm1) {
  if (hi32m1 < ref) {
    loc = 0;
    wm1 = 0;
    return false;
  }
  uint32_t lc = lo32 > ref ? lo32 - ref : 0u;
  uint32_t hc = hi32m1 - ref;
  if (hc > width_mask<B>()) hc = width_mask<B>();
  loc = lc;
  wm1 = hc - lc;
  return lc <= hc;
}

// Zone-map survivors among blocks k0 .. k0+cnt-1 (cnt <= 64): bit i set iff
// block k0+i must be read.  Uniform result.
__device__ __forceinline__ uint64_t survivors_u32(const uint32_t* zmin, const uint32_t* zmax,
                                                  uint64_t k0, uint32_t cnt, uint32_t lo32,
                                                  uint32_t hi32m1) {
  const uint32_t l = lane_id();
  bool keep = false;
  if (l < cnt) {
    uint32_t mn = zmin[k0 + l], mx = zmax[k0 + l];
    keep = !(mx < lo32 || mn > hi32m1);
  }
  return ballot(keep);
}

__device__ __forceinline__ uint64_t survivors_i64(const int64_t* zmin, const int64_t* zmax, uint64_t k0,
                                                  uint32_t cnt, int64_t lo, int64_t hi) {
  const uint32_t l = lane_id();
  bool keep = false;
  if (l < cnt) {
    int64_t mn = zmin[k0 + l], mx = zmax[k0 + l];
    keep = !(mx < lo || mn >= hi);
  }
  return ballot(keep);
}

__device__ __forceinline__ uint64_t all_blocks(uint32_t cnt) {
  return cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
}

// Folds partials[0, n) into *out (one work-group; fold.hip).  Enqueued after
// every kernel that ends in write_partial, on the same stream.
hipError_t launch_fold(const Partial* partials, uint32_t n, Result* out, uint64_t blocks_total, int32_t strategy,
                       hipStream_t st);

// Work-group reduction of the per-wave (count, sum, blocks) into the
// work-group's partial; a second launch (fold_partials_kernel, enqueued right
// after on the same stream) folds the partials into the result.  A
// last-work-group ticket instead needs an agent-scope release per
// work-group, i.e. an L2 write-back on this multi-XCD part, and cost 5-11 us
// per launch; stream order makes the partials visible to the fold for free.
// `count` and `blocks` are wave-uniform, `lane_sum` per lane.  `red`: LDS
// for 16 x 3 values (kRedBytes); the scan kernels place it at the end of their
// dynamic LDS, which leaves their own LDS data at address 0 (no base add in
// the dictionary gathers' addresses).
constexpr uint32_t kRedBytes = 16u * 3u * 8u;
__device__ __forceinline__ void write_partial(Partial* partials, uint64_t count, uint64_t lane_sum, uint64_t blocks,
                                              uint64_t (*red)[3]) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t s = wave_sum_u64(lane_sum);
  if (lane == 0) {
    red[wave][0] = count;
    red[wave][1] = s;
    red[wave][2] = blocks;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t c = 0, t = 0, b = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      c += red[w][0];
      t += red[w][1];
      b += red[w][2];
    }
    Partial* q = partials + blockIdx.x;
    q->count = c;
    q->sum = t;
    q->blocks = b;
  }
}

__device__ __forceinline__ void write_partial(Partial* partials, uint64_t count, uint64_t lane_sum, uint64_t blocks) {
  __shared__ uint64_t red[16][3];
  write_partial(partials, count, lane_sum, blocks, red);
}

__device__ __forceinline__ void finish_scan(const Params& p, uint64_t count, uint64_t lane_sum, uint64_t blocks,
                                            uint64_t (*red)[3]) {
  write_partial(p.partials, count, lane_sum, blocks, red);
}

}  // namespace scan_dev
