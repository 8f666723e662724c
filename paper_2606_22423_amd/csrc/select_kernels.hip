// Materializing select: the ascending positions of the rows that pass a
// range predicate, written to HBM, and late materialization on a position
// list (refine by another column's predicate, gather values).
//
// Select runs in three steps so that the output order is the row order:
//  1. mark (one kernel per width b): every wavefront takes two blocks at a
//     time, half a wavefront each; after the zone-map test, lane l' of a
//     half marks the 32 values 32 l' .. 32 l' + 31 of its block from codes
//     in registers and stores them as one 32-bit word (the block's 1024-bit
//     mark string, 128 bytes, one bit per value), and the half's popcount
//     sum is the block's match count.  Codes of 8 and 16 bits are read
//     coalesced by groups of b / 4 lanes per mark word, 32-bit codes by the
//     whole half with one ballot per word, other widths as each lane's own
//     slice of b words;
//  2. an exclusive scan of the counts gives each block its output offset
//     (tiles of 1024 counts per work-group, one work-group over the tile
//     totals, then the tile offsets added back);
//  3. write: groups of 16 consecutive blocks per wavefront; the marks of the
//     group's blocks with matches arrive in one round of loads, read as 16
//     64-bit words per block; four consecutive blocks fill one contiguous
//     output range, expanded in the wavefront's LDS buffer and copied out
//     with coalesced stores, so every position lands at its rank in row
//     order.  The payload is not read again.
//     A block entirely inside the predicate (all-match, with zone maps) has
//     no marks: its position range is written without being read.
// Work loops use a wave-uniform block index (readfirstlane), so their
// control flow is the same in every lane.
#include "device_common.h"
#include "runtime_decode.h"
#include "select_kernels.h"

#include <utility>

namespace scan_dev {

namespace {

constexpr int kSelWaves = 4;
constexpr uint32_t kWriteGroup = 16;  // blocks per wavefront step of the write pass

// The predicate in the zone-map / code domain, as written by the setup kernel.
struct ZRange {
  int64_t lo, hi;
};

__device__ __forceinline__ ZRange load_range(const SelParams& p) {
  return ZRange{p.zrange[0], p.zrange[1]};
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

// Pass marks of one lane's 32 codes (held in w, stream bits [32 B l', ...) of
// its block, values 32 l' .. 32 l' + 31) for the code window [lo32, lo32 +
// wm1]: bit t of the result for value 32 l' + t; with VALID, values at or
// past `valid` (the block's valid count) fail.
template <uint32_t B, bool VALID>
__device__ __forceinline__ uint32_t lane_marks(const uint32_t (&w)[B], uint32_t lo32, uint32_t wm1, uint32_t v0,
                                               uint32_t valid) {
  uint32_t bits = 0;
#pragma unroll
  for (uint32_t t = 0; t < 32u; ++t) {
    const uint32_t bit = t * B, wi = bit >> 5, sh = bit & 31u;
    uint32_t c;
    if (B == 32) c = w[t];
    else if (sh + B <= 32) c = (w[wi] >> sh) & ((1u << (B & 31u)) - 1u);
    else c = __builtin_amdgcn_alignbit(w[wi + 1 < B ? wi + 1 : wi], w[wi], sh) & ((1u << (B & 31u)) - 1u);
    bool hit = (c - lo32) <= wm1;
    if (VALID) hit = hit && (v0 + t < valid);
    bits |= (hit ? 1u : 0u) << t;
  }
  return bits;
}

// The lane's B words, in 16-byte (B a multiple of 4) or 8-byte (B even)
// pieces; the slice starts at a multiple of 4 B bytes of a 16-byte aligned
// payload.  A load instruction touches one line per lane.  In one or two
// pieces the lines are used up at once and the loads are nontemporal (the
// payload stream then leaves the marks in the last-level cache for the write
// pass); in more pieces they are plain, so that the lane's later pieces hit
// the lines in the L1 instead of fetching them again.
typedef uint32_t SelU32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t SelU32x2 __attribute__((ext_vector_type(2)));
template <typename T, bool NT>
__device__ __forceinline__ T load_piece(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <uint32_t B>
__device__ __forceinline__ void load_lane_words(const uint32_t* __restrict__ src, uint32_t (&w)[B]) {
  constexpr uint32_t kPieces = B % 4u == 0u ? B / 4u : B % 2u == 0u ? B / 2u : B;
  constexpr bool kNT = kPieces <= 2u;
  if constexpr (B % 4u == 0u) {
#pragma unroll
    for (uint32_t i = 0; i < B / 4u; ++i) {
      const SelU32x4 v = load_piece<SelU32x4, kNT>(reinterpret_cast<const SelU32x4*>(src) + i);
      w[4u * i] = v.x;
      w[4u * i + 1u] = v.y;
      w[4u * i + 2u] = v.z;
      w[4u * i + 3u] = v.w;
    }
  } else if constexpr (B % 2u == 0u) {
#pragma unroll
    for (uint32_t i = 0; i < B / 2u; ++i) {
      const SelU32x2 v = load_piece<SelU32x2, kNT>(reinterpret_cast<const SelU32x2*>(src) + i);
      w[2u * i] = v.x;
      w[2u * i + 1u] = v.y;
    }
  } else {
#pragma unroll
    for (uint32_t i = 0; i < B; ++i) w[i] = load_piece<uint32_t, kNT>(src + i);
  }
}

// 32-bit codes, one per word: lane l' of the half-wavefront reads words
// 32 i + l' (coalesced, nontemporal), and the half's ballot of pass i is mark word i,
// which lane i keeps.  Every lane of the half takes the same branch, so
// the ballot's other half (the other block, or inactive) is dropped.
template <bool VALID>
__device__ __forceinline__ uint32_t wide_marks(const uint32_t* __restrict__ blk, uint32_t l, uint32_t half,
                                               uint32_t lo32, uint32_t wm1, uint32_t valid) {
  uint32_t c[32];
#pragma unroll
  for (uint32_t i = 0; i < 32u; ++i) c[i] = __builtin_nontemporal_load(blk + 32u * i + l);
  uint32_t bits = 0;
#pragma unroll
  for (uint32_t i = 0; i < 32u; ++i) {
    bool hit = (c[i] - lo32) <= wm1;
    if (VALID) hit = hit && (32u * i + l < valid);
    const uint64_t bal = __ballot(hit);
    const uint32_t mine = half ? (uint32_t)(bal >> 32) : (uint32_t)bal;
    bits = l == i ? mine : bits;
  }
  return bits;
}

// B = 8 or 16: the 4 B bytes of a mark word are read by a group of
// P = B / 4 lanes, 16 bytes each; in pass i (of P) lane l' reads piece
// 32 i + l' of the block (coalesced, nontemporal), the 32 / P codes of
// values (32 i + l') 32 / P + c, which are bits (l' mod P) 32 / P + c of
// mark word (32 i + l') / P.  Shuffles within the group join the pieces,
// and lane l' then takes word l' from the group that built it.
template <uint32_t B, bool VALID>
__device__ __forceinline__ uint32_t group_marks(const uint32_t* __restrict__ blk, uint32_t l, uint32_t lo32,
                                                uint32_t wm1, uint32_t valid) {
  static_assert(B == 8u || B == 16u, "group marks take 8- or 16-bit codes");
  constexpr uint32_t P = B / 4u, kCodes = 32u / P, kPerWord = 32u / B, kMask = (1u << B) - 1u;
  SelU32x4 v[P];
#pragma unroll
  for (uint32_t i = 0; i < P; ++i) v[i] = __builtin_nontemporal_load(reinterpret_cast<const SelU32x4*>(blk) + 32u * i + l);
  uint32_t r[P];
#pragma unroll
  for (uint32_t i = 0; i < P; ++i) {
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t c = 0; c < kCodes; ++c) {
      const uint32_t code = (v[i][c / kPerWord] >> (B * (c % kPerWord))) & kMask;
      bool hit = (code - lo32) <= wm1;
      if (VALID) hit = hit && ((32u * i + l) * kCodes + c < valid);
      bits |= (hit ? 1u : 0u) << c;
    }
    uint32_t x = bits << (kCodes * (l % P));
#pragma unroll
    for (uint32_t o = 1; o < P; o <<= 1) x |= __shfl_xor(x, (int)o, 32);
    r[i] = x;
  }
  uint32_t out = 0;
#pragma unroll
  for (uint32_t i = 0; i < P; ++i) {
    const uint32_t t = __shfl(r[i], (int)(P * (l % kCodes)), 32);
    out = l / kCodes == i ? t : out;
  }
  return out;
}

}  // namespace

// Mark pass: a wavefront takes two blocks at a time, half a wavefront each;
// lane l' of a half holds the 32 consecutive codes of values 32 l' .. 32 l' +
// 31 (the block's words l' B .. l' B + B - 1, read straight into registers)
// and writes their marks as one 32-bit word, word l' of the block's 1024-bit
// mark string, which the write pass reads as 16 words of 64 bits (bit l of
// word t: value 64 t + l).  The block's count is the half-wavefront's sum.
// Zone maps decide per block: skipped (count 0, no marks), decoded, or, with
// the all-match shortcut, taken whole (count = its valid values, no marks).
template <uint32_t B>
__global__ __launch_bounds__(256) void select_mark_kernel(const SelParams p) {
  const uint32_t lane = threadIdx.x & 63u, l = lane & 31u, half = lane >> 5;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const ZRange zr = load_range(p);
  const int64_t top = int64_t(1) << B;
  const uint64_t npairs = (p.nb + 1u) / 2u;
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  uint32_t* marks32 = reinterpret_cast<uint32_t*>(p.marks);
  for (uint64_t q = (uint64_t)blockIdx.x * kSelWaves + wave; q < npairs; q += tw) {
    const uint64_t k = 2u * q + half;
    const bool in = k < p.nb;
    const int cls = in ? block_class(p, zr, k) : 0;
    const uint32_t valid = k == p.nb - 1u ? (uint32_t)(p.n - k * kBlockValues) : kBlockValues;
    uint32_t cnt = 0;
    if (cls == 1) {
      int64_t clo = zr.lo, chi = zr.hi;
      if (p.enc != ENC_DICT && p.refs) {
        const int64_t ref = (int64_t)p.refs[k];
        clo = clo - ref > 0 ? clo - ref : 0;
        chi = chi - ref < top ? chi - ref : top;
      }
      if (clo < chi) {
        const uint32_t lo32 = (uint32_t)clo, wm1 = (uint32_t)(chi - clo - 1);
        uint32_t bits;
        if constexpr (B == 32u) {
          bits = valid == kBlockValues ? wide_marks<false>(p.payload + k * 1024u, l, half, lo32, wm1, valid)
                                       : wide_marks<true>(p.payload + k * 1024u, l, half, lo32, wm1, valid);
        } else if constexpr (B == 8u || B == 16u) {
          bits = valid == kBlockValues ? group_marks<B, false>(p.payload + k * (32u * B), l, lo32, wm1, valid)
                                       : group_marks<B, true>(p.payload + k * (32u * B), l, lo32, wm1, valid);
        } else {
          const uint32_t* src = p.payload + k * (32u * B) + l * B;
          uint32_t w[B];
          load_lane_words<B>(src, w);
          bits = valid == kBlockValues ? lane_marks<B, false>(w, lo32, wm1, 32u * l, valid)
                                       : lane_marks<B, true>(w, lo32, wm1, 32u * l, valid);
        }
        marks32[k * 32u + l] = bits;
        cnt = (uint32_t)__builtin_popcount(bits);
      }
    }
    // the half-wavefront's sum (lanes of the other half hold the other block)
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 32);
    if (cls == 2) cnt = valid;
    if (in && l == 0u) p.counts[k] = cnt;
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

// Write pass: wavefront step = kWriteGroup consecutive blocks.  Lane j < 16
// holds block g + j's count, offset and class; the ballots of the blocks that
// have matches and no all-match shortcut arrive in four 8-byte loads per lane
// (load i, lane l: block 4 i + l / 16, step l % 16).  The offsets are an
// exclusive scan of the counts in block order, so the positions of four
// consecutive blocks fill one contiguous range of the output: each quarter
// (four blocks) is expanded into the wavefront's LDS buffer (every lane
// writes the set bits of its own ballot word, whole blocks are filled with
// their consecutive positions) and then copied out with coalesced stores.
// The buffer holds each position's offset from the quarter's first row (12
// bits, in 16-bit slots; sparse quarters writing their few positions
// straight to the output measured slower).  Only the wavefront itself
// touches its buffer: no work-group barrier.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ __launch_bounds__(256) void select_write_kernel(const SelParams p, uint32_t* positions) {
  __shared__ uint16_t stage_all[kSelWaves][4u * kBlockValues];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint16_t* stage = stage_all[wave];
  const ZRange zr = load_range(p);
  const uint64_t ngroups = (p.nb + kWriteGroup - 1) / kWriteGroup;
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  for (uint64_t g = (uint64_t)blockIdx.x * kSelWaves + wave; g < ngroups; g += tw) {
    const uint64_t k0 = g * kWriteGroup;
    const uint64_t kl = k0 + lane;
    const bool in = lane < kWriteGroup && kl < p.nb;
    const uint32_t cnt = in ? p.counts[kl] : 0u;
    const uint32_t off = in ? p.offsets[kl] : 0u;
    const bool whole = cnt > 0u && p.use_am && block_class(p, zr, kl) == 2;
    const uint64_t has = ballot(cnt > 0u);          // blocks with matches
    const uint64_t read = has & ~ballot(whole);     // ... that have ballots
    uint64_t mk[4];
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i) {
      const uint32_t blk = 4u * i + (lane >> 4);
      mk[i] = ((read >> blk) & 1ull) ? p.marks[(k0 + blk) * 16u + (lane & 15u)] : 0ull;
    }
#pragma unroll
    for (uint32_t i = 0; i < 4u; ++i) {
      const uint32_t q0 = 4u * i;
      if (!((has >> q0) & 0xFull)) continue;  // uniform: no match in the quarter
      // the quarter's output range: from the offset of its first block with
      // matches, as many positions as its blocks hold
      const uint32_t first_blk = q0 + (uint32_t)__builtin_ctzll((has >> q0) & 0xFull);
      const uint32_t base = __builtin_amdgcn_readlane(off, first_blk);
      uint32_t span = 0;
#pragma unroll
      for (uint32_t j = 0; j < 4u; ++j) span += __builtin_amdgcn_readlane(cnt, q0 + j);
      // ballot words: each lane places its word's positions after the
      // matches of its block's earlier steps (prefix sum over 16 lanes)
      uint64_t w = mk[i];
      const uint32_t pc = (uint32_t)__builtin_popcountll(w);
      uint32_t incl = pc;
#pragma unroll
      for (uint32_t d = 1; d < 16u; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 16);
        if ((lane & 15u) >= d) incl += y;
      }
      const uint32_t wo = __shfl(off, q0 + (lane >> 4), 64) + incl - pc;  // this word's first output slot
      const uint32_t qrow = (uint32_t)((k0 + q0) * kBlockValues);         // the quarter's first row
      const uint32_t wrow = 1024u * (lane >> 4) + 64u * (lane & 15u);      // this word's first row, from qrow
      const uint64_t whole_q = (has & ~read) & (0xFull << q0);
      uint32_t at = wo - base;
      while (w) {
        stage[at++] = (uint16_t)(wrow + (uint32_t)__builtin_ctzll(w));
        w &= w - 1ull;
      }
      // whole blocks of the quarter: their rows are consecutive
      for (uint64_t rest = whole_q; rest; rest &= rest - 1) {
        const uint32_t j = (uint32_t)__builtin_ctzll(rest);
        const uint32_t c = __builtin_amdgcn_readlane(cnt, j);
        const uint32_t o = __builtin_amdgcn_readlane(off, j) - base;
        const uint32_t r = 1024u * (j - q0);
        for (uint32_t q = lane; q < c; q += 64u) stage[o + q] = (uint16_t)(r + q);
      }
      wave_lds_order();
      for (uint32_t q = lane; q < span; q += 64u) positions[base + q] = qrow + stage[q];
      wave_lds_order();  // the copy has read the buffer before the next quarter fills it
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

namespace {
using MarkFn = void (*)(SelParams);
template <uint32_t... Bs>
struct MarkTable {
  static constexpr MarkFn fns[sizeof...(Bs)] = {select_mark_kernel<Bs + 1>...};
};
template <size_t... I>
constexpr auto make_mark_table(std::index_sequence<I...>) {
  return MarkTable<(uint32_t)I...>{};
}
using MarkTableT = decltype(make_mark_table(std::make_index_sequence<32>{}));
}  // namespace

hipError_t launch_select_mark(const SelParams& p, uint32_t grid, hipStream_t st) {
  if (p.b < 1 || p.b > 32) return hipErrorInvalidValue;
  // no more work-groups than fit at once (the registers limit them): a
  // grid-strided loop with a late second wave of work-groups runs that wave
  // on a part of the chip
  static int fit[32] = {};
  const void* fn = reinterpret_cast<const void*>(MarkTableT::fns[p.b - 1]);
  if (fit[p.b - 1] == 0) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64 * kSelWaves, 0) == hipSuccess && occ > 0 &&
        cus > 0)
      fit[p.b - 1] = cus * occ;
    else
      fit[p.b - 1] = -1;
  }
  if (fit[p.b - 1] > 0 && grid > (uint32_t)fit[p.b - 1]) grid = (uint32_t)fit[p.b - 1];
  hipLaunchKernelGGL(MarkTableT::fns[p.b - 1], dim3(grid), dim3(64 * kSelWaves), 0, st, p);
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
  // no more work-groups than fit at once (the LDS buffers limit them): the
  // grid-strided loop then has no late second wave
  static int fit = 0;
  if (fit == 0) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, select_write_kernel, 64 * kSelWaves, 0) == hipSuccess &&
        occ > 0 && cus > 0)
      fit = cus * occ;
    else
      fit = -1;
  }
  if (fit > 0 && grid > (uint32_t)fit) grid = (uint32_t)fit;
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
