// Materializing select: the ascending positions of the rows that pass a
// range predicate, written to HBM, and late materialization on a position
// list (refine by another column's predicate, gather values).
//
// Select runs in three steps so that the output order is the row order:
//  1. mark (one kernel per width b): every wavefront takes groups of
//     G = max(1, 32 / b) consecutive blocks (at most 4 KB of words), groups
//     g = w, w + W, ... (W wavefronts); it tests the zone maps, stages the
//     blocks that need decoding in LDS, decodes them (values j = lane + 64 t)
//     and stores each block's 16 pass ballots (one bit per value, 128 bytes)
//     and match count.  The next group's words are in flight in registers
//     while the current group decodes from LDS, and the zone maps and block
//     references arrive one group further ahead, so no load waits in the
//     steady state;
//  2. an exclusive scan of the counts gives each block its output offset
//     (tiles of 1024 counts per work-group, one work-group over the tile
//     totals, then the tile offsets added back);
//  3. write: groups of 16 consecutive blocks per wavefront; the ballots of the
//     group's blocks with matches arrive in one round of loads, each nonzero
//     ballot gets its output offset (the block's offset plus a prefix sum of
//     the popcounts of the block's earlier steps) and its matches leave with
//     mbcnt, so every position lands at its rank in row order.  The payload
//     is not read again.
//     A block entirely inside the predicate (all-match, with zone maps) has
//     no ballots: its position range is written without being read.
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

// Pass ballots of a staged block (b = B, `valid` values) for the code window
// [clo, chi): lane t < 16 receives the ballot of step t (bit l: value l + 64 t
// passes), `cnt` (uniform) the number of passing values.
template <uint32_t B>
__device__ __forceinline__ uint64_t block_marks(int64_t clo, int64_t chi, const uint32_t* st, uint32_t valid,
                                                uint32_t lane, uint32_t& cnt) {
  cnt = 0;
  if (clo >= chi) return 0;
  const Extract ex(st, lane, B);
  const uint32_t lo32 = (uint32_t)clo, wm1 = (uint32_t)(chi - clo - 1);
  uint64_t mine = 0;
  if (valid == kBlockValues) {
#pragma unroll
    for (uint32_t t = 0; t < 16u; ++t) {
      const uint64_t m = ballot((ex(t) - lo32) <= wm1);
      mine = lane == t ? m : mine;
      cnt += (uint32_t)__builtin_popcountll(m);
    }
  } else {
#pragma unroll
    for (uint32_t t = 0; t < 16u; ++t) {
      const uint64_t m = ballot(((ex(t) - lo32) <= wm1) && (lane + 64u * t < valid));
      mine = lane == t ? m : mine;
      cnt += (uint32_t)__builtin_popcountll(m);
    }
  }
  return mine;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Group geometry of the mark pass for width B.
template <uint32_t B>
struct MarkGroup {
  static constexpr uint32_t kBlocks = B >= 32u ? 1u : 32u / B;      // G
  static constexpr uint32_t kWords = 32u * B;                       // words per block
  static constexpr uint32_t kPiecesPerBlock = 8u * B;               // 16-byte pieces per block
  static constexpr uint32_t kPieces = kBlocks * kPiecesPerBlock;    // at most 256
};

// Zone maps and reference of one group's blocks: lane j < G holds block
// k0 + j's (loads issued by `issue`, consumed later by `classify` and the
// decode).
struct GroupInfo {
  uint32_t zmn, zmx, ref;
  __device__ __forceinline__ void issue(const SelParams& p, uint64_t k0, uint32_t G, uint32_t lane) {
    const uint64_t k = k0 + lane;
    const bool in = lane < G && k < p.nb;
    zmn = in && p.use_zm ? p.zmin[k] : 0u;
    zmx = in && p.use_zm ? p.zmax[k] : 0u;
    ref = in && p.refs ? p.refs[k] : 0u;
  }
  // 0: skip, 1: decode, 2: all-match (lanes past the group or the column: 0)
  __device__ __forceinline__ uint32_t classify(const SelParams& p, const ZRange& zr, uint64_t k0, uint32_t G,
                                               uint32_t lane) const {
    if (!(lane < G && k0 + lane < p.nb) || zr.lo >= zr.hi) return 0u;
    if (!p.use_zm) return 1u;
    if ((int64_t)zmx < zr.lo || (int64_t)zmn >= zr.hi) return 0u;
    if (p.use_am && (int64_t)zmn >= zr.lo && (int64_t)zmx < zr.hi) return 2u;
    return 1u;
  }
};

// A group's words in registers: lane takes 16-byte pieces lane + 64 q, only
// those of blocks whose bit is set in `need` (pieces of other blocks are
// neither loaded nor staged).  A native vector type, so that the copies stay
// register moves (HIP's uint4 is a struct copied by memcpy).
template <uint32_t B>
struct GroupRegs {
  using Geo = MarkGroup<B>;
  u32x4 r0, r1, r2, r3;
  __device__ __forceinline__ static bool has(uint32_t need, uint32_t q) {
    return q < Geo::kPieces && ((need >> (q / Geo::kPiecesPerBlock)) & 1u);
  }
  __device__ __forceinline__ void load(const SelParams& p, uint64_t k0, uint32_t need, uint32_t lane) {
    // adjacent lanes read adjacent 16 bytes: whole lines, streamed (non-temporal)
    const u32x4* src = reinterpret_cast<const u32x4*>(p.payload + k0 * Geo::kWords);
    if (has(need, lane)) r0 = __builtin_nontemporal_load(src + lane);
    if (Geo::kPieces > 64u && has(need, lane + 64u)) r1 = __builtin_nontemporal_load(src + lane + 64u);
    if (Geo::kPieces > 128u && has(need, lane + 128u)) r2 = __builtin_nontemporal_load(src + lane + 128u);
    if (Geo::kPieces > 192u && has(need, lane + 192u)) r3 = __builtin_nontemporal_load(src + lane + 192u);
  }
  __device__ __forceinline__ void store(uint32_t* st, uint32_t need, uint32_t lane) const {
    u32x4* dst = reinterpret_cast<u32x4*>(st);
    __builtin_amdgcn_wave_barrier();
    if (has(need, lane)) dst[lane] = r0;
    if (Geo::kPieces > 64u && has(need, lane + 64u)) dst[lane + 64u] = r1;
    if (Geo::kPieces > 128u && has(need, lane + 128u)) dst[lane + 128u] = r2;
    if (Geo::kPieces > 192u && has(need, lane + 192u)) dst[lane + 192u] = r3;
    st[Geo::kBlocks * Geo::kWords] = 0u;  // the funnel's spill word; every lane writes the same value
    __builtin_amdgcn_wave_barrier();
  }
};

}  // namespace

template <uint32_t B>
__global__ __launch_bounds__(256) void select_mark_kernel(const SelParams p) {
  using Geo = MarkGroup<B>;
  constexpr uint32_t G = Geo::kBlocks;
  __shared__ __align__(16) uint32_t lds[kSelWaves][kRtStageWords];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* st = lds[wave];
  const ZRange zr = load_range(p);
  const uint64_t ng = (p.nb + G - 1) / G;
  const uint64_t tw = (uint64_t)gridDim.x * kSelWaves;
  const int64_t top = int64_t(1) << B;
  uint64_t g = (uint64_t)blockIdx.x * kSelWaves + wave;
  if (g >= ng) return;
  GroupRegs<B> regs;
  GroupInfo cur, nxt;
  cur.issue(p, g * G, G, lane);
  uint32_t cls = cur.classify(p, zr, g * G, G, lane);
  uint32_t need = (uint32_t)ballot(cls == 1u);
  if (need) regs.load(p, g * G, need, lane);
  nxt.issue(p, (g + tw) * G, G, lane);
  // Vector loads retire in order: a group's words are issued before the zone
  // maps of the group after it, and whatever a group's decode needs was loaded
  // an iteration earlier, so the waits below are for loads long in flight.
  for (; g < ng; g += tw) {
    regs.store(st, need, lane);
    const uint64_t k0 = g * G;
    const uint32_t cls_c = cls, need_c = need, ref_c = cur.ref;
    const uint64_t gn = g + tw;
    cls = nxt.classify(p, zr, gn * G, G, lane);
    need = (uint32_t)ballot(cls == 1u);
    if (need) regs.load(p, gn * G, need, lane);  // in flight while this group decodes
    cur = nxt;
    nxt.issue(p, (gn + tw) * G, G, lane);
    uint32_t cnt_v = 0;
#pragma unroll 1
    for (uint32_t j = 0; j < G; ++j) {
      const uint64_t k = k0 + j;
      if (k >= p.nb) break;
      const uint32_t c = __builtin_amdgcn_readlane(cls_c, j);
      const uint32_t valid = k == p.nb - 1 ? (uint32_t)(p.n - k * kBlockValues) : kBlockValues;
      uint32_t cnt = c == 2u ? valid : 0u;
      if ((need_c >> j) & 1u) {
        int64_t clo = zr.lo, chi = zr.hi;
        if (p.enc != ENC_DICT) {
          const int64_t ref = (int64_t)__builtin_amdgcn_readlane(ref_c, j);
          clo = clo - ref > 0 ? clo - ref : 0;
          chi = chi - ref < top ? chi - ref : top;
        }
        const uint64_t mine = block_marks<B>(clo, chi, st + j * Geo::kWords, valid, lane, cnt);
        if (lane < 16u) p.marks[k * 16u + lane] = mine;
      }
      cnt_v = lane == j ? cnt : cnt_v;
    }
    if (lane < G && k0 + lane < p.nb) p.counts[k0 + lane] = cnt_v;
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
