// Fused decode + predicate + aggregate kernels (gfx950, wave64).
//
// One launch scans one column.  The grid is persistent (sized to the resident
// capacity of the device) and every wavefront owns one contiguous range of
// 1024-value blocks, so the static split is balanced to one block.  A
// wavefront walks its range in windows of 64 blocks: one ballot over the
// window's zone maps gives the survivors (all blocks with zone maps off),
// which are compacted into a per-wavefront LDS list (mbcnt positions).
//
// Survivors are decoded in steps of about 4 KiB of payload per wavefront, and
// the next step's words are loaded into registers while the current step is
// decoded (software pipelining), so every wavefront keeps a load in flight:
//  * RM-direct / lane-interleaved: two blocks per wavefront pass, one per
//    half-wavefront; lane l holds 32 codes in B registers and extracts them
//    with compile-time shifts;
//  * RM-LDS: the wavefront stages whole blocks in LDS with coalesced loads and
//    lane l extracts values j = l + 64 t with a funnel shift;
//  * byte-aligned (B = 8, 16, 32): plain u8/u16/u32 vector loads.
// The decoders whose loads read whole cache lines across the wavefront
// (lane-interleaved, the RM-LDS staging, byte-aligned) load non-temporally.
// Per value: extract, one unsigned compare in code space
// ((c - lo_c) <= w - 1; just c <= w - 1 when lo_c = 0), ballot of the compare
// (the compare's lane mask), scalar popcount for COUNT, and the selected value
// added under the mask (branch-free) or compacted into an LDS selection-vector
// ring that is drained 64 entries at a time (compaction).
// The partial last block of a column is excluded from the pipelined loop and
// decoded once, with a per-value validity test, by the wavefront that owns it.
#pragma once

#include <type_traits>

#include "device_common.h"

namespace scan_dev {

// Predicate forms of the FOR/DICT kernels.
enum PredForm {
  PF_REFS = 0,   // FOR with per-block references: code range per block
  PF_RANGE = 1,  // one code range for the whole column: (c - lo) <= w - 1
  PF_LO0 = 2     // one code range starting at 0: c <= w - 1
};

template <int B>
struct Geo {
  // block pairs per step (half-wavefront decoders).  Branch-free: about
  // 8 KiB per wavefront below b = 16 (32/b pairs, at most 8), one pair at
  // b = 16-23, two from b = 24 (12-16 KiB); with the one or two wavefronts per
  // SIMD the autotuner picks, these deeper steps measured faster (b = 12:
  // 18 %).  Compaction keeps about 4 KiB (its ring and masks need the
  // registers; deeper steps spill).
  static constexpr int kPairs = B >= 24 ? 2 : B >= 16 ? 1 : (32 / B > 8 ? 8 : 32 / B);
  // the alternative step depth the autotuner may pick instead (branch-free
  // frame-of-reference, register decoders): half as deep below b = 16, one
  // pair deeper at b = 16-23, one pair from b = 24 on.  Branch-free dictionary
  // scans (row-major direct) swap the two below b = 16: the shallower step is
  // their default (its LDS gathers measured 1-2 us faster at b = 4 and 8,
  // 10 % at b = 12) and kPairs their alternative.
  static constexpr int kPairsAlt = B >= 24 ? 1 : B >= 16 ? kPairs + 1 : (kPairs / 2 > 1 ? kPairs / 2 : 1);
  static constexpr int kPairsSV = B >= 16 ? 1 : (16 / B > 4 ? 4 : 16 / B);
  // the delta decoders (prefix scan per pair) keep one pair per step from b = 16
  static constexpr int kDeltaPairs = B >= 16 ? 1 : (16 / B > 4 ? 4 : 16 / B);
  // blocks staged per step (RM-LDS), at most 8
  static constexpr int kLdsBlocks = B >= 32 ? 1 : (32 / B > 8 ? 8 : 32 / B);
  static constexpr int kStageWords = 32 * B + 4;            // one staged block plus an over-read pad
  static constexpr int kStageLoads = (32 * B + 63) / 64;    // words per lane to stage one block
  static constexpr int kByteBlocks = B >= 32 ? 1 : 32 / B;  // blocks per step (byte-aligned, B = 8/16/32)
};

// Empty register constraint: pins `x` to VGPRs at this point so the compiler
// cannot defer and re-associate the per-value adds (which would keep every
// value's compare mask alive and spill them).  Emits no instruction; applied
// every fourth value, so the scheduler still interleaves four values.
template <typename T>
__device__ __forceinline__ void pin(T& x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "one VGPR or an aligned VGPR pair");
  asm volatile("" : "+v"(x));
}

// ------------------------------------------------------------------ loads

template <int B>
__device__ __forceinline__ void load_slice(const uint32_t* __restrict__ src, uint32_t (&w)[B]) {
  if constexpr (B % 4 == 0) {
#pragma unroll
    for (int i = 0; i < B / 4; ++i) {
      uint4 v = reinterpret_cast<const uint4*>(src)[i];
      w[4 * i] = v.x;
      w[4 * i + 1] = v.y;
      w[4 * i + 2] = v.z;
      w[4 * i + 3] = v.w;
    }
  } else if constexpr (B % 2 == 0) {
#pragma unroll
    for (int i = 0; i < B / 2; ++i) {
      uint2 v = reinterpret_cast<const uint2*>(src)[i];
      w[2 * i] = v.x;
      w[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < B; ++i) w[i] = src[i];
  }
}

// Code t of a run of codes held in registers: bits [t*B, t*B + B).  Every
// shift is a compile-time constant (one v_bfe_u32, or alignbit + and).
template <int B, int N>
__device__ __forceinline__ uint32_t run_code(const uint32_t (&y)[N], int t) {
  const int bit = t * B;
  const int wi = bit >> 5, sh = bit & 31;
  if (B == 32) return y[t];
  if (sh + B <= 32) return (y[wi] >> sh) & width_mask<B>();
  return funnel(y[wi + 1], y[wi], sh) & width_mask<B>();
}

// ------------------------------------------------------ per-wave state

template <typename EntryT>
struct WaveState {
  uint64_t count = 0;   // uniform
  uint64_t blocks = 0;  // uniform
  uint64_t refsum = 0;  // uniform: sum over blocks of (matches in block) * (reference or base)
  uint64_t lsum = 0;    // per lane
  uint64_t lcount = 0;  // per lane (branch-free mode counts per lane, no ballot)
  uint32_t head = 0, tail = 0;  // selection-vector ring counters (uniform)
  EntryT* ring = nullptr;
  // branch-free dictionary scans: the LDS dictionary holds packed entries
  // (see stage_dictionary) relative to dict_base (uniform)
  bool dict_packed = false;
  uint64_t dict_base = 0;
  // packed dictionaries of b <= kDictPairMaxB: a table of code pairs staged
  // beside the entries (see stage_dictionary_pairs)
  bool dict_pairs = false;
};

// Value of a selected code: FOR adds the code (references are added through
// counts); DICT adds the dictionary entry staged in LDS (index clamped).
template <int ENC>
__device__ __forceinline__ uint64_t code_value(uint32_t c, const int64_t* dict_lds, uint32_t dict_last) {
  if constexpr (ENC == ENC_DICT) return (uint64_t)dict_lds[c < dict_last ? c : dict_last];
  else return (uint64_t)c;
}

// Packed dictionary for branch-free scans: an entry inside the code window
// [clo, chi) becomes (entry - base) + 2^58 with base the window's first
// entry, every other slot 0.  One 64-bit add per code then accumulates both
// results: over one block (at most 32 codes per lane) the high six bits hold
// the matches and the low 58 bits the sum of (entry - base), which cannot
// carry into them while the window's range (last - first entry) is below
// 2^53.  SUM = that sum + base x COUNT (mod 2^64).  A window of larger range
// is only masked: its entries as they are, every other slot 0.
constexpr int kDictCountShift = 58;
constexpr uint64_t kDictSumMask = (1ull << kDictCountShift) - 1ull;
constexpr uint64_t kDictMaxRange = 1ull << 53;

// Smallest and largest of a value over the wavefront.
__device__ __forceinline__ void wave_min_max_i64(int64_t& mn, int64_t& mx) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t a = (uint64_t)mn, b = (uint64_t)mx;
    const int64_t pa = (int64_t)(((uint64_t)__shfl_xor((uint32_t)(a >> 32), o, 64) << 32) | __shfl_xor((uint32_t)a, o, 64));
    const int64_t pb = (int64_t)(((uint64_t)__shfl_xor((uint32_t)(b >> 32), o, 64) << 32) | __shfl_xor((uint32_t)b, o, 64));
    mn = pa < mn ? pa : mn;
    mx = pb > mx ? pb : mx;
  }
}

// Stage a dictionary in LDS, in the form the scan reads (packed when PACK and
// the window qualifies, else masked, up to and including the zero slot), for
// the code window [clo, chi) of the predicate [lo, hi).  The entries are
// sorted and distinct, so clo and chi are the numbers of entries below lo and
// below hi, and the window's first and last entries are the smallest and
// largest entries inside [lo, hi): all four come out of one reduction over the
// entries as they arrive (a thread's loads in flight together), with no
// binary search.  Each thread stores its entries as they are and rewrites the
// same slots after the reduction, so there are two barriers.  Slots from len
// up to `reach` (the codes' range, at most kMaxDict) and the zero slot are 0.
// `red`: the work-group reduction area (16 x 3 words of 64 bits).  Every
// thread of the work-group must call it.
template <bool PACK>
__device__ __forceinline__ void stage_dictionary(const int64_t* __restrict__ src, uint32_t len, uint32_t reach,
                                                 int64_t lo, int64_t hi, int64_t* dict_lds, uint64_t (*red)[3],
                                                 uint32_t& clo, uint32_t& chi, bool& packed, uint64_t& base) {
  constexpr uint32_t kPer = 16;  // a 4096-entry dictionary in one round at 256 threads
  const uint32_t bd = blockDim.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nw = bd >> 6;
  const uint32_t span = bd * kPer;
  // entries below lo (bits 0-15) and below hi (bits 16-31): at most kMaxDict each
  uint32_t n = 0;
  int64_t mn = INT64_MAX, mx = INT64_MIN;
  // Rounds of kPer entries per thread (slots c0 + tid + j*bd), every load of
  // a round in flight together; each entry is tallied and stored in its slot
  // as it is, to be rewritten after the reduction by the same thread.
  for (uint32_t c0 = 0; c0 < len; c0 += span) {
    const uint32_t rem = len - c0;
    const uint32_t nv0 = tid < rem ? (rem - tid - 1u) / bd + 1u : 0u;
    const uint32_t nv = nv0 < kPer ? nv0 : kPer;  // this thread's real entries of the round
    int64_t x[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) x[j] = j < nv ? src[c0 + tid + j * bd] : 0;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      if (j < nv) {
        const int64_t v = x[j];
        n += (v < lo ? 1u : 0u) + (v < hi ? 0x10000u : 0u);
        const bool in = v >= lo && v < hi;
        mn = in && v < mn ? v : mn;
        mx = in && v > mx ? v : mx;
        dict_lds[c0 + tid + j * bd] = v;
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o, 64);
  wave_min_max_i64(mn, mx);
  if (lane == 0) {
    red[wave][0] = n;
    red[wave][1] = (uint64_t)mn;
    red[wave][2] = (uint64_t)mx;
  }
  __syncthreads();
  uint32_t tot = 0;
  // work-groups of at most 256 threads: four wavefronts
#pragma unroll
  for (uint32_t w = 0; w < 4u; ++w) {
    if (w >= nw) break;
    tot += (uint32_t)red[w][0];
    const int64_t a = (int64_t)red[w][1], b = (int64_t)red[w][2];
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  clo = tot & 0xFFFFu;
  chi = tot >> 16;
  base = clo < chi ? (uint64_t)mn : 0ull;
  packed = PACK && (clo >= chi || (uint64_t)mx - base < kDictMaxRange);
  // Every slot below top in the form the scan reads: an entry inside
  // [lo, hi) is inside the code window (sorted, distinct entries).
  const uint32_t top = len > reach ? len : reach;
  for (uint32_t c0 = 0; c0 < top; c0 += span) {
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint32_t i = c0 + tid + j * bd;
      if (i < top) {
        const int64_t v = i < len ? dict_lds[i] : 0;
        int64_t o = 0;
        if (i < len && v >= lo && v < hi)
          o = packed ? (int64_t)(((uint64_t)v - base) | (1ull << kDictCountShift)) : v;
        dict_lds[i] = o;
      }
    }
  }
  if (tid == 0) dict_lds[kDictZeroSlot] = 0;
  __syncthreads();
}

typedef __attribute__((address_space(3))) const int64_t LdsI64;
__device__ __forceinline__ uint64_t dict_at(uint32_t idx) {
  return (uint64_t)*reinterpret_cast<LdsI64*>((uintptr_t)(idx * 8u));
}

// Code pairs of a packed dictionary of b <= kDictPairMaxB: slot
// kDictPairBase + (c0 | c1 << b) holds entry c0 + entry c1 (both packed, so
// the match counts add too; 16 pairs per lane and block keep the count field
// at most 32), so one gather serves two codes.  The table sits between the
// entries (at most 2^b <= kDictPairBase slots) and the zero slot.
constexpr int kDictPairMaxB = 5;
constexpr uint32_t kDictPairBase = 64;
static_assert(kDictPairBase + (1u << (2 * kDictPairMaxB)) <= kDictZeroSlot, "pair table overlaps the zero slot");

// Build the pair table from the staged (packed) entries; every thread of the
// work-group calls it after stage_dictionary.  Ends with a barrier.
template <int B>
__device__ __forceinline__ void stage_dictionary_pairs(int64_t* dict_lds) {
  constexpr uint32_t kMask = (1u << B) - 1u;
  for (uint32_t q = threadIdx.x; q < (1u << (2 * B)); q += blockDim.x)
    dict_lds[kDictPairBase + q] = (int64_t)((uint64_t)dict_lds[q & kMask] + (uint64_t)dict_lds[q >> B]);
  __syncthreads();
}

// Index of a code's entry in the masked LDS dictionary: codes of b <= 12 bits
// stay inside the area; wider codes at or past the zero slot read it.
template <int B>
__device__ __forceinline__ uint32_t dict_index(uint32_t c) {
  if constexpr (B > 12) return c < kDictZeroSlot ? c : kDictZeroSlot;
  else return c;
}


// Selection-vector push: compact the selected lanes' entries into the ring at
// mbcnt positions; when 64 or more are pending, every lane consumes one.
template <int ENC, typename EntryT>
__device__ __forceinline__ void sv_push(WaveState<EntryT>& s, EntryT e, bool pass, uint64_t m, uint32_t lane,
                                        const int64_t* dict_lds, uint32_t dict_last) {
  if (m) {
    const uint32_t pos = mbcnt(m);
    if (pass) s.ring[(s.head + pos) & (kRingEntries - 1)] = e;
    s.head += (uint32_t)__builtin_popcountll(m);
    if (s.head - s.tail >= 64u) {
      __builtin_amdgcn_wave_barrier();
      const EntryT x = s.ring[(s.tail + lane) & (kRingEntries - 1)];
      if constexpr (ENC == ENC_DICT) s.lsum += code_value<ENC>((uint32_t)x, dict_lds, dict_last);
      else s.lsum += (uint64_t)x;
      s.tail += 64u;
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <int ENC, typename EntryT>
__device__ __forceinline__ void sv_drain_rest(WaveState<EntryT>& s, uint32_t lane, const int64_t* dict_lds,
                                              uint32_t dict_last) {
  const uint32_t rem = s.head - s.tail;
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) {
    const EntryT x = s.ring[(s.tail + lane) & (kRingEntries - 1)];
    if constexpr (ENC == ENC_DICT) s.lsum += code_value<ENC>((uint32_t)x, dict_lds, dict_last);
    else s.lsum += (uint64_t)x;
  }
  s.tail = s.head;
}

// Per-lane partial sum of one decode pass: u32 is exact for FOR codes of
// B <= 26 bits (a lane adds at most 64 of them before folding).
template <int B, int ENC>
using PartT = typename std::conditional<(ENC == ENC_FOR && B <= 26), uint32_t, uint64_t>::type;

// Code-space predicate of one block.
struct CodeRange {
  uint32_t loc, wm1;
  bool nonempty;
};

template <int B, int ENC, int PF>
__device__ __forceinline__ CodeRange block_range(const Params& p, uint32_t ref, uint32_t clo, uint32_t chi) {
  CodeRange r;
  if constexpr (ENC == ENC_DICT) {
    r.nonempty = clo < chi;
    r.loc = clo;
    r.wm1 = chi - clo - 1u;
  } else {
    r.nonempty = for_code_range<B>(PF == PF_REFS ? ref : 0u, p.lo32, p.hi32m1, r.loc, r.wm1);
  }
  return r;
}

// ------------------------------------------------------ block windows

// Survivors among blocks k0 .. k0+cnt-1 (cnt <= 64) of a FOR/DICT column,
// without block `excl` (the partial last block, decoded separately).  With
// the all-match shortcut, a surviving block whose [min, max] lies inside the
// predicate is not returned: the lane testing it adds the block's 1024 values
// to am_count and its stored sum to am_sum (per-lane accumulators).
template <int ENC>
__device__ __forceinline__ uint64_t window_live(const Params& p, uint64_t k0, uint32_t cnt, uint32_t clo, uint32_t chi,
                                                uint64_t excl, uint64_t& am_count, uint64_t& am_sum) {
  const uint32_t lane = lane_id();
  bool keep = lane < cnt && (k0 + lane) != excl;
  if (p.use_zm && keep) {
    const uint32_t mn = static_cast<const uint32_t*>(p.zmin)[k0 + lane];
    const uint32_t mx = static_cast<const uint32_t*>(p.zmax)[k0 + lane];
    bool inside;
    if constexpr (ENC == ENC_DICT) {
      keep = !(mx < clo || mn >= chi);
      inside = mn >= clo && mx < chi;
    } else {
      keep = !(mx < p.lo32 || mn > p.hi32m1);
      inside = mn >= p.lo32 && mx <= p.hi32m1;
    }
    if (p.use_am && keep && inside) {
      am_count += kBlockValues;
      am_sum += p.bsum[k0 + lane];
      keep = false;
    }
  }
  return ballot(keep);
}

__device__ __forceinline__ uint64_t window_live_i64(const Params& p, uint64_t k0, uint32_t cnt, uint64_t excl,
                                                    uint64_t& am_count, uint64_t& am_sum) {
  const uint32_t lane = lane_id();
  bool keep = lane < cnt && (k0 + lane) != excl;
  if (p.use_zm && keep) {
    const int64_t mn = static_cast<const int64_t*>(p.zmin)[k0 + lane];
    const int64_t mx = static_cast<const int64_t*>(p.zmax)[k0 + lane];
    keep = !(mx < p.lo || mn >= p.hi);
    if (p.use_am && keep && mn >= p.lo && mx < p.hi) {
      am_count += kBlockValues;
      am_sum += p.bsum[k0 + lane];
      keep = false;
    }
  }
  return ballot(keep);
}

// Zone-map test of one block (uniform), for the separately decoded last block.
template <int ENC>
__device__ __forceinline__ bool block_survives(const Params& p, uint64_t k, uint32_t clo, uint32_t chi) {
  if (!p.use_zm) return true;
  if constexpr (ENC == ENC_DELTA) {
    const int64_t mn = static_cast<const int64_t*>(p.zmin)[k], mx = static_cast<const int64_t*>(p.zmax)[k];
    return !(mx < p.lo || mn >= p.hi);
  } else {
    const uint32_t mn = static_cast<const uint32_t*>(p.zmin)[k], mx = static_cast<const uint32_t*>(p.zmax)[k];
    if constexpr (ENC == ENC_DICT) return !(mx < clo || mn >= chi);
    else return !(mx < p.lo32 || mn > p.hi32m1);
  }
}

// Whether a surviving block lies entirely inside the predicate (uniform; only
// with the all-match shortcut).
template <int ENC>
__device__ __forceinline__ bool block_inside(const Params& p, uint64_t k, uint32_t clo, uint32_t chi) {
  if (!p.use_am) return false;
  if constexpr (ENC == ENC_DELTA) {
    const int64_t mn = static_cast<const int64_t*>(p.zmin)[k], mx = static_cast<const int64_t*>(p.zmax)[k];
    return mn >= p.lo && mx < p.hi;
  } else {
    const uint32_t mn = static_cast<const uint32_t*>(p.zmin)[k], mx = static_cast<const uint32_t*>(p.zmax)[k];
    if constexpr (ENC == ENC_DICT) return mn >= clo && mx < chi;
    else return mn >= p.lo32 && mx <= p.hi32m1;
  }
}

// Whether block k lies in one of the windows [a + j*stride, a + j*stride + win)
// that end before e.
__device__ __forceinline__ bool owns_block(uint64_t k, uint64_t a, uint64_t e, uint64_t stride, uint32_t win) {
  return k >= a && k < e && ((k - a) % stride) < win;
}

// Walks the wavefront's windows (win blocks each, `stride` blocks apart, up to
// end_k) and hands out the surviving blocks in steps of up to NPER per
// half-wavefront (lanes 0-31 take list entries pos, pos+2, ...; lanes 32-63
// take pos+1, pos+3, ...).
template <int NPER, typename LiveFn>
struct PairCursor {
  uint64_t next_k, end_k, k0;
  uint32_t nsurv, pos;
  uint32_t* list;   // per-wavefront LDS, 64 entries
  uint64_t safe;    // a block this lane was last handed (valid once a fetch succeeded)
  uint64_t stride;  // distance between this wavefront's windows
  uint32_t win;     // blocks per window (1..64)

  __device__ __forceinline__ bool fetch(uint64_t (&kb)[NPER], uint32_t& actbits, uint64_t& blocks, LiveFn& live_fn,
                                        uint32_t lane) {
    while (pos >= nsurv) {
      if (next_k >= end_k) {
        // Exhausted: hand out the last valid block again so the caller's
        // unconditional prefetch stays in bounds (its result is not decoded).
#pragma unroll
        for (int q = 0; q < NPER; ++q) kb[q] = safe;
        actbits = 0;
        return false;
      }
      const uint64_t left = end_k - next_k;
      const uint32_t cnt = left < win ? (uint32_t)left : win;
      k0 = next_k;
      next_k += stride;
      const uint64_t live = live_fn(k0, cnt);
      blocks += (uint64_t)__builtin_popcountll(live);
      __builtin_amdgcn_wave_barrier();
      if ((live >> lane) & 1ull) list[mbcnt(live)] = lane;
      __builtin_amdgcn_wave_barrier();
      nsurv = (uint32_t)__builtin_popcountll(live);
      pos = 0;
    }
    const uint32_t h = lane >> 5;
    actbits = 0;
#pragma unroll
    for (int q = 0; q < NPER; ++q) {
      const uint32_t idx = pos + 2u * q + h;
      const bool a = idx < nsurv;
      kb[q] = k0 + list[a ? idx : pos];
      actbits |= (a ? 1u : 0u) << q;
    }
    pos += 2u * NPER;
    safe = kb[0];
    return true;
  }
};

// Same walk for decoders that take one block per wavefront pass: a step is a
// uniform mask of up to NB window bits.
template <int NB, typename LiveFn>
struct BlockCursor {
  uint64_t next_k, end_k, k0, live;
  uint64_t stride;  // distance between this wavefront's windows
  uint32_t win;     // blocks per window (1..64)

  __device__ __forceinline__ bool fetch(uint64_t& sk0, uint64_t& smask, uint64_t& blocks, LiveFn& live_fn) {
    while (live == 0) {
      if (next_k >= end_k) return false;
      const uint64_t left = end_k - next_k;
      const uint32_t cnt = left < win ? (uint32_t)left : win;
      k0 = next_k;
      next_k += stride;
      live = live_fn(k0, cnt);
      blocks += (uint64_t)__builtin_popcountll(live);
    }
    uint64_t m = 0, l = live;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const uint64_t bit = l & (~l + 1ull);
      m |= bit;
      l ^= bit;
    }
    live = l;
    sk0 = k0;
    smask = m;
    return true;
  }
};

// Branch-free COUNT and SUM of the 32 codes a lane holds, for B <= 15 (frame
// of reference, full blocks): SIMD within a register.  The codes are spread
// into fields with spare bits above each code (B = 2, 4, 8: fields of 2B
// bits, odd and even codes apart; B = 3: eight consecutive codes into the
// eight nibbles of a register; B = 5, 6, 7: four consecutive codes shifted
// into the four bytes of a register; B = 9-15: two consecutive codes into the
// two halves), so one subtraction tests all fields of a register
// against the code window with no borrow between fields, and the top bit of
// each field is its pass flag.  v_bcnt counts the flags; an unsigned dot
// product of the fields with the 0/1 flags (dot8 of nibbles, dot4 of bytes,
// dot2 of halves) adds the passing codes.  B = 1 needs only a popcount per
// word.  Code c passes iff (c - loc) <= wm1 (PF_LO0: loc = 0).
template <int B, int PF>
__device__ __forceinline__ void swar_count_sum(const uint32_t (&w)[B], uint32_t loc, uint32_t wm1, uint32_t& lc,
                                               uint32_t& part) {
  if constexpr (B == 1) {
    const uint32_t pc = (uint32_t)__builtin_popcount(w[0]);
    const bool p0 = loc == 0u;                         // code 0 in the window
    const bool p1 = loc <= 1u && loc + wm1 >= 1u;      // code 1 in the window
    lc += (p0 ? 32u - pc : 0u) + (p1 ? pc : 0u);
    part += p1 ? pc : 0u;
  } else if constexpr (B == 3) {
    // eight codes (24 stream bits) into the eight nibbles of a register, bit 3
    // of each the spare: 12 + 12 bits to the two halves, 6 + 6 to the bytes
    // of each half, 3 + 3 to the nibbles of each byte
    constexpr uint32_t hm = 0x88888888u;
    const uint32_t locr = loc * 0x11111111u;
    const uint32_t wr = (0x8u + wm1) * 0x11111111u;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int bit = 24 * g, wi = bit >> 5, sh = bit & 31;
      const int wn = wi + 1 < B ? wi + 1 : wi;  // only read when the group straddles a word
      const uint32_t chunk = sh + 24 <= 32 ? (w[wi] >> sh) : funnel(w[wn], w[wi], sh);
      uint32_t x = (chunk & 0xFFFu) | ((chunk & 0xFFF000u) << 4);
      x = (x & 0x003F003Fu) | ((x & 0x0FC00FC0u) << 2);
      x = (x & 0x07070707u) | ((x & 0x38383838u) << 1);
      const uint32_t g4 = PF == PF_LO0 ? x : (((x | hm) - locr) & ~hm);
      const uint32_t flags = (wr - g4) & hm;
      lc += (uint32_t)__builtin_popcount(flags);
      part = __builtin_amdgcn_udot8(x, flags >> 3, part, false);
    }
  } else if constexpr (B == 5 || B == 6 || B == 7) {
    constexpr uint32_t m0 = (1u << B) - 1u;
    constexpr uint32_t hm = 0x80808080u;
    const uint32_t locr = loc * 0x01010101u;
    const uint32_t wr = (0x80u + wm1) * 0x01010101u;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      // codes 4g .. 4g+3: stream bits [4Bg, 4Bg + 4B)
      const int bit = 4 * B * g, wi = bit >> 5, sh = bit & 31;
      const int wn = wi + 1 < B ? wi + 1 : wi;  // only read when the group straddles a word
      const uint32_t chunk = sh + 4 * B <= 32 ? (w[wi] >> sh) : funnel(w[wn], w[wi], sh);
      uint32_t x = chunk & m0;
      x |= (chunk << (8 - B)) & (m0 << 8);
      x |= (chunk << (16 - 2 * B)) & (m0 << 16);
      x |= (chunk << (24 - 3 * B)) & (m0 << 24);
      const uint32_t g8 = PF == PF_LO0 ? x : (((x | hm) - locr) & ~hm);
      const uint32_t flags = (wr - g8) & hm;
      lc += (uint32_t)__builtin_popcount(flags);
      part = __builtin_amdgcn_udot4(x, flags >> 7, part, false);
    }
  } else if constexpr (B >= 9 && B <= 15) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    constexpr uint32_t m0 = (1u << B) - 1u;
    constexpr uint32_t hm = 0x80008000u;
    const uint32_t locr = loc * 0x00010001u;
    const uint32_t wr = (0x8000u + wm1) * 0x00010001u;
#pragma unroll
    for (int g = 0; g < 16; ++g) {
      // codes 2g, 2g+1: stream bits [2Bg, 2Bg + 2B), into the two halves
      const int bit = 2 * B * g, wi = bit >> 5, sh = bit & 31;
      const int wn = wi + 1 < B ? wi + 1 : wi;  // only read when the pair straddles a word
      const uint32_t chunk = sh + 2 * B <= 32 ? (w[wi] >> sh) : funnel(w[wn], w[wi], sh);
      const uint32_t x = (chunk & m0) | ((chunk << (16 - B)) & (m0 << 16));
      const uint32_t g16 = PF == PF_LO0 ? x : (((x | hm) - locr) & ~hm);
      const uint32_t flags = (wr - g16) & hm;
      lc += (uint32_t)__builtin_popcount(flags);
      part = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, x), __builtin_bit_cast(u16x2, flags >> 15), part,
                                    false);
    }
  } else {
    constexpr int F = 2 * B;
    constexpr uint32_t rep = F == 4 ? 0x11111111u : F == 8 ? 0x01010101u : 0x00010001u;
    constexpr uint32_t vmask = ((1u << B) - 1u) * rep;  // the code bits of every field
    constexpr uint32_t hm = (1u << (F - 1)) * rep;      // the flag bit of every field
    const uint32_t locr = loc * rep;
    const uint32_t wr = ((1u << (F - 1)) + wm1) * rep;
#pragma unroll
    for (int i = 0; i < B; ++i) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t x = (k ? (w[i] >> B) : w[i]) & vmask;
        // field: c - loc when c >= loc; when c < loc the field value exceeds
        // any wm1 (its flag bit is clear and the rest is >= 2^(F-1) - loc)
        const uint32_t g = PF == PF_LO0 ? x : (((x | hm) - locr) & ~hm);
        const uint32_t flags = (wr - g) & hm;  // flag set iff field <= wm1
        lc += (uint32_t)__builtin_popcount(flags);
        const uint32_t f01 = flags >> (F - 1);
        if constexpr (F == 4) {
          part = __builtin_amdgcn_udot8(x, f01, part, false);
        } else if constexpr (F == 8) {
          part = __builtin_amdgcn_udot4(x, f01, part, false);
        } else {
          typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
          part = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, x), __builtin_bit_cast(u16x2, f01), part, false);
        }
      }
    }
  }
}

// -------------------------------------------- half-wavefront pair decoding

// Decode the 32 codes each lane holds for one block (lanes 0-31: one block,
// lanes 32-63: another).  `act`: this lane's block is real and may match.
// `ref`: the block's reference (PF_REFS; loaded with its words, a step ahead).
template <int B, int DEC, int MODE, int ENC, int PF, bool TAIL>
__device__ __forceinline__ void decode_pair(const Params& p, WaveState<uint32_t>& s, uint32_t lane,
                                            const uint32_t (&w)[B], uint64_t kb, bool act, uint32_t ref,
                                            const int64_t* dict_lds, uint32_t dict_last, uint32_t clo, uint32_t chi) {
  const uint32_t l = lane & 31u;
  const CodeRange cr = block_range<B, ENC, PF>(p, ref, clo, chi);
  act = act && cr.nonempty;
  const uint64_t act_m = ballot(act);
  if (act_m == 0) return;
  const uint32_t limit = (TAIL && kb == p.nb - 1) ? p.tail : kBlockValues;
  PartT<B, ENC> part = 0;
  if constexpr (MODE == MODE_BF && ENC == ENC_FOR && !TAIL && B <= 15) {
    uint32_t lc = 0, sp = 0;
    swar_count_sum<B, PF>(w, cr.loc, cr.wm1, lc, sp);
    if (act) {
      s.lcount += lc;
      s.lsum += (uint64_t)sp;
      if constexpr (PF == PF_REFS) s.lsum += (uint64_t)lc * ref;
    }
  } else if constexpr (MODE == MODE_BF && ENC == ENC_DICT) {
    // Branch-free dictionary, in three forms: (1) b <= kDictPairMaxB with a
    // pair table on full blocks, one gather per two codes; (2) packed entries,
    // one gather and one 64-bit add per code giving COUNT and SUM; (3) masked
    // entries (windows spanning 2^53 or more): SUM adds every code's entry (no
    // compare, no select; a partial last block's padding slots read the zero
    // slot) and COUNT comes from packed fields for b <= 8 on full blocks, else
    // one compare per code and a scalar popcount of the wavefront's mask; a
    // lane whose block is absent or cannot match compares against an empty
    // window (a dictionary's code window is at most kMaxDict wide, so its
    // width does not overflow).
    if constexpr (!TAIL && B <= kDictPairMaxB) {
      if (s.dict_pairs) {
        // one gather per two consecutive codes (see stage_dictionary_pairs)
#pragma unroll
        for (int g = 0; g < 16; g += 8) {
          uint64_t e[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) e[k] = dict_at(kDictPairBase + run_code<2 * B, B>(w, g + k));
          part += ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
          pin(part);
        }
        if (act) {
          const uint32_t lc = (uint32_t)(part >> kDictCountShift);
          s.lcount += lc;
          s.lsum += (part & kDictSumMask) + s.dict_base * lc;
        }
        return;
      }
    }
    if (s.dict_packed) {
      // packed entries: one 64-bit add per code (see stage_dictionary); the
      // reads go out in groups of eight before their adds
#pragma unroll
      for (int g = 0; g < 32; g += 8) {
        uint64_t e[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int t = g + k;
          const uint32_t c = run_code<B, B>(w, t);
          uint32_t idx = dict_index<B>(c);
          if (TAIL) idx = (((DEC == DEC_RM_DIRECT) ? (32u * l + t) : (32u * t + l)) < limit) ? idx : kDictZeroSlot;
          e[k] = dict_at(idx);
        }
        part += ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
        pin(part);
      }
      if (act) {
        const uint32_t lc = (uint32_t)(part >> kDictCountShift);
        s.lcount += lc;
        s.lsum += (part & kDictSumMask) + s.dict_base * lc;
      }
      return;
    }
    constexpr bool kFields = !TAIL && B <= 8;
    uint32_t lc = 0;   // per lane (packed fields)
    uint32_t cnt = 0;  // uniform (compares)
    if constexpr (kFields) {
      uint32_t unused = 0;
      swar_count_sum<B, PF>(w, cr.loc, cr.wm1, lc, unused);
    }
    uint32_t width = act ? cr.wm1 + 1u : 0u;
    pin(width);  // a per-lane bound: keeps the compiler from splitting it back into act && compare
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const uint32_t c = run_code<B, B>(w, t);
      bool valid = true;
      if (TAIL) valid = (((DEC == DEC_RM_DIRECT) ? (32u * l + t) : (32u * t + l)) < limit);
      if constexpr (!kFields) cnt += (uint32_t)__builtin_popcountll(ballot(valid && (c - cr.loc) < width));
      uint32_t idx = dict_index<B>(c);
      if (TAIL) idx = valid ? idx : kDictZeroSlot;
      part += (uint64_t)dict_lds[idx];
      if ((t & 7) == 7) pin(part);
    }
    s.count += cnt;
    if (act) {
      s.lcount += lc;
      s.lsum += (uint64_t)part;
    }
  } else if constexpr (MODE == MODE_BF) {
    // Branch-free: per-lane count and masked add; the compare's mask stays in
    // VCC and feeds a select and a carry-add (no ballot, no scalar work).
    uint32_t lc = 0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const uint32_t c = run_code<B, B>(w, t);
      bool ok = (PF == PF_LO0) ? (c <= cr.wm1) : ((c - cr.loc) <= cr.wm1);
      if (TAIL) ok = ok && (((DEC == DEC_RM_DIRECT) ? (32u * l + t) : (32u * t + l)) < limit);
      lc += ok ? 1u : 0u;
      const uint64_t v = code_value<ENC>(c, dict_lds, dict_last);
      part += ok ? (PartT<B, ENC>)v : (PartT<B, ENC>)0;
      if ((t & 3) == 3) {
        pin(part);
        pin(lc);
      }
    }
    if (act) {
      s.lcount += lc;
      s.lsum += (uint64_t)part;
      if constexpr (PF == PF_REFS) s.lsum += (uint64_t)lc * ref;
    }
  } else {
    uint32_t cA = 0, cB = 0, call = 0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const uint32_t c = run_code<B, B>(w, t);
      const bool hit = (PF == PF_LO0) ? (c <= cr.wm1) : ((c - cr.loc) <= cr.wm1);
      uint64_t m = ballot(hit) & act_m;
      bool valid = true;
      if (TAIL) {
        const uint32_t j = (DEC == DEC_RM_DIRECT) ? (32u * l + t) : (32u * t + l);
        valid = j < limit;
        m &= ballot(valid);
      }
      if constexpr (PF == PF_REFS) {
        cA += (uint32_t)__builtin_popcount((uint32_t)m);
        cB += (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
      } else {
        call += (uint32_t)__builtin_popcountll(m);
      }
      sv_push<ENC, uint32_t>(s, c, hit && act && valid, m, lane, dict_lds, dict_last);
    }
    if constexpr (PF == PF_REFS) {
      s.count += (uint64_t)cA + cB;
      s.refsum += (uint64_t)cA * readlane(ref, 0) + (uint64_t)cB * readlane(ref, 32);
    } else {
      s.count += call;
    }
  }
}

// Row-major: each lane reads its own contiguous slice, so one load touches a
// part of several cache lines whose rest the lane's next loads read: the
// lines must stay cached (non-temporal loads measured 2.5x slower).  The
// transposed layout reads each line whole in one instruction (32 lanes x 4
// bytes), nothing is re-read, and non-temporal loads stream 5-12 % faster
// from b = 12 on (they do not displace other lines in the caches).
template <int B, int DEC>
__device__ __forceinline__ void load_pair_words(const Params& p, uint64_t kb, uint32_t l, uint32_t (&w)[B]) {
  const uint32_t* __restrict__ blk = p.payload + kb * (32u * B);
  if constexpr (DEC == DEC_RM_DIRECT) {
    load_slice<B>(blk + l * B, w);
  } else {
#pragma unroll
    for (int r = 0; r < B; ++r) w[r] = __builtin_nontemporal_load(blk + 32 * r + l);
  }
}

template <int B, int DEC, int MODE, int ENC, int PF, int P>
__device__ __forceinline__ void run_pairs(const Params& p, WaveState<uint32_t>& s, uint32_t lane, uint32_t* list,
                                          uint64_t ka, uint64_t ke, uint64_t stride, uint32_t win, uint64_t excl,
                                          const int64_t* dict_lds, uint32_t dict_last, uint32_t clo, uint32_t chi) {
  const uint32_t l = lane & 31u;
  auto live_fn = [&](uint64_t k0, uint32_t cnt) {
    return window_live<ENC>(p, k0, cnt, clo, chi, excl, s.lcount, s.lsum);
  };
  PairCursor<P, decltype(live_fn)> cur{ka, ke, 0, 0, 0, list, ka, stride, win};
  // Two register buffers used alternately: the next step's loads are always
  // issued (a harmless reload of a valid block when there is no next step)
  // before the current step is decoded, so exactly one step is in flight.
  uint64_t k0b[P], k1b[P];
  uint32_t a0 = 0, a1 = 0;
  uint32_t w0[P][B], w1[P][B];
  uint32_t r0[P], r1[P];  // block references (PF_REFS), in flight with the words
  auto load = [&](const uint64_t (&kb)[P], uint32_t (&w)[P][B], uint32_t (&r)[P]) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      load_pair_words<B, DEC>(p, kb[q], l, w[q]);
      r[q] = PF == PF_REFS ? p.refs[kb[q]] : 0u;
    }
  };
  auto decode = [&](const uint32_t (&w)[P][B], const uint64_t (&kb)[P], uint32_t ab, const uint32_t (&r)[P]) {
#pragma unroll
    for (int q = 0; q < P; ++q)
      decode_pair<B, DEC, MODE, ENC, PF, false>(p, s, lane, w[q], kb[q], (ab >> q) & 1u, r[q], dict_lds, dict_last,
                                                clo, chi);
  };
  if (!cur.fetch(k0b, a0, s.blocks, live_fn, lane)) return;
  load(k0b, w0, r0);
  while (true) {
    const bool more1 = cur.fetch(k1b, a1, s.blocks, live_fn, lane);
    load(k1b, w1, r1);
    decode(w0, k0b, a0, r0);
    if (!more1) break;
    const bool more0 = cur.fetch(k0b, a0, s.blocks, live_fn, lane);
    load(k0b, w0, r0);
    decode(w1, k1b, a1, r1);
    if (!more0) break;
  }
}

// ---------------------------------------------- wavefront block decoding

// RM-LDS: decode one staged block; lane l takes values j = l + 64 t (t < 16),
// which share the shift (l*B mod 32) and sit 2*B*t words apart.
template <int B, int MODE, int ENC, int PF, bool TAIL>
__device__ __forceinline__ void decode_staged(const Params& p, WaveState<uint32_t>& s, uint32_t lane,
                                              const uint32_t* st, uint64_t k, uint32_t ref, const int64_t* dict_lds,
                                              uint32_t dict_last, uint32_t clo, uint32_t chi) {
  const CodeRange cr = block_range<B, ENC, PF>(p, ref, clo, chi);
  if (!cr.nonempty) return;
  const uint32_t limit = TAIL ? p.tail : kBlockValues;
  const uint32_t bit0 = lane * B;
  const uint32_t* sp = st + (bit0 >> 5);
  const uint32_t sh = bit0 & 31u;
  uint32_t cnt = 0;
  uint32_t ucnt = 0;  // branch-free dictionary: uniform count
  PartT<B, ENC> part = 0;
  if constexpr (MODE == MODE_BF && ENC == ENC_DICT) {
    if (s.dict_packed) {
      // packed entries: one 64-bit add per code (see stage_dictionary); the
      // reads go out in groups of eight before their adds
#pragma unroll
      for (int g = 0; g < 16; g += 8) {
        uint64_t e[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int t = g + k;
          uint32_t c;
          if (B == 32) c = sp[64 * t];
          else c = funnel(sp[2 * B * t + 1], sp[2 * B * t], sh) & width_mask<B>();
          uint32_t idx = dict_index<B>(c);
          if (TAIL) idx = (lane + 64u * t < limit) ? idx : kDictZeroSlot;
          e[k] = dict_at(idx);
        }
        part += ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
        pin(part);
      }
      const uint32_t lc = (uint32_t)(part >> kDictCountShift);
      s.lcount += lc;
      s.lsum += (part & kDictSumMask) + s.dict_base * lc;
      return;
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    uint32_t c;
    if (B == 32) c = sp[64 * t];
    else c = funnel(sp[2 * B * t + 1], sp[2 * B * t], sh) & width_mask<B>();
    const bool hit = (PF == PF_LO0) ? (c <= cr.wm1) : ((c - cr.loc) <= cr.wm1);
    const bool valid = !TAIL || (lane + 64u * t < limit);
    if constexpr (MODE == MODE_BF && ENC == ENC_DICT) {
      // a window too wide to pack: scalar popcount of the compare mask and
      // the masked entry (padding slots read the zero slot)
      ucnt += (uint32_t)__builtin_popcountll(ballot(hit && valid));
      uint32_t idx = dict_index<B>(c);
      if (TAIL) idx = valid ? idx : kDictZeroSlot;
      part += (uint64_t)dict_lds[idx];
      if ((t & 3) == 3) pin(part);
    } else if constexpr (MODE == MODE_BF) {
      const bool ok = hit && valid;
      cnt += ok ? 1u : 0u;
      const uint64_t v = code_value<ENC>(c, dict_lds, dict_last);
      part += ok ? (PartT<B, ENC>)v : (PartT<B, ENC>)0;
      if ((t & 3) == 3) {
        pin(part);
        pin(cnt);
      }
    } else {
      uint64_t m = ballot(hit);
      if (TAIL) m &= ballot(valid);
      cnt += (uint32_t)__builtin_popcountll(m);
      sv_push<ENC, uint32_t>(s, c, hit && valid, m, lane, dict_lds, dict_last);
    }
  }
  if constexpr (MODE == MODE_BF && ENC == ENC_DICT) {
    s.count += ucnt;
    s.lsum += (uint64_t)part;
  } else if constexpr (MODE == MODE_BF) {
    s.lcount += cnt;  // per lane
    s.lsum += (uint64_t)part + (uint64_t)cnt * ref;
  } else {
    s.count += cnt;   // uniform
    s.refsum += (uint64_t)cnt * ref;
  }
}

// Byte-aligned: one 16-byte load per lane per KiB of the block.
template <int B, int MODE, int ENC, int PF, bool TAIL>
__device__ __forceinline__ void decode_bytes(const Params& p, WaveState<uint32_t>& s, uint32_t lane,
                                             const uint4 (&x)[B / 8], uint64_t k, uint32_t ref) {
  const CodeRange cr = block_range<B, ENC, PF>(p, ref, 0, 0);
  if (!cr.nonempty) return;
  const uint32_t limit = TAIL ? p.tail : kBlockValues;
  uint32_t cnt = 0;
  PartT<B, ENC> part = 0;
  constexpr int V = 128 / B;  // values per 16-byte load
#pragma unroll
  for (int q = 0; q < B / 8; ++q) {
    const uint32_t xs[4] = {x[q].x, x[q].y, x[q].z, x[q].w};
    const uint32_t idx0 = q * (8192 / B) + lane * V;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      uint32_t c;
      if (B == 8) c = (xs[e >> 2] >> (8 * (e & 3))) & 0xFFu;
      else if (B == 16) c = (xs[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
      else c = xs[e];
      const bool hit = (PF == PF_LO0) ? (c <= cr.wm1) : ((c - cr.loc) <= cr.wm1);
      const bool valid = !TAIL || (idx0 + e < limit);
      if constexpr (MODE == MODE_BF) {
        const bool ok = hit && valid;
        cnt += ok ? 1u : 0u;
        part += ok ? (PartT<B, ENC>)c : (PartT<B, ENC>)0;
        if ((e & 3) == 3) {
          pin(part);
          pin(cnt);
        }
      } else {
        uint64_t m = ballot(hit);
        if (TAIL) m &= ballot(valid);
        cnt += (uint32_t)__builtin_popcountll(m);
        sv_push<ENC, uint32_t>(s, c, hit && valid, m, lane, nullptr, 0);
      }
    }
  }
  if constexpr (MODE == MODE_BF) {
    s.lcount += cnt;
    s.lsum += (uint64_t)part + (uint64_t)cnt * ref;
  } else {
    s.count += cnt;
    s.refsum += (uint64_t)cnt * ref;
  }
}

// Coalesced staging loads of one block into registers (lane takes words
// lane + 64 i), and their store into the block's LDS slot.
// 16-byte non-temporal load (whole-line streaming reads, see load_pair_words).
__device__ __forceinline__ uint4 load_stream16(const uint4* p) {
  typedef uint32_t v4 __attribute__((ext_vector_type(4)));
  const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

template <int B>
__device__ __forceinline__ void stage_load(const uint32_t* __restrict__ blk, uint32_t lane,
                                           uint32_t (&r)[Geo<B>::kStageLoads]) {
#pragma unroll
  for (int i = 0; i < Geo<B>::kStageLoads; ++i) {
    const uint32_t w = lane + 64u * i;
    r[i] = ((32 * B) % 64 == 0 || w < 32u * B) ? __builtin_nontemporal_load(blk + w) : 0u;
  }
}

template <int B>
__device__ __forceinline__ void stage_store(uint32_t* st, uint32_t lane, const uint32_t (&r)[Geo<B>::kStageLoads]) {
#pragma unroll
  for (int i = 0; i < Geo<B>::kStageLoads; ++i) {
    const uint32_t w = lane + 64u * i;
    if ((32 * B) % 64 == 0 || w < 32u * B) st[w] = r[i];
  }
}

// The j-th block of a step: the j-th set bit of the step mask, or (past the
// last one) the step's first block, so that every step issues the same loads.
__device__ __forceinline__ uint64_t step_block(uint64_t k0, uint64_t mask, int j) {
  uint64_t m = mask;
  for (int i = 0; i < j && (m & (m - 1ull)); ++i) m &= m - 1ull;
  return k0 + (uint64_t)__builtin_ctzll(m);
}

template <int B, int MODE, int ENC, int PF, int NB>
__device__ __forceinline__ void run_staged(const Params& p, WaveState<uint32_t>& s, uint32_t lane, uint32_t* st,
                                           uint64_t ka, uint64_t ke, uint64_t stride, uint32_t win, uint64_t excl,
                                           const int64_t* dict_lds, uint32_t dict_last, uint32_t clo, uint32_t chi) {
  constexpr int NL = Geo<B>::kStageLoads, SW = Geo<B>::kStageWords;
  auto live_fn = [&](uint64_t k0, uint32_t cnt) {
    return window_live<ENC>(p, k0, cnt, clo, chi, excl, s.lcount, s.lsum);
  };
  BlockCursor<NB, decltype(live_fn)> cur{ka, ke, 0, 0, stride, win};
  uint64_t k0 = 0, m0 = 0, k1 = 0, m1 = 0;
  uint32_t r0[NB][NL], r1[NB][NL];
  uint32_t f0[NB], f1[NB];  // block references (PF_REFS), in flight with the words
  auto load = [&](uint64_t base, uint64_t mask, uint32_t (&dst)[NB][NL], uint32_t (&f)[NB]) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint64_t k = step_block(base, mask, j);
      stage_load<B>(p.payload + k * (32u * B), lane, dst[j]);
      f[j] = PF == PF_REFS ? p.refs[k] : 0u;
    }
  };
  auto decode = [&](uint64_t base, uint64_t mask, const uint32_t (&src)[NB][NL], const uint32_t (&f)[NB]) {
    const int n = __builtin_popcountll(mask);
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < n) stage_store<B>(st + j * SW, lane, src[j]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (mask) {
        const uint64_t k = base + (uint64_t)__builtin_ctzll(mask);
        mask &= mask - 1ull;
        decode_staged<B, MODE, ENC, PF, false>(p, s, lane, st + j * SW, k, f[j], dict_lds, dict_last, clo, chi);
      }
    }
    __builtin_amdgcn_wave_barrier();
  };
  if (!cur.fetch(k0, m0, s.blocks, live_fn)) return;
  load(k0, m0, r0, f0);
  while (true) {
    const bool more1 = cur.fetch(k1, m1, s.blocks, live_fn);
    if (!more1) { k1 = k0; m1 = m0; }
    load(k1, m1, r1, f1);
    decode(k0, m0, r0, f0);
    if (!more1) break;
    const bool more0 = cur.fetch(k0, m0, s.blocks, live_fn);
    if (!more0) { k0 = k1; m0 = m1; }
    load(k0, m0, r0, f0);
    decode(k1, m1, r1, f1);
    if (!more0) break;
  }
}

template <int B, int MODE, int ENC, int PF, int NB>
__device__ __forceinline__ void run_bytes(const Params& p, WaveState<uint32_t>& s, uint32_t lane, uint64_t ka,
                                          uint64_t ke, uint64_t stride, uint32_t win, uint64_t excl) {
  constexpr int Q = B / 8;
  auto live_fn = [&](uint64_t k0, uint32_t cnt) {
    return window_live<ENC>(p, k0, cnt, 0, 0, excl, s.lcount, s.lsum);
  };
  BlockCursor<NB, decltype(live_fn)> cur{ka, ke, 0, 0, stride, win};
  uint64_t k0 = 0, m0 = 0, k1 = 0, m1 = 0;
  uint4 x0[NB][Q], x1[NB][Q];
  uint32_t f0[NB], f1[NB];  // block references (PF_REFS), in flight with the words
  auto load = [&](uint64_t base, uint64_t mask, uint4 (&dst)[NB][Q], uint32_t (&f)[NB]) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint64_t k = step_block(base, mask, j);
      const uint4* blk = reinterpret_cast<const uint4*>(p.payload + k * (32u * B));
#pragma unroll
      for (int q = 0; q < Q; ++q) dst[j][q] = load_stream16(blk + 64 * q + lane);
      f[j] = PF == PF_REFS ? p.refs[k] : 0u;
    }
  };
  auto decode = [&](uint64_t base, uint64_t mask, const uint4 (&src)[NB][Q], const uint32_t (&f)[NB]) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (mask) {
        const uint64_t k = base + (uint64_t)__builtin_ctzll(mask);
        mask &= mask - 1ull;
        decode_bytes<B, MODE, ENC, PF, false>(p, s, lane, src[j], k, f[j]);
      }
    }
  };
  if (!cur.fetch(k0, m0, s.blocks, live_fn)) return;
  load(k0, m0, x0, f0);
  while (true) {
    const bool more1 = cur.fetch(k1, m1, s.blocks, live_fn);
    if (!more1) { k1 = k0; m1 = m0; }
    load(k1, m1, x1, f1);
    decode(k0, m0, x0, f0);
    if (!more1) break;
    const bool more0 = cur.fetch(k0, m0, s.blocks, live_fn);
    if (!more0) { k0 = k1; m0 = m1; }
    load(k0, m0, x0, f0);
    decode(k1, m1, x1, f1);
    if (!more0) break;
  }
}

// ------------------------------------------------------------ FOR / DICT

constexpr uint32_t kListWords = 64;  // per-wavefront survivor list

template <int B, int DEC, int MODE>
__host__ __device__ constexpr uint32_t wave_lds_words() {
  return kListWords + (DEC == DEC_RM_LDS ? Geo<B>::kLdsBlocks * Geo<B>::kStageWords : 0u) +
         (MODE == MODE_SV ? kRingEntries : 0u);
}

// Dynamic LDS bytes of code_scan for a work-group of `waves` wavefronts.
template <int B, int DEC, int MODE, int ENC>
__host__ __device__ constexpr uint32_t code_scan_lds(uint32_t waves) {
  return (ENC == ENC_DICT ? kDictLdsBytes : 0u) + waves * wave_lds_words<B, DEC, MODE>() * 4u + kRedBytes;
}

// Step depth of scan_range: the default pipelined steps, the alternative
// depth of the register decoders' branch-free frame-of-reference kernels
// (Geo<B>::kPairsAlt; a tuning choice), or one block pair / staged block per
// step (the batched kernels, to bound code size).
enum StepForm { STEP_DEFAULT = 0, STEP_ALT = 1, STEP_SMALL = 2 };

// Scan blocks [ka, ke) of a FOR/DICT column into the wavefront state, with
// steps of the given form.  The partial
// last block, when it lies in the range, is decoded here with per-value
// validity after the pipelined loop.
template <int B, int DEC, int MODE, int ENC, int PF, int STEP>
__device__ __forceinline__ void scan_range(const Params& p, WaveState<uint32_t>& s, uint32_t lane, uint32_t* list,
                                           uint32_t* st, uint64_t ka, uint64_t ke, uint64_t stride, uint32_t win,
                                           const int64_t* dict_lds, uint32_t dict_last, uint32_t clo, uint32_t chi) {
  const uint64_t last = p.nb - 1;
  const bool tail_partial = p.tail != kBlockValues;
  const uint64_t excl = tail_partial ? last : ~0ull;
  if constexpr (DEC == DEC_RM_DIRECT || DEC == DEC_LI) {
    constexpr bool kSwap = ENC == ENC_DICT && MODE == MODE_BF && B < 16;
    constexpr int P = STEP == STEP_SMALL ? 1
                      : MODE == MODE_SV ? Geo<B>::kPairsSV
                      : (STEP == STEP_ALT) != kSwap ? Geo<B>::kPairsAlt : Geo<B>::kPairs;
    run_pairs<B, DEC, MODE, ENC, PF, P>(p, s, lane, list, ka, ke, stride, win, excl, dict_lds, dict_last, clo, chi);
  } else if constexpr (DEC == DEC_RM_LDS) {
    run_staged<B, MODE, ENC, PF, STEP == STEP_SMALL ? 1 : Geo<B>::kLdsBlocks>(p, s, lane, st, ka, ke, stride, win, excl, dict_lds,
                                                                 dict_last, clo, chi);
  } else {
    run_bytes<B, MODE, ENC, PF, STEP == STEP_SMALL ? 1 : Geo<B>::kByteBlocks>(p, s, lane, ka, ke, stride, win, excl);
  }
  if (tail_partial && owns_block(last, ka, ke, stride, win) && block_survives<ENC>(p, last, clo, chi)) {
    if (block_inside<ENC>(p, last, clo, chi)) {
      // all-match: every valid value passes; lane 0 takes the block (no branch on the lane)
      const uint64_t bs = p.bsum[last];
      s.lcount += lane == 0 ? (uint64_t)p.tail : 0ull;
      s.lsum += lane == 0 ? bs : 0ull;
    } else if constexpr (DEC == DEC_RM_DIRECT || DEC == DEC_LI) {
      s.blocks += 1;
      uint32_t w[B];
      load_pair_words<B, DEC>(p, last, lane & 31u, w);
      decode_pair<B, DEC, MODE, ENC, PF, true>(p, s, lane, w, last, lane < 32u, PF == PF_REFS ? p.refs[last] : 0u,
                                               dict_lds, dict_last, clo, chi);
    } else if constexpr (DEC == DEC_RM_LDS) {
      s.blocks += 1;
      uint32_t r[Geo<B>::kStageLoads];
      stage_load<B>(p.payload + last * (32u * B), lane, r);
      __builtin_amdgcn_wave_barrier();
      stage_store<B>(st, lane, r);
      __builtin_amdgcn_wave_barrier();
      decode_staged<B, MODE, ENC, PF, true>(p, s, lane, st, last, PF == PF_REFS ? p.refs[last] : 0u, dict_lds,
                                            dict_last, clo, chi);
      __builtin_amdgcn_wave_barrier();
    } else {
      s.blocks += 1;
      uint4 x[B / 8];
      const uint4* blk = reinterpret_cast<const uint4*>(p.payload + last * (32u * B));
#pragma unroll
      for (int q = 0; q < B / 8; ++q) x[q] = blk[64 * q + lane];
      decode_bytes<B, MODE, ENC, PF, true>(p, s, lane, x, last, PF == PF_REFS ? p.refs[last] : 0u);
    }
  }
}

template <int B, int DEC, int MODE, int ENC, int PF, int STEP = STEP_DEFAULT>
__global__ __launch_bounds__(256) void code_scan(const Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t* dict_lds = reinterpret_cast<int64_t*>(smem);
  uint32_t* wave_area = reinterpret_cast<uint32_t*>(smem + (ENC == ENC_DICT ? kDictLdsBytes : 0u)) +
                        wave * wave_lds_words<B, DEC, MODE>();
  uint32_t* list = wave_area;
  uint32_t* st = wave_area + kListWords;  // 16-byte aligned: the list is 256 bytes
  WaveState<uint32_t> s;
  s.ring = st + (DEC == DEC_RM_LDS ? Geo<B>::kLdsBlocks * Geo<B>::kStageWords : 0u);

  // LDS after the wavefront areas: the work-group reduction of the result
  // (and, before the scan, the dictionary staging's counts)
  auto* red = reinterpret_cast<uint64_t(*)[3]>(smem + (ENC == ENC_DICT ? kDictLdsBytes : 0u) +
                                               nw * wave_lds_words<B, DEC, MODE>() * 4u);
  uint32_t clo = 0, chi = 0, dict_last = 0;
  if constexpr (ENC == ENC_DICT) {
    stage_dictionary<MODE == MODE_BF>(p.dict, p.dict_len, B <= 12 ? (1u << B) : kMaxDict, p.lo, p.hi, dict_lds, red,
                                      clo, chi, s.dict_packed, s.dict_base);
    dict_last = p.dict_len - 1u;
    if constexpr (MODE == MODE_BF && DEC == DEC_RM_DIRECT && B <= kDictPairMaxB) {
      if (s.dict_packed) {  // uniform: the same window in every work-group
        stage_dictionary_pairs<B>(dict_lds);
        s.dict_pairs = true;
      }
    }
  }
  // Grid-strided windows of p.G blocks: at any moment the wavefronts read one
  // compact region of the column (DRAM row locality), like a streaming copy.
  const uint64_t gw = (uint64_t)blockIdx.x * nw + wave, tw = (uint64_t)gridDim.x * nw;
  scan_range<B, DEC, MODE, ENC, PF, STEP>(p, s, lane, list, st, gw * p.G, p.nb, tw * p.G, p.G, dict_lds, dict_last,
                                           clo, chi);
  if constexpr (MODE == MODE_SV) sv_drain_rest<ENC, uint32_t>(s, lane, dict_lds, dict_last);
  finish_scan(p, s.count + wave_sum_u64(s.lcount), s.lsum + (lane == 0 ? s.refsum : 0ull), s.blocks, red);
}

// ------------------------------------------------------------- delta scan

// Block-relative value rel = v - base_k < 1024 * 2^B: u32 for B <= 22.
template <int B>
using RelT = typename std::conditional<(B <= 22), uint32_t, uint64_t>::type;

template <int B>
struct RelRange {
  RelT<B> loc, wm1;
  bool nonempty;
};

// [lo, hi) on values -> [loc, loc + wm1] on rel = v - base (exact for any int64 inputs).
template <int B>
__device__ __forceinline__ RelRange<B> rel_range(int64_t base, int64_t lo, int64_t hi) {
  constexpr uint64_t kCap = (B <= 22) ? (1ull << 32) : (1ull << 43);
  uint64_t dlo = lo > base ? (uint64_t)lo - (uint64_t)base : 0ull;
  uint64_t dhi = hi > base ? (uint64_t)hi - (uint64_t)base : 0ull;
  if (dlo > kCap) dlo = kCap;
  if (dhi > kCap) dhi = kCap;
  RelRange<B> r;
  r.nonempty = dlo < dhi;
  r.loc = (RelT<B>)dlo;
  r.wm1 = (RelT<B>)(dhi - dlo - 1ull);
  return r;
}

template <typename T>
__device__ __forceinline__ T shfl_up_t(T x, int d, int width) {
  if constexpr (sizeof(T) == 4) {
    return (T)__shfl_up((uint32_t)x, d, width);
  } else {
    const uint32_t lo = __shfl_up((uint32_t)x, d, width), hi = __shfl_up((uint32_t)(x >> 32), d, width);
    return ((T)hi << 32) | lo;
  }
}

// Inclusive scan of x over segments of WIDTH lanes.
template <typename T, int WIDTH>
__device__ __forceinline__ T seg_inclusive_scan(T x, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < WIDTH; d <<= 1) {
    const T y = shfl_up_t<T>(x, d, WIDTH);
    if ((lane & (WIDTH - 1)) >= (uint32_t)d) x += y;
  }
  return x;
}

// Delta, half-wavefront per block: lane l holds deltas 32 l .. 32 l + 31,
// forms its local inclusive prefix, the half-wavefront scans the slice totals,
// rel = exclusive + local prefix.  `base`: the block's base, loaded with its
// words (a step ahead of the decode).
template <int B, int MODE, bool TAIL>
__device__ __forceinline__ void decode_delta_pair(const Params& p, WaveState<RelT<B>>& s, uint32_t lane,
                                                  const uint32_t (&w)[B], uint64_t kb, bool act, int64_t base) {
  using R = RelT<B>;
  const uint32_t l = lane & 31u;
  const RelRange<B> rr = rel_range<B>(base, p.lo, p.hi);
  act = act && rr.nonempty;
  const uint64_t act_m = ballot(act);
  if (act_m == 0) return;
  const uint32_t limit = (TAIL && kb == p.nb - 1) ? p.tail : kBlockValues;
  R pre[32];
  R run = 0;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    run += (R)run_code<B, B>(w, t);
    pre[t] = run;
  }
  const R excl = seg_inclusive_scan<R, 32>(run, lane) - run;
  using PT = typename std::conditional<(B <= 16), uint32_t, uint64_t>::type;
  PT part = 0;
  if constexpr (MODE == MODE_BF) {
    uint32_t lc = 0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const R rel = excl + pre[t];
      bool ok = (R)(rel - rr.loc) <= rr.wm1;
      if (TAIL) ok = ok && (32u * l + t < limit);
      lc += ok ? 1u : 0u;
      part += ok ? (PT)rel : (PT)0;
      if ((t & 3) == 3) {
        pin(part);
        pin(lc);
      }
    }
    if (act) {
      s.lcount += lc;
      s.lsum += (uint64_t)part + (uint64_t)lc * (uint64_t)base;
    }
  } else {
    uint32_t cA = 0, cB = 0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const R rel = excl + pre[t];
      const bool hit = (R)(rel - rr.loc) <= rr.wm1;
      uint64_t m = ballot(hit) & act_m;
      bool valid = true;
      if (TAIL) {
        valid = 32u * l + t < limit;
        m &= ballot(valid);
      }
      cA += (uint32_t)__builtin_popcount((uint32_t)m);
      cB += (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
      sv_push<ENC_DELTA, R>(s, rel, hit && act && valid, m, lane, nullptr, 0);
    }
    s.count += (uint64_t)cA + cB;
    s.refsum += (uint64_t)cA * readlane64((uint64_t)base, 0) + (uint64_t)cB * readlane64((uint64_t)base, 32);
  }
}

// Delta, wavefront per staged block: lane l takes the contiguous run
// 16 l .. 16 l + 15, realigns its words with one funnel shift so every code
// sits at a compile-time offset, and the wavefront scans the run totals.
template <int B, int MODE, bool TAIL>
__device__ __forceinline__ void decode_delta_staged(const Params& p, WaveState<RelT<B>>& s, uint32_t lane,
                                                    const uint32_t* st, int64_t base) {
  using R = RelT<B>;
  const RelRange<B> rr = rel_range<B>(base, p.lo, p.hi);
  if (!rr.nonempty) return;
  constexpr int NY = (16 * B + 31) / 32;
  const uint32_t bit0 = 16u * lane * B;
  const uint32_t* sp = st + (bit0 >> 5);
  const uint32_t sh = bit0 & 31u;
  uint32_t y[NY + 1];
#pragma unroll
  for (int i = 0; i < NY; ++i) y[i] = funnel(sp[i + 1], sp[i], sh);
  y[NY] = 0;
  const uint32_t limit = TAIL ? p.tail : kBlockValues;
  R pre[16];
  R run = 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    run += (R)run_code<B, NY + 1>(y, t);
    pre[t] = run;
  }
  const R excl = seg_inclusive_scan<R, 64>(run, lane) - run;
  uint32_t cnt = 0;
  using PT = typename std::conditional<(B <= 16), uint32_t, uint64_t>::type;
  PT part = 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const R rel = excl + pre[t];
    const bool hit = (R)(rel - rr.loc) <= rr.wm1;
    const bool valid = !TAIL || (16u * lane + t < limit);
    if constexpr (MODE == MODE_BF) {
      const bool ok = hit && valid;
      cnt += ok ? 1u : 0u;
      part += ok ? (PT)rel : (PT)0;
      if ((t & 3) == 3) {
        pin(part);
        pin(cnt);
      }
    } else {
      uint64_t m = ballot(hit);
      if (TAIL) m &= ballot(valid);
      cnt += (uint32_t)__builtin_popcountll(m);
      sv_push<ENC_DELTA, R>(s, rel, hit && valid, m, lane, nullptr, 0);
    }
  }
  if constexpr (MODE == MODE_BF) {
    s.lcount += cnt;
    s.lsum += (uint64_t)part + (uint64_t)cnt * (uint64_t)base;
  } else {
    s.count += cnt;
    s.refsum += (uint64_t)cnt * (uint64_t)base;
  }
}

template <int B, int DEC, int MODE>
__host__ __device__ constexpr uint32_t delta_wave_words() {
  return kListWords + (DEC == DEC_RM_LDS ? Geo<B>::kLdsBlocks * Geo<B>::kStageWords : 0u) +
         (MODE == MODE_SV ? kRingEntries * (uint32_t)sizeof(RelT<B>) / 4u : 0u);
}

template <int B, int DEC, int MODE>
__host__ __device__ constexpr uint32_t delta_scan_lds(uint32_t waves) {
  return waves * delta_wave_words<B, DEC, MODE>() * 4u + kRedBytes;
}

// Scan blocks [ka, ke) of a delta column into the wavefront state (see
// scan_range for SMALL and the partial last block).
template <int B, int DEC, int MODE, bool SMALL>
__device__ __forceinline__ void delta_range(const Params& p, WaveState<RelT<B>>& s, uint32_t lane, uint32_t* list,
                                            uint32_t* st, uint64_t ka, uint64_t ke, uint64_t stride, uint32_t win) {
  const uint64_t last = p.nb - 1;
  const bool tail_partial = p.tail != kBlockValues;
  const uint64_t excl = tail_partial ? last : ~0ull;
  auto live_fn = [&](uint64_t k0, uint32_t cnt) { return window_live_i64(p, k0, cnt, excl, s.lcount, s.lsum); };
  if constexpr (DEC == DEC_RM_DIRECT) {
    constexpr int P = SMALL ? 1 : Geo<B>::kDeltaPairs;
    const uint32_t l = lane & 31u;
    PairCursor<P, decltype(live_fn)> cur{ka, ke, 0, 0, 0, list, ka, stride, win};
    uint64_t k0b[P], k1b[P];
    uint32_t a0 = 0, a1 = 0;
    uint32_t w0[P][B], w1[P][B];
    int64_t b0[P], b1[P];  // block bases, in flight with the words
    auto load = [&](const uint64_t (&kb)[P], uint32_t (&w)[P][B], int64_t (&bb)[P]) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        load_pair_words<B, DEC_RM_DIRECT>(p, kb[q], l, w[q]);
        bb[q] = p.bases[kb[q]];
      }
    };
    auto decode = [&](const uint32_t (&w)[P][B], const uint64_t (&kb)[P], uint32_t ab, const int64_t (&bb)[P]) {
#pragma unroll
      for (int q = 0; q < P; ++q)
        decode_delta_pair<B, MODE, false>(p, s, lane, w[q], kb[q], (ab >> q) & 1u, bb[q]);
    };
    if (cur.fetch(k0b, a0, s.blocks, live_fn, lane)) {
      load(k0b, w0, b0);
      while (true) {
        const bool more1 = cur.fetch(k1b, a1, s.blocks, live_fn, lane);
        load(k1b, w1, b1);
        decode(w0, k0b, a0, b0);
        if (!more1) break;
        const bool more0 = cur.fetch(k0b, a0, s.blocks, live_fn, lane);
        load(k0b, w0, b0);
        decode(w1, k1b, a1, b1);
        if (!more0) break;
      }
    }
  } else {
    constexpr int NB = SMALL ? 1 : Geo<B>::kLdsBlocks, NL = Geo<B>::kStageLoads, SW = Geo<B>::kStageWords;
    BlockCursor<NB, decltype(live_fn)> cur{ka, ke, 0, 0, stride, win};
    uint64_t k0 = 0, m0 = 0, k1 = 0, m1 = 0;
    uint32_t r0[NB][NL], r1[NB][NL];
    int64_t b0[NB], b1[NB];  // block bases, in flight with the words (step_block j: the j-th decoded block)
    auto load = [&](uint64_t base, uint64_t mask, uint32_t (&dst)[NB][NL], int64_t (&bb)[NB]) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const uint64_t k = step_block(base, mask, j);
        stage_load<B>(p.payload + k * (32u * B), lane, dst[j]);
        bb[j] = p.bases[k];
      }
    };
    auto decode = [&](uint64_t mask, const uint32_t (&src)[NB][NL], const int64_t (&bb)[NB]) {
      const int n = __builtin_popcountll(mask);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < n) stage_store<B>(st + j * SW, lane, src[j]);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < n) decode_delta_staged<B, MODE, false>(p, s, lane, st + j * SW, bb[j]);
      __builtin_amdgcn_wave_barrier();
    };
    if (cur.fetch(k0, m0, s.blocks, live_fn)) {
      load(k0, m0, r0, b0);
      while (true) {
        const bool more1 = cur.fetch(k1, m1, s.blocks, live_fn);
        if (!more1) { k1 = k0; m1 = m0; }
        load(k1, m1, r1, b1);
        decode(m0, r0, b0);
        if (!more1) break;
        const bool more0 = cur.fetch(k0, m0, s.blocks, live_fn);
        if (!more0) { k0 = k1; m0 = m1; }
        load(k0, m0, r0, b0);
        decode(m1, r1, b1);
        if (!more0) break;
      }
    }
  }
  if (tail_partial && owns_block(last, ka, ke, stride, win) && block_survives<ENC_DELTA>(p, last, 0, 0)) {
    if (block_inside<ENC_DELTA>(p, last, 0, 0)) {
      // all-match: every valid value passes; lane 0 takes the block (no branch on the lane)
      const uint64_t bs = p.bsum[last];
      s.lcount += lane == 0 ? (uint64_t)p.tail : 0ull;
      s.lsum += lane == 0 ? bs : 0ull;
    } else if constexpr (DEC == DEC_RM_DIRECT) {
      s.blocks += 1;
      uint32_t w[B];
      load_pair_words<B, DEC_RM_DIRECT>(p, last, lane & 31u, w);
      decode_delta_pair<B, MODE, true>(p, s, lane, w, last, lane < 32u, p.bases[last]);
    } else {
      s.blocks += 1;
      uint32_t r[Geo<B>::kStageLoads];
      stage_load<B>(p.payload + last * (32u * B), lane, r);
      stage_store<B>(st, lane, r);
      __builtin_amdgcn_wave_barrier();
      decode_delta_staged<B, MODE, true>(p, s, lane, st, p.bases[last]);
    }
  }
}

template <int B, int DEC, int MODE>
__global__ __launch_bounds__(256) void delta_scan(const Params p) {
  using R = RelT<B>;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t* wave_area = reinterpret_cast<uint32_t*>(smem) + wave * delta_wave_words<B, DEC, MODE>();
  uint32_t* list = wave_area;
  uint32_t* st = wave_area + kListWords;
  WaveState<R> s;
  s.ring = reinterpret_cast<R*>(st + (DEC == DEC_RM_LDS ? Geo<B>::kLdsBlocks * Geo<B>::kStageWords : 0u));
  const uint64_t gw = (uint64_t)blockIdx.x * nw + wave, tw = (uint64_t)gridDim.x * nw;
  delta_range<B, DEC, MODE, false>(p, s, lane, list, st, gw * p.G, p.nb, tw * p.G, p.G);
  if constexpr (MODE == MODE_SV) sv_drain_rest<ENC_DELTA, R>(s, lane, nullptr, 0);
  auto* red = reinterpret_cast<uint64_t(*)[3]>(smem + nw * delta_wave_words<B, DEC, MODE>() * 4u);
  finish_scan(p, s.count + wave_sum_u64(s.lcount), s.lsum + (lane == 0 ? s.refsum : 0ull), s.blocks, red);
}

}  // namespace scan_dev
