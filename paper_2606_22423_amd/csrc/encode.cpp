// Host-side column encoders (frame of reference, delta, dictionary codes) and
// zone maps, written from the column format in include/scan.h.  Each block is
// packed as 32 slices of 32 codes with a 64-bit bit accumulator; work is split
// over host threads by block ranges.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/scan.h"

namespace {

constexpr uint64_t kL = SCAN_BLOCK_VALUES;

uint64_t blocks_of(uint64_t n) { return (n + kL - 1) / kL; }

uint64_t code_limit(uint32_t b) { return b == 32 ? 0xFFFFFFFFull : ((1ull << b) - 1ull); }

// Pack 32 codes into b consecutive words, LSB first.
inline void pack32(const uint32_t* codes, uint32_t b, uint32_t* out) {
  uint64_t acc = 0;
  uint32_t fill = 0, o = 0;
  for (int t = 0; t < 32; ++t) {
    acc |= (uint64_t)codes[t] << fill;
    fill += b;
    while (fill >= 32) {
      out[o++] = (uint32_t)acc;
      acc >>= 32;
      fill -= 32;
    }
  }
}

// Pack one block's codes (cnt valid, the rest zero) in the requested layout.
inline void pack_block(const uint32_t* codes, uint32_t cnt, uint32_t b, uint32_t layout, uint32_t* out) {
  uint32_t tmp[32];
  uint32_t words[32];
  for (uint32_t s = 0; s < 32; ++s) {
    for (uint32_t t = 0; t < 32; ++t) {
      // RM: slice s holds codes 32 s .. 32 s + 31; LI: lane s holds codes s, s + 32, ...
      const uint32_t j = layout == SCAN_LAYOUT_LI ? 32u * t + s : 32u * s + t;
      tmp[t] = j < cnt ? codes[j] : 0u;
    }
    if (layout == SCAN_LAYOUT_LI) {
      pack32(tmp, b, words);
      for (uint32_t r = 0; r < b; ++r) out[32u * r + s] = words[r];
    } else {
      pack32(tmp, b, out + s * b);
    }
  }
}

template <typename F>
bool parallel_blocks(uint64_t nb, F&& fn) {
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  uint64_t per = std::max<uint64_t>(64, (nb + hw - 1) / hw);
  std::atomic<bool> ok{true};
  std::vector<std::thread> th;
  for (uint64_t a = 0; a < nb; a += per) {
    uint64_t e = std::min(nb, a + per);
    th.emplace_back([&, a, e] {
      for (uint64_t k = a; k < e && ok.load(std::memory_order_relaxed); ++k)
        if (!fn(k)) ok = false;
    });
  }
  for (auto& t : th) t.join();
  return ok;
}

}  // namespace

extern "C" {

uint64_t scan_payload_words(uint64_t n, uint32_t b) { return blocks_of(n) * 32ull * b; }

scan_status scan_encode_for(const uint32_t* values, uint64_t n, uint32_t b, uint32_t layout, int32_t ref_policy,
                            uint32_t* payload, uint32_t* block_ref, uint32_t* zone_min, uint32_t* zone_max) {
  if (b < 1 || b > 32 || (n && (!values || !payload)) || layout > 1 || ref_policy < 0 || ref_policy > 1 ||
      (ref_policy == 1 && !block_ref))
    return SCAN_EINVAL;
  const uint64_t nb = blocks_of(n);
  const uint64_t lim = code_limit(b);
  bool ok = parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * kL;
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(kL, n - a);
    uint32_t mn = values[a], mx = values[a];
    for (uint32_t j = 0; j < cnt; ++j) {
      mn = std::min(mn, values[a + j]);
      mx = std::max(mx, values[a + j]);
    }
    const uint32_t ref = ref_policy == 1 ? mn : 0u;
    if ((uint64_t)mx - ref > lim) return false;
    uint32_t codes[kL];
    for (uint32_t j = 0; j < cnt; ++j) codes[j] = values[a + j] - ref;
    pack_block(codes, cnt, b, layout, payload + k * 32ull * b);
    if (block_ref) block_ref[k] = ref;
    if (zone_min) zone_min[k] = mn;
    if (zone_max) zone_max[k] = mx;
    return true;
  });
  return ok ? SCAN_OK : SCAN_EINVAL;
}

scan_status scan_encode_delta(const int64_t* values, uint64_t n, uint32_t b, uint32_t* payload, int64_t* block_base,
                              int64_t* zone_min, int64_t* zone_max) {
  if (b < 1 || b > 32 || (n && (!values || !payload || !block_base))) return SCAN_EINVAL;
  const uint64_t nb = blocks_of(n);
  const uint64_t lim = code_limit(b);
  bool ok = parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * kL;
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(kL, n - a);
    uint32_t codes[kL];
    codes[0] = 0;
    for (uint32_t j = 1; j < cnt; ++j) {
      const int64_t prev = values[a + j - 1], cur = values[a + j];
      if (cur < prev) return false;
      const uint64_t d = (uint64_t)cur - (uint64_t)prev;
      if (d > lim) return false;
      codes[j] = (uint32_t)d;
    }
    pack_block(codes, cnt, b, SCAN_LAYOUT_RM, payload + k * 32ull * b);
    block_base[k] = values[a];
    if (zone_min) zone_min[k] = values[a];
    if (zone_max) zone_max[k] = values[a + cnt - 1];
    return true;
  });
  return ok ? SCAN_OK : SCAN_EINVAL;
}

scan_status scan_encode_dict(const uint32_t* codes, uint64_t n, uint32_t b, uint32_t dict_len, uint32_t* payload,
                             uint32_t* zone_min, uint32_t* zone_max) {
  if (b < 1 || b > 32 || (n && (!codes || !payload)) || dict_len == 0 || dict_len > SCAN_MAX_DICT ||
      (uint64_t)dict_len > code_limit(b) + 1ull)
    return SCAN_EINVAL;
  const uint64_t nb = blocks_of(n);
  bool ok = parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * kL;
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(kL, n - a);
    uint32_t mn = codes[a], mx = codes[a];
    for (uint32_t j = 0; j < cnt; ++j) {
      if (codes[a + j] >= dict_len) return false;
      mn = std::min(mn, codes[a + j]);
      mx = std::max(mx, codes[a + j]);
    }
    pack_block(codes + a, cnt, b, SCAN_LAYOUT_RM, payload + k * 32ull * b);
    if (zone_min) zone_min[k] = mn;
    if (zone_max) zone_max[k] = mx;
    return true;
  });
  return ok ? SCAN_OK : SCAN_EINVAL;
}

scan_status scan_block_sums(int32_t enc, const void* values, uint64_t n, const int64_t* dict, uint32_t dict_len,
                            uint64_t* out) {
  if (n && (!values || !out)) return SCAN_EINVAL;
  if (enc == SCAN_ENC_DICT && n && !dict) return SCAN_EINVAL;
  if (enc != SCAN_ENC_FOR && enc != SCAN_ENC_DELTA_FOR && enc != SCAN_ENC_DICT) return SCAN_EINVAL;
  const uint64_t nb = blocks_of(n);
  bool ok = parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * 1024ull, e = std::min<uint64_t>(n, a + 1024ull);
    uint64_t sum = 0;  // mod 2^64
    for (uint64_t i = a; i < e; ++i) {
      if (enc == SCAN_ENC_FOR) {
        sum += static_cast<const uint32_t*>(values)[i];
      } else if (enc == SCAN_ENC_DELTA_FOR) {
        sum += (uint64_t) static_cast<const int64_t*>(values)[i];
      } else {
        const uint32_t c = static_cast<const uint32_t*>(values)[i];
        if (c >= dict_len) return false;
        sum += (uint64_t)dict[c];
      }
    }
    out[k] = sum;
    return true;
  });
  return ok ? SCAN_OK : SCAN_EINVAL;
}

scan_status scan_rle_encode(const uint32_t* values, uint64_t n, uint32_t* run_value, uint16_t* run_len,
                            uint64_t* block_run, uint32_t* zone_min, uint32_t* zone_max, uint64_t* n_runs) {
  if (!n_runs || !block_run || (n && (!values || !run_value || !run_len))) return SCAN_EINVAL;
  const uint64_t nb = blocks_of(n);
  // pass 1: runs per block (in parallel), then block starts; pass 2: the runs
  std::vector<uint64_t> per(nb + 1, 0);
  parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * 1024ull, e = std::min<uint64_t>(n, a + 1024ull);
    uint64_t r = 0;
    for (uint64_t i = a; i < e; ++i) r += (i == a || values[i] != values[i - 1]) ? 1u : 0u;
    per[k] = r;
    return true;
  });
  uint64_t acc = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    block_run[k] = acc;
    acc += per[k];
  }
  block_run[nb] = acc;
  *n_runs = acc;
  parallel_blocks(nb, [&](uint64_t k) {
    const uint64_t a = k * 1024ull, e = std::min<uint64_t>(n, a + 1024ull);
    uint64_t r = block_run[k];
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    for (uint64_t i = a; i < e; ++i) {
      if (i == a || values[i] != values[i - 1]) {
        run_value[r] = values[i];
        run_len[r] = 0;
        ++r;
      }
      ++run_len[r - 1];
      mn = std::min(mn, values[i]);
      mx = std::max(mx, values[i]);
    }
    if (zone_min) zone_min[k] = mn;
    if (zone_max) zone_max[k] = mx;
    return true;
  });
  return SCAN_OK;
}

}  // extern "C"
