/*
 * CPU ORACLE for the fused columnar scan -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code, header, table or helper with
 * the GPU library: it is written from the definitions below, in plain scalar
 * C, one value at a time, for a reader to check against the paper by eye.
 *
 * What it computes (the paper, "Problem and Model" and "Method"): a scan
 * reads a compressed column, decodes every value, evaluates a predicate and
 * aggregates, in one pass.  For decoded values v_0..v_{n-1} and the half-open
 * predicate [lo, hi):
 *     COUNT = #{ i : lo <= v_i < hi }
 *     SUM   = (sum of those v_i) mod 2^64, reported as two's-complement int64
 * Zone maps (per-block min/max, "Method") are a speed device: a block whose
 * [min, max] misses [lo, hi) holds no match.  With zone maps on, the oracle
 * reports blocks_read = #{ k : not (max_k < lo or min_k >= hi) }; with zone
 * maps off, blocks_read = number of blocks.  An empty predicate (lo >= hi)
 * reads nothing: every output is 0.
 * All-match shortcut (an extension of the zone-map idea, not in the paper): a
 * block whose [min, max] lies inside [lo, hi) matches entirely, so a scan
 * can take its count and its stored sum without decoding it.  COUNT and SUM
 * are unchanged by definition; blocks_read then counts only the surviving
 * blocks that are not entirely inside: #{ k : survives and not (min_k >= lo
 * and max_k < hi) }.
 *
 * Format (the paper fixes only 1024-value blocks and the idea of a
 * row-major and a lane-transposed packing; the bit order below is this
 * project's reading, chosen so that widths 8/16/32 coincide with plain
 * little-endian u8/u16/u32 arrays as the paper requires of byte-aligned widths):
 *   block k holds values kL .. kL+L-1 (L = 1024) in 32*b u32 words;
 *   row-major (RM): value j of the block occupies block bits [j*b, j*b+b);
 *     block bit t is bit (t mod 32) of block word (t div 32);
 *   lane-interleaved (LI): value j goes to lane j mod 32, slot j div 32; a
 *     lane's slots fill its own bit stream, lane bit t being bit (t mod 32)
 *     of block word 32*(t div 32) + lane;
 *   tail slots past n are zero.
 *   frame of reference: v = ref_k + code (u32; ref_k = 0 when refs is NULL);
 *   delta: v = base_k + (d_0 + ... + d_j) with d_0 = 0 (int64);
 *   dictionary: v = D[code], D strictly increasing int64.
 *
 * Parity pins for every function live in tests/ (round trips, the byte-aligned
 * identity, closed-form COUNT/SUM, brute force against an independent
 * big-integer decoder, zone-map on == off).
 */
#include <stdint.h>
#include <string.h>

#define ORC_L 1024u

typedef struct {
  uint64_t count;
  int64_t sum;
  uint64_t blocks_read;
  uint64_t blocks_total;
  int32_t sum_overflow; /* 1 if the exact sum lies outside int64 (SUM is then the wrapped value) */
} orc_result;

static uint64_t nblocks(uint64_t n) { return (n + ORC_L - 1u) / ORC_L; }

static uint32_t width_mask(uint32_t b) { return b == 32u ? 0xFFFFFFFFu : ((1u << b) - 1u); }

/* ------------------------------------------------------------ bit packing */

/* Set every bit of every code individually (slow, obviously correct). */
int orc_pack_rm(const uint32_t* codes, uint64_t n, uint32_t b, uint32_t* words) {
  if (b < 1u || b > 32u) return -1;
  memset(words, 0, (size_t)(nblocks(n) * 32u * b * 4u));
  for (uint64_t i = 0; i < n; i++) {
    if (codes[i] & ~width_mask(b)) return -2;
    uint32_t* blk = words + (i / ORC_L) * 32u * b;
    uint64_t j = i % ORC_L;
    for (uint32_t q = 0; q < b; q++) {
      uint64_t t = j * b + q;
      if ((codes[i] >> q) & 1u) blk[t / 32u] |= 1u << (t % 32u);
    }
  }
  return 0;
}

int orc_pack_li(const uint32_t* codes, uint64_t n, uint32_t b, uint32_t* words) {
  if (b < 1u || b > 32u) return -1;
  memset(words, 0, (size_t)(nblocks(n) * 32u * b * 4u));
  for (uint64_t i = 0; i < n; i++) {
    if (codes[i] & ~width_mask(b)) return -2;
    uint32_t* blk = words + (i / ORC_L) * 32u * b;
    uint64_t j = i % ORC_L;
    uint64_t lane = j % 32u, slot = j / 32u;
    for (uint32_t q = 0; q < b; q++) {
      uint64_t t = slot * b + q; /* bit of the lane's own stream */
      if ((codes[i] >> q) & 1u) blk[32u * (t / 32u) + lane] |= 1u << (t % 32u);
    }
  }
  return 0;
}

/* Serial variable-shift extractor (the paper's scalar row-major decoder):
 * the code starting at block bit j*b, joined across a word boundary. */
static uint32_t extract_rm(const uint32_t* blk, uint32_t j, uint32_t b) {
  uint64_t bit = (uint64_t)j * b;
  uint32_t w = (uint32_t)(bit / 32u), off = (uint32_t)(bit % 32u);
  uint32_t x = blk[w] >> off;
  if (off + b > 32u) x |= blk[w + 1u] << (32u - off);
  return x & width_mask(b);
}

static uint32_t extract_li(const uint32_t* blk, uint32_t j, uint32_t b) {
  uint32_t lane = j % 32u, slot = j / 32u;
  uint64_t bit = (uint64_t)slot * b;
  uint32_t r = (uint32_t)(bit / 32u), off = (uint32_t)(bit % 32u);
  uint32_t x = blk[32u * r + lane] >> off;
  if (off + b > 32u) x |= blk[32u * (r + 1u) + lane] << (32u - off);
  return x & width_mask(b);
}

static uint32_t extract(const uint32_t* payload, uint64_t i, uint32_t b, int layout) {
  const uint32_t* blk = payload + (i / ORC_L) * 32u * b;
  uint32_t j = (uint32_t)(i % ORC_L);
  return layout == 1 ? extract_li(blk, j, b) : extract_rm(blk, j, b);
}

int orc_unpack(const uint32_t* words, uint64_t n, uint32_t b, int layout, uint32_t* codes) {
  if (b < 1u || b > 32u || (layout != 0 && layout != 1)) return -1;
  for (uint64_t i = 0; i < n; i++) codes[i] = extract(words, i, b, layout);
  return 0;
}

/* ----------------------------------------------------------------- encodings */

/* Frame of reference.  policy 0: ref_k = 0; policy 1: ref_k = min of block k.
 * Fails (-2) if some v - ref_k does not fit in b bits. */
int orc_for_encode(const uint32_t* v, uint64_t n, uint32_t b, int policy, uint32_t* refs,
                   uint32_t* codes) {
  if (b < 1u || b > 32u) return -1;
  for (uint64_t k = 0; k < nblocks(n); k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    uint32_t ref = 0;
    if (policy == 1) {
      ref = v[a];
      for (uint64_t i = a; i < e; i++)
        if (v[i] < ref) ref = v[i];
    }
    if (refs) refs[k] = ref;
    for (uint64_t i = a; i < e; i++) {
      uint64_t c = (uint64_t)v[i] - ref;
      if (c > width_mask(b)) return -2;
      codes[i] = (uint32_t)c;
    }
  }
  return 0;
}

/* Delta: base_k = first value of block k; d_0 = 0, d_j = v_j - v_{j-1} in [0, 2^b). */
int orc_delta_encode(const int64_t* v, uint64_t n, uint32_t b, int64_t* bases, uint32_t* codes) {
  if (b < 1u || b > 32u) return -1;
  for (uint64_t k = 0; k < nblocks(n); k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    bases[k] = v[a];
    codes[a] = 0;
    for (uint64_t i = a + 1u; i < e; i++) {
      if (v[i] < v[i - 1u]) return -3;
      __int128 d = (__int128)v[i] - (__int128)v[i - 1u];
      if (d > (__int128)width_mask(b)) return -2;
      codes[i] = (uint32_t)d;
    }
  }
  return 0;
}

int orc_delta_decode(const uint32_t* codes, const int64_t* bases, uint64_t n, int64_t* v) {
  for (uint64_t k = 0; k < nblocks(n); k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    int64_t run = bases[k];
    for (uint64_t i = a; i < e; i++) {
      run += (int64_t)codes[i];
      v[i] = run;
    }
  }
  return 0;
}

/* Dictionary: code = position of v in the strictly increasing D[0..m). */
int orc_dict_encode(const int64_t* v, uint64_t n, const int64_t* dict, uint32_t m, uint32_t* codes) {
  for (uint32_t c = 1; c < m; c++)
    if (dict[c - 1u] >= dict[c]) return -3;
  for (uint64_t i = 0; i < n; i++) {
    uint32_t a = 0, e = m; /* first c with dict[c] >= v[i] */
    while (a < e) {
      uint32_t mid = a + (e - a) / 2u;
      if (dict[mid] < v[i]) a = mid + 1u; else e = mid;
    }
    if (a == m || dict[a] != v[i]) return -2;
    codes[i] = a;
  }
  return 0;
}

/* Per-block min/max of the decoded values over the block's valid slots. */
int orc_zonemap_u32(const uint32_t* v, uint64_t n, uint32_t* zmin, uint32_t* zmax) {
  for (uint64_t k = 0; k < nblocks(n); k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    uint32_t mn = v[a], mx = v[a];
    for (uint64_t i = a; i < e; i++) {
      if (v[i] < mn) mn = v[i];
      if (v[i] > mx) mx = v[i];
    }
    zmin[k] = mn;
    zmax[k] = mx;
  }
  return 0;
}

int orc_zonemap_i64(const int64_t* v, uint64_t n, int64_t* zmin, int64_t* zmax) {
  for (uint64_t k = 0; k < nblocks(n); k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    int64_t mn = v[a], mx = v[a];
    for (uint64_t i = a; i < e; i++) {
      if (v[i] < mn) mn = v[i];
      if (v[i] > mx) mx = v[i];
    }
    zmin[k] = mn;
    zmax[k] = mx;
  }
  return 0;
}

/* ------------------------------------------------------------------- scans */

typedef struct {
  __int128 sum;
  uint64_t count;
} acc_t;

static void finish(const acc_t* a, uint64_t read, uint64_t total, orc_result* out) {
  out->count = a->count;
  out->sum = (int64_t)(uint64_t)(unsigned __int128)a->sum; /* low 64 bits */
  out->sum_overflow = (a->sum > (__int128)INT64_MAX || a->sum < (__int128)INT64_MIN) ? 1 : 0;
  out->blocks_read = read;
  out->blocks_total = total;
}

/* Decoded value i of a packed column.  enc: 0 frame of reference, 1 delta, 2 dictionary.
 * Delta needs the running prefix, so it is decoded block by block in the scan below. */
static int64_t decode_for(const uint32_t* payload, const uint32_t* refs, uint64_t i, uint32_t b,
                          int layout) {
  uint32_t ref = refs ? refs[i / ORC_L] : 0u;
  return (int64_t)(uint32_t)(ref + extract(payload, i, b, layout));
}

/* One column scan.  The block's values are decoded first (into vals), its zone
 * map is taken from them, and only then is the block tested and aggregated. */
static int scan_generic(int enc, const uint32_t* payload, const uint32_t* refs, const int64_t* bases,
                        const int64_t* dict, uint32_t m, uint64_t n, uint32_t b, int layout,
                        int64_t lo, int64_t hi, int flags, orc_result* out) {
  /* flags: bit 0 zone maps, bit 1 all-match shortcut (with zone maps) */
  const int use_zm = flags & 1, use_am = (flags & 3) == 3;
  acc_t acc = {0, 0};
  uint64_t nb = nblocks(n), read = 0;
  if (b < 1u || b > 32u) return -1;
  if (lo >= hi || n == 0) {
    finish(&acc, 0, nb, out);
    return 0;
  }
  int64_t vals[ORC_L];
  for (uint64_t k = 0; k < nb; k++) {
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    int64_t run = (enc == 1) ? bases[k] : 0;
    for (uint64_t i = a; i < e; i++) {
      if (enc == 0) {
        vals[i - a] = decode_for(payload, refs, i, b, layout);
      } else if (enc == 1) {
        run += (int64_t)extract(payload, i, b, layout);
        vals[i - a] = run;
      } else {
        uint32_t c = extract(payload, i, b, layout);
        if (c >= m) return -2;
        vals[i - a] = dict[c];
      }
    }
    if (use_zm) {
      int64_t mn = vals[0], mx = vals[0];
      for (uint64_t i = 0; i < e - a; i++) {
        if (vals[i] < mn) mn = vals[i];
        if (vals[i] > mx) mx = vals[i];
      }
      if (mx < lo || mn >= hi) continue; /* skipped: contributes nothing */
      if (use_am && mn >= lo && mx < hi) {
        /* entirely inside: every value matches; not a block read */
        for (uint64_t i = 0; i < e - a; i++) {
          acc.count++;
          acc.sum += vals[i];
        }
        continue;
      }
    }
    read++;
    for (uint64_t i = 0; i < e - a; i++) {
      if (lo <= vals[i] && vals[i] < hi) {
        acc.count++;
        acc.sum += vals[i];
      }
    }
  }
  finish(&acc, read, nb, out);
  return 0;
}

int orc_scan_for(const uint32_t* payload, const uint32_t* refs, uint64_t n, uint32_t b, int layout,
                 int64_t lo, int64_t hi, int flags, orc_result* out) {
  return scan_generic(0, payload, refs, NULL, NULL, 0, n, b, layout, lo, hi, flags, out);
}

int orc_scan_delta(const uint32_t* payload, const int64_t* bases, uint64_t n, uint32_t b, int64_t lo,
                   int64_t hi, int flags, orc_result* out) {
  return scan_generic(1, payload, NULL, bases, NULL, 0, n, b, 0, lo, hi, flags, out);
}

int orc_scan_dict(const uint32_t* payload, const int64_t* dict, uint32_t m, uint64_t n, uint32_t b,
                  int64_t lo, int64_t hi, int flags, orc_result* out) {
  return scan_generic(2, payload, NULL, NULL, dict, m, n, b, 0, lo, hi, flags, out);
}

/* The plain definition on raw values, with no packing at all. */
int orc_count_sum_u32(const uint32_t* v, uint64_t n, int64_t lo, int64_t hi, orc_result* out) {
  acc_t acc = {0, 0};
  for (uint64_t i = 0; i < n && lo < hi; i++)
    if (lo <= (int64_t)v[i] && (int64_t)v[i] < hi) {
      acc.count++;
      acc.sum += v[i];
    }
  finish(&acc, 0, nblocks(n), out);
  return 0;
}

int orc_count_sum_i64(const int64_t* v, uint64_t n, int64_t lo, int64_t hi, orc_result* out) {
  acc_t acc = {0, 0};
  for (uint64_t i = 0; i < n && lo < hi; i++)
    if (lo <= v[i] && v[i] < hi) {
      acc.count++;
      acc.sum += v[i];
    }
  finish(&acc, 0, nblocks(n), out);
  return 0;
}

/* -------------------------------------------------- multi-column query */

/* A packed table column as the query oracle sees it: enc 0 (frame of
 * reference, RM) or 2 (dictionary, RM). */
typedef struct {
  int32_t enc;
  uint32_t b;
  const uint32_t* payload;
  const uint32_t* refs;
  const int64_t* dict;
  uint32_t m;
} orc_column;

static int64_t column_value(const orc_column* c, uint64_t i) {
  if (c->enc == 2) return c->dict[extract(c->payload, i, c->b, 0)];
  return decode_for(c->payload, c->refs, i, c->b, 0);
}

/* COUNT and SUM(sum_col) over the rows where every conjunct lo_f <= v_f < hi_f holds. */
int orc_query(const orc_column* cols, uint64_t n, int nf, const int32_t* fcol, const int64_t* flo,
              const int64_t* fhi, int32_t sum_col, orc_result* out) {
  acc_t acc = {0, 0};
  for (uint64_t i = 0; i < n; i++) {
    int ok = 1;
    for (int f = 0; f < nf && ok; f++) {
      int64_t v = column_value(&cols[fcol[f]], i);
      ok = (flo[f] <= v && v < fhi[f]);
    }
    if (ok) {
      acc.count++;
      acc.sum += column_value(&cols[sum_col], i);
    }
  }
  finish(&acc, 0, nblocks(n), out);
  return 0;
}

/* ------------------------------------------------ materializing select */

/* Decoded value i of a frame-of-reference (enc 0) or dictionary (enc 2)
 * column; one value at a time, nothing shared with the scan above. */
static int64_t value_at(int enc, const uint32_t* payload, const uint32_t* refs, const int64_t* dict, uint64_t i,
                        uint32_t b, int layout) {
  if (enc == 2) return dict[extract(payload, i, b, layout)];
  return decode_for(payload, refs, i, b, layout);
}

/* Materializing select: the ascending positions i < n with lo <= v_i < hi.
 * Writes at most cap of them to out and returns how many there are
 * (negative on a bad width or encoding). */
int64_t orc_select(int enc, const uint32_t* payload, const uint32_t* refs, const int64_t* dict, uint64_t n,
                   uint32_t b, int layout, int64_t lo, int64_t hi, uint32_t* out, uint64_t cap) {
  if (b < 1u || b > 32u || (enc != 0 && enc != 2)) return -1;
  int64_t count = 0;
  for (uint64_t i = 0; i < n && lo < hi; i++) {
    int64_t v = value_at(enc, payload, refs, dict, i, b, layout);
    if (lo <= v && v < hi) {
      if ((uint64_t)count < cap) out[count] = (uint32_t)i;
      count++;
    }
  }
  return count;
}

/* Late materialization: the positions of pos[0..m) (ascending) whose value
 * in this column lies in [lo, hi), in the same order. */
int64_t orc_refine(int enc, const uint32_t* payload, const uint32_t* refs, const int64_t* dict, uint32_t b,
                   int layout, int64_t lo, int64_t hi, const uint32_t* pos, uint64_t m, uint32_t* out) {
  if (b < 1u || b > 32u || (enc != 0 && enc != 2)) return -1;
  int64_t count = 0;
  for (uint64_t q = 0; q < m && lo < hi; q++) {
    int64_t v = value_at(enc, payload, refs, dict, pos[q], b, layout);
    if (lo <= v && v < hi) out[count++] = pos[q];
  }
  return count;
}

/* The values at pos[0..m). */
int orc_gather(int enc, const uint32_t* payload, const uint32_t* refs, const int64_t* dict, uint32_t b, int layout,
               const uint32_t* pos, uint64_t m, int64_t* out) {
  if (b < 1u || b > 32u || (enc != 0 && enc != 2)) return -1;
  for (uint64_t q = 0; q < m; q++) out[q] = value_at(enc, payload, refs, dict, pos[q], b, layout);
  return 0;
}

/* ------------------------------------------------------------- run length */

/* Run-length encoding of a u32 column, block by block (runs never cross a
 * 1024-value block): run r has value rv[r] and length rl[r] (1..1024);
 * block k owns runs br[k] .. br[k+1]-1.  Returns the number of runs.  The
 * arrays must hold n runs and nb + 1 block starts. */
int64_t orc_rle_encode(const uint32_t* v, uint64_t n, uint32_t* rv, uint16_t* rl, uint64_t* br) {
  uint64_t runs = 0, nb = nblocks(n);
  for (uint64_t k = 0; k < nb; k++) {
    br[k] = runs;
    uint64_t a = k * ORC_L, e = (a + ORC_L < n) ? a + ORC_L : n;
    for (uint64_t i = a; i < e; i++) {
      if (i == a || v[i] != v[i - 1]) {
        rv[runs] = v[i];
        rl[runs] = 0;
        runs++;
      }
      rl[runs - 1]++;
    }
  }
  br[nb] = runs;
  return (int64_t)runs;
}

/* Expand the runs back into values (the definition of the format). */
int orc_rle_decode(const uint32_t* rv, const uint16_t* rl, const uint64_t* br, uint64_t nb, uint32_t* v) {
  uint64_t i = 0;
  for (uint64_t k = 0; k < nb; k++)
    for (uint64_t r = br[k]; r < br[k + 1]; r++)
      for (uint32_t t = 0; t < rl[r]; t++) v[i++] = rv[r];
  return 0;
}
