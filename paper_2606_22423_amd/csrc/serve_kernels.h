// Conjunctive multi-column queries over one table, many queries per launch.
//
// A query: COUNT and SUM(sum column) over the rows where every conjunct
// lo_f <= v_f < hi_f (1..3 filter columns) holds.  Table columns are
// row-major, frame of reference (u32 values, optional per-block reference)
// or dictionary (codes into a sorted int64 dictionary), each with its own
// width, all with the same row count; every column has zone maps.
//
// Work item = (window of G blocks, query), numbered window-major, so that the
// queries of a batch walk the table together and concurrent wavefronts read
// the same blocks of shared columns from the caches.  A wavefront:
//  1. tests the window's blocks against every conjunct's zone map (lane i:
//     block i of the window) -> ballot of surviving blocks;
//  2. per surviving block, stages the first conjunct's block in LDS, decodes
//     values j = lane + 64 t (t < 16) with a funnel shift (the shift is the
//     same for all t of a lane), tests the predicate in code space and keeps
//     a 16-bit row mask per lane; if no lane has a row left the block ends
//     here (early out: later conjuncts and the SUM column are not loaded);
//  3. repeats for the next conjuncts, then decodes the SUM column under the
//     mask, adds the selected values (FOR: codes, plus reference x count;
//     dictionary: entries) and popcounts the mask;
//  4. adds (count, sum mod 2^64, blocks) to the query's slot with atomics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scan_dev {

constexpr int kQueryMaxFilters = 3;

struct QCol {
  const uint32_t* payload;
  const uint32_t* refs;  // FOR: per-block references or null (all 0)
  const int64_t* dict;   // dictionary entries
  const uint32_t* zmin;  // per-block min / max (values for FOR, codes for dictionary)
  const uint32_t* zmax;
  uint32_t b, enc, dict_len;
  uint32_t stage_off;    // shared-decode kernel: word offset of this column's block in the LDS staging area
};

struct QDesc {
  uint32_t nf;                    // filter conjuncts, 1..3
  uint32_t sum_col;
  uint32_t col[kQueryMaxFilters];
  uint32_t empty;                 // set by setup when a conjunct can match nothing
  int64_t lo[kQueryMaxFilters], hi[kQueryMaxFilters];
  // predicate in the zone-map / code domain (set by setup): FOR [lo, hi)
  // clamped to [0, 2^32]; dictionary [lower_bound(lo), lower_bound(hi))
  int64_t zlo[kQueryMaxFilters], zhi[kQueryMaxFilters];
};

struct QOut {
  uint64_t count, sum, blocks, pad;
};

struct QArgs {
  const QCol* cols;
  QDesc* q;
  QOut* out;
  uint32_t* cursor;  // one counter, zero before the scan
  uint32_t nq;
  uint32_t G;        // blocks per window (1..64)
  uint64_t n, nb;    // rows and blocks of the table
  uint64_t items;    // windows x queries (shared-decode kernel: windows)
  uint32_t stage_words;  // shared-decode kernel: LDS words of the staging area (every column's block)
  uint32_t pad;
};

hipError_t launch_query_setup(const QArgs& a, hipStream_t st);
hipError_t launch_query_scan(const QArgs& a, uint32_t grid, hipStream_t st);
hipError_t query_scan_occupancy(int* wgs_per_cu);

// Shared-decode form: work item = a window of G blocks for every query of
// the launch (at most kSharedMaxQueries; tables of at most kSharedMaxCols
// columns whose blocks fit the staging area together).  Per block, a
// work-group reads each column block that any surviving query needs once and
// evaluates every query on it:
//  1. zone maps: lane q of every wavefront tests its query's conjuncts on the
//     window's blocks (a bit per block), so each block starts with a ballot of
//     the queries that survive it (the same in every wavefront);
//  2. the union of those queries' filter and SUM columns is staged in LDS,
//     packed, at each column's fixed offset: one round of loads (eight
//     columns' loads in flight at a time) and one barrier per block;
//  3. the i-th surviving query runs on wavefront i mod 4, entirely: its
//     conjuncts in order on the staged blocks (funnel-shift extraction, a
//     16-bit row mask per lane, early out when no row is left), then its SUM
//     column under the mask, into the work-group's accumulator of the query;
//  4. at the end the work-group adds its accumulators to the result slots.
// Every column block a batch needs is read from memory once per work-group
// item instead of once per query; results are identical (integer sums).
constexpr uint32_t kSharedMaxQueries = 64;
constexpr uint32_t kSharedMaxCols = 64;
constexpr uint32_t kSharedWindow = 8;
constexpr uint32_t kSharedMaxStageWords = 16384;  // 64 KiB of LDS
hipError_t launch_query_shared(const QArgs& a, uint32_t grid, hipStream_t st);
hipError_t query_shared_occupancy(int* wgs_per_cu, uint32_t stage_words);

}  // namespace scan_dev
