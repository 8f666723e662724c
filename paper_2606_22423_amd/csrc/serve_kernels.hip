// Conjunctive multi-column query kernels (see serve_kernels.h).
#include "device_common.h"
#include "runtime_decode.h"
#include "serve_kernels.h"

namespace scan_dev {

namespace {
constexpr int kWavesPerWg = 4;
}  // namespace

__global__ __launch_bounds__(256) void query_setup_kernel(QArgs a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *a.cursor = 0u;
  if (i >= a.nq) return;
  a.out[i] = QOut{0, 0, 0, 0};
  QDesc& d = a.q[i];
  uint32_t empty = 0;
  for (uint32_t f = 0; f < d.nf; ++f) {
    const QCol c = a.cols[d.col[f]];
    int64_t zl, zh;
    if (c.enc == ENC_DICT) {
      zl = lower_bound_global(c.dict, c.dict_len, d.lo[f]);
      zh = lower_bound_global(c.dict, c.dict_len, d.hi[f]);
    } else {
      zl = d.lo[f] > 0 ? d.lo[f] : 0;
      zh = d.hi[f] < (int64_t(1) << 32) ? d.hi[f] : (int64_t(1) << 32);
    }
    if (d.lo[f] >= d.hi[f] || zl >= zh) empty = 1;
    d.zlo[f] = zl;
    d.zhi[f] = zh;
  }
  d.empty = empty;
}

// At most 64 VGPRs (the occupancy hint), so that eight work-groups (32
// wavefronts, the most a CU holds) are resident: the kernel waits on
// dependent loads and every resident wavefront hides latency.
__global__ __launch_bounds__(256, 8) void query_scan_kernel(const QArgs a) {
  __shared__ __align__(16) uint32_t lds[kWavesPerWg][kRtStageWords];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint32_t* st = lds[wave];
  while (true) {
    const uint32_t item = wave_next_item(a.cursor, lane);
    if (item >= a.items) break;
    const uint32_t qi = item % a.nq;
    const uint64_t k0 = (uint64_t)(item / a.nq) * a.G;
    const QDesc& d = a.q[qi];
    if (d.empty) continue;
    const uint32_t nf = d.nf;
    const uint32_t cnt = (uint32_t)((a.nb - k0) < a.G ? (a.nb - k0) : a.G);
    // 1. zone maps of every conjunct; lane i tests block k0 + i
    bool live = lane < cnt;
    for (uint32_t f = 0; f < nf; ++f) {
      const QCol& c = a.cols[d.col[f]];
      if (live) {
        const int64_t mn = c.zmin[k0 + lane], mx = c.zmax[k0 + lane];
        live = !(mx < d.zlo[f] || mn >= d.zhi[f]);
      }
    }
    uint64_t lm = ballot(live);
    const uint64_t blocks = (uint64_t)__builtin_popcountll(lm);
    uint32_t lcount = 0;
    uint64_t lsum = 0;
    while (lm) {
      const uint64_t k = k0 + (uint64_t)__builtin_ctzll(lm);
      lm &= lm - 1ull;
      const uint32_t valid = (k == a.nb - 1) ? (uint32_t)(a.n - k * kBlockValues) : kBlockValues;
      uint32_t rows = 0;  // bit t: value lane + 64 t is still selected
      for (uint32_t t = 0; t < 16u; ++t) rows |= (lane + 64u * t < valid) ? (1u << t) : 0u;
      // 2./3. conjuncts in order, with an early out once no row is left
      for (uint32_t f = 0; f < nf && ballot(rows != 0u); ++f) {
        const QCol& c = a.cols[d.col[f]];
        int64_t clo = d.zlo[f], chi = d.zhi[f];
        if (c.enc != ENC_DICT) {
          const int64_t ref = c.refs ? (int64_t)c.refs[k] : 0;
          const int64_t top = int64_t(1) << c.b;
          clo = clo - ref > 0 ? clo - ref : 0;
          chi = chi - ref < top ? chi - ref : top;
        }
        if (clo >= chi) {
          rows = 0u;
          break;
        }
        stage_rt_block(st, c.payload, c.b, k, lane);
        const Extract ex(st, lane, c.b);
        const uint32_t lo32 = (uint32_t)clo, wm1 = (uint32_t)(chi - clo - 1);
        uint32_t keep = 0;
#pragma unroll
        for (uint32_t t = 0; t < 16u; ++t) keep |= ((ex(t) - lo32) <= wm1) ? (1u << t) : 0u;
        rows &= keep;
      }
      if (!ballot(rows != 0u)) continue;
      // the SUM column under the mask
      const QCol& s = a.cols[d.sum_col];
      stage_rt_block(st, s.payload, s.b, k, lane);
      const Extract ex(st, lane, s.b);
      const uint32_t nsel = (uint32_t)__builtin_popcount(rows);
      lcount += nsel;
      if (s.enc == ENC_DICT) {
        const uint32_t last = s.dict_len - 1u;  // codes index the dictionary (clamped)
        for (uint32_t t = 0; t < 16u; ++t)
          if ((rows >> t) & 1u) {
            const uint32_t code = ex(t);
            lsum += (uint64_t)s.dict[code < last ? code : last];
          }
      } else {
        uint64_t part = 0;
#pragma unroll
        for (uint32_t t = 0; t < 16u; ++t) part += ((rows >> t) & 1u) ? (uint64_t)ex(t) : 0ull;
        const uint64_t ref = s.refs ? (uint64_t)s.refs[k] : 0ull;
        lsum += part + ref * nsel;
      }
    }
    const uint64_t count = wave_sum_u64(lcount);
    const uint64_t sum = wave_sum_u64(lsum);
    if (lane == 0) {
      QOut* o = a.out + qi;
      atomicAdd(reinterpret_cast<unsigned long long*>(&o->count), (unsigned long long)count);
      atomicAdd(reinterpret_cast<unsigned long long*>(&o->sum), (unsigned long long)sum);
      atomicAdd(reinterpret_cast<unsigned long long*>(&o->blocks), (unsigned long long)blocks);
    }
  }
}

hipError_t launch_query_setup(const QArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(query_setup_kernel, dim3(a.nq / 256u + 1u), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Work-groups of the query kernel that fit on one CU (registers and LDS).
// The kernel waits on dependent loads (zone maps, then each conjunct's
// block, then the SUM column), so it runs best with every one of them
// resident: on MI355X a 64-query batch took 7.8 ms at 7 work-groups per CU
// against 18.1 ms at 2.
hipError_t query_scan_occupancy(int* wgs_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, query_scan_kernel, 64 * kWavesPerWg, 0);
}

hipError_t launch_query_scan(const QArgs& a, uint32_t grid, hipStream_t st) {
  if (a.items == 0) return hipSuccess;
  hipLaunchKernelGGL(query_scan_kernel, dim3(grid), dim3(64 * kWavesPerWg), 0, st, a);
  return hipGetLastError();
}

}  // namespace scan_dev
