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

// Sum of the dictionary entries of a lane's selected rows (bit t of rows:
// row lane + 64 t).  Every one of the 16 entries is loaded, an unselected row
// reading entry 0, before any is added: the loads are in flight together
// instead of one memory latency per selected row (codes index the dictionary,
// clamped to its last entry).
__device__ __forceinline__ uint64_t dict_sum_masked(const int64_t* dict, uint32_t dict_len, const Extract& ex,
                                                    uint32_t rows) {
  const uint32_t last = dict_len - 1u;
  int64_t e[16];
#pragma unroll
  for (uint32_t t = 0; t < 16u; ++t) {
    const uint32_t code = ((rows >> t) & 1u) ? ex(t) : 0u;
    e[t] = dict[code < last ? code : last];
  }
  uint64_t sum = 0;
#pragma unroll
  for (uint32_t t = 0; t < 16u; ++t) sum += ((rows >> t) & 1u) ? (uint64_t)e[t] : 0ull;
  return sum;
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
        lsum += dict_sum_masked(s.dict, s.dict_len, ex, rows);
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

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)x, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), o, 64);
    x |= ((uint64_t)hi << 32) | lo;
  }
  return x;
}

// Stage block k of every column in `need` into its slot of the LDS staging
// area (32 b words at cols[c].stage_off, then a zero spill word for the
// funnel shift of the block's last code), and each staged FOR column's block
// reference into col_ref.  Direct global-to-LDS loads: thread t takes the
// block's 16-byte piece t (a block has at most 256), which lands at byte
// 1024 w + 16 lane of the slot for thread t = 64 w + lane (the load's lane
// layout); every column's loads are in flight together and none goes through
// registers.  Ends with this wavefront's loads complete; the caller's
// barrier then makes the whole stage visible.
__device__ __forceinline__ void stage_columns(uint32_t* stage, uint32_t* col_ref, const QCol* cols, uint64_t need,
                                              uint64_t k) {
  typedef __attribute__((address_space(1))) const void GlobalV;
  typedef __attribute__((address_space(3))) void LdsV;
  const uint32_t tid = threadIdx.x, wave = tid >> 6;
  while (need) {
    const uint32_t c = (uint32_t)__builtin_ctzll(need);
    need &= need - 1ull;
    const QCol& col = cols[c];
    const uint32_t words = 32u * col.b;
    uint32_t* slot = stage + col.stage_off;
    if (tid < words / 4u)
      __builtin_amdgcn_global_load_lds((GlobalV*)(col.payload + k * words + 4u * tid), (LdsV*)(slot + 256u * wave),
                                       16u, 0, 0);
    if (tid == 0) {
      slot[words] = 0u;
      col_ref[c] = (col.enc != ENC_DICT && col.refs) ? col.refs[k] : 0u;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
}

__global__ __launch_bounds__(256) void query_shared_kernel(const QArgs a) {
  extern __shared__ __align__(16) uint32_t stage[];
  __shared__ uint64_t acc_count[kSharedMaxQueries], acc_sum[kSharedMaxQueries];
  __shared__ uint32_t col_ref[kSharedMaxCols];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // lane q of every wavefront holds query q
  const uint32_t ql = lane < a.nq ? lane : 0u;
  const QDesc& dq = a.q[ql];
  const bool has_q = lane < a.nq && !dq.empty;
  const uint32_t nf = has_q ? dq.nf : 0u;
  uint32_t fcol[kQueryMaxFilters];
  int64_t flo[kQueryMaxFilters], fhi[kQueryMaxFilters];
  uint64_t need_bits = 0;
#pragma unroll
  for (int f = 0; f < kQueryMaxFilters; ++f) {
    fcol[f] = (uint32_t)f < nf ? dq.col[f] : 0u;
    flo[f] = dq.zlo[f];
    fhi[f] = dq.zhi[f];
    if ((uint32_t)f < nf) need_bits |= 1ull << fcol[f];
  }
  const uint32_t scol = dq.sum_col;
  if (has_q) need_bits |= 1ull << scol;
  for (uint32_t i = threadIdx.x; i < kSharedMaxQueries; i += blockDim.x) {
    acc_count[i] = 0;
    acc_sum[i] = 0;
  }
  uint64_t blocks_acc = 0;  // wavefront 0, lane q: blocks that survive query q's zone maps
  for (uint64_t w = blockIdx.x; w < a.items; w += gridDim.x) {
    const uint64_t k0 = w * a.G;
    const uint32_t cnt = (uint32_t)((a.nb - k0) < a.G ? (a.nb - k0) : a.G);
    // 1. zone maps: bit j of live = block k0 + j meets every conjunct
    uint32_t live = has_q ? (cnt >= 32u ? ~0u : ((1u << cnt) - 1u)) : 0u;
#pragma unroll
    for (int f = 0; f < kQueryMaxFilters; ++f) {
      if ((uint32_t)f >= nf) continue;
      const QCol& c = a.cols[fcol[f]];
      for (uint32_t j = 0; j < cnt; ++j) {
        const int64_t mn = c.zmin[k0 + j], mx = c.zmax[k0 + j];
        if (mx < flo[f] || mn >= fhi[f]) live &= ~(1u << j);
      }
    }
    if (wave == 0) blocks_acc += (uint64_t)__builtin_popcount(live);
    for (uint32_t j = 0; j < cnt; ++j) {
      const uint64_t qmask = ballot((live >> j) & 1u);
      if (qmask == 0) continue;  // uniform: every wavefront holds the same masks
      const uint64_t k = k0 + j;
      const uint32_t valid = (k == a.nb - 1) ? (uint32_t)(a.n - k * kBlockValues) : kBlockValues;
      uint32_t vrows = 0;
      for (uint32_t t = 0; t < 16u; ++t) vrows |= (lane + 64u * t < valid) ? (1u << t) : 0u;
      const bool lq = (qmask >> lane) & 1ull;
      const uint64_t need = wave_or_u64(lq ? need_bits : 0ull);
      // 2. stage the block of every column a surviving query needs
      __syncthreads();  // every wavefront is done with the previous block's staging
      stage_columns(stage, col_ref, a.cols, need, k);
      __syncthreads();
      // 3. the i-th surviving query on wavefront i mod nw, conjuncts then SUM
      uint32_t idx = 0;
      for (uint64_t m = qmask; m; m &= m - 1, ++idx) {
        if (idx % nw != wave) continue;
        const int q = (int)__builtin_ctzll(m);
        const uint32_t nfq = readlane(nf, q);
        uint32_t rows = vrows;
#pragma unroll
        for (int f = 0; f < kQueryMaxFilters; ++f) {
          if ((uint32_t)f >= nfq) break;
          const uint32_t ci = readlane(fcol[f], q);
          const QCol& c = a.cols[ci];
          int64_t clo = (int64_t)readlane64((uint64_t)flo[f], q), chi = (int64_t)readlane64((uint64_t)fhi[f], q);
          if (c.enc != ENC_DICT) {
            const int64_t ref = (int64_t)col_ref[ci];
            const int64_t top = int64_t(1) << c.b;
            clo = clo - ref > 0 ? clo - ref : 0;
            chi = chi - ref < top ? chi - ref : top;
          }
          if (clo >= chi) {
            rows = 0u;
            break;
          }
          const Extract ex(stage + c.stage_off, lane, c.b);
          const uint32_t lo32 = (uint32_t)clo, wm1 = (uint32_t)(chi - clo - 1);
          uint32_t keep = 0;
#pragma unroll
          for (uint32_t t = 0; t < 16u; ++t) keep |= ((ex(t) - lo32) <= wm1) ? (1u << t) : 0u;
          rows &= keep;
          if (!ballot(rows != 0u)) break;
        }
        if (!ballot(rows != 0u)) continue;
        const uint32_t si = readlane(scol, q);
        const QCol& s = a.cols[si];
        const Extract ex(stage + s.stage_off, lane, s.b);
        const uint32_t nsel = (uint32_t)__builtin_popcount(rows);
        uint64_t lsum = 0;
        if (s.enc == ENC_DICT) {
          lsum += dict_sum_masked(s.dict, s.dict_len, ex, rows);
        } else {
#pragma unroll
          for (uint32_t t = 0; t < 16u; ++t) lsum += ((rows >> t) & 1u) ? (uint64_t)ex(t) : 0ull;
          lsum += (uint64_t)col_ref[si] * nsel;
        }
        const uint64_t tc = wave_sum_u64(nsel), ts = wave_sum_u64(lsum);
        if (lane == 0) {
          acc_count[q] += tc;
          acc_sum[q] += ts;
        }
      }
    }
  }
  __syncthreads();
  if (wave == 0 && has_q && blocks_acc)
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.out[lane].blocks), (unsigned long long)blocks_acc);
  for (uint32_t i = threadIdx.x; i < a.nq; i += blockDim.x) {
    if (acc_count[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.out[i].count), (unsigned long long)acc_count[i]);
    if (acc_sum[i]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.out[i].sum), (unsigned long long)acc_sum[i]);
  }
}

hipError_t query_shared_occupancy(int* wgs_per_cu, uint32_t stage_words) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, query_shared_kernel, 256, stage_words * 4u);
}

hipError_t launch_query_shared(const QArgs& a, uint32_t grid, hipStream_t st) {
  if (a.items == 0 || a.nq == 0) return hipSuccess;
  if (a.stage_words > kSharedMaxStageWords) return hipErrorInvalidValue;
  hipLaunchKernelGGL(query_shared_kernel, dim3(grid), dim3(256), a.stage_words * 4u, st, a);
  return hipGetLastError();
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
