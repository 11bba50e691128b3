// UT raw-bank decoding (Section IV of the paper) for gfx950.
//
// Work unit: one (event, layer) = S consecutive banks whose words are contiguous.
//   k_decode_count : per bank, the number of valid words (size != 0), written into hit_offsets as
//                    scratch; per unit, their sum.
//   k_decode_scan  : exclusive scan of the unit sums -> first hit of every unit.
//   k_decode_write : per unit, local scan of the bank counts -> final hit_offsets; then, chunk by
//                    chunk of banks staged in LDS: stable compaction of the valid words (block scan),
//                    rank sort of each bank by word value, decode and coalesced SoA store.
// The paper's seven kernels (count, three-kernel prefix sum, pre-decode, find permutation, decode in
// order) map onto these three; the sort is by x (the word value) rather than by y.
#include "common.hpp"

namespace utc {

constexpr uint32_t kMaxBankWords = UTC_MAX_BANK_WORDS;
constexpr int kChunkWords = UTC_MAX_BANK_WORDS;  // LDS staging capacity per chunk (words)
constexpr int kScanTmp = 17;                      // block_exclusive_scan scratch (<= 1024 threads)

__device__ inline bool bank_ok(uint32_t a, uint32_t e) { return e >= a && e - a <= kMaxBankWords; }

__global__ void __launch_bounds__(1024)
k_decode_count(const uint16_t* __restrict__ words, const uint32_t* __restrict__ bank_offsets, int S,
               int n_units, uint32_t* __restrict__ bank_count, uint32_t* __restrict__ unit_count,
               uint32_t* flags)
{
  __shared__ uint32_t tmp[kScanTmp];
  for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
    const int64_t b0 = (int64_t)unit * S;
    uint32_t local = 0;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
      const uint32_t a = bank_offsets[b0 + s], e = bank_offsets[b0 + s + 1];
      uint32_t c = 0;
      if (e < a) {
        raise_flag(flags, UTC_FLAG_BANK_ORDER);
      } else if (e - a > kMaxBankWords) {
        raise_flag(flags, UTC_FLAG_BANK_SIZE);
      } else {
        for (uint32_t i = a; i < e; ++i) c += (words[i] & 0xFu) != 0u;
      }
      bank_count[b0 + s] = c;
      local += c;
    }
    const uint32_t total = block_sum(local, tmp);
    if (threadIdx.x == 0) unit_count[unit] = total;
  }
}

// Single workgroup: exclusive scan of the unit sums.  Each thread owns kItems consecutive entries.
__global__ void __launch_bounds__(1024)
k_decode_scan(const uint32_t* __restrict__ unit_count, int n_units, uint32_t* __restrict__ unit_base,
              uint32_t* __restrict__ hit_offsets_end)
{
  constexpr int kItems = 16;
  __shared__ uint32_t tmp[kScanTmp];
  uint32_t carry = 0;
  for (int base = 0; base < n_units; base += blockDim.x * kItems) {
    const int i0 = base + threadIdx.x * kItems;
    uint32_t ex[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      ex[k] = sum;
      sum += (i0 + k < n_units) ? unit_count[i0 + k] : 0u;
    }
    uint32_t tot;
    const uint32_t pre = block_exclusive_scan(sum, tmp, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if (i0 + k < n_units) unit_base[i0 + k] = carry + pre + ex[k];
    carry += tot;
  }
  if (threadIdx.x == 0) {
    unit_base[n_units] = carry;
    *hit_offsets_end = carry;
  }
}

__global__ void __launch_bounds__(1024)
k_decode_write(Geom g, const uint16_t* __restrict__ words, const uint32_t* __restrict__ bank_offsets,
               int n_units, int64_t capacity, const uint32_t* __restrict__ unit_base,
               uint32_t* __restrict__ hit_offsets, uint32_t* __restrict__ lhcbid,
               float* __restrict__ z, float* __restrict__ u, float* __restrict__ y_begin,
               float* __restrict__ y_end, float* __restrict__ weight, uint32_t* flags)
{
  extern __shared__ uint32_t smem[];
  const int S = g.S;
  uint32_t* s_off = smem;                 // [S+1] raw word offsets of the unit's banks
  uint32_t* s_hoff = s_off + (S + 1);     // [S+1] first local hit of each bank
  uint32_t* s_tmp = s_hoff + (S + 1);     // scan scratch
  uint16_t* s_words = reinterpret_cast<uint16_t*>(s_tmp + kScanTmp);  // staged words, then sorted
  uint16_t* s_comp = s_words + kChunkWords;   // valid words in bank order
  uint16_t* s_cbank = s_comp + kChunkWords;   // their bank (sector)
  uint16_t* s_sbank = s_cbank + kChunkWords;  // bank of the sorted words
  const int tid = threadIdx.x, bs = blockDim.x;

  for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
    const int layer = unit % kLayers;
    const int64_t b0 = (int64_t)unit * S;
    for (int s = tid; s <= S; s += bs) s_off[s] = bank_offsets[b0 + s];
    // local exclusive scan of the bank counts (left in hit_offsets by k_decode_count)
    uint32_t carry = 0;
    for (int base = 0; base < S; base += bs) {
      const int s = base + tid;
      const uint32_t c = s < S ? hit_offsets[b0 + s] : 0u;
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan(c, s_tmp, &tot);
      if (s < S) s_hoff[s] = carry + ex;
      carry += tot;
    }
    if (tid == 0) s_hoff[S] = carry;
    __syncthreads();
    const uint32_t H = unit_base[unit];
    for (int s = tid; s < S; s += bs) hit_offsets[b0 + s] = H + s_hoff[s];

    int s0 = 0;
    while (s0 < S) {
      if (!bank_ok(s_off[s0], s_off[s0 + 1])) { ++s0; continue; }
      // a chunk: consecutive well-formed banks whose words fit in LDS
      int s1 = s0 + 1;
      uint32_t nw = s_off[s0 + 1] - s_off[s0];
      while (s1 < S) {
        const uint32_t a = s_off[s1], e = s_off[s1 + 1];
        if (!bank_ok(a, e) || nw + (e - a) > (uint32_t)kChunkWords) break;
        nw += e - a;
        ++s1;
      }
      const uint32_t cs = s_off[s0];
      for (uint32_t i = tid; i < nw; i += bs) s_words[i] = words[cs + i];
      __syncthreads();

      // stable compaction of the valid words; thread tid owns a contiguous run of raw words
      const uint32_t per = (nw + bs - 1) / bs;
      const uint32_t i0 = min(tid * per, nw), i1 = min(i0 + per, nw);
      uint32_t nv = 0;
      for (uint32_t i = i0; i < i1; ++i) nv += (s_words[i] & 0xFu) != 0u;
      uint32_t tot;
      uint32_t pos = block_exclusive_scan(nv, s_tmp, &tot);
      if (i0 < i1) {
        int lo = s0, hi = s1;  // last bank b in [s0, s1) with s_off[b] <= cs + i0
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[mid] <= cs + i0) lo = mid; else hi = mid;
        }
        int b = lo;
        for (uint32_t i = i0; i < i1; ++i) {
          while (cs + i >= s_off[b + 1]) ++b;
          const uint16_t w = s_words[i];
          if (w & 0xFu) {
            s_comp[pos] = w;
            s_cbank[pos] = (uint16_t)b;
            ++pos;
          }
        }
      }
      __syncthreads();

      // order each bank's hits by word value (ties keep bank order): rank of each hit in its bank
      const uint32_t hb = s_hoff[s0];
      for (uint32_t k = tid; k < tot; k += bs) {
        const uint16_t w = s_comp[k];
        const int bk = s_cbank[k];
        const uint32_t lo = s_hoff[bk] - hb, hi = s_hoff[bk + 1] - hb;
        uint32_t rank = 0;
        for (uint32_t j = lo; j < hi; ++j) {
          const uint16_t o = s_comp[j];
          rank += (o < w) | ((o == w) & (j < k));
        }
        s_words[lo + rank] = w;
        s_sbank[lo + rank] = (uint16_t)bk;
      }
      __syncthreads();

      // decode and store the chunk's hits, consecutive threads on consecutive hits
      for (uint32_t k = tid; k < tot; k += bs) {
        const int64_t h = (int64_t)H + hb + k;
        if (h >= capacity) { raise_flag(flags, UTC_FLAG_CAPACITY); continue; }
        const uint32_t w = s_words[k];
        const uint32_t s = s_sbank[k];
        const uint32_t size = w & 0xFu, frac = (w >> 4) & 7u, strip = w >> 7;
        lhcbid[h] = ((uint32_t)layer << 28) | (s << 12) | (strip << 3) | frac;
        z[h] = g.z_layer[layer];
        u[h] = fmaf((float)(strip * 8u + frac), g.pitch8, g.u0[layer * S + s]);
        y_begin[h] = g.y_begin;
        y_end[h] = g.y_end;
        weight[h] = g.weight_by_size[size];
      }
      __syncthreads();
      s0 = s1;
    }
    __syncthreads();
  }
}

size_t decode_lds_bytes(int S) {
  return sizeof(uint32_t) * (2 * (size_t)(S + 1) + kScanTmp) + 4 * sizeof(uint16_t) * kChunkWords;
}

}  // namespace utc

using namespace utc;

extern "C" size_t ut_decode_workspace_bytes(int32_t n_events, int32_t n_sectors)
{
  (void)n_sectors;
  if (n_events < 0) return 0;
  const size_t units = (size_t)n_events * kLayers;
  return ((2 * units + 1) * sizeof(uint32_t) + 255) / 256 * 256;
}

extern "C" utc_status ut_decode(const utc_geometry* geom, const uint16_t* words,
                                const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                                uint32_t* hit_offsets, uint32_t* lhcbid, float* z, float* u,
                                float* y_begin, float* y_end, float* weight, uint32_t* error_flags,
                                void* workspace, size_t workspace_bytes,
                                const utc_launch_config* launch, hipStream_t stream)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      !geom->u0 || n_events < 0 || hit_capacity < 0 || !bank_offsets || !hit_offsets)
    return UTC_ERR_ARG;
  if (n_events > 0 && hit_capacity > 0 && (!words || !lhcbid || !z || !u || !y_begin || !y_end || !weight))
    return UTC_ERR_ARG;
  if (launch && (launch->block < 64 || launch->block > 1024 || launch->block % 64 || launch->grid < 0))
    return UTC_ERR_ARG;
  const size_t need = ut_decode_workspace_bytes(n_events, geom->n_sectors);
  if (!workspace || workspace_bytes < need) return UTC_ERR_WORKSPACE;
  const int S = geom->n_sectors;
  const int n_units = n_events * kLayers;
  uint32_t* unit_count = static_cast<uint32_t*>(workspace);
  uint32_t* unit_base = unit_count + n_units;
  const Geom g = make_geom(*geom);
  const int block = launch ? launch->block : 256;
  const int grid = (launch && launch->grid > 0) ? launch->grid : (n_units > 0 ? n_units : 1);
  const int64_t n_banks = (int64_t)n_units * S;

  if (n_units > 0) {
    hipLaunchKernelGGL(k_decode_count, dim3(grid), dim3(block), 0, stream, words, bank_offsets, S,
                       n_units, hit_offsets, unit_count, error_flags);
  }
  hipLaunchKernelGGL(k_decode_scan, dim3(1), dim3(1024), 0, stream, unit_count, n_units, unit_base,
                     hit_offsets + n_banks);
  if (n_units > 0) {
    const size_t lds = decode_lds_bytes(S);
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_decode_write),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      attr_set = true;
    }
    hipLaunchKernelGGL(k_decode_write, dim3(grid), dim3(block), lds, stream, g, words, bank_offsets,
                       n_units, hit_capacity, unit_base, hit_offsets, lhcbid, z, u, y_begin, y_end,
                       weight, error_flags);
  }
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}
