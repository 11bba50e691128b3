// The steps on either side of the UT chain (Section VI, "UT decoding and tracking performance"):
// the global event cut before decoding and the consolidation of the found upstream tracks into a
// dense container after the tracking.  Both are prefix sums plus gathers: bandwidth-bound copies.
#include "common.hpp"

namespace utc {

// Exclusive scan of n values in place by one workgroup; the total goes to *total.  All threads of
// the workgroup must call it.  Each wave scans kRows consecutive rows of 64 values (coalesced, a DPP
// scan per row carried along the rows), then the wave totals are scanned across the workgroup.
__device__ inline void block_scan_inplace(uint32_t* a, int64_t n, uint32_t* total, uint32_t* tmp) {
  constexpr int kRows = 16;
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)nw * kWave * kRows) {
    const int64_t seg = base + (int64_t)wid * kWave * kRows;
    uint32_t v[kRows], ex[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int64_t i = seg + r * kWave + lane;
      v[r] = i < n ? a[i] : 0u;
    }
    uint32_t run = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const uint32_t x = wave_inclusive_scan(v[r]);
      ex[r] = run + x - v[r];
      run += (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
    }
    uint32_t tot;
    const uint32_t woff = block_exclusive_scan(lane == kWave - 1 ? run : 0u, tmp, &tot);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int64_t i = seg + r * kWave + lane;
      if (i < n) a[i] = carry + woff + ex[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// ---- global event cut ----

// One thread per event: keep flag, kept word and track counts (0 for a rejected event).
__global__ void k_gec_count(const uint32_t* __restrict__ bank_offsets, const uint32_t* __restrict__ velo_offsets,
                            int n_events, int64_t banks_per_event, uint32_t max_words,
                            uint32_t* __restrict__ n_words, uint32_t* __restrict__ n_tracks,
                            uint8_t* __restrict__ keep, uint32_t* flags) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  const uint32_t a = bank_offsets[(int64_t)e * banks_per_event];
  const uint32_t b = bank_offsets[(int64_t)(e + 1) * banks_per_event];
  const bool ordered = b >= a;
  if (!ordered) raise_flag(flags, UTC_FLAG_BANK_ORDER);
  const bool ok = ordered && (b - a) <= max_words;
  n_words[e] = ok ? b - a : 0u;
  n_tracks[e] = ok ? velo_offsets[e + 1] - velo_offsets[e] : 0u;
  keep[e] = ok ? 1 : 0;
}

// One workgroup: kept counts to bases (exclusive scans), totals, and the number of kept events.
__global__ void __launch_bounds__(1024)
k_gec_scan(uint32_t* __restrict__ n_words, uint32_t* __restrict__ n_tracks, const uint8_t* __restrict__ keep,
           int n_events, uint32_t* __restrict__ totals, int32_t* n_kept) {
  __shared__ uint32_t tmp[17];
  block_scan_inplace(n_words, n_events, &totals[0], tmp);
  block_scan_inplace(n_tracks, n_events, &totals[1], tmp);
  uint32_t c = 0;
  for (int e = threadIdx.x; e < n_events; e += blockDim.x) c += keep[e];
  uint32_t tot;
  (void)block_exclusive_scan(c, tmp, &tot);
  if (threadIdx.x == 0 && n_kept) *n_kept = (int32_t)tot;
}

// Offsets of the compact batch: one thread per bank, plus the event entries.
__global__ void k_gec_offsets(const uint32_t* __restrict__ bank_offsets, const uint8_t* __restrict__ keep,
                              const uint32_t* __restrict__ word_base, const uint32_t* __restrict__ track_base,
                              const uint32_t* __restrict__ totals, int n_events, int64_t banks_per_event,
                              uint32_t* __restrict__ out_bank_offsets, uint32_t* __restrict__ out_velo_offsets) {
  const int64_t nb = (int64_t)n_events * banks_per_event;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) {
    const int64_t e = i / banks_per_event;
    // a kept event keeps its bank layout; a rejected one has all its banks empty at its base
    out_bank_offsets[i] = keep[e] ? word_base[e] + (bank_offsets[i] - bank_offsets[e * banks_per_event])
                                  : word_base[e];
  } else if (i == nb) {
    out_bank_offsets[nb] = totals[0];
  }
  if (i < n_events) out_velo_offsets[i] = track_base[i];
  if (i == n_events) out_velo_offsets[n_events] = totals[1];
}

// Words and VELO states of the kept events (one workgroup per event, grid-strided).
__global__ void k_gec_copy(const uint16_t* __restrict__ words, const uint32_t* __restrict__ bank_offsets,
                           const float* __restrict__ vx, const float* __restrict__ vy,
                           const float* __restrict__ vtx, const float* __restrict__ vty,
                           const uint32_t* __restrict__ velo_offsets, const uint8_t* __restrict__ keep,
                           const uint32_t* __restrict__ word_base, const uint32_t* __restrict__ track_base,
                           int n_events, int64_t banks_per_event, uint16_t* __restrict__ out_words,
                           float* __restrict__ ox, float* __restrict__ oy, float* __restrict__ otx,
                           float* __restrict__ oty) {
  for (int e = blockIdx.x; e < n_events; e += gridDim.x) {
    if (!keep[e]) continue;
    const uint32_t src = bank_offsets[(int64_t)e * banks_per_event];
    const uint32_t nw = bank_offsets[(int64_t)(e + 1) * banks_per_event] - src;
    const uint32_t dst = word_base[e];
    for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) out_words[(int64_t)dst + k] = words[(int64_t)src + k];
    const uint32_t t0 = velo_offsets[e], nt = velo_offsets[e + 1] - t0, d0 = track_base[e];
    for (uint32_t k = threadIdx.x; k < nt; k += blockDim.x) {
      ox[d0 + k] = vx[t0 + k];
      oy[d0 + k] = vy[t0 + k];
      otx[d0 + k] = vtx[t0 + k];
      oty[d0 + k] = vty[t0 + k];
    }
  }
}

// ---- consolidation ----

constexpr int kConsItems = 2;     // tracks per thread in the consolidation kernels
constexpr int kConsThreads = 256; // threads per workgroup: many workgroups even for 1e5 tracks

// Found tracks of each block of kConsThreads * kConsItems tracks.
__global__ void __launch_bounds__(kConsThreads)
k_cons_count(const int32_t* __restrict__ nhits, int64_t n_tracks, uint32_t* __restrict__ block_sum) {
  __shared__ uint32_t tmp[17];
  const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kConsItems;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kConsItems; ++k) c += (t0 + k < n_tracks && nhits[t0 + k] > 0) ? 1u : 0u;
  uint32_t tot;
  (void)block_exclusive_scan(c, tmp, &tot);
  if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024)
k_cons_scan(uint32_t* __restrict__ block_sum, int64_t n_blocks, uint32_t* __restrict__ total,
            int32_t* n_found) {
  __shared__ uint32_t tmp[17];
  block_scan_inplace(block_sum, n_blocks, total, tmp);
  __syncthreads();
  if (threadIdx.x == 0 && n_found) *n_found = (int32_t)*total;
}

// Scatter of the found tracks to their dense slots; the dense position of every track (found or
// not) is kept for the per-event offsets.  hit_idx rows move as one 16-byte vector when both
// arrays are 16-byte aligned.
__global__ void __launch_bounds__(kConsThreads)
k_cons_scatter(const int32_t* __restrict__ nhits, const int32_t* __restrict__ hit_idx,
               const float* __restrict__ qop, const float* __restrict__ chi2, int64_t n_tracks,
               const uint32_t* __restrict__ block_base, uint32_t* __restrict__ pos,
               int32_t* __restrict__ out_velo, int32_t* __restrict__ out_hit_idx,
               float* __restrict__ out_qop, float* __restrict__ out_chi2, int32_t* __restrict__ out_nhits) {
  __shared__ uint32_t tmp[17];
  const int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kConsItems;
  bool f[kConsItems];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kConsItems; ++k) {
    f[k] = t0 + k < n_tracks && nhits[t0 + k] > 0;
    c += f[k] ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t p = block_base[blockIdx.x] + block_exclusive_scan(c, tmp, &tot);
  const bool vec = ((reinterpret_cast<uintptr_t>(hit_idx) | reinterpret_cast<uintptr_t>(out_hit_idx)) & 15u) == 0;
#pragma unroll
  for (int k = 0; k < kConsItems; ++k) {
    const int64_t t = t0 + k;
    if (t >= n_tracks) break;
    pos[t] = p;
    if (f[k]) {
      if (vec) {
        reinterpret_cast<int4*>(out_hit_idx)[p] = reinterpret_cast<const int4*>(hit_idx)[t];
      } else {
#pragma unroll
        for (int l = 0; l < kLayers; ++l) out_hit_idx[4 * (int64_t)p + l] = hit_idx[4 * t + l];
      }
      out_velo[p] = (int32_t)t;
      out_qop[p] = qop[t];
      out_chi2[p] = chi2[t];
      out_nhits[p] = nhits[t];
      ++p;
    }
  }
}

__global__ void k_cons_offsets(const uint32_t* __restrict__ velo_offsets, int n_events, int64_t n_tracks,
                               const uint32_t* __restrict__ pos, const uint32_t* __restrict__ total,
                               uint32_t* __restrict__ out_offsets) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > n_events) return;
  const uint32_t t = velo_offsets[e];
  out_offsets[e] = ((int64_t)t < n_tracks) ? pos[t] : *total;
}

}  // namespace utc

using namespace utc;

extern "C" size_t ut_global_event_cut_workspace_bytes(int32_t n_events)
{
  if (n_events < 0) return 0;
  const size_t e = (size_t)n_events + 1;
  return ((2 * e + 2) * sizeof(uint32_t) + e + 255) / 256 * 256;
}

extern "C" utc_status ut_global_event_cut(const utc_geometry* geom, int32_t n_events, const uint16_t* words,
                                          const uint32_t* bank_offsets, const float* vx, const float* vy,
                                          const float* vtx, const float* vty, const uint32_t* velo_offsets,
                                          uint32_t max_words, uint16_t* out_words, uint32_t* out_bank_offsets,
                                          float* out_vx, float* out_vy, float* out_vtx, float* out_vty,
                                          uint32_t* out_velo_offsets, uint8_t* keep, int32_t* n_kept,
                                          uint32_t* error_flags, void* workspace, size_t workspace_bytes,
                                          hipStream_t stream)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      n_events < 0 || !bank_offsets || !velo_offsets || !out_bank_offsets || !out_velo_offsets)
    return UTC_ERR_ARG;
  if (n_events > 0 && (!words || !vx || !vy || !vtx || !vty || !out_words || !out_vx || !out_vy ||
                       !out_vtx || !out_vty))
    return UTC_ERR_ARG;
  if (!workspace || workspace_bytes < ut_global_event_cut_workspace_bytes(n_events)) return UTC_ERR_WORKSPACE;
  const int64_t bpe = (int64_t)kLayers * geom->n_sectors;
  const int64_t nb = (int64_t)n_events * bpe;
  if (nb + 2 > (int64_t)INT32_MAX * 256) return UTC_ERR_ARG;
  (void)hipGetLastError();  // report only errors of this call
  uint32_t* word_base = static_cast<uint32_t*>(workspace);      // [E + 1]
  uint32_t* track_base = word_base + (n_events + 1);            // [E + 1]
  uint32_t* totals = track_base + (n_events + 1);               // [2]
  uint8_t* kflag = keep ? keep : reinterpret_cast<uint8_t*>(totals + 2);   // [E]
  if (n_events > 0)
    hipLaunchKernelGGL(k_gec_count, dim3((n_events + 255) / 256), dim3(256), 0, stream, bank_offsets,
                       velo_offsets, n_events, bpe, max_words, word_base, track_base, kflag, error_flags);
  hipLaunchKernelGGL(k_gec_scan, dim3(1), dim3(1024), 0, stream, word_base, track_base, kflag, n_events,
                     totals, n_kept);
  const int64_t n_off = (nb + 1 > (int64_t)n_events + 1) ? nb + 1 : (int64_t)n_events + 1;
  hipLaunchKernelGGL(k_gec_offsets, dim3((unsigned)((n_off + 255) / 256)), dim3(256), 0, stream,
                     bank_offsets, kflag, word_base, track_base, totals, n_events, bpe, out_bank_offsets,
                     out_velo_offsets);
  if (n_events > 0) {
    const int grid = n_events < 4096 ? n_events : 4096;
    hipLaunchKernelGGL(k_gec_copy, dim3(grid), dim3(256), 0, stream, words, bank_offsets, vx, vy, vtx, vty,
                       velo_offsets, kflag, word_base, track_base, n_events, bpe, out_words, out_vx,
                       out_vy, out_vtx, out_vty);
  }
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}

extern "C" size_t compass_consolidate_workspace_bytes(int64_t n_tracks)
{
  if (n_tracks < 0) return 0;
  const int64_t per_block = kConsThreads * kConsItems;
  const int64_t blocks = (n_tracks + per_block - 1) / per_block;
  return (((size_t)n_tracks + (size_t)blocks + 2) * sizeof(uint32_t) + 255) / 256 * 256;
}

extern "C" utc_status compass_consolidate(int32_t n_events, const uint32_t* velo_offsets, int64_t n_tracks,
                                          const int32_t* nhits, const int32_t* hit_idx, const float* qop,
                                          const float* chi2, uint32_t* out_offsets, int32_t* out_velo,
                                          int32_t* out_hit_idx, float* out_qop, float* out_chi2,
                                          int32_t* out_nhits, int32_t* n_found, void* workspace,
                                          size_t workspace_bytes, hipStream_t stream)
{
  if (n_events < 0 || n_tracks < 0 || n_tracks > INT32_MAX || !velo_offsets || !out_offsets) return UTC_ERR_ARG;
  if (n_tracks > 0 && (!nhits || !hit_idx || !qop || !chi2 || !out_velo || !out_hit_idx || !out_qop ||
                       !out_chi2 || !out_nhits))
    return UTC_ERR_ARG;
  if (!workspace || workspace_bytes < compass_consolidate_workspace_bytes(n_tracks)) return UTC_ERR_WORKSPACE;
  (void)hipGetLastError();  // report only errors of this call
  const int64_t per_block = kConsThreads * kConsItems;
  const int64_t blocks = (n_tracks + per_block - 1) / per_block;
  uint32_t* pos = static_cast<uint32_t*>(workspace);   // [n_tracks]
  uint32_t* block_sum = pos + n_tracks;                // [blocks]
  uint32_t* total = block_sum + blocks;                // [1]
  if (blocks > 0)
    hipLaunchKernelGGL(k_cons_count, dim3((unsigned)blocks), dim3(kConsThreads), 0, stream, nhits, n_tracks,
                       block_sum);
  hipLaunchKernelGGL(k_cons_scan, dim3(1), dim3(1024), 0, stream, block_sum, blocks, total, n_found);
  if (blocks > 0)
    hipLaunchKernelGGL(k_cons_scatter, dim3((unsigned)blocks), dim3(kConsThreads), 0, stream, nhits, hit_idx, qop,
                       chi2, n_tracks, block_sum, pos, out_velo, out_hit_idx, out_qop, out_chi2, out_nhits);
  hipLaunchKernelGGL(k_cons_offsets, dim3((n_events + 1 + 255) / 256), dim3(256), 0, stream, velo_offsets,
                     n_events, n_tracks, pos, total, out_offsets);
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}
