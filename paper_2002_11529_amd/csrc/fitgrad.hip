// Track-fit chi2 with per-sector alignment offsets and its hand-written adjoint, for gfx950.
//
// The fit of the tracklet search (Sections III-C and V-B) with the hit assignment frozen, seen as a
// function of the per-sector x offsets delta and the per-track q/p.  One thread per track computes
// its chi2 and d chi2/d qop directly; the per-sector sums of w*r and the total chi2 are accumulated
// exactly as integers in units of 2^-40 (a hi/lo pair of 64-bit words per sum), first in LDS per
// workgroup, then as one row of partial sums per workgroup that a second kernel adds up, so the
// result is the same for every schedule and launch shape.
#include "common.hpp"

namespace utc {

constexpr double kFix = 1099511627776.0;           // 2^40
constexpr double kTwo32 = 4294967296.0;            // 2^32
constexpr int kMaxRows = 512;                      // workgroups of the adjoint kernel (partial rows)

// Split x * 2^40 into hi * 2^32 + lo with 0 <= lo < 2^32 (lo rounded to an integer).
__device__ inline void to_fixed(double x, uint64_t& hi_out, uint64_t& lo_out) {
  const double c = x * kFix;
  double hi = floor(c * (1.0 / kTwo32));
  double lo = rint(c - hi * kTwo32);
  if (lo >= kTwo32) { lo -= kTwo32; hi += 1.0; }
  hi_out = (uint64_t)(int64_t)hi;
  lo_out = (uint64_t)lo;
}

__device__ inline double from_fixed(uint64_t hi, uint64_t lo) {
  return ((double)(int64_t)hi * kTwo32 + (double)lo) / kFix;
}

// The hits of the frozen fits, either gathered through the hit indices from the hit arrays, or
// already in track-major form (compass_fit_freeze): u, weight and global sector of the four layers
// of each track, 40 bytes per track read as three vectors.
struct FitHits {
  const int32_t* idx;        // [4n] hit indices (gathered form)
  int64_t n_hits;
  const float* u;            // hit arrays (gathered form)
  const float* w;
  const uint32_t* id;
  const float4* tu;          // [n] per-track u (frozen form)
  const float4* tw;          // [n] per-track weights
  const short4* ts;          // [n] per-track global sectors, -1 = no hit
};

// Layer-l hit of track t: its u, weight and global sector, or false when the slot holds no hit.
template <bool kFrozen>
__device__ inline bool fit_hit(const Geom& g, const FitHits& h, int64_t t, int l, const float4& tu,
                               const float4& tw, const short4& ts, float& u, float& w, int& sec) {
  if constexpr (kFrozen) {
    sec = l == 0 ? ts.x : l == 1 ? ts.y : l == 2 ? ts.z : ts.w;
    u = l == 0 ? tu.x : l == 1 ? tu.y : l == 2 ? tu.z : tu.w;
    w = l == 0 ? tw.x : l == 1 ? tw.y : l == 2 ? tw.z : tw.w;
    return sec >= 0 && sec < kLayers * g.S;
  } else {
    const int32_t hi = h.idx[t * kLayers + l];
    if (hi < 0 || hi >= h.n_hits) return false;
    const uint32_t id = h.id[hi];
    if ((id >> 28) >= (uint32_t)kLayers || ((id >> 12) & 0xFFFFu) >= (uint32_t)g.S) return false;
    sec = (int)(id >> 28) * g.S + (int)((id >> 12) & 0xFFFFu);
    u = h.u[hi];
    w = h.w[hi];
    return true;
  }
}

// Per-workgroup partial sums: workgroup b writes row b of part[grid][2*(4S+1)], the (hi, lo)
// pairs of the 4S sector sums and, last, of the total chi2.  The sums are accumulated in LDS when
// they fit (kLdsAcc), else with integer atomics directly in the workgroup's own row, cleared
// beforehand by k_fitgrad_clear; either way a workgroup writes its own row and nothing else.
template <bool kLdsAcc, bool kFrozen>
__global__ void __launch_bounds__(1024)
k_fitgrad(Geom g, int64_t n_tracks, FitHits fh, const float* __restrict__ vx,
          const float* __restrict__ vy, const float* __restrict__ vtx,
          const float* __restrict__ vty, const float* __restrict__ qop,
          const float* __restrict__ offsets, float m2s, float* __restrict__ chi2_track,
          float* __restrict__ grad_qop, bool want_sums, uint64_t* __restrict__ part)
{
  extern __shared__ uint64_t s_acc[];  // [2 * (4S + 1)] when want_sums and kLdsAcc
  const int S = g.S;
  const int n_sums = kLayers * S + 1;
  uint64_t* col = part + (size_t)blockIdx.x * 2 * n_sums;   // this workgroup's row (contiguous)
  auto acc_add = [&](int i, uint64_t v) {
    if constexpr (kLdsAcc) atomicAdd((unsigned long long*)&s_acc[i], (unsigned long long)v);
    else atomicAdd((unsigned long long*)&col[i], (unsigned long long)v);
  };
  if (kLdsAcc && want_sums) {
    for (int i = threadIdx.x; i < 2 * n_sums; i += blockDim.x) s_acc[i] = 0;
    __syncthreads();
  }
  double dz[kLayers];
#pragma unroll
  for (int l = 0; l < kLayers; ++l) dz[l] = (double)g.z_layer[l] - (double)g.z_velo;

  uint64_t tot_hi = 0, tot_lo = 0;  // this thread's share of the total chi2, fixed point
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tracks;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double x0 = vx[t], y0 = vy[t], tx = vtx[t], ty = vty[t];
    const double q = qop[t];
    float4 tu{}, tw{};
    short4 ts{};
    if constexpr (kFrozen) {
      tu = fh.tu[t];
      tw = fh.tw[t];
      ts = fh.ts[t];
    }
    float c2 = 0.0f, gq = 0.0f;
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      float hu, hw;
      int sec;
      if (!fit_hit<kFrozen>(g, fh, t, l, tu, tw, ts, hu, hw, sec)) continue;
      const double xs = x0 + tx * dz[l];
      const double yl = y0 + ty * dz[l];
      const double m = (double)hu + yl * (double)g.dxdy[l];
      const float r = (float)(((m - (double)offsets[sec]) - xs) - (double)g.a_kick[l] * q);
      const float wr = hw * r;
      c2 = c2 + wr * r;
      gq = gq + wr * g.a_kick[l];
      if (want_sums) {
        uint64_t hi, lo;
        to_fixed((double)wr, hi, lo);
        acc_add(2 * sec, hi);
        acc_add(2 * sec + 1, lo);
      }
    }
    if (chi2_track) chi2_track[t] = c2;
    if (grad_qop) grad_qop[t] = m2s * gq;
    if (want_sums) {
      uint64_t hi, lo;
      to_fixed((double)c2, hi, lo);
      tot_hi += hi;
      tot_lo += lo;
    }
  }
  if (!want_sums) return;
  // integer sums over the wavefront, then one LDS atomic pair per wavefront
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    tot_hi += __shfl_xor(tot_hi, o, kWave);
    tot_lo += __shfl_xor(tot_lo, o, kWave);
  }
  if (lane_id() == 0) {
    acc_add(2 * (n_sums - 1), tot_hi);
    acc_add(2 * (n_sums - 1) + 1, tot_lo);
  }
  if constexpr (!kLdsAcc) return;
  __syncthreads();
  // row blockIdx.x of the workgroup-major partial array part[gridDim.x][2*n_sums], written whole
  for (int i = threadIdx.x; i < 2 * n_sums; i += blockDim.x)
    col[i] = s_acc[i];
}

// Zeroes n words (the partial rows when they are accumulated in place).
__global__ void k_fitgrad_clear(uint64_t* __restrict__ part, int64_t n)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    part[i] = 0;
}

// One wavefront per sum: add the workgroups' partials (integers, so in any order) and convert.
__global__ void k_fitgrad_finalize(const uint64_t* __restrict__ part, int n_rows, int n_sums,
                                   double scale2, float* __restrict__ grad_offsets,
                                   double* __restrict__ chi2_total)
{
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (i >= n_sums) return;
  const int lane = lane_id();
  uint64_t hi = 0, lo = 0;
  for (int r = lane; r < n_rows; r += kWave) {
    hi += part[(size_t)r * 2 * n_sums + 2 * i];
    lo += part[(size_t)r * 2 * n_sums + 2 * i + 1];
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    hi += __shfl_xor(hi, o, kWave);
    lo += __shfl_xor(lo, o, kWave);
  }
  if (lane != 0) return;
  const double v = from_fixed(hi, lo);
  if (i == n_sums - 1) {
    if (chi2_total) *chi2_total = v;
  } else if (grad_offsets) {
    grad_offsets[i] = (float)(scale2 * v);
  }
}

}  // namespace utc

using namespace utc;

extern "C" size_t compass_fit_grad_workspace_bytes(int32_t n_sectors)
{
  if (n_sectors < 1) return 0;
  const size_t n = (size_t)kMaxRows * 2 * ((size_t)kLayers * n_sectors + 1) * sizeof(uint64_t);
  return (n + 255) / 256 * 256;
}

// Checks, launches and the sum finalisation shared by compass_fit_grad and compass_fit_grad_frozen.
template <bool kFrozen>
static utc_status fit_grad_launch(const utc_geometry* geom, int64_t n_tracks, const FitHits& fh,
                                  const float* vx, const float* vy, const float* vtx, const float* vty,
                                  const float* qop, const float* offsets, float grad_scale,
                                  float* chi2_track, double* chi2_total, float* grad_qop,
                                  float* grad_offsets, void* workspace, size_t workspace_bytes,
                                  hipStream_t stream)
{
  if (n_tracks > 0 && (!vx || !vy || !vtx || !vty || !qop || !offsets)) return UTC_ERR_ARG;
  if (!workspace || workspace_bytes < compass_fit_grad_workspace_bytes(geom->n_sectors))
    return UTC_ERR_WORKSPACE;
  const Geom g = make_geom(*geom);
  const int S = geom->n_sectors;
  const int n_sums = kLayers * S + 1;
  uint64_t* part = static_cast<uint64_t*>(workspace);
  const bool want_sums = grad_offsets != nullptr || chi2_total != nullptr;
  const float m2s = -2.0f * grad_scale;
  // the sums in LDS when they fit (up to 2559 sectors per layer), else in the workspace rows
  const size_t lds_need = want_sums ? 2 * (size_t)n_sums * sizeof(uint64_t) : 0;
  const bool lds_acc = lds_need <= 160 * 1024;
  const size_t lds = lds_acc ? lds_need : 0;
  (void)hipGetLastError();  // report only errors of this call
  const int block = 1024;
  int64_t blocks = (n_tracks + block - 1) / block;
  if (blocks > kMaxRows) blocks = kMaxRows;
  if (blocks < 1) blocks = 1;
  if (lds_acc && !allow_dynamic_lds(reinterpret_cast<const void*>(k_fitgrad<true, kFrozen>), lds))
    return UTC_ERR_HIP;
  if (want_sums && !lds_acc) {
    const int64_t n = 2 * (int64_t)n_sums * blocks;
    hipLaunchKernelGGL(k_fitgrad_clear, dim3((unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096)),
                       dim3(256), 0, stream, part, n);
  }
  if (lds_acc)
    hipLaunchKernelGGL((k_fitgrad<true, kFrozen>), dim3((unsigned)blocks), dim3(block), lds, stream, g,
                       n_tracks, fh, vx, vy, vtx, vty, qop, offsets, m2s, chi2_track, grad_qop,
                       want_sums, part);
  else
    hipLaunchKernelGGL((k_fitgrad<false, kFrozen>), dim3((unsigned)blocks), dim3(block), 0, stream, g,
                       n_tracks, fh, vx, vy, vtx, vty, qop, offsets, m2s, chi2_track, grad_qop,
                       want_sums, part);
  if (want_sums)
    hipLaunchKernelGGL(k_fitgrad_finalize, dim3((n_sums + 3) / 4), dim3(256), 0, stream, part,
                       (int)blocks, n_sums, -2.0 * (double)grad_scale, grad_offsets, chi2_total);
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}

extern "C" utc_status compass_fit_grad(const utc_geometry* geom, int64_t n_tracks,
                                       const int32_t* track_hit_idx, int64_t n_hits,
                                       const float* hit_u, const float* hit_weight,
                                       const uint32_t* hit_lhcbid,
                                       const float* vx, const float* vy, const float* vtx,
                                       const float* vty, const float* qop, const float* offsets,
                                       float grad_scale, float* chi2_track, double* chi2_total,
                                       float* grad_qop, float* grad_offsets, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      n_tracks < 0 || n_hits < 0)
    return UTC_ERR_ARG;
  if (n_tracks > 0 && (!track_hit_idx || !hit_u || !hit_weight || !hit_lhcbid)) return UTC_ERR_ARG;
  FitHits fh{track_hit_idx, n_hits, hit_u, hit_weight, hit_lhcbid, nullptr, nullptr, nullptr};
  return fit_grad_launch<false>(geom, n_tracks, fh, vx, vy, vtx, vty, qop, offsets, grad_scale,
                                chi2_track, chi2_total, grad_qop, grad_offsets, workspace,
                                workspace_bytes, stream);
}

// One thread per track: the u, weight and global sector of its four hits, as compass_fit_grad
// reads them, written track-major.
__global__ void k_fit_freeze(Geom g, int64_t n_tracks, FitHits fh, float4* __restrict__ tu,
                             float4* __restrict__ tw, short4* __restrict__ ts)
{
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tracks;
       t += (int64_t)gridDim.x * blockDim.x) {
    float u[kLayers], w[kLayers];
    int sec[kLayers];
    const float4 z4{};
    const short4 s4{};
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      if (!fit_hit<false>(g, fh, t, l, z4, z4, s4, u[l], w[l], sec[l])) {
        u[l] = 0.0f;
        w[l] = 0.0f;
        sec[l] = -1;
      }
    }
    tu[t] = make_float4(u[0], u[1], u[2], u[3]);
    tw[t] = make_float4(w[0], w[1], w[2], w[3]);
    ts[t] = make_short4((short)sec[0], (short)sec[1], (short)sec[2], (short)sec[3]);
  }
}

extern "C" utc_status compass_fit_freeze(const utc_geometry* geom, int64_t n_tracks,
                                         const int32_t* track_hit_idx, int64_t n_hits,
                                         const float* hit_u, const float* hit_weight,
                                         const uint32_t* hit_lhcbid, float* track_u,
                                         float* track_weight, int16_t* track_sector,
                                         hipStream_t stream)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      n_tracks < 0 || n_hits < 0)
    return UTC_ERR_ARG;
  if (n_tracks > 0 && (!track_hit_idx || !hit_u || !hit_weight || !hit_lhcbid || !track_u ||
                       !track_weight || !track_sector))
    return UTC_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(track_u) | reinterpret_cast<uintptr_t>(track_weight)) & 15u ||
      reinterpret_cast<uintptr_t>(track_sector) & 7u)
    return UTC_ERR_ARG;
  if (n_tracks == 0) return UTC_OK;
  (void)hipGetLastError();
  const Geom g = make_geom(*geom);
  FitHits fh{track_hit_idx, n_hits, hit_u, hit_weight, hit_lhcbid, nullptr, nullptr, nullptr};
  int64_t blocks = (n_tracks + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fit_freeze, dim3((unsigned)blocks), dim3(256), 0, stream, g, n_tracks, fh,
                     reinterpret_cast<float4*>(track_u), reinterpret_cast<float4*>(track_weight),
                     reinterpret_cast<short4*>(track_sector));
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}

extern "C" utc_status compass_fit_grad_frozen(const utc_geometry* geom, int64_t n_tracks,
                                              const float* track_u, const float* track_weight,
                                              const int16_t* track_sector,
                                              const float* vx, const float* vy, const float* vtx,
                                              const float* vty, const float* qop,
                                              const float* offsets, float grad_scale,
                                              float* chi2_track, double* chi2_total,
                                              float* grad_qop, float* grad_offsets,
                                              void* workspace, size_t workspace_bytes,
                                              hipStream_t stream)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      n_tracks < 0)
    return UTC_ERR_ARG;
  if (n_tracks > 0 && (!track_u || !track_weight || !track_sector)) return UTC_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(track_u) | reinterpret_cast<uintptr_t>(track_weight)) & 15u ||
      reinterpret_cast<uintptr_t>(track_sector) & 7u)
    return UTC_ERR_ARG;
  FitHits fh{nullptr, 0, nullptr, nullptr, nullptr, reinterpret_cast<const float4*>(track_u),
             reinterpret_cast<const float4*>(track_weight), reinterpret_cast<const short4*>(track_sector)};
  return fit_grad_launch<true>(geom, n_tracks, fh, vx, vy, vtx, vty, qop, offsets, grad_scale,
                               chi2_track, chi2_total, grad_qop, grad_offsets, workspace,
                               workspace_bytes, stream);
}
