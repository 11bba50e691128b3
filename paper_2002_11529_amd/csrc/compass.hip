// Compass tracking (Section V of the paper) for gfx950.
//
// For every VELO track: straight-line extrapolation to the four layers, acceptance filter, hit
// windows (binary searches over the x-sorted hits of the central sector and its neighbours, cut to
// the max_hits hits nearest to the prediction), then the tracklet search: anchor pairs in the first
// and third panel (forward) or fourth and second (backward), slope test against the VELO slope,
// completion hits in the other two panels inside the interval spanned by the pair-slope and
// VELO-slope extrapolations, one-parameter chi2 fit in q/p for each candidate, and selection under
// a total order (more hits, lower chi2, smaller hit indices).
#include "common.hpp"

namespace utc {

struct CPar {
  float W;            // window half-width (mm)
  int max_hits;       // per-layer window cap
  int half;           // (n_sectors_search - 1) / 2
  float slope_tol;
  float eps;          // completion interval margin (mm)
};

// anchor A, anchor B, completion C1, completion C2 for the forward and backward directions
__constant__ int kDirs[2][4] = {{0, 2, 1, 3}, {3, 1, 2, 0}};

// First index i in [lo, hi) with pred(i) true for a predicate that is false then true.
template <class P>
__device__ inline int64_t first_true(int64_t lo, int64_t hi, P pred) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (pred(mid)) hi = mid; else lo = mid + 1;
  }
  return lo;
}

struct Best {
  int n;          // 0 = none
  float q, chi2;
  int32_t idx[kLayers];
};

__device__ inline bool better(int n, float chi2, const int32_t idx[kLayers], const Best& b) {
  if (b.n == 0) return true;
  if (n != b.n) return n > b.n;
  if (chi2 < b.chi2) return true;
  if (chi2 > b.chi2) return false;
#pragma unroll
  for (int l = 0; l < kLayers; ++l)
    if (idx[l] != b.idx[l]) return idx[l] < b.idx[l];
  return false;
}

__device__ inline void fit(const Geom& g, const float xs[kLayers], const float yl[kLayers],
                           const float* __restrict__ hu, const float* __restrict__ hw,
                           const int32_t idx[kLayers], float& q_out, float& chi2_out) {
  float r[kLayers];
  float Sar = 0.0f, Saa = 0.0f;
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    if (idx[l] < 0) continue;
    const float m = hu[idx[l]] + yl[l] * g.dxdy[l];
    r[l] = m - xs[l];
    const float wa = hw[idx[l]] * g.a_kick[l];
    Sar = Sar + wa * r[l];
    Saa = Saa + wa * g.a_kick[l];
  }
  const float q = Sar / Saa;
  float chi2 = 0.0f;
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    if (idx[l] < 0) continue;
    const float e = r[l] - g.a_kick[l] * q;
    chi2 = chi2 + (hw[idx[l]] * e) * e;
  }
  q_out = q;
  chi2_out = chi2;
}

__device__ inline bool y_ok(const float* __restrict__ yb, const float* __restrict__ ye, int64_t i, float y) {
  return yb[i] <= y && y <= ye[i];
}

// One thread processes one VELO track.
__global__ void __launch_bounds__(256)
k_compass_thread(Geom g, CPar p, int n_events, const uint32_t* __restrict__ hit_offsets,
                 const float* __restrict__ hu, const float* __restrict__ hw,
                 const float* __restrict__ hyb, const float* __restrict__ hye,
                 const float* __restrict__ vx, const float* __restrict__ vy,
                 const float* __restrict__ vtx, const float* __restrict__ vty,
                 const uint32_t* __restrict__ velo_offsets, int32_t* __restrict__ hit_idx,
                 float* __restrict__ qop, float* __restrict__ chi2, int32_t* __restrict__ nhits,
                 int16_t* __restrict__ windows, uint32_t* flags)
{
  const int S = g.S;
  const float u_max = g.u_min + (float)S * g.sector_width;
  for (int e = blockIdx.x; e < n_events; e += gridDim.x) {
    int64_t layer_first[kLayers];
    bool overflow = false;
#pragma unroll
    for (int l = 0; l < kLayers; ++l) {
      const int64_t b0 = ((int64_t)e * kLayers + l) * S;
      layer_first[l] = hit_offsets[b0];
      if ((int64_t)hit_offsets[b0 + S] - layer_first[l] > 32767) overflow = true;
    }
    if (overflow && threadIdx.x == 0) raise_flag(flags, UTC_FLAG_LAYER_OVERFLOW);
    const uint32_t t1 = velo_offsets[e + 1];
    for (uint32_t t = velo_offsets[e] + threadIdx.x; t < t1; t += blockDim.x) {
      const float x0 = vx[t], y0 = vy[t], tx = vtx[t], ty = vty[t];
      float xs[kLayers], yl[kLayers], up[kLayers];
#pragma unroll
      for (int l = 0; l < kLayers; ++l) {
        const float dz = g.z_layer[l] - g.z_velo;
        xs[l] = x0 + tx * dz;
        yl[l] = y0 + ty * dz;
        up[l] = xs[l] - yl[l] * g.dxdy[l];
      }
      bool active = !overflow;
      if (active) {
        const int chk[2] = {0, kLayers - 1};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int l = chk[k];
          if (!(g.y_begin <= yl[l] && yl[l] <= g.y_end)) active = false;
          if (!(g.u_min <= up[l] && up[l] <= u_max)) active = false;
        }
      }
      int64_t wf[kLayers];
      int wn[kLayers];
      Best best;
      best.n = 0;
      best.q = 0.0f;
      best.chi2 = 0.0f;
#pragma unroll
      for (int l = 0; l < kLayers; ++l) { best.idx[l] = -1; wf[l] = -1; wn[l] = 0; }

      if (active) {
        // windows (Section V-A)
#pragma unroll
        for (int l = 0; l < kLayers; ++l) {
          const float ts = floorf((up[l] - g.u_min) * g.inv_sector_width);
          const int c = ts < 0.0f ? 0 : (ts > (float)(S - 1) ? S - 1 : (int)ts);
          const int s_lo = c - p.half < 0 ? 0 : c - p.half;
          const int s_hi = c + p.half > S - 1 ? S - 1 : c + p.half;
          const int64_t b0 = ((int64_t)e * kLayers + l) * S;
          const int64_t H0 = hit_offsets[b0 + s_lo], H1 = hit_offsets[b0 + s_hi + 1];
          const float lo = up[l] - p.W, hi = up[l] + p.W;
          const float upl = up[l];
          int64_t first = first_true(H0, H1, [&](int64_t i) { return hu[i] >= lo; });
          int64_t end = first_true(first, H1, [&](int64_t i) { return hu[i] > hi; });
          const int N = p.max_hits;
          if (end - first > N) {
            // the N nearest: first start f whose left hit is no farther than the hit just past
            // the window; equals dropping the farther end one at a time, the right one on ties
            const int64_t a = first_true(first, end - N, [&](int64_t f) {
              return (upl - hu[f]) <= (hu[f + N] - upl);
            });
            first = a;
            end = a + N;
          }
          wf[l] = first;
          wn[l] = (int)(end - first);
        }

        // tracklet search (Section V-B)
        for (int dir = 0; dir < 2 && best.n == 0; ++dir) {
          const int A = kDirs[dir][0], B = kDirs[dir][1];
          const int C[2] = {kDirs[dir][2], kDirs[dir][3]};
          const float inv_dz_ab = 1.0f / (g.z_layer[B] - g.z_layer[A]);
          for (int ja = 0; ja < wn[A]; ++ja) {
            const int64_t iA = wf[A] + ja;
            if (!y_ok(hyb, hye, iA, yl[A])) continue;
            const float mA = hu[iA] + yl[A] * g.dxdy[A];
            for (int jb = 0; jb < wn[B]; ++jb) {
              const int64_t iB = wf[B] + jb;
              if (!y_ok(hyb, hye, iB, yl[B])) continue;
              const float mB = hu[iB] + yl[B] * g.dxdy[B];
              const float slope = (mB - mA) * inv_dz_ab;
              if (!(fabsf(slope - tx) <= p.slope_tol)) continue;
              uint32_t mask[2];
#pragma unroll
              for (int k = 0; k < 2; ++k) {
                const int Cl = C[k];
                const float d = g.z_layer[Cl] - g.z_layer[A];
                const float xt = mA + slope * d;
                const float xv = mA + tx * d;
                const float lo = fminf(xt, xv) - p.eps;
                const float hi = fmaxf(xt, xv) + p.eps;
                uint32_t mk = 0;
                for (int j = 0; j < wn[Cl]; ++j) {
                  const int64_t i = wf[Cl] + j;
                  if (!y_ok(hyb, hye, i, yl[Cl])) continue;
                  const float m = hu[i] + yl[Cl] * g.dxdy[Cl];
                  if (lo <= m && m <= hi) mk |= 1u << j;
                }
                mask[k] = mk;
              }
              // every candidate: each completion panel one compatible hit or none, >= 3 hits
              for (int k1 = -1; k1 < wn[C[0]]; ++k1) {
                if (k1 >= 0 && !((mask[0] >> k1) & 1u)) continue;
                for (int k2 = -1; k2 < wn[C[1]]; ++k2) {
                  if (k2 >= 0 && !((mask[1] >> k2) & 1u)) continue;
                  const int n = 2 + (k1 >= 0) + (k2 >= 0);
                  if (n < 3) continue;
                  int32_t idx[kLayers];
#pragma unroll
                  for (int l = 0; l < kLayers; ++l) idx[l] = -1;
                  idx[A] = (int32_t)iA;
                  idx[B] = (int32_t)iB;
                  if (k1 >= 0) idx[C[0]] = (int32_t)(wf[C[0]] + k1);
                  if (k2 >= 0) idx[C[1]] = (int32_t)(wf[C[1]] + k2);
                  float q, c2;
                  fit(g, xs, yl, hu, hw, idx, q, c2);
                  if (better(n, c2, idx, best)) {
                    best.n = n;
                    best.q = q;
                    best.chi2 = c2;
#pragma unroll
                    for (int l = 0; l < kLayers; ++l) best.idx[l] = idx[l];
                  }
                }
              }
            }
          }
        }
      }

#pragma unroll
      for (int l = 0; l < kLayers; ++l) hit_idx[(int64_t)t * kLayers + l] = best.idx[l];
      qop[t] = best.q;
      chi2[t] = best.chi2;
      nhits[t] = best.n;
      if (windows) {
#pragma unroll
        for (int l = 0; l < kLayers; ++l) {
          const int64_t o = ((int64_t)t * kLayers + l) * 2;
          windows[o] = active ? (int16_t)(wf[l] - layer_first[l]) : (int16_t)-1;
          windows[o + 1] = (int16_t)wn[l];
        }
      }
    }
  }
}

}  // namespace utc

using namespace utc;

extern "C" size_t compass_find_workspace_bytes(int32_t n_events, int64_t n_tracks)
{
  (void)n_events;
  (void)n_tracks;
  return 256;
}

extern "C" utc_status compass_find(const utc_geometry* geom, const utc_compass_params* params,
                                   int32_t n_events, const uint32_t* hit_offsets, const float* hit_u,
                                   const float* hit_weight, const float* hit_y_begin,
                                   const float* hit_y_end, const float* vx, const float* vy,
                                   const float* vtx, const float* vty, const uint32_t* velo_offsets,
                                   int64_t n_tracks, int32_t* hit_idx, float* qop, float* chi2,
                                   int32_t* nhits, int16_t* windows, uint32_t* error_flags,
                                   void* workspace, size_t workspace_bytes,
                                   const utc_launch_config* launch, hipStream_t stream)
{
  if (!geom || !params || geom->n_layers != kLayers || geom->n_sectors < 1 ||
      geom->n_sectors > 8192 || n_events < 0 || n_tracks < 0 || n_tracks > INT32_MAX)
    return UTC_ERR_ARG;
  if (params->max_hits < 1 || params->max_hits > UTC_MAX_WINDOW_HITS ||
      params->n_sectors_search < 1 || params->n_sectors_search % 2 == 0)
    return UTC_ERR_ARG;
  if (n_events > 0 && (!hit_offsets || !velo_offsets)) return UTC_ERR_ARG;
  if (n_tracks > 0 && (!hit_u || !hit_weight || !hit_y_begin || !hit_y_end || !vx || !vy || !vtx ||
                       !vty || !hit_idx || !qop || !chi2 || !nhits))
    return UTC_ERR_ARG;
  if (launch && (launch->block < 64 || launch->block > 256 || launch->block % 64 || launch->grid < 0))
    return UTC_ERR_ARG;
  if (!workspace || workspace_bytes < compass_find_workspace_bytes(n_events, n_tracks))
    return UTC_ERR_WORKSPACE;
  if (n_events == 0 || n_tracks == 0) return UTC_OK;
  const Geom g = make_geom(*geom);
  CPar p;
  p.W = params->w0 + params->kw / params->p_min;
  p.max_hits = params->max_hits;
  p.half = (params->n_sectors_search - 1) / 2;
  p.slope_tol = params->slope_tol;
  p.eps = params->completion_tol;
  const int block = launch ? launch->block : 256;
  const int grid = (launch && launch->grid > 0) ? launch->grid : n_events;
  hipLaunchKernelGGL(k_compass_thread, dim3(grid), dim3(block), 0, stream, g, p, n_events,
                     hit_offsets, hit_u, hit_weight, hit_y_begin, hit_y_end, vx, vy, vtx, vty,
                     velo_offsets, hit_idx, qop, chi2, nhits, windows, error_flags);
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}
