// Compass tracking (Section V of the paper) for gfx950: stand-alone kernel over decoded hits.
//
// One workgroup per event at a time (events strided over the grid): the event's bank offsets and, when
// they fit, the u (and weights) of its hits are staged in LDS; then each wavefront runs the search for groups of
// 16 VELO tracks (compass_group.hpp): windows by binary search over the staged hits, tracklets by
// anchor pairs spread over the lanes, selection by an LDS atomic minimum of a total-order key.
#include <cmath>

#include "compass_group.hpp"

namespace utc {

// LDS words of the event's bank offsets (nb + 1) and the six control words after them, rounded to
// 16 bytes.
__host__ __device__ inline int hoff_words(int nb) { return (nb + 1 + 6 + 3) & ~3; }

// kGreedy: the paper's search variant (max_tracklets > 0), a kernel of its own so that its code
// does not weigh on the register allocation of the default search
// The next group of tracks for the calling wave: groups are handed out in order from a counter in
// LDS, so the waves of a workgroup finish an event together whatever each group costs.
__device__ inline uint32_t claim_group(uint32_t* counter) {
  uint32_t v = 0;
  if (lane_id() == 0) v = atomicAdd(counter, 1u);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);   // every lane is active here
}

template <bool kGreedy>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_compass(Geom g, CPar p, int n_events, const uint32_t* __restrict__ hit_offsets,
          const float* __restrict__ hu, const float* __restrict__ hw,
          const float* __restrict__ hyb, const float* __restrict__ hye,
          const uint32_t* __restrict__ velo_offsets, TrackIO io, uint32_t* flags, int u_cap,
          uint32_t* ev_counter)
{
  extern __shared__ __align__(16) char smem[];
  const int S = g.S;
  const int nb = kLayers * S;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int wid = tid / kWave, nwaves = bs / kWave;
  uint32_t* s_hoff = reinterpret_cast<uint32_t*>(smem);
  float* s_u = reinterpret_cast<float*>(s_hoff + hoff_words(nb));
  uint32_t* s_next = s_hoff + nb + 1;   // group counter, after the offsets
  uint32_t* s_event = s_hoff + nb + 2;  // the workgroup's next event (persistent grids)
  uint32_t* s_ycov = s_hoff + nb + 3;   // [3] y range every strip of the event covers (ordered
                                        // keys of the largest y_begin and the smallest y_end), and
                                        // whether some strip's range is not a number
  char* gbase = reinterpret_cast<char*>(s_u + u_cap);
  const GroupScratch gs = carve_group(gbase + (size_t)wid * group_scratch_bytes(p.max_hits, kGreedy),
                                      p.max_hits, kGreedy);

  // a persistent grid (ev_counter set, cleared to gridDim.x beforehand) takes events 0..grid-1 in
  // order and then claims the next event whenever a workgroup finishes one, so uneven events
  // spread over the workgroups as they free up; otherwise one workgroup per event
  for (int e = blockIdx.x; e < n_events;) {
    const int64_t eb = (int64_t)e * nb;
    const uint32_t H = hit_offsets[eb];
    for (int j0 = 0; j0 <= nb; j0 += 4 * bs) {
      uint32_t v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + q * bs + tid;
        v[q] = j <= nb ? hit_offsets[eb + j] : 0u;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + q * bs + tid;
        if (j <= nb) s_hoff[j] = v[q] - H;
      }
    }
    if (tid == 0) {
      *s_next = (uint32_t)nwaves;   // groups 0 .. nwaves-1 go to the waves in order
      s_ycov[0] = 0u;
      s_ycov[1] = ~0u;
      s_ycov[2] = 0u;
    }
    __syncthreads();
    const uint32_t nh = s_hoff[nb];
    bool overflow = false;
#pragma unroll
    for (int l = 0; l < kLayers; ++l)
      if (s_hoff[(l + 1) * S] - s_hoff[l * S] > 32767u) overflow = true;
    const bool staged = nh <= (uint32_t)u_cap;
    const bool staged_w = 2 * (uint64_t)nh <= (uint64_t)u_cap;   // the weights too, after the u
    // u of every hit when the event fits, else of every stride-th hit (a coarse index for the
    // window searches, which then finish with a few steps in global memory)
    uint32_t stride = 1;
    while (u_cap > 0 && (nh + stride - 1) / stride > (uint32_t)u_cap) stride *= 2;
    const uint32_t ncoarse = u_cap > 0 ? (nh + stride - 1) / stride : 0u;
    for (uint32_t k0 = 0; k0 < ncoarse; k0 += 8 * bs) {
      float v[8], w[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t k = k0 + q * bs + tid;
        v[q] = k < ncoarse ? hu[(int64_t)H + (int64_t)k * stride] : 0.0f;
        w[q] = (staged_w && k < ncoarse) ? hw[(int64_t)H + k] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t k = k0 + q * bs + tid;
        if (k < ncoarse) {
          s_u[k] = v[q];
          if (staged_w) s_u[nh + k] = w[q];
        }
      }
    }
    // the y range that every strip of the event covers: a track whose y lies inside it at a layer
    // passes the per-hit y test of every hit there, so the window tile then skips the per-hit
    // y_begin / y_end loads (one coalesced pass over the event's ranges instead of gathers per
    // window slot; with a range that is not a number the per-hit test is kept for every track)
    if (hyb) {
      uint32_t kb = 0u, ke = ~0u;
      bool bad = false;
      for (uint32_t k0 = 0; k0 < nh; k0 += 4 * bs) {
        float vb[4], ve[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t k = k0 + q * bs + tid;
          vb[q] = k < nh ? hyb[(int64_t)H + k] : -INFINITY;
          ve[q] = k < nh ? hye[(int64_t)H + k] : INFINITY;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bad |= !(vb[q] == vb[q]) || !(ve[q] == ve[q]);
          kb = max(kb, float_order_key(vb[q]));
          ke = min(ke, float_order_key(ve[q]));
        }
      }
      kb = wave_max_u32(kb);
      ke = ~wave_max_u32(~ke);
      const bool any_bad = wave_any(bad);
      if (lane_id() == 0) {
        atomicMax(&s_ycov[0], kb);
        atomicMin(&s_ycov[1], ke);
        if (any_bad) atomicOr(&s_ycov[2], 1u);
      }
    }
    if (overflow && tid == 0) raise_flag(flags, UTC_FLAG_LAYER_OVERFLOW);
    __syncthreads();
    EventView ev;
    ev.u_lds = s_u;
    ev.u_glb = hu;
    ev.w_lds = staged_w ? s_u + nh : nullptr;
    ev.w_glb = hw;
    ev.yb_glb = hyb;
    ev.ye_glb = hye;
    ev.hoff = s_hoff;
    ev.first = H;
    ev.overflow = overflow;
    // an empty or all-NaN-free range gives y_lo > y_hi, which no track lies inside
    ev.y_lo = (hyb && s_ycov[2] == 0u) ? float_from_order_key(s_ycov[0]) : INFINITY;
    ev.y_hi = (hyb && s_ycov[2] == 0u) ? float_from_order_key(s_ycov[1]) : -INFINITY;
    ev.stride = staged ? 1u : (ncoarse > 0 ? stride : 0u);
    const uint32_t t0 = velo_offsets[e], t1 = velo_offsets[e + 1];
    const uint32_t ngroups = (t1 - t0 + kGroupTracks - 1) / kGroupTracks;
    // a wave claims its next group before searching the current one (the group's VELO states are
    // loaded after the search: held in registers across it they cost more in spilled registers
    // than their load latency)
    uint32_t grp = (uint32_t)wid;
    uint32_t nxt = grp < ngroups ? claim_group(s_next) : ngroups;
    LaneState st = load_state(io, t0 + grp * kGroupTracks, t1);
    if (staged_w) {
      while (grp < ngroups) {
        compass_group<true, true, kGreedy>(g, p, ev, gs, t0 + grp * kGroupTracks, t1, io, st);
        st = load_state(io, t0 + nxt * kGroupTracks, t1);
        grp = nxt;
        nxt = grp < ngroups ? claim_group(s_next) : ngroups;
      }
    } else if (staged) {
      while (grp < ngroups) {
        compass_group<true, false, kGreedy>(g, p, ev, gs, t0 + grp * kGroupTracks, t1, io, st);
        st = load_state(io, t0 + nxt * kGroupTracks, t1);
        grp = nxt;
        nxt = grp < ngroups ? claim_group(s_next) : ngroups;
      }
    } else {
      while (grp < ngroups) {
        compass_group<false, false, kGreedy>(g, p, ev, gs, t0 + grp * kGroupTracks, t1, io, st);
        st = load_state(io, t0 + nxt * kGroupTracks, t1);
        grp = nxt;
        nxt = grp < ngroups ? claim_group(s_next) : ngroups;
      }
    }
    __syncthreads();
    if (ev_counter) {
      if (tid == 0) *s_event = atomicAdd(ev_counter, 1u);
      __syncthreads();
      e = (int)min(*s_event, (uint32_t)n_events);
    } else {
      e += gridDim.x;
    }
  }
}

// Sets the event counter of a persistent launch to its grid size.
__global__ void k_compass_start(uint32_t* ev_counter, uint32_t grid) {
  if (threadIdx.x == 0) *ev_counter = grid;
}

size_t compass_lds_bytes(int S, int max_hits, int waves, int u_cap, bool greedy) {
  const size_t hoff = 4 * (size_t)hoff_words(kLayers * S);
  return hoff + 4 * (size_t)u_cap + (size_t)waves * group_scratch_bytes(max_hits, greedy);
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
  if (params->max_tracklets < 0) return UTC_ERR_ARG;
  if (params->max_hits < 1 || params->max_hits > UTC_MAX_WINDOW_HITS ||
      params->n_sectors_search < 1 || params->n_sectors_search % 2 == 0)
    return UTC_ERR_ARG;
  if (n_events > 0 && (!hit_offsets || !velo_offsets)) return UTC_ERR_ARG;
  if (n_tracks > 0 && (!hit_u || !hit_weight || !vx || !vy || !vtx || !vty || !hit_idx || !qop ||
                       !chi2 || !nhits))
    return UTC_ERR_ARG;
  if ((hit_y_begin == nullptr) != (hit_y_end == nullptr)) return UTC_ERR_ARG;
  if (launch && (launch->block < 64 || launch->block > 512 || launch->block % 64 || launch->grid < 0 ||
                 launch->window_tile < 0 || launch->window_tile > 40 ||
                 (launch->window_tile > 0 && launch->window_tile < 4)))
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
  p.max_tracklets = params->max_tracklets;
  const bool greedy = p.max_tracklets > 0;
  // the pruning bound needs positive kick factors
  p.prune = 1;
  for (int l = 0; l < kLayers; ++l)
    if (!(geom->a_kick[l] > 0.0f) || !std::isfinite(geom->a_kick[l])) p.prune = 0;
  // without a given launch shape, fewer wavefronts per workgroup when the bank offsets of a large
  // geometry and the tiles of large windows do not fit the LDS of four
  int block = launch ? launch->block : 256;
  while (!launch && block > kWave && compass_lds_bytes(g.S, p.max_hits, block / kWave, 0, greedy) > 160 * 1024)
    block -= kWave;
  const int waves = block / kWave;
  // stage u of events up to u_cap hits (and their weights up to u_cap / 2), keeping the
  // workgroup's LDS at the window tile per wavefront (by default 10 KiB: four 256-thread workgroups
  // share a CU's 160 KiB, the occupancy the kernel's registers allow); larger events search
  // global memory
  const int tile_kib = (launch && launch->window_tile > 0) ? launch->window_tile : 10;
  const size_t budget = (size_t)waves * tile_kib * 1024;
  const size_t fixed = compass_lds_bytes(g.S, p.max_hits, waves, 0, greedy);
  const int u_cap = fixed < budget ? (int)((budget - fixed) / sizeof(float)) / 64 * 64 : 0;
  const size_t lds = compass_lds_bytes(g.S, p.max_hits, waves, u_cap, greedy);
  if (lds > 160 * 1024) return UTC_ERR_ARG;
  (void)hipGetLastError();  // report only errors of this call
  const int grid = (launch && launch->grid > 0) ? launch->grid : n_events;
  // persistent launches hand out events from a counter in the workspace
  uint32_t* ev_counter = grid < n_events ? static_cast<uint32_t*>(workspace) : nullptr;
  TrackIO io{vx, vy, vtx, vty, hit_idx, qop, chi2, nhits, windows};
  const void* kern = p.max_tracklets > 0 ? reinterpret_cast<const void*>(k_compass<true>)
                                          : reinterpret_cast<const void*>(k_compass<false>);
  if (!allow_dynamic_lds(kern, lds)) return UTC_ERR_HIP;
  if (ev_counter)
    hipLaunchKernelGGL(k_compass_start, dim3(1), dim3(64), 0, stream, ev_counter, (uint32_t)grid);
  if (p.max_tracklets > 0)
    hipLaunchKernelGGL(k_compass<true>, dim3(grid), dim3(block), lds, stream, g, p, n_events,
                       hit_offsets, hit_u, hit_weight, hit_y_begin, hit_y_end, velo_offsets, io,
                       error_flags, u_cap, ev_counter);
  else
    hipLaunchKernelGGL(k_compass<false>, dim3(grid), dim3(block), lds, stream, g, p, n_events,
                       hit_offsets, hit_u, hit_weight, hit_y_begin, hit_y_end, velo_offsets, io,
                       error_flags, u_cap, ev_counter);
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}
