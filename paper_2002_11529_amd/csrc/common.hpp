// Device-side helpers shared by the kernels of libutcompass (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

#include "ut_compass.h"

namespace utc {

constexpr int kLayers = 4;
constexpr int kWave = 64;

// Geometry as a by-value kernel argument (the device table u0 stays a pointer).
struct Geom {
  int32_t S;
  float z_layer[4];
  float dxdy[4];
  float a_kick[4];
  float z_velo;
  float pitch8;
  float u_min;
  float sector_width;
  float inv_sector_width;
  float y_begin, y_end;
  float weight_by_size[16];
  float inv_a_up[4];   // 1 / a_kick rounded up (upper bounds for the pruning; unused if a <= 0)
  const float* u0;
};

inline Geom make_geom(const utc_geometry& g) {
  Geom d;
  d.S = g.n_sectors;
  for (int l = 0; l < 4; ++l) {
    d.z_layer[l] = g.z_layer[l];
    d.dxdy[l] = g.dxdy[l];
    d.a_kick[l] = g.a_kick[l];
  }
  d.z_velo = g.z_velo;
  d.pitch8 = g.pitch8;
  d.u_min = g.u_min;
  d.sector_width = g.sector_width;
  d.inv_sector_width = g.inv_sector_width;
  d.y_begin = g.y_begin;
  d.y_end = g.y_end;
  for (int i = 0; i < 16; ++i) d.weight_by_size[i] = g.weight_by_size[i];
  for (int l = 0; l < 4; ++l)
    d.inv_a_up[l] = g.a_kick[l] > 0.0f ? nextafterf(1.0f / g.a_kick[l], INFINITY) : 0.0f;
  d.u0 = g.u0;
  return d;
}

// Allow `bytes` of dynamic LDS for `func` (needed above 64 KiB).  Clears the error state on failure.
inline bool allow_dynamic_lds(const void* func, size_t bytes) {
  if (bytes <= 64 * 1024) return true;
  if (hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

__device__ inline void raise_flag(uint32_t* flags, uint32_t bit) {
  if (flags) atomicOr(flags, bit);
}

// Inclusive scans across one wavefront with all 64 lanes active, in DPP data movement (no LDS
// round trips): shifts right by 1, 2, 4 and 8 lanes inside each row of 16 lanes (lanes without a
// source keep the identity), then the last lane of row 0 is added into row 1 and of row 2 into row
// 3, then lane 31 into rows 2 and 3.
template <class Op>
__device__ inline uint32_t dpp_inclusive_scan(uint32_t v, uint32_t identity, Op op) {
  const int id = (int)identity;
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return v;
}

__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
  return dpp_inclusive_scan(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ inline uint32_t wave_inclusive_max(uint32_t x) {
  return dpp_inclusive_scan(x, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

__device__ inline uint32_t wave_max_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_inclusive_max(x), 63);
}

// Unsigned keys in the order of the floats they stand for (-0 before +0; not for NaN).
__device__ inline uint32_t float_order_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ inline float float_from_order_key(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ inline uint32_t wave_sum(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_inclusive_scan(x), 63);
}

// Exclusive scan across the workgroup.  `tmp` holds blockDim.x/64 + 1 words of LDS.  All threads
// must call it; it ends with a barrier so `tmp` may be reused right after.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  uint32_t x = wave_inclusive_scan(v);
  if (lane == kWave - 1) tmp[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t t = lane < nw ? tmp[lane] : 0u;
    t = wave_inclusive_scan(t);
    if (lane < nw) tmp[lane] = t;
  }
  __syncthreads();
  uint32_t before = wid > 0 ? tmp[wid - 1] : 0u;
  *total = tmp[nw - 1];
  __syncthreads();
  return before + x - v;
}

__device__ inline uint32_t block_sum(uint32_t v, uint32_t* tmp) {
  uint32_t total;
  block_exclusive_scan(v, tmp, &total);
  return total;
}

}  // namespace utc

namespace utc {

// ---- wavefront helpers (wave64) ----
__device__ inline int lane_id() { return __lane_id(); }

// Orders the LDS accesses of one wavefront: the compiler may not move memory operations across it
// and earlier LDS writes of any lane are visible to later reads of any lane of the same wave.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

__device__ inline uint32_t lanes_before(uint64_t mask) {
  return (uint32_t)__popcll(mask & __lanemask_lt());
}

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0ull; }

template <class T>
__device__ inline T wave_bcast(T v, int src) { return __shfl(v, src, kWave); }

__device__ inline uint32_t wave_excl_scan(uint32_t x, uint32_t* total) {
  const uint32_t inc = wave_inclusive_scan(x);
  *total = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
  return inc - x;
}

// First index i in [lo, hi) with pred(i) true for a predicate that is false then true.
template <class P>
__device__ inline int64_t first_true(int64_t lo, int64_t hi, P pred) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (pred(mid)) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// The same over 32-bit indices.
template <class P>
__device__ inline uint32_t first_true_u32(uint32_t lo, uint32_t hi, P pred) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (pred(mid)) hi = mid; else lo = mid + 1;
  }
  return lo;
}

}  // namespace utc
