// Launch-shape autotuner for the batched path: times candidate (block, grid) shapes of ut_decode
// and compass_find on the caller's own buffers with HIP events and keeps the fastest.  A set-up
// call: it synchronises the stream, unlike the other entry points.
#include "common.hpp"

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

template <class F>
float median_us(F&& run, int reps, hipStream_t stream, Timer& tm, bool& ok) {
  float best[32];
  const int n = reps < 1 ? 1 : (reps > 32 ? 32 : reps);
  if (run() != UTC_OK) { ok = false; return 0.0f; }  // warm-up, also checks the shape
  for (int i = 0; i < n; ++i) {
    (void)hipEventRecord(tm.a, stream);
    if (run() != UTC_OK) { ok = false; return 0.0f; }
    (void)hipEventRecord(tm.b, stream);
    (void)hipEventSynchronize(tm.b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, tm.a, tm.b);
    best[i] = ms * 1000.0f;
  }
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && best[j] < best[j - 1]; --j) {
      const float t = best[j]; best[j] = best[j - 1]; best[j - 1] = t;
    }
  ok = true;
  return best[n / 2];
}

}  // namespace

extern "C" utc_status ut_decode_autotune(const utc_geometry* geom, const uint16_t* words,
                                         const uint32_t* bank_offsets, int32_t n_events,
                                         int64_t hit_capacity, uint32_t* hit_offsets,
                                         uint32_t* lhcbid, float* z, float* u, float* y_begin,
                                         float* y_end, float* weight, uint32_t* error_flags,
                                         void* workspace, size_t workspace_bytes, int32_t reps,
                                         utc_launch_config* best, float* best_us,
                                         hipStream_t stream)
{
  if (!best || !best_us) return UTC_ERR_ARG;
  static const int blocks[] = {64, 128, 256, 512};
  static const int grids[] = {0, 256, 512, 1024, 2048};
  Timer tm;
  float t_best = 3.0e38f;
  bool any = false;
  for (int b : blocks)
    for (int gsz : grids) {
      utc_launch_config c{b, gsz, 0, 0};
      bool ok = false;
      const float t = median_us([&] {
        return ut_decode(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, z,
                         u, y_begin, y_end, weight, error_flags, workspace, workspace_bytes, &c,
                         stream);
      }, reps, stream, tm, ok);
      if (ok && t < t_best) {
        t_best = t;
        *best = c;
        any = true;
      }
    }
  if (!any) return UTC_ERR_ARG;
  *best_us = t_best;
  return UTC_OK;
}

extern "C" utc_status compass_find_autotune(const utc_geometry* geom, const utc_compass_params* params,
                                            int32_t n_events, const uint32_t* hit_offsets,
                                            const float* hit_u, const float* hit_weight,
                                            const float* hit_y_begin, const float* hit_y_end,
                                            const float* vx, const float* vy, const float* vtx,
                                            const float* vty, const uint32_t* velo_offsets,
                                            int64_t n_tracks, int32_t* hit_idx, float* qop,
                                            float* chi2, int32_t* nhits, uint32_t* error_flags,
                                            void* workspace, size_t workspace_bytes, int32_t reps,
                                            utc_launch_config* best, float* best_us,
                                            hipStream_t stream)
{
  if (!best || !best_us) return UTC_ERR_ARG;
  static const int blocks[] = {64, 128, 256, 512};
  static const int grids[] = {0, 512, 1024, 2048};
  Timer tm;
  float t_best = 3.0e38f;
  bool any = false;
  for (int b : blocks)
    for (int gsz : grids) {
      utc_launch_config c{b, gsz, 0, 0};
      bool ok = false;
      const float t = median_us([&] {
        return compass_find(geom, params, n_events, hit_offsets, hit_u, hit_weight, hit_y_begin,
                            hit_y_end, vx, vy, vtx, vty, velo_offsets, n_tracks, hit_idx, qop, chi2,
                            nhits, nullptr, error_flags, workspace, workspace_bytes, &c, stream);
      }, reps, stream, tm, ok);
      if (ok && t < t_best) {
        t_best = t;
        *best = c;
        any = true;
      }
    }
  if (!any) return UTC_ERR_ARG;
  *best_us = t_best;
  return UTC_OK;
}
