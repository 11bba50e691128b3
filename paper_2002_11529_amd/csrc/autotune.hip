// Launch-shape autotuner for the batched path: times candidate (window tile, block, grid) shapes of
// ut_decode and compass_find on the caller's own buffers with HIP events and keeps the first candidate, in
// the listed order, within kTieFrac of the fastest (near-equal shapes are within the timing noise;
// the rule keeps the choice from flipping between them from run to run).  A set-up call: it
// synchronises the stream, unlike the other entry points.
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

constexpr float kTieFrac = 0.02f;

constexpr int kMaxShapes = 128;

// Times every (window tile, block, grid) of the three lists with run(config) and picks as described
// above (tiles outermost, so the first tile listed wins a tie).
template <class F>
utc_status tune_shapes(const int* tiles, int nt, const int* blocks, int nb, const int* grids, int ng,
                       F&& run, int reps, hipStream_t stream, utc_launch_config* best,
                       float* best_us) {
  if (nt * nb * ng > kMaxShapes) return UTC_ERR_ARG;
  Timer tm;
  float t[kMaxShapes];
  bool okc[kMaxShapes];
  utc_launch_config cfg[kMaxShapes];
  float t_min = 3.0e38f;
  int n = 0;
  for (int a = 0; a < nt; ++a)
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < ng; ++j, ++n) {
        cfg[n] = utc_launch_config{blocks[i], grids[j], tiles[a], 0};
        bool ok = false;
        t[n] = median_us([&] { return run(&cfg[n]); }, reps, stream, tm, ok);
        okc[n] = ok;
        if (ok && t[n] < t_min) t_min = t[n];
      }
  for (int k = 0; k < n; ++k)
    if (okc[k] && t[k] <= t_min * (1.0f + kTieFrac)) {
      *best = cfg[k];
      *best_us = t[k];
      return UTC_OK;
    }
  return UTC_ERR_ARG;
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
  static const int tiles[] = {10, 6, 16};
  static const int blocks[] = {64, 128, 256, 512};
  static const int grids[] = {0, 512, 2048};
  return tune_shapes(tiles, 3, blocks, 4, grids, 3, [&](const utc_launch_config* c) {
    return ut_decode(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, z, u,
                     y_begin, y_end, weight, error_flags, workspace, workspace_bytes, c, stream);
  }, reps, stream, best, best_us);
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
  static const int tiles[] = {10, 8, 16, 24};
  static const int blocks[] = {64, 128, 256, 512};
  static const int grids[] = {0, 512, 1024, 2048};
  return tune_shapes(tiles, 4, blocks, 4, grids, 4, [&](const utc_launch_config* c) {
    return compass_find(geom, params, n_events, hit_offsets, hit_u, hit_weight, hit_y_begin, hit_y_end,
                        vx, vy, vtx, vty, velo_offsets, n_tracks, hit_idx, qop, chi2, nhits, nullptr,
                        error_flags, workspace, workspace_bytes, c, stream);
  }, reps, stream, best, best_us);
}
