/* Plain CPU oracle for UT raw-bank decoding and Compass tracking.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference the GPU path is checked
 * against.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product library never calls it and shares no source with it.
 *
 * Paper: "A parallel-computing algorithm for high-energy physics particle tracking and decoding
 * using GPU architectures" (Fernandez Declara et al., IEEE Access 2019).
 *   decode   : Section IV (hit parameters; count, prefix sum, sort within sector groups, decode)
 *   windows  : Section V-A (extrapolate, locate region by binary search, bound, refine; 1/3/5 sectors)
 *   tracklets: Section V-B (anchors in the first and third panel, tolerance window from the pair
 *              slope and the VELO slope, completion in the second and fourth panel, forward then
 *              backward, prefer 4 hits over 3 and then lowest chi2)
 *   fit      : Section III-C (p-kick chi2 fit giving the momentum) and Section V-B (fit in
 *              combination with the VELO track)
 * The paper states the method in prose only.  The precise arithmetic below is the reading written
 * down in the design notes; every floating-point step is IEEE binary32, round to nearest, no
 * contraction, in the order written in oracle.c.
 *
 * All pointers are host pointers owned by the caller.
 */
#ifndef UT_ORACLE_H
#define UT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status bits returned by the oracle (same meaning as the library's device error flags). */
#define ORA_FLAG_BANK_ORDER     1u  /* bank_offsets decrease: that bank is treated as empty */
#define ORA_FLAG_CAPACITY       2u  /* more hits than hit_capacity: extra hits are not stored */
#define ORA_FLAG_LAYER_OVERFLOW 4u  /* an (event, layer) holds >= 32768 hits: event gets no tracks */
#define ORA_FLAG_BANK_SIZE      8u  /* a bank holds more than ORA_MAX_BANK_WORDS words: treated as empty */
#define ORA_MAX_BANK_WORDS   8192u  /* twice the 4096 distinct 1/8-strip positions of a sector */
#define ORA_ERR_ARG          (-1)

typedef struct {
  int32_t n_layers;            /* must be 4 */
  int32_t n_sectors;           /* S */
  float z_layer[4];            /* mm */
  float dxdy[4];               /* tan(stereo angle): x = u + y*dxdy */
  float a_kick[4];             /* x deflection per unit q/p at each layer (mm*MeV) */
  float z_velo;                /* z of the VELO state (mm) */
  float pitch8;                /* 1/8-strip pitch (mm) */
  float u_min;                 /* left edge of sector 0 (mm) */
  float sector_width;          /* mm */
  float inv_sector_width;      /* 1/mm */
  float y_begin, y_end;        /* y extent of every strip (mm) */
  float weight_by_size[16];    /* hit weight by cluster size */
  const float* u0;             /* [4*S]: u of the first 1/8-strip bin centre of each sector */
} ora_detector;

typedef struct {
  float w0, kw, p_min;         /* window half-width W = w0 + kw/p_min */
  int32_t max_hits;            /* N_max: per-layer window cap, 1..32 */
  int32_t n_sectors_search;    /* 1, 3 or 5 */
  float slope_tol;             /* |t_pair - tx| bound */
  float completion_tol;        /* completion interval margin (mm) */
  int32_t max_tracklets;       /* 0: every compatible combination; N > 0: the paper's search with
                                  the closest completion hit per layer, stopping after N tracklets */
} ora_params;

/* Decode: banks b = (e*4 + l)*S + s hold words[bank_offsets[b] .. bank_offsets[b+1]).
 * Writes hit_offsets[E*4*S + 1] (exclusive scan of valid words per bank) and the hit SoA.
 * Returns a bitmask of ORA_FLAG_* (0 = clean) or ORA_ERR_ARG. */
int ora_ut_decode(const ora_detector* det, const uint16_t* words, const uint32_t* bank_offsets,
                  int32_t n_events, int64_t hit_capacity, uint32_t* hit_offsets,
                  uint32_t* lhcbid, float* z, float* u, float* y_begin, float* y_end, float* weight);

/* Compass: per VELO track (global order, velo_offsets[E+1]) writes hit_idx[4] (global hit index
 * or -1), qop, chi2, nhits (0 = no upstream track).  Optional outputs (NULL to skip):
 * win_first[n*4] (global index of the first window hit), win_size[n*4], active[n].
 * Returns a bitmask of ORA_FLAG_* or ORA_ERR_ARG. */
int ora_compass_find(const ora_detector* det, const ora_params* par, int32_t n_events,
                     const uint32_t* hit_offsets, const float* hit_u, const float* hit_weight,
                     const float* hit_y_begin, const float* hit_y_end,
                     const float* vx, const float* vy, const float* vtx, const float* vty,
                     const uint32_t* velo_offsets,
                     int32_t* hit_idx, float* qop, float* chi2, int32_t* nhits,
                     int32_t* win_first, int32_t* win_size, uint8_t* active);

/* Track-fit chi2 with per-sector x offsets and its adjoint in binary32.  Hit slots with an index
 * outside [0, n_hits) or an LHCbID naming no sector are skipped.  The residual of each hit
 * is evaluated in binary64 and rounded once to binary32; everything after that is binary32.  Any of
 * the outputs may be NULL.  Returns the total chi2 summed in double in track order. */
double ora_fit_grad_f32(const ora_detector* det, int64_t n_tracks, const int32_t* track_hit_idx,
                        int64_t n_hits, const float* hit_u, const float* hit_weight, const uint32_t* hit_lhcbid,
                        const float* vx, const float* vy, const float* vtx, const float* vty,
                        const float* qop, const float* offsets, float grad_scale,
                        float* chi2_track, float* grad_qop, float* grad_offsets);

/* The same quantities in binary64 throughout: the reference gradient. */
double ora_fit_grad_f64(const ora_detector* det, int64_t n_tracks, const int32_t* track_hit_idx,
                        int64_t n_hits, const float* hit_u, const float* hit_weight, const uint32_t* hit_lhcbid,
                        const float* vx, const float* vy, const float* vtx, const float* vty,
                        const double* qop, const double* offsets, double grad_scale,
                        double* chi2_track, double* grad_qop, double* grad_offsets);

#ifdef __cplusplus
}
#endif
#endif
