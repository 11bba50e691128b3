/* ut_compass.h — C ABI of libutcompass.so: UT raw-bank decoding and Compass upstream tracking on
 * AMD Instinct MI355X (gfx950).
 *
 * Paper: "A parallel-computing algorithm for high-energy physics particle tracking and decoding
 * using GPU architectures" (Fernandez Declara et al., IEEE Access 2019).
 *
 * Conventions shared by every entry point:
 *  - Array pointers are DEVICE pointers owned by the caller.  Structs are host memory, read during
 *    the call only.  No entry point allocates device memory or synchronises the host: all work is
 *    enqueued on `stream` in order, so a caller may capture the calls in a HIP graph.
 *  - Argument errors that the host can see (NULL where required, negative sizes, parameters out of
 *    range, workspace too small) return a negative utc_status and enqueue nothing.
 *  - Data errors that only the device can see set bits in *error_flags (a device uint32 that is
 *    OR-ed, never cleared by the library; may be NULL).  They never trap; the affected bank or event
 *    gets empty results and everything else is unaffected.
 *  - Every output is deterministic: identical inputs give bit-identical outputs on every run and
 *    for every launch configuration.
 */
#ifndef UT_COMPASS_H
#define UT_COMPASS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UTC_OK = 0,
  UTC_ERR_ARG = -1,        /* NULL pointer, negative size or parameter out of range */
  UTC_ERR_WORKSPACE = -2,  /* workspace NULL or smaller than the matching *_workspace_bytes() */
  UTC_ERR_HIP = -3         /* a HIP launch failed (see hipGetLastError) */
} utc_status;

/* Device error-flag bits. */
#define UTC_FLAG_BANK_ORDER     1u  /* bank_offsets[b+1] < bank_offsets[b]: bank b decoded as empty */
#define UTC_FLAG_CAPACITY       2u  /* more hits than hit_capacity: hits past the capacity not stored */
#define UTC_FLAG_LAYER_OVERFLOW 4u  /* an (event, layer) holds > 32767 hits: the event gets no tracks */
#define UTC_FLAG_BANK_SIZE      8u  /* a bank holds > UTC_MAX_BANK_WORDS words: decoded as empty */

#define UTC_MAX_BANK_WORDS 8192     /* a sector has 4096 distinct 1/8-strip positions */
#define UTC_MAX_WINDOW_HITS 32      /* upper bound of utc_compass_params.max_hits */

/* Detector description (synthetic stand-in for the UT geometry of Section III-A and the field
 * look-up tables of Section III-C).  Four layers of n_sectors sectors side by side in x. */
typedef struct {
  int32_t n_layers;          /* must be 4 */
  int32_t n_sectors;         /* S, 1..8192 */
  float z_layer[4];          /* mm */
  float dxdy[4];             /* tan(stereo angle); x = u + y*dxdy */
  float a_kick[4];           /* x deflection per unit q/p at each layer (mm*MeV) */
  float z_velo;              /* z of the VELO states (mm) */
  float pitch8;              /* 1/8-strip pitch (mm) */
  float u_min;               /* left edge of sector 0 (mm) */
  float sector_width;        /* mm */
  float inv_sector_width;    /* 1/mm */
  float y_begin, y_end;      /* y extent of the strips (mm) */
  float weight_by_size[16];  /* hit weight (1/sigma^2) by cluster size; [0] unused */
  const float* u0;           /* DEVICE [4*S]: u of the centre of the first 1/8-strip bin of each sector */
} utc_geometry;

/* Compass knobs (Section V: number of sectors, number of hit candidates; tolerances of V-B). */
typedef struct {
  float w0, kw, p_min;       /* window half-width W = w0 + kw/p_min (mm) */
  int32_t max_hits;          /* hits kept per layer window (nearest to the prediction), 1..32 */
  int32_t n_sectors_search;  /* 1, 3 or 5 */
  float slope_tol;           /* anchor pair accepted if |t_pair - tx_velo| <= slope_tol */
  float completion_tol;      /* completion interval margin (mm) */
  int32_t max_tracklets;     /* 0: minimum over every compatible combination; N > 0: the search of
                                Section V-B: each window walked central sector first, then its
                                neighbours at growing distance (left first), ascending x inside a
                                sector; anchor pairs A-major in that order; per pair the compatible
                                hit closest to the pair-slope extrapolation in each completion
                                layer (first in walk order on a tie); stop after N tracklets */
} utc_compass_params;

/* Launch shape.  NULL selects the defaults.  block: threads per workgroup, a multiple of 64, at
 * most 1024 for ut_decode and 512 for compass_find (a shape outside these limits, or one whose LDS
 * does not fit a CU, is rejected with UTC_ERR_ARG); grid: workgroups (0 = one per work item, > 0 =
 * persistent grid of that many workgroups striding over the work items); window_tile: KiB of LDS
 * per wavefront for the staged data (ut_decode: the chunk of raw words a wavefront sorts at once;
 * compass_find: the window cache, i.e. the positions, and when they fit the weights, of the
 * event's hits that the window searches and the tile read), 0 = 10, else 4 .. 40.  More LDS per
 * wavefront stages larger events and chunks, less keeps more wavefronts per CU. */
typedef struct {
  int32_t block;
  int32_t grid;
  int32_t window_tile;
  int32_t reserved;
} utc_launch_config;

/* ---------------------------------------------------------------------------------------------
 * ut_decode — Section IV (Table "Kernel configuration for UT decoding": count hits, prefix sum,
 * pre-decode, find permutation, decode in order).
 *
 * Input: n_events * 4 * S raw banks, bank b = (e*4 + l)*S + s holding the uint16 words
 * words[bank_offsets[b] .. bank_offsets[b+1]) (offsets in words, absolute indices into `words`).
 * A word is strip<<7 | fraction<<4 | size (9, 3, 4 bits); size 0 marks padding.
 * Output: hit_offsets[E*4*S + 1] = exclusive prefix sum of the valid words per bank (hit_offsets[0]
 * = 0), and the hit structure of arrays of Section IV at index hit_offsets[b] + k for the k-th hit
 * of bank b in ascending word order (i.e. ascending x):
 *   lhcbid = l<<28 | s<<12 | strip<<3 | fraction;  z = z_layer[l];
 *   u = fmaf(8*strip + fraction, pitch8, u0[l*S + s]) (x at y = 0);  y_begin, y_end;
 *   weight = weight_by_size[size].
 * The six output arrays must hold hit_capacity elements; hits past it are not stored
 * (UTC_FLAG_CAPACITY).  Pass hit_capacity >= number of words to be safe.  z, y_begin and y_end
 * are layer / geometry constants and may be NULL (not written): the compact form of the hit
 * structure, 12 instead of 24 bytes per hit.
 * Workspace: ut_decode_workspace_bytes(n_events, S) bytes of device memory, any content.
 * --------------------------------------------------------------------------------------------- */
size_t ut_decode_workspace_bytes(int32_t n_events, int32_t n_sectors);

utc_status ut_decode(const utc_geometry* geom, const uint16_t* words, const uint32_t* bank_offsets,
                     int32_t n_events, int64_t hit_capacity, uint32_t* hit_offsets,
                     uint32_t* lhcbid, float* z, float* u, float* y_begin, float* y_end,
                     float* weight, uint32_t* error_flags, void* workspace, size_t workspace_bytes,
                     const utc_launch_config* launch, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * ut_decode_noalloc — ut_decode for callers that cannot allocate device memory (code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as ut_decode, without the workspace: the unit sums and bases go to a fixed scratch
 * array inside the library, 4 * (8 * UTC_NOALLOC_MAX_EVENTS + 1) bytes (about 1 MiB) of device
 * memory on each GPU the call runs on, held until the process ends.  The call allocates nothing;
 * its first call on a device looks up that device's copy of the array (hipGetSymbolAddress, with the
 * device current).  n_events > UTC_NOALLOC_MAX_EVENTS returns UTC_ERR_ARG; a failed lookup returns
 * UTC_ERR_HIP.  Every call on one GPU shares the array, so calls that may run at the same time on
 * one GPU (on different streams, or from different threads) race and give wrong results: order them
 * on one stream, or use ut_decode with a workspace each.
 * --------------------------------------------------------------------------------------------- */
#define UTC_NOALLOC_MAX_EVENTS 32768

utc_status ut_decode_noalloc(const utc_geometry* geom, const uint16_t* words,
                             const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                             uint32_t* hit_offsets, uint32_t* lhcbid, float* z, float* u,
                             float* y_begin, float* y_end, float* weight, uint32_t* error_flags,
                             const utc_launch_config* launch, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * compass_find — Section V: per VELO track, hit windows in the four layers (V-A), tracklet search
 * with the p-kick chi2 fit and selection (V-B).
 *
 * Hits: the structure of arrays and hit_offsets[E*4*S+1] as written by ut_decode (u non-decreasing
 * inside each (event, layer)).  VELO tracks: states x, y, tx, ty at z_velo, tracks of event e at
 * velo_offsets[e] .. velo_offsets[e+1] (velo_offsets[E] = n_tracks).
 * Output per track t (dense, VELO order): hit_idx[4t + l] = index of the layer-l hit (-1 = none),
 * nhits (0 = no upstream track, else 3 or 4), qop (MeV^-1, its sign is the charge) and chi2 of the
 * fit; zeros for tracks without a tracklet.  windows (optional, NULL to skip): int16 pairs
 * [4t + l] = (first hit - first hit of its (event, layer), size), (-1, 0) when not searched.
 * hit_y_begin and hit_y_end may both be NULL: every strip then spans the geometry's
 * [y_begin, y_end] (what ut_decode writes; the compact form of the hits).
 * Workspace: compass_find_workspace_bytes() bytes, any content.  A persistent launch (grid > 0 and
 * fewer workgroups than events) keeps its event counter there (reset by the call, on the stream):
 * calls in flight at the same time need workspaces of their own.
 * --------------------------------------------------------------------------------------------- */
size_t compass_find_workspace_bytes(int32_t n_events, int64_t n_tracks);

utc_status compass_find(const utc_geometry* geom, const utc_compass_params* params, int32_t n_events,
                        const uint32_t* hit_offsets, const float* hit_u, const float* hit_weight,
                        const float* hit_y_begin, const float* hit_y_end,
                        const float* vx, const float* vy, const float* vtx, const float* vty,
                        const uint32_t* velo_offsets, int64_t n_tracks,
                        int32_t* hit_idx, float* qop, float* chi2, int32_t* nhits, int16_t* windows,
                        uint32_t* error_flags, void* workspace, size_t workspace_bytes,
                        const utc_launch_config* launch, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * compass_fit_grad — the track-fit chi2 of Sections III-C / V-B as a function of per-sector x
 * offsets delta (4*S) and per-track q/p, with the hit assignment frozen, and its adjoint:
 *   r_h = ((m_h - delta_s(h)) - xs_l) - a_l * qop_t,  m_h = u_h + y_l * dxdy_l,
 *   chi2_t = sum_h w_h r_h^2,  chi2 = sum_t chi2_t,
 *   grad_qop_t = grad_scale * d chi2 / d qop_t = -2 grad_scale sum_h w_h a_l r_h,
 *   grad_offsets_s = -2 grad_scale sum_{h in s} w_h r_h.
 * r is evaluated in binary64 and rounded once to binary32; the rest of the per-track arithmetic is
 * binary32; chi2_total and grad_offsets are summed exactly (integer fixed point, 2^-40) and
 * rounded at the end, so results do not depend on thread scheduling.
 * track_hit_idx[4t + l]: index into the hit arrays (length n_hits) of the layer-l hit of track t,
 * or -1; the sector of a hit is taken from its LHCbID.  Slots whose index is outside [0, n_hits) or
 * whose LHCbID names no sector of the geometry are skipped.  Every output may be NULL; a call with
 * all gradient pointers NULL is the forward pass.  The sums are accumulated per workgroup in LDS up
 * to 2559 sectors per layer and in the workspace beyond (same results).
 * Workspace: compass_fit_grad_workspace_bytes(S) bytes, any content.
 * --------------------------------------------------------------------------------------------- */
size_t compass_fit_grad_workspace_bytes(int32_t n_sectors);

utc_status compass_fit_grad(const utc_geometry* geom, int64_t n_tracks, const int32_t* track_hit_idx,
                            int64_t n_hits, const float* hit_u, const float* hit_weight,
                            const uint32_t* hit_lhcbid,
                            const float* vx, const float* vy, const float* vtx, const float* vty,
                            const float* qop, const float* offsets, float grad_scale,
                            float* chi2_track, double* chi2_total, float* grad_qop,
                            float* grad_offsets, void* workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * compass_fit_freeze / compass_fit_grad_frozen — the same fit chi2 and adjoint as compass_fit_grad
 * (same formulas, same roundings, the same results bit for bit), with the frozen hits gathered
 * once into track-major form: compass_fit_freeze writes, for every track t and layer l, the u,
 * weight and global sector l*S+s of its layer-l hit to track_u[4t+l], track_weight[4t+l] and
 * track_sector[4t+l] (0, 0 and -1 for a slot that compass_fit_grad skips); compass_fit_grad_frozen
 * then reads 40 bytes per track instead of gathering from the hit arrays, and skips slots whose
 * sector is outside [0, 4S).  track_u and track_weight must be 16-byte aligned and track_sector
 * 8-byte aligned (UTC_ERR_ARG otherwise).  Outputs, workspace and errors as compass_fit_grad.
 * --------------------------------------------------------------------------------------------- */
utc_status compass_fit_freeze(const utc_geometry* geom, int64_t n_tracks, const int32_t* track_hit_idx,
                              int64_t n_hits, const float* hit_u, const float* hit_weight,
                              const uint32_t* hit_lhcbid, float* track_u, float* track_weight,
                              int16_t* track_sector, hipStream_t stream);

utc_status compass_fit_grad_frozen(const utc_geometry* geom, int64_t n_tracks, const float* track_u,
                                   const float* track_weight, const int16_t* track_sector,
                                   const float* vx, const float* vy, const float* vtx,
                                   const float* vty, const float* qop, const float* offsets,
                                   float grad_scale, float* chi2_track, double* chi2_total,
                                   float* grad_qop, float* grad_offsets, void* workspace,
                                   size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Autotuning of the batched launch (not in the paper, which tuned its kernel parameters by hand,
 * Section VI-C).  Each call runs the matching entry point on the caller's buffers (same arguments
 * and meaning as ut_decode / compass_find) for every candidate launch shape: window tile in
 * {10, 6, 16} KiB (decode) or {10, 8, 16, 24} KiB (Compass), block in {64, 128, 256, 512}, grid
 * in {one workgroup per work item, 512, 2048} (decode) or {one per item, 512, 1024, 2048}
 * (Compass) persistent workgroups; shapes whose LDS does not fit a CU are skipped.  Each shape
 * runs once to warm up and then `reps` times (1..32).  *best receives the first shape, in the
 * order tile, block, grid of the lists above, whose median time is within 2 % of the lowest
 * median (near-equal shapes are within the timing noise; the rule keeps repeated tunings on one
 * shape), *best_us its median in microseconds.
 * Results do not depend on the shape.  Unlike the other calls these synchronise
 * the stream (set-up calls); the outputs hold the last run's results.
 * --------------------------------------------------------------------------------------------- */
utc_status ut_decode_autotune(const utc_geometry* geom, const uint16_t* words,
                              const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                              uint32_t* hit_offsets, uint32_t* lhcbid, float* z, float* u,
                              float* y_begin, float* y_end, float* weight, uint32_t* error_flags,
                              void* workspace, size_t workspace_bytes, int32_t reps,
                              utc_launch_config* best, float* best_us, hipStream_t stream);

utc_status compass_find_autotune(const utc_geometry* geom, const utc_compass_params* params,
                                 int32_t n_events, const uint32_t* hit_offsets, const float* hit_u,
                                 const float* hit_weight, const float* hit_y_begin,
                                 const float* hit_y_end, const float* vx, const float* vy,
                                 const float* vtx, const float* vty, const uint32_t* velo_offsets,
                                 int64_t n_tracks, int32_t* hit_idx, float* qop, float* chi2,
                                 int32_t* nhits, uint32_t* error_flags, void* workspace,
                                 size_t workspace_bytes, int32_t reps, utc_launch_config* best,
                                 float* best_us, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * ut_global_event_cut — the global event cut that precedes decoding (Section VI: events are
 * selected before the UT chain runs).  An event is kept when its raw banks hold at most max_words
 * words in total (padding included); kept events are copied, in order, into a compact batch of the
 * same n_events events in which every rejected event is empty (no words, no VELO tracks), so the
 * following ut_decode / compass_find calls take the same event count and need no host round trip.
 *
 * Inputs: the raw-bank batch of ut_decode (words, bank_offsets [n_events*4*S + 1]) and the VELO
 * states of compass_find (vx, vy, vtx, vty, velo_offsets [n_events + 1]).
 * Outputs: out_words (capacity: bank_offsets[n_events*4*S] words), out_bank_offsets
 * [n_events*4*S + 1], out_vx/vy/vtx/vty (capacity: velo_offsets[n_events]), out_velo_offsets
 * [n_events + 1], keep [n_events] (1 kept, 0 rejected; may be NULL), n_kept (device int32, the
 * number of kept events; may be NULL).  Output arrays must not overlap the inputs.
 * Bank offsets that decrease are treated as an empty event (and flagged UTC_FLAG_BANK_ORDER).
 * Workspace: ut_global_event_cut_workspace_bytes(n_events) bytes, any content.
 * --------------------------------------------------------------------------------------------- */
size_t ut_global_event_cut_workspace_bytes(int32_t n_events);

utc_status ut_global_event_cut(const utc_geometry* geom, int32_t n_events, const uint16_t* words,
                               const uint32_t* bank_offsets, const float* vx, const float* vy,
                               const float* vtx, const float* vty, const uint32_t* velo_offsets,
                               uint32_t max_words, uint16_t* out_words, uint32_t* out_bank_offsets,
                               float* out_vx, float* out_vy, float* out_vtx, float* out_vty,
                               uint32_t* out_velo_offsets, uint8_t* keep, int32_t* n_kept,
                               uint32_t* error_flags, void* workspace, size_t workspace_bytes,
                               hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * compass_consolidate — the found upstream tracks of compass_find gathered into a dense container
 * (the prefix sum and consolidation step that follows the tracking, Section VI): the tracks with
 * nhits > 0, in VELO order, with per-event offsets.
 *
 * Inputs: velo_offsets [n_events + 1] and compass_find's per-track outputs nhits [n_tracks],
 * hit_idx [n_tracks*4], qop, chi2 [n_tracks].
 * Outputs (capacity n_tracks each; only the first *n_found entries are written): out_velo
 * (the VELO index of each found track), out_hit_idx [*4], out_qop, out_chi2, out_nhits; and
 * out_offsets [n_events + 1], out_offsets[e] = number of found tracks in events before e
 * (out_offsets[n_events] = *n_found); n_found (device int32; may be NULL).
 * Workspace: compass_consolidate_workspace_bytes(n_tracks) bytes, any content.
 * --------------------------------------------------------------------------------------------- */
size_t compass_consolidate_workspace_bytes(int64_t n_tracks);

utc_status compass_consolidate(int32_t n_events, const uint32_t* velo_offsets, int64_t n_tracks,
                               const int32_t* nhits, const int32_t* hit_idx, const float* qop,
                               const float* chi2, uint32_t* out_offsets, int32_t* out_velo,
                               int32_t* out_hit_idx, float* out_qop, float* out_chi2,
                               int32_t* out_nhits, int32_t* n_found, void* workspace,
                               size_t workspace_bytes, hipStream_t stream);

/* Human-readable name of a status code. */
const char* utc_status_string(int status);

/* Library version string. */
const char* utc_version(void);

#ifdef __cplusplus
}
#endif
#endif
