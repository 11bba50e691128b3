/* Plain CPU oracle: UT raw-bank decoding and Compass tracking.  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).  Single-threaded, scalar, written for reading rather than speed.  Build with
 * -ffp-contract=off and without fast-math so that every float expression below is evaluated as
 * written, one IEEE binary32 rounding per operation. */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NL 4

/* ------------------------------------------------------------------------------------------------
 * Decoding (Section IV).  A raw word carries strip (9 bits), interstrip fraction (3 bits) and
 * cluster size (4 bits); size 0 marks padding.  Per bank: count the hits, prefix-sum the counts
 * into hit offsets, order the hits of the bank by position, and store the six hit parameters
 * (LHCbID, z, x at y=0, yBegin, yEnd, weight) as a structure of arrays.
 * ------------------------------------------------------------------------------------------------ */
int ora_ut_decode(const ora_detector* det, const uint16_t* words, const uint32_t* bank_offsets,
                  int32_t n_events, int64_t hit_capacity, uint32_t* hit_offsets,
                  uint32_t* lhcbid, float* z, float* u, float* y_begin, float* y_end, float* weight)
{
  if (!det || det->n_layers != NL || det->n_sectors <= 0 || n_events < 0 || !bank_offsets ||
      !hit_offsets || hit_capacity < 0)
    return ORA_ERR_ARG;
  const int64_t S = det->n_sectors;
  const int64_t n_banks = (int64_t)n_events * NL * S;
  unsigned flags = 0;

  /* count valid words per bank and take the exclusive prefix sum */
  uint32_t running = 0;
  uint32_t largest = 0;
  for (int64_t b = 0; b < n_banks; ++b) {
    hit_offsets[b] = running;
    uint32_t start = bank_offsets[b], end = bank_offsets[b + 1];
    if (end < start) { flags |= ORA_FLAG_BANK_ORDER; continue; }
    if (end - start > ORA_MAX_BANK_WORDS) { flags |= ORA_FLAG_BANK_SIZE; continue; }
    if (end - start > largest) largest = end - start;
    for (uint32_t i = start; i < end; ++i)
      if (words[i] & 0xFu) running++;
  }
  hit_offsets[n_banks] = running;
  if ((int64_t)running > hit_capacity) flags |= ORA_FLAG_CAPACITY;

  uint16_t* sorted = (uint16_t*)malloc(sizeof(uint16_t) * (largest ? largest : 1));
  if (!sorted) return ORA_ERR_ARG;
  for (int64_t b = 0; b < n_banks; ++b) {
    uint32_t start = bank_offsets[b], end = bank_offsets[b + 1];
    if (end < start || end - start > ORA_MAX_BANK_WORDS) continue;
    const int32_t l = (int32_t)((b / S) % NL);
    const int32_t s = (int32_t)(b % S);
    /* keep the valid words in bank order */
    uint32_t n = 0;
    for (uint32_t i = start; i < end; ++i)
      if (words[i] & 0xFu) sorted[n++] = words[i];
    /* stable insertion sort by the whole word: the position bits are the high bits, so this
       orders the hits of a sector by x */
    for (uint32_t i = 1; i < n; ++i) {
      uint16_t w = sorted[i];
      uint32_t j = i;
      while (j > 0 && sorted[j - 1] > w) { sorted[j] = sorted[j - 1]; --j; }
      sorted[j] = w;
    }
    for (uint32_t k = 0; k < n; ++k) {
      int64_t h = (int64_t)hit_offsets[b] + k;
      if (h >= hit_capacity) continue;
      uint32_t w = sorted[k];
      uint32_t size = w & 0xFu, frac = (w >> 4) & 7u, strip = w >> 7;
      lhcbid[h] = ((uint32_t)l << 28) | ((uint32_t)s << 12) | (strip << 3) | frac;
      z[h] = det->z_layer[l];
      /* x at y=0: sector origin plus position in 1/8 strips, one rounding */
      u[h] = fmaf((float)(strip * 8u + frac), det->pitch8, det->u0[l * S + s]);
      y_begin[h] = det->y_begin;
      y_end[h] = det->y_end;
      weight[h] = det->weight_by_size[size];
    }
  }
  free(sorted);
  return (int)flags;
}

/* ------------------------------------------------------------------------------------------------
 * Compass (Section V).
 * ------------------------------------------------------------------------------------------------ */

/* VELO straight line at each layer (Section V-A: extrapolation of the VELO track to the panels). */
typedef struct {
  float xs[NL];   /* x of the straight line */
  float yl[NL];   /* y of the straight line */
  float up[NL];   /* predicted measured coordinate u = x - y*dxdy */
} ora_extrap;

static void extrapolate(const ora_detector* det, float vx, float vy, float vtx, float vty,
                        ora_extrap* x)
{
  for (int l = 0; l < NL; ++l) {
    float dz = det->z_layer[l] - det->z_velo;
    x->xs[l] = vx + vtx * dz;
    x->yl[l] = vy + vty * dz;
    x->up[l] = x->xs[l] - x->yl[l] * det->dxdy[l];
  }
}

/* A track is kept when it crosses the first and the last layer inside the planes (Section V-A:
   tracks outside the UT acceptance are filtered out before the window search). */
static int in_acceptance(const ora_detector* det, const ora_extrap* x)
{
  const float u_max = det->u_min + (float)det->n_sectors * det->sector_width;
  static const int check[2] = {0, NL - 1};
  for (int k = 0; k < 2; ++k) {
    int l = check[k];
    if (!(det->y_begin <= x->yl[l] && x->yl[l] <= det->y_end)) return 0;
    if (!(det->u_min <= x->up[l] && x->up[l] <= u_max)) return 0;
  }
  return 1;
}

/* Window of one layer (Section V-A): the sector the prediction points to and its neighbours
   (1, 3 or 5 sectors, fewer at the layer edges), the hits with u in [up - W, up + W], cut to the
   max_hits hits nearest to the prediction.  Linear scans stand in for the paper's binary searches. */
static void find_window(const ora_detector* det, const ora_params* par, const uint32_t* hit_offsets,
                        const float* hit_u, int64_t layer_bank0, float up, float W,
                        int64_t* first_out, int64_t* end_out)
{
  const int32_t S = det->n_sectors;
  const int32_t half = (par->n_sectors_search - 1) / 2;
  float t = floorf((up - det->u_min) * det->inv_sector_width);
  int32_t c = t < 0.0f ? 0 : (t > (float)(S - 1) ? S - 1 : (int32_t)t);
  int32_t s_lo = c - half < 0 ? 0 : c - half;
  int32_t s_hi = c + half > S - 1 ? S - 1 : c + half;
  int64_t H0 = hit_offsets[layer_bank0 + s_lo];
  int64_t H1 = hit_offsets[layer_bank0 + s_hi + 1];
  float lo = up - W, hi = up + W;
  int64_t first = H0;
  while (first < H1 && !(hit_u[first] >= lo)) ++first;
  int64_t end = first;
  while (end < H1 && !(hit_u[end] > hi)) ++end;
  /* keep the max_hits hits nearest to the prediction: drop the farther end, the right one on a tie */
  while (end - first > par->max_hits) {
    float dl = up - hit_u[first];
    float dr = hit_u[end - 1] - up;
    if (dr >= dl) --end; else ++first;
  }
  *first_out = first;
  *end_out = end;
}

typedef struct {
  int valid;
  int nhits;
  float qop, chi2;
  int32_t idx[NL];
} ora_candidate;

/* One-parameter weighted least squares in q/p with the VELO state held fixed (the p-kick chi2 fit
   of Section III-C, done "in combination with the VELO track" as in Section V-B).  Residual of a
   hit: r = m - xs, model r = a_kick * qop.  Layers are summed in order 0..3. */
static void fit_candidate(const ora_detector* det, const ora_extrap* x, const float* hit_u,
                          const float* hit_weight, const int32_t idx[NL], float* qop_out,
                          float* chi2_out)
{
  float r[NL];
  float Sar = 0.0f, Saa = 0.0f;
  for (int l = 0; l < NL; ++l) {
    if (idx[l] < 0) continue;
    float m = hit_u[idx[l]] + x->yl[l] * det->dxdy[l];
    r[l] = m - x->xs[l];
    float wa = hit_weight[idx[l]] * det->a_kick[l];
    Sar = Sar + wa * r[l];
    Saa = Saa + wa * det->a_kick[l];
  }
  float qop = Sar / Saa;
  float chi2 = 0.0f;
  for (int l = 0; l < NL; ++l) {
    if (idx[l] < 0) continue;
    float e = r[l] - det->a_kick[l] * qop;
    chi2 = chi2 + (hit_weight[idx[l]] * e) * e;
  }
  *qop_out = qop;
  *chi2_out = chi2;
}

/* Selection order (Section V-B: prefer 4 hits over 3, then the lowest chi2); remaining ties go to
   the lexicographically smallest hit-index tuple (missing hit = -1) so the choice is unique. */
static int better(int nhits, float chi2, const int32_t idx[NL], const ora_candidate* best)
{
  if (!best->valid) return 1;
  if (nhits != best->nhits) return nhits > best->nhits;
  if (chi2 < best->chi2) return 1;
  if (chi2 > best->chi2) return 0;
  for (int l = 0; l < NL; ++l)
    if (idx[l] != best->idx[l]) return idx[l] < best->idx[l];
  return 0;
}

/* anchor A, anchor B, completion C1, completion C2: forward uses the first and third panel as
   anchors, backward the same scheme with the panel order reversed (Section V-B) */
static const int DIRS[2][4] = {{0, 2, 1, 3}, {3, 1, 2, 0}};

#define MAX_WIN 32

int ora_compass_find(const ora_detector* det, const ora_params* par, int32_t n_events,
                     const uint32_t* hit_offsets, const float* hit_u, const float* hit_weight,
                     const float* hit_y_begin, const float* hit_y_end,
                     const float* vx, const float* vy, const float* vtx, const float* vty,
                     const uint32_t* velo_offsets,
                     int32_t* hit_idx, float* qop, float* chi2, int32_t* nhits,
                     int32_t* win_first, int32_t* win_size, uint8_t* active)
{
  if (!det || !par || det->n_layers != NL || det->n_sectors <= 0 || n_events < 0 ||
      par->max_hits < 1 || par->max_hits > MAX_WIN || par->n_sectors_search < 1 ||
      par->n_sectors_search % 2 == 0 || !hit_offsets || !velo_offsets)
    return ORA_ERR_ARG;
  const int64_t S = det->n_sectors;
  const float W = par->w0 + par->kw / par->p_min;
  unsigned flags = 0;

  for (int32_t e = 0; e < n_events; ++e) {
    /* window starts are stored relative to their (event, layer) as 16-bit values (Section V-A),
       so an (event, layer) may hold at most 32767 hits */
    int overflow = 0;
    for (int l = 0; l < NL; ++l) {
      int64_t b0 = ((int64_t)e * NL + l) * S;
      if ((int64_t)hit_offsets[b0 + S] - (int64_t)hit_offsets[b0] > 32767) overflow = 1;
    }
    if (overflow) flags |= ORA_FLAG_LAYER_OVERFLOW;

    for (uint32_t t = velo_offsets[e]; t < velo_offsets[e + 1]; ++t) {
      ora_candidate best;
      memset(&best, 0, sizeof best);
      for (int l = 0; l < NL; ++l) {
        hit_idx[(int64_t)t * NL + l] = -1;
        if (win_first) win_first[(int64_t)t * NL + l] = -1;
        if (win_size) win_size[(int64_t)t * NL + l] = 0;
      }
      qop[t] = 0.0f; chi2[t] = 0.0f; nhits[t] = 0;
      if (active) active[t] = 0;
      if (overflow) continue;

      ora_extrap x;
      extrapolate(det, vx[t], vy[t], vtx[t], vty[t], &x);
      if (!in_acceptance(det, &x)) continue;
      if (active) active[t] = 1;

      int64_t wf[NL], we[NL];
      for (int l = 0; l < NL; ++l) {
        find_window(det, par, hit_offsets, hit_u, ((int64_t)e * NL + l) * S, x.up[l], W,
                    &wf[l], &we[l]);
        if (win_first) win_first[(int64_t)t * NL + l] = (int32_t)wf[l];
        if (win_size) win_size[(int64_t)t * NL + l] = (int32_t)(we[l] - wf[l]);
      }

      for (int dir = 0; dir < 2 && !best.valid; ++dir) {
        const int A = DIRS[dir][0], B = DIRS[dir][1], C[2] = {DIRS[dir][2], DIRS[dir][3]};
        int n_tracklets = 0;
        const float inv_dz_ab = 1.0f / (det->z_layer[B] - det->z_layer[A]);
        for (int64_t iA = wf[A]; iA < we[A]; ++iA) {
          /* the strip must cover the track's y (the VELO tolerance check of Section V-A) */
          if (!(hit_y_begin[iA] <= x.yl[A] && x.yl[A] <= hit_y_end[iA])) continue;
          float mA = hit_u[iA] + x.yl[A] * det->dxdy[A];
          for (int64_t iB = wf[B]; iB < we[B]; ++iB) {
            if (!(hit_y_begin[iB] <= x.yl[B] && x.yl[B] <= hit_y_end[iB])) continue;
            float mB = hit_u[iB] + x.yl[B] * det->dxdy[B];
            float slope = (mB - mA) * inv_dz_ab;
            if (!(fabsf(slope - vtx[t]) <= par->slope_tol)) continue;
            /* tolerance window in each completion panel, spanned by the pair slope and the VELO
               slope extrapolated from the first anchor, widened by completion_tol */
            int32_t compat[2][MAX_WIN];
            int ncompat[2] = {0, 0};
            for (int k = 0; k < 2; ++k) {
              int Cl = C[k];
              float d = det->z_layer[Cl] - det->z_layer[A];
              float xt = mA + slope * d;
              float xv = mA + vtx[t] * d;
              float lo = fminf(xt, xv) - par->completion_tol;
              float hi = fmaxf(xt, xv) + par->completion_tol;
              for (int64_t i = wf[Cl]; i < we[Cl]; ++i) {
                if (!(hit_y_begin[i] <= x.yl[Cl] && x.yl[Cl] <= hit_y_end[i])) continue;
                float m = hit_u[i] + x.yl[Cl] * det->dxdy[Cl];
                if (lo <= m && m <= hi) compat[k][ncompat[k]++] = (int32_t)i;
              }
            }
            if (par->max_tracklets > 0) {
              /* the paper's search (Section V-B): in each completion panel the compatible hit
                 closest to the pair-slope extrapolation (the first one on a tie); the pair makes a
                 tracklet when at least one is found; the search stops after max_tracklets tracklets */
              int32_t best_hit[2] = {-1, -1};
              for (int k = 0; k < 2; ++k) {
                float d = det->z_layer[C[k]] - det->z_layer[A];
                float xt = mA + slope * d;
                float bd = 0.0f;
                for (int q = 0; q < ncompat[k]; ++q) {
                  int32_t i = compat[k][q];
                  float m = hit_u[i] + x.yl[C[k]] * det->dxdy[C[k]];
                  float dist = fabsf(m - xt);
                  if (best_hit[k] < 0 || dist < bd) { best_hit[k] = i; bd = dist; }
                }
              }
              if (best_hit[0] < 0 && best_hit[1] < 0) continue;
              int32_t idx[NL];
              idx[A] = (int32_t)iA;
              idx[B] = (int32_t)iB;
              idx[C[0]] = best_hit[0];
              idx[C[1]] = best_hit[1];
              int n = 2 + (best_hit[0] >= 0) + (best_hit[1] >= 0);
              float q, c2;
              fit_candidate(det, &x, hit_u, hit_weight, idx, &q, &c2);
              if (better(n, c2, idx, &best)) {
                best.valid = 1; best.nhits = n; best.qop = q; best.chi2 = c2;
                memcpy(best.idx, idx, sizeof idx);
              }
              if (++n_tracklets >= par->max_tracklets) goto direction_done;
              continue;
            }
            /* every candidate: both anchors, each completion panel with one compatible hit or
               none, at least three hits */
            for (int k1 = -1; k1 < ncompat[0]; ++k1) {
              for (int k2 = -1; k2 < ncompat[1]; ++k2) {
                int n = 2 + (k1 >= 0) + (k2 >= 0);
                if (n < 3) continue;
                int32_t idx[NL];
                idx[A] = (int32_t)iA;
                idx[B] = (int32_t)iB;
                idx[C[0]] = k1 >= 0 ? compat[0][k1] : -1;
                idx[C[1]] = k2 >= 0 ? compat[1][k2] : -1;
                float q, c2;
                fit_candidate(det, &x, hit_u, hit_weight, idx, &q, &c2);
                if (better(n, c2, idx, &best)) {
                  best.valid = 1; best.nhits = n; best.qop = q; best.chi2 = c2;
                  memcpy(best.idx, idx, sizeof idx);
                }
              }
            }
          }
        }
      direction_done:;
        /* the backward direction is only tried when the forward one found nothing */
      }
      if (best.valid) {
        for (int l = 0; l < NL; ++l) hit_idx[(int64_t)t * NL + l] = best.idx[l];
        qop[t] = best.qop;
        chi2[t] = best.chi2;
        nhits[t] = best.nhits;
      }
    }
  }
  return (int)flags;
}

/* ------------------------------------------------------------------------------------------------
 * Fit chi2 with per-sector alignment offsets, and its adjoint.  The hit assignment is frozen; the
 * residual of hit h (layer l, sector s) of track t is
 *     r = ((m_h - offset_s) - xs_l) - a_l * qop_t,   m_h = u_h + y_l * dxdy_l,
 * chi2_t = sum_h w_h r^2,  d chi2 / d qop_t = -2 sum_h w_h a_l r,  d chi2 / d offset_s =
 * -2 sum_{h in s} w_h r, each multiplied by grad_scale.
 * ------------------------------------------------------------------------------------------------ */
double ora_fit_grad_f32(const ora_detector* det, int64_t n_tracks, const int32_t* track_hit_idx,
                        int64_t n_hits, const float* hit_u, const float* hit_weight, const uint32_t* hit_lhcbid,
                        const float* vx, const float* vy, const float* vtx, const float* vty,
                        const float* qop, const float* offsets, float grad_scale,
                        float* chi2_track, float* grad_qop, float* grad_offsets)
{
  const int64_t S = det->n_sectors;
  double* acc = NULL;
  if (grad_offsets) acc = (double*)calloc((size_t)(NL * S), sizeof(double));
  double total = 0.0;
  const float m2s = -2.0f * grad_scale;
  for (int64_t t = 0; t < n_tracks; ++t) {
    float c2 = 0.0f, gq = 0.0f;
    for (int l = 0; l < NL; ++l) {
      int32_t h = track_hit_idx[t * NL + l];
      if (h < 0 || h >= n_hits) continue;
      if ((hit_lhcbid[h] >> 28) >= NL || ((hit_lhcbid[h] >> 12) & 0xFFFFu) >= (uint32_t)S) continue;
      uint32_t id = hit_lhcbid[h];
      int64_t sec = (int64_t)(id >> 28) * S + ((id >> 12) & 0xFFFFu);
      /* The residual is a small difference of terms of a few hundred mm; it is evaluated in
         binary64 (products of binary32 inputs are exact there) and rounded once, so that its
         relative error is one binary32 rounding rather than the cancellation of the large terms. */
      double dz = (double)det->z_layer[l] - (double)det->z_velo;
      double xs = (double)vx[t] + (double)vtx[t] * dz;
      double yl = (double)vy[t] + (double)vty[t] * dz;
      double m = (double)hit_u[h] + yl * (double)det->dxdy[l];
      float r = (float)(((m - (double)offsets[sec]) - xs) - (double)det->a_kick[l] * (double)qop[t]);
      float wr = hit_weight[h] * r;
      c2 = c2 + wr * r;
      gq = gq + wr * det->a_kick[l];
      if (acc) acc[sec] += (double)wr;
    }
    if (chi2_track) chi2_track[t] = c2;
    if (grad_qop) grad_qop[t] = m2s * gq;
    total += (double)c2;
  }
  if (acc) {
    for (int64_t s = 0; s < NL * S; ++s) grad_offsets[s] = (float)(-2.0 * (double)grad_scale * acc[s]);
    free(acc);
  }
  return total;
}

double ora_fit_grad_f64(const ora_detector* det, int64_t n_tracks, const int32_t* track_hit_idx,
                        int64_t n_hits, const float* hit_u, const float* hit_weight, const uint32_t* hit_lhcbid,
                        const float* vx, const float* vy, const float* vtx, const float* vty,
                        const double* qop, const double* offsets, double grad_scale,
                        double* chi2_track, double* grad_qop, double* grad_offsets)
{
  const int64_t S = det->n_sectors;
  if (grad_offsets) memset(grad_offsets, 0, sizeof(double) * (size_t)(NL * S));
  double total = 0.0;
  for (int64_t t = 0; t < n_tracks; ++t) {
    double c2 = 0.0, gq = 0.0;
    for (int l = 0; l < NL; ++l) {
      int32_t h = track_hit_idx[t * NL + l];
      if (h < 0 || h >= n_hits) continue;
      if ((hit_lhcbid[h] >> 28) >= NL || ((hit_lhcbid[h] >> 12) & 0xFFFFu) >= (uint32_t)S) continue;
      double dz = (double)det->z_layer[l] - (double)det->z_velo;
      double xs = (double)vx[t] + (double)vtx[t] * dz;
      double yl = (double)vy[t] + (double)vty[t] * dz;
      uint32_t id = hit_lhcbid[h];
      int64_t sec = (int64_t)(id >> 28) * S + ((id >> 12) & 0xFFFFu);
      double m = (double)hit_u[h] + yl * (double)det->dxdy[l];
      double r = ((m - offsets[sec]) - xs) - (double)det->a_kick[l] * qop[t];
      double wr = (double)hit_weight[h] * r;
      c2 += wr * r;
      gq += wr * (double)det->a_kick[l];
      if (grad_offsets) grad_offsets[sec] += -2.0 * grad_scale * wr;
    }
    if (chi2_track) chi2_track[t] = c2;
    if (grad_qop) grad_qop[t] = -2.0 * grad_scale * gq;
    total += c2;
  }
  return total;
}
