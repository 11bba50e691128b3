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

/* Window of one layer (Section V-A): the sector the prediction points to (the central sector c) and
   its neighbours (1, 3 or 5 sectors, fewer at the layer edges), the hits with u in [up - W, up + W],
   cut to the max_hits hits nearest to the prediction.  Linear scans stand in for the paper's binary
   searches. */
typedef struct {
  int64_t first, end;     /* window hits [first, end), global indices, ascending x */
  int32_t c, s_lo, s_hi;  /* central sector and the allowed sector range */
} ora_window;

static void find_window(const ora_detector* det, const ora_params* par, const uint32_t* hit_offsets,
                        const float* hit_u, int64_t layer_bank0, float up, float W, ora_window* win)
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
  win->first = first;
  win->end = end;
  win->c = c;
  win->s_lo = s_lo;
  win->s_hi = s_hi;
}

/* The hits of a window in the order the paper's search walks its combined ranges (Section V-B): the
   central sector first, then its immediate neighbours, the extreme sectors of a five-sector search
   last; of two neighbours at the same distance the left one (lower sector) first; ascending x
   inside a sector.  Returns the number of hits written to out. */
static int walk_order(const ora_params* par, const uint32_t* hit_offsets, int64_t layer_bank0,
                      const ora_window* win, int64_t* out)
{
  const int32_t half = (par->n_sectors_search - 1) / 2;
  int n = 0;
  for (int32_t k = 0; k <= half; ++k) {
    for (int side = -1; side <= 1; side += 2) {
      if (k == 0 && side == 1) continue;
      int32_t s = win->c + side * k;
      if (s < win->s_lo || s > win->s_hi) continue;
      int64_t lo = hit_offsets[layer_bank0 + s], hi = hit_offsets[layer_bank0 + s + 1];
      if (lo < win->first) lo = win->first;
      if (hi > win->end) hi = win->end;
      for (int64_t i = lo; i < hi; ++i) out[n++] = i;
    }
  }
  return n;
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

/* Selection order (Section V-B: prefer 4 hits over 3, then the lowest chi2).  A chi2 that is not a
   number (a candidate whose hits all weigh 0 fits 0/0) comes after every number; remaining ties go
   to the lexicographically smallest hit-index tuple (missing hit = -1), so the choice is unique. */
static int better(int nhits, float chi2, const int32_t idx[NL], const ora_candidate* best)
{
  if (!best->valid) return 1;
  if (nhits != best->nhits) return nhits > best->nhits;
  int nan_new = isnan(chi2), nan_best = isnan(best->chi2);
  if (nan_new != nan_best) return nan_best;
  if (!nan_new) {
    if (chi2 < best->chi2) return 1;
    if (chi2 > best->chi2) return 0;
  }
  for (int l = 0; l < NL; ++l)
    if (idx[l] != best->idx[l]) return idx[l] < best->idx[l];
  return 0;
}

static void consider(const ora_detector* det, const ora_extrap* x, const float* hit_u,
                     const float* hit_weight, const int32_t idx[NL], ora_candidate* best)
{
  int n = 0;
  for (int l = 0; l < NL; ++l) n += idx[l] >= 0;
  float q, c2;
  fit_candidate(det, x, hit_u, hit_weight, idx, &q, &c2);
  if (better(n, c2, idx, best)) {
    best->valid = 1; best->nhits = n; best->qop = q; best->chi2 = c2;
    memcpy(best->idx, idx, sizeof(int32_t) * NL);
  }
}

/* A hit takes part in the search when its strip covers the track's y (the VELO tolerance check that
   Section V-A repeats in the tracking kernel) and its weight is a usable inverse variance: a
   negative or NaN weight makes the hit unusable, like a strip that misses the track. */
static int usable(const float* hit_y_begin, const float* hit_y_end, const float* hit_weight,
                  int64_t i, float y)
{
  return hit_y_begin[i] <= y && y <= hit_y_end[i] && hit_weight[i] >= 0.0f;
}

/* anchor A, anchor B, completion C1, completion C2: forward uses the first and third panel as
   anchors, backward the same scheme with the panel order reversed (Section V-B) */
static const int DIRS[2][4] = {{0, 2, 1, 3}, {3, 1, 2, 0}};

#define MAX_WIN 32

/* Everything one track's search reads. */
typedef struct {
  const ora_detector* det;
  const ora_params* par;
  const float *u, *w, *yb, *ye;
  float vtx;
  ora_extrap x;
  int64_t walk[NL][MAX_WIN];   /* window hits of each layer in walk order */
  int nwalk[NL];
} ora_track;

/* Slope of an anchor pair and the test of Section V-B: the pair passes when its slope is within
   slope_tol of the VELO slope. */
static int pair_slope(const ora_track* T, int A, int B, int64_t iA, int64_t iB, float* mA_out,
                      float* slope_out)
{
  const ora_detector* det = T->det;
  const float inv_dz_ab = 1.0f / (det->z_layer[B] - det->z_layer[A]);
  float mA = T->u[iA] + T->x.yl[A] * det->dxdy[A];
  float mB = T->u[iB] + T->x.yl[B] * det->dxdy[B];
  float slope = (mB - mA) * inv_dz_ab;
  *mA_out = mA;
  *slope_out = slope;
  return fabsf(slope - T->vtx) <= T->par->slope_tol;
}

/* Completion hits of a passing pair in panel Cl: inside the tolerance window spanned by the pair
   slope and the VELO slope extrapolated from the first anchor, widened by completion_tol.  Written
   to out in walk order; returns their number. */
static int compatible(const ora_track* T, int A, int Cl, float mA, float slope, int64_t* out)
{
  const ora_detector* det = T->det;
  float d = det->z_layer[Cl] - det->z_layer[A];
  float xt = mA + slope * d;
  float xv = mA + T->vtx * d;
  float lo = fminf(xt, xv) - T->par->completion_tol;
  float hi = fmaxf(xt, xv) + T->par->completion_tol;
  int n = 0;
  for (int k = 0; k < T->nwalk[Cl]; ++k) {
    int64_t i = T->walk[Cl][k];
    if (!usable(T->yb, T->ye, T->w, i, T->x.yl[Cl])) continue;
    float m = T->u[i] + T->x.yl[Cl] * det->dxdy[Cl];
    if (lo <= m && m <= hi) out[n++] = i;
  }
  return n;
}

/* Every candidate of one direction (reading R11): both anchors, in each completion panel one
   compatible hit or none, at least three hits; the best one under the selection order. */
static void search_every_combination(const ora_track* T, int dir, ora_candidate* best)
{
  const int A = DIRS[dir][0], B = DIRS[dir][1], C[2] = {DIRS[dir][2], DIRS[dir][3]};
  for (int a = 0; a < T->nwalk[A]; ++a) {
    int64_t iA = T->walk[A][a];
    if (!usable(T->yb, T->ye, T->w, iA, T->x.yl[A])) continue;
    for (int b = 0; b < T->nwalk[B]; ++b) {
      int64_t iB = T->walk[B][b];
      if (!usable(T->yb, T->ye, T->w, iB, T->x.yl[B])) continue;
      float mA, slope;
      if (!pair_slope(T, A, B, iA, iB, &mA, &slope)) continue;
      int64_t compat[2][MAX_WIN];
      int ncompat[2];
      for (int k = 0; k < 2; ++k) ncompat[k] = compatible(T, A, C[k], mA, slope, compat[k]);
      for (int k1 = -1; k1 < ncompat[0]; ++k1) {
        for (int k2 = -1; k2 < ncompat[1]; ++k2) {
          if (k1 < 0 && k2 < 0) continue;
          int32_t idx[NL];
          idx[A] = (int32_t)iA;
          idx[B] = (int32_t)iB;
          idx[C[0]] = k1 >= 0 ? (int32_t)compat[0][k1] : -1;
          idx[C[1]] = k2 >= 0 ? (int32_t)compat[1][k2] : -1;
          consider(T->det, &T->x, T->u, T->w, idx, best);
        }
      }
    }
  }
}

/* The search as the paper runs it (Section V-B), reading R23: the combined ranges are walked in walk
   order, anchor-A hits outermost; for each passing pair the compatible hit closest to the pair-slope
   extrapolation is taken in each completion panel (the first in walk order on a tie); a pair with at
   least one completion hit is a tracklet and is fitted; the search stops after max_tracklets
   tracklets, the best of them by the selection order being kept. */
static void search_as_the_paper(const ora_track* T, int dir, ora_candidate* best)
{
  const ora_detector* det = T->det;
  const int A = DIRS[dir][0], B = DIRS[dir][1], C[2] = {DIRS[dir][2], DIRS[dir][3]};
  int n_tracklets = 0;
  for (int a = 0; a < T->nwalk[A]; ++a) {
    int64_t iA = T->walk[A][a];
    if (!usable(T->yb, T->ye, T->w, iA, T->x.yl[A])) continue;
    for (int b = 0; b < T->nwalk[B]; ++b) {
      int64_t iB = T->walk[B][b];
      if (!usable(T->yb, T->ye, T->w, iB, T->x.yl[B])) continue;
      float mA, slope;
      if (!pair_slope(T, A, B, iA, iB, &mA, &slope)) continue;
      int32_t pick[2] = {-1, -1};
      for (int k = 0; k < 2; ++k) {
        int64_t compat[MAX_WIN];
        int nc = compatible(T, A, C[k], mA, slope, compat);
        float xt = mA + slope * (det->z_layer[C[k]] - det->z_layer[A]);
        float bd = 0.0f;
        for (int q = 0; q < nc; ++q) {
          float m = T->u[compat[q]] + T->x.yl[C[k]] * det->dxdy[C[k]];
          float dist = fabsf(m - xt);
          if (pick[k] < 0 || dist < bd) { pick[k] = (int32_t)compat[q]; bd = dist; }
        }
      }
      if (pick[0] < 0 && pick[1] < 0) continue;
      int32_t idx[NL];
      idx[A] = (int32_t)iA;
      idx[B] = (int32_t)iB;
      idx[C[0]] = pick[0];
      idx[C[1]] = pick[1];
      consider(det, &T->x, T->u, T->w, idx, best);
      if (++n_tracklets >= T->par->max_tracklets) return;
    }
  }
}

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
      par->n_sectors_search % 2 == 0 || par->max_tracklets < 0 || !hit_offsets || !velo_offsets)
    return ORA_ERR_ARG;
  const int64_t S = det->n_sectors;
  const float W = par->w0 + par->kw / par->p_min;
  unsigned flags = 0;
  ora_track T;
  T.det = det;
  T.par = par;
  T.u = hit_u;
  T.w = hit_weight;
  T.yb = hit_y_begin;
  T.ye = hit_y_end;

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

      extrapolate(det, vx[t], vy[t], vtx[t], vty[t], &T.x);
      if (!in_acceptance(det, &T.x)) continue;
      if (active) active[t] = 1;
      T.vtx = vtx[t];

      for (int l = 0; l < NL; ++l) {
        int64_t b0 = ((int64_t)e * NL + l) * S;
        ora_window win;
        find_window(det, par, hit_offsets, hit_u, b0, T.x.up[l], W, &win);
        T.nwalk[l] = walk_order(par, hit_offsets, b0, &win, T.walk[l]);
        if (win_first) win_first[(int64_t)t * NL + l] = (int32_t)win.first;
        if (win_size) win_size[(int64_t)t * NL + l] = (int32_t)(win.end - win.first);
      }

      /* forward first; the backward direction is only tried when the forward one found nothing */
      for (int dir = 0; dir < 2 && !best.valid; ++dir) {
        if (par->max_tracklets > 0) search_as_the_paper(&T, dir, &best);
        else search_every_combination(&T, dir, &best);
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
