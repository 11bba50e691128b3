// Compass tracklet search for a group of 16 VELO tracks by one wavefront (Section V of the paper).
//
// Lane layout for windows: lane = 4*t + l (track t of the group, layer l).  Each lane extrapolates
// its track to its layer, does the binary searches for its window and copies the window's hits
// (x at the track's y, weight or -1 when the strip does not cover the track's y) into an LDS tile.
// Tracklets: the work items (track, anchor-A hit) are spread over the lanes; each finds its passing
// anchor-B hits as a slot range, the passing pairs are handed out in batches of at most 64, each
// pair's completion hits are found as slot ranges, the 4-hit candidates are pruned exactly against
// a seed (see run_batch), and the remaining candidates are flattened over the lanes, fitted, and
// their 64-bit selection keys folded into the track's minimum with an LDS atomic.  The key orders
// candidates exactly like the reference selection (more hits, then lower chi2, then the
// lexicographically smaller hit-index tuple), so the minimum is the same for every schedule.
#pragma once

#include "common.hpp"

namespace utc {

constexpr int kGroupTracks = 16;
constexpr int kPruneMinCandidates = 256;   // 4-hit candidates of a batch below which no pruning
constexpr uint32_t kFilterMinPairs = 128;   // anchor pairs of a group below which no seeds

struct CPar {
  float W;            // window half-width (mm)
  int max_hits;       // per-layer window cap (<= 32)
  int half;           // (n_sectors_search - 1) / 2
  float slope_tol;
  float eps;          // completion interval margin (mm)
  int prune;          // lower-bound pruning of 4-hit candidates allowed (kick factors > 0)
  int max_tracklets;  // 0: every compatible combination; N > 0: the paper's search, N tracklets
};

// Hits of the current event as seen by the search.  kULds / kWLds: u / weight read from LDS
// (event-local index) rather than global memory; the choice is a template parameter so that each
// instantiation addresses one memory space directly.  Hit offsets of the event's 4*S banks are in
// LDS, relative to the event's first hit.
struct EventView {
  const float* u_lds;          // staged u (event-local index)
  const float* u_glb;          // global u
  const float* w_lds;          // staged weights (event-local index)
  const float* w_glb;
  const float* yb_glb;         // nullptr: every strip spans [g.y_begin, g.y_end]
  const float* ye_glb;
  const uint32_t* hoff;        // [4S+1] event-local first hit of each bank
  int64_t first;               // global index of the event's first hit
  bool overflow;               // an (event, layer) holds more than 32767 hits
  float y_lo, y_hi;            // every strip of the event covers [y_lo, y_hi] (empty if unknown)
  uint32_t stride;             // u_lds[k] = u of hit k*stride (1: every hit; 0: nothing staged)
};

template <bool kULds>
__device__ inline float ev_u(const EventView& ev, uint32_t k) {
  if constexpr (kULds) return ev.u_lds[k];
  else return ev.u_glb[ev.first + k];
}

template <bool kWLds>
__device__ inline float ev_w(const EventView& ev, uint32_t k) {
  if constexpr (kWLds) return ev.w_lds[k];
  else return ev.w_glb[ev.first + k];
}

// Per-wavefront LDS of the group.  Tile entries are slot-major (slot j of lane 4t+l at
// j*64 + 4t + l) so that the 64 lanes filling one slot hit 64 different banks.
struct GroupScratch {
  float* tm;          // [max_hits][64] x at the track's y of each window hit
  float* tw;          // [max_hits][64] weight, -1 when unusable
  float* xs;          // [64] straight-line x at each layer
  float* tx;          // [16] VELO slope tx of each track
  int32_t* nwin;      // [64] window sizes
  unsigned long long* best;  // [16] selection key minimum
  unsigned long long* lbk;   // [16] per track: the seed pair proposed so far (two-anchor chi2 bits
                             // << 32 | anchor-A slot << 8 | anchor-B slot), or, in the paper's
                             // search, the number of tracklets found
  uint32_t* umask;    // [64] usable window slots (strip covers the track's y)
  uint32_t* wfirst;   // [64] first hit of each window (event-local), kept here across the search
  uint32_t* poff;     // [17] pair offsets of the tracks
  uint32_t* bp;       // [128] anchor pairs that passed the slope test: t | jA<<8 | jB<<16 (a batch
                      // of at most 64 at the front; in the pruned 4-hit search the pairs kept so
                      // far followed by the next pairs to test)
  uint32_t* bm1;      // [64] their completion masks in layer C1
  uint32_t* bm2;      // [64] their completion masks in layer C2
  uint32_t* boff;     // [65] candidate offsets of the batch
  uint32_t* mk;       // [64] pair starting at each candidate slot of a chunk (index + 1, 0 = none)
  uint32_t* irem;     // [16 * max_hits] passing anchor-B slots of each work item (pruned search)
  float* tz;          // [16] bound of |q| sqrt(Saa) over every candidate of each track
  // the paper's search only: window slots in the order the search walks them (central sector
  // first, see build_walk_order), walk[p] = slot at walk position p, iwalk[slot] = its position
  uint8_t* walk;      // [max_hits][64]
  uint8_t* iwalk;     // [max_hits][64]
};

__host__ __device__ inline size_t group_scratch_bytes(int max_hits, bool greedy) {
  const size_t b = 16 * kGroupTracks + 8 * 64 + 2 * sizeof(float) * 64 * (size_t)max_hits + 4 * 64 +
                   4 * kGroupTracks + 4 * 64 + 4 * (kGroupTracks + 1) + 4 * 128 + 2 * 4 * 64 + 4 * 65 +
                   4 * 64 + 4 * kGroupTracks * (size_t)max_hits + 4 * kGroupTracks +
                   (greedy ? 2 * 64 * (size_t)max_hits : 0);
  return (b + 15) / 16 * 16;
}

__device__ inline GroupScratch carve_group(char* p, int max_hits, bool greedy) {
  GroupScratch s;
  s.best = reinterpret_cast<unsigned long long*>(p);
  s.lbk = s.best + kGroupTracks;
  s.umask = reinterpret_cast<uint32_t*>(s.lbk + kGroupTracks);
  s.wfirst = s.umask + 64;
  s.tm = reinterpret_cast<float*>(s.wfirst + 64);
  s.tw = s.tm + 64 * max_hits;
  s.xs = s.tw + 64 * max_hits;
  s.tx = s.xs + 64;
  s.nwin = reinterpret_cast<int32_t*>(s.tx + kGroupTracks);
  s.poff = reinterpret_cast<uint32_t*>(s.nwin + 64);
  s.bp = s.poff + kGroupTracks + 1;
  s.bm1 = s.bp + 128;
  s.bm2 = s.bm1 + 64;
  s.boff = s.bm2 + 64;
  s.mk = s.boff + 65;
  s.irem = s.mk + 64;
  s.tz = reinterpret_cast<float*>(s.irem + kGroupTracks * max_hits);
  s.walk = greedy ? reinterpret_cast<uint8_t*>(s.tz + kGroupTracks) : nullptr;
  s.iwalk = greedy ? s.walk + 64 * max_hits : nullptr;
  return s;
}

__device__ inline int tile_at(int t, int l, int j) { return j * 64 + t * 4 + l; }

// Walk position <-> window slot of lane 4t+l (the paper's search only).
__device__ inline uint32_t walk_slot(const GroupScratch& s, int t, int l, uint32_t pos) {
  return s.walk[tile_at(t, l, (int)pos)];
}

// A mask of window slots of lane 4t+l as a mask of walk positions.
__device__ inline uint32_t to_walk_mask(const GroupScratch& s, int t, int l, uint32_t m) {
  uint32_t w = 0u;
  for (; m; m &= m - 1u) w |= 1u << s.iwalk[tile_at(t, l, __builtin_ctz(m))];
  return w;
}

// anchor A, anchor B, completion C1, completion C2; forward then backward (panel order reversed)
__device__ inline void dir_layers(int dir, int& A, int& B, int& C1, int& C2) {
  if (dir == 0) { A = 0; B = 2; C1 = 1; C2 = 3; }
  else { A = 3; B = 1; C1 = 2; C2 = 0; }
}

constexpr unsigned long long kNoKey = ~0ull;

// Fit of one candidate (codes: window slot + 1 per layer, 0 = no hit): one-parameter weighted
// least squares in q/p with the VELO state fixed; layers summed in order 0..3.
__device__ inline void fit_codes(const Geom& g, const GroupScratch& s, int t,
                                 const uint32_t code[4], float& q_out, float& chi2_out) {
  float r[kLayers], w[kLayers];
  float Sar = 0.0f, Saa = 0.0f;
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    if (code[l] == 0) continue;
    const int o = tile_at(t, l, (int)code[l] - 1);
    w[l] = s.tw[o];
    r[l] = s.tm[o] - s.xs[t * 4 + l];
    const float wa = w[l] * g.a_kick[l];
    Sar = Sar + wa * r[l];
    Saa = Saa + wa * g.a_kick[l];
  }
  const float q = Sar / Saa;
  float chi2 = 0.0f;
#pragma unroll
  for (int l = 0; l < kLayers; ++l) {
    if (code[l] == 0) continue;
    const float e = r[l] - g.a_kick[l] * q;
    chi2 = chi2 + (w[l] * e) * e;
  }
  q_out = q;
  chi2_out = chi2;
}

__device__ inline unsigned long long make_key(int nh, float chi2, const uint32_t code[4]) {
  return ((unsigned long long)(nh == 4 ? 0u : 1u) << 63) |
         ((unsigned long long)__float_as_uint(chi2) << 24) |
         ((unsigned long long)code[0] << 18) | ((unsigned long long)code[1] << 12) |
         ((unsigned long long)code[2] << 6) | (unsigned long long)code[3];
}

// Position of the n-th (from 0) set bit of m.
__device__ inline uint32_t nth_set_bit(uint32_t m, uint32_t n) {
  for (uint32_t i = 0; i < n; ++i) m &= m - 1;
  return (uint32_t)__builtin_ctz(m);
}

// Bit mask of the window slots [lo, hi) (0 <= lo, hi <= 32).
__device__ inline uint32_t range_mask(uint32_t lo, uint32_t hi) {
  if (hi <= lo) return 0u;
  const uint32_t up = hi >= 32u ? ~0u : ((1u << hi) - 1u);
  return up & ~((1u << lo) - 1u);
}

// Window slots hold the hits in ascending u, so their x at the track's y (u plus one constant,
// rounded) is non-decreasing, and every test of the search that compares a monotone function of
// that x with bounds selects a contiguous slot range; the ranges are found by binary search with
// the test itself as predicate, so they contain exactly the slots the test accepts.

// Anchor-B slots that pass the slope test with anchor-A hit mA: |(mB - mA)/dz - tx| <= slope_tol,
// evaluated as (mB - mA) * (1/dz) - tx in binary32.  The deviation is monotone in mB (decreasing
// when dz < 0, i.e. in the backward direction).
__device__ inline uint32_t slope_range(const GroupScratch& s, int t, int B, float mA, float inv_dz,
                                       float tx, float tol) {
  const uint32_t n = (uint32_t)s.nwin[t * 4 + B];
  // both ends searched in one loop over [0, n) (independent searches, loads issued together); with
  // dz < 0 the deviation decreases along the slots and the two tests swap roles
  const bool up = inv_dz >= 0.0f;
  uint32_t a0 = 0, a1 = n, b0 = 0, b1 = n;
  while (a0 < a1 || b0 < b1) {
    const uint32_t am = a0 + ((a1 - a0) >> 1), bm = b0 + ((b1 - b0) >> 1);
    const float da = a0 < a1 ? (s.tm[tile_at(t, B, (int)am)] - mA) * inv_dz - tx : 0.0f;
    const float db = b0 < b1 ? (s.tm[tile_at(t, B, (int)bm)] - mA) * inv_dz - tx : 0.0f;
    if (a0 < a1) {
      if (up ? (da >= -tol) : (da <= tol)) a1 = am; else a0 = am + 1;
    }
    if (b0 < b1) {
      if (up ? (db > tol) : (db < -tol)) b1 = bm; else b0 = bm + 1;
    }
  }
  return range_mask(a0, b0);
}

// Completion interval of layer Cl for a pair (the one completion_ranges searches).
__device__ inline void completion_bounds(const Geom& g, const CPar& p, const GroupScratch& s, int t,
                                         int A, int Cl, float mA, float slope, float& lo, float& hi) {
  const float d = g.z_layer[Cl] - g.z_layer[A];
  const float xt = mA + slope * d;
  const float xv = mA + s.tx[t] * d;
  lo = fminf(xt, xv) - p.eps;
  hi = fmaxf(xt, xv) + p.eps;
}

// Completion slots of a passing pair in layer Cl: x inside the interval spanned by the pair-slope
// and VELO-slope extrapolations from the first anchor, widened by the completion tolerance.
// Completion slots of a passing pair in both completion layers; the four range ends are searched
// in one loop (independent searches, loads issued together).  In each layer the slots with
// x > hi are a subset of those with x >= lo unless the interval is empty, in which case the mask
// comes out empty either way.
__device__ inline void completion_ranges(const Geom& g, const CPar& p, const GroupScratch& s, int t,
                                         int A, int C1, int C2, float mA, float slope, uint32_t& m1,
                                         uint32_t& m2) {
  float lo1, hi1, lo2, hi2;
  completion_bounds(g, p, s, t, A, C1, mA, slope, lo1, hi1);
  completion_bounds(g, p, s, t, A, C2, mA, slope, lo2, hi2);
  const uint32_t n1 = (uint32_t)s.nwin[t * 4 + C1], n2 = (uint32_t)s.nwin[t * 4 + C2];
  uint32_t a0 = 0, a1 = n1, b0 = 0, b1 = n1, c0 = 0, c1 = n2, d0 = 0, d1 = n2;
  while (a0 < a1 || b0 < b1 || c0 < c1 || d0 < d1) {
    const uint32_t am = a0 + ((a1 - a0) >> 1), bm = b0 + ((b1 - b0) >> 1);
    const uint32_t cm = c0 + ((c1 - c0) >> 1), dm = d0 + ((d1 - d0) >> 1);
    const float xa = a0 < a1 ? s.tm[tile_at(t, C1, (int)am)] : 0.0f;
    const float xb = b0 < b1 ? s.tm[tile_at(t, C1, (int)bm)] : 0.0f;
    const float xc = c0 < c1 ? s.tm[tile_at(t, C2, (int)cm)] : 0.0f;
    const float xd = d0 < d1 ? s.tm[tile_at(t, C2, (int)dm)] : 0.0f;
    if (a0 < a1) { if (xa >= lo1) a1 = am; else a0 = am + 1; }
    if (b0 < b1) { if (xb > hi1) b1 = bm; else b0 = bm + 1; }
    if (c0 < c1) { if (xc >= lo2) c1 = cm; else c0 = cm + 1; }
    if (d0 < d1) { if (xd > hi2) d1 = dm; else d0 = dm + 1; }
  }
  m1 = range_mask(a0, b0);
  m2 = range_mask(c0, d0);
}

// Exact pruning of the 4-hit candidates of one passing anchor pair.
//
// For fixed inputs r_l (x of the hit at the track's y minus the straight line), w_l and a_l, the
// fit's chi2 is the minimum over q of sum_l w_l (r_l - a_l q)^2 (Sections III-C, V-B).  Adding a hit
// adds a non-negative term, so the chi2 of (A, B, c1, c2) is at least that of (A, B, c1), which in
// closed form is chi2_AB + S w e^2 / (S + w a^2), e = r - a q_AB, with S = k_A + k_B, k = w a^2, and
// q_AB = N / S, N = sum w a r, chi2_AB the two-anchor fit; in particular it is at least chi2_AB.  A
// candidate can only be selected if its binary32 chi2 is <= U, the binary32 chi2 of a 4-hit
// candidate of the track already evaluated.  The binary32 evaluation undershoots the real minimum
// by at most
//   E <= 7u chi2 + 2.02u sqrt(chi2) |q| sqrt(Saa),   u = 2^-24,
// (roundings of the products and sums, and of r - a*q at the computed q), with |q| <= max |r/a| over
// the candidate's hits and Saa <= S + the largest k of each completion layer.  Both are bounded per
// pair from the completion intervals (|r| of a completion hit is at most the larger distance of the
// interval ends from the straight line) and the largest weight of the layer's window.  So a
// completion hit whose bound exceeds T = U + 4E (+ a relative 1e-6) cannot be in the selected
// candidate, whatever the other hit is, and a pair whose chi2_AB alone exceeds T has no such hit.
// The test is evaluated in binary64 from the binary32 inputs, multiplied through by S^2 (S + k) so
// that it needs no division:  C (S + k) + S w (r S - a N)^2 <= T S^2 (S + k),  C = chi2_AB S^2.
// E only enters as a margin and is bounded from above in binary32.  Pruning changes which
// candidates are evaluated, never the result; it is skipped where its premises fail (non-finite
// values).
struct AnchorFit {
  double S, N, C;    // k_A + k_B, sum w a r, chi2_AB * S^2
};

__device__ inline AnchorFit anchor_fit(const Geom& g, const GroupScratch& s, int t, int A, int B,
                                       int jA, int jB) {
  const int oA = tile_at(t, A, jA), oB = tile_at(t, B, jB);
  const double rA = s.tm[oA] - s.xs[t * 4 + A], rB = s.tm[oB] - s.xs[t * 4 + B];
  const double wA = s.tw[oA], wB = s.tw[oB];
  const double aA = g.a_kick[A], aB = g.a_kick[B];
  AnchorFit f;
  f.S = wA * aA * aA + wB * aB * aB;
  f.N = wA * aA * rA + wB * aB * rB;
  const double eA = rA * f.S - aA * f.N, eB = rB * f.S - aB * f.N;
  f.C = wA * eA * eA + wB * eB * eB;
  return f;
}

// The part of the test that is common to every completion hit of a pair: T, the pair-level test,
// and the right-hand side of the hit test divided through by (S + k).  In exact arithmetic the hit
// test  C (S + k) + S w e^2 <= T S^2 (S + k)  is  S w e^2 <= (S + k) D,  D = T S^2 - C; D is taken
// with an added 2^-50 (T S^2 + C), more than its rounding errors, and the right-hand side with a
// factor 1 + 1e-12, so that the binary64 evaluation keeps every hit the exact test keeps.
// Z, the bound of |q| sqrt(Saa) that the margin E takes, is per track: every hit of a candidate is
// a usable window slot, so |q| <= max |r / a| over the track's usable window slots of the four
// layers (q is a weighted mean of the r / a of its hits), and Saa <= sum over layers of the largest
// usable weight times a^2.  Computed in binary32 from reciprocals of the kick factors rounded up on
// the host and the hardware square root (within 1 ulp); the factor 1.001 covers those roundings.
struct PruneBound {
  double S, N;     // the pair's k_A + k_B and sum w a r
  double D;        // slackened T S^2 - C, times 1 + 1e-12
  int state;       // 0: test each hit; 1: keep every hit (premises fail); 2: no hit can be kept
};

__device__ inline PruneBound prune_bound(const AnchorFit& f, float Z, float U) {
  constexpr float u = 5.9604644775390625e-08f;   // 2^-24
  // the hardware square root is within 1 ulp; the factor 1.001 covers it
  const float E = (7.0f * u * (2.0f * U + 1.0f) + 2.02f * u * __builtin_amdgcn_sqrtf(2.0f * U + 1.0f) * Z) *
                  1.001f;
  PruneBound b;
  b.S = f.S;
  b.N = f.N;
  b.D = 0.0;
  b.state = 1;
  if (!(E <= U + 1.0f) || !isfinite(f.C)) return b;   // premises fail: keep all
  const double T = (double)U + 4.0 * (double)E + 1e-6 * ((double)U + 1.0);
  const double TS2 = T * (f.S * f.S);
  if (f.C > TS2) {   // chi2_AB alone exceeds the bound
    b.state = 2;
    return b;
  }
  b.D = ((TS2 - f.C) + 0x1p-50 * (TS2 + f.C)) * (1.0 + 1e-12);
  b.state = 0;
  return b;
}

// Completion hits of layer Cl (mask m) that can still be in a selected candidate.
__device__ inline uint32_t prune_mask(const Geom& g, const GroupScratch& s, int t, int Cl, uint32_t m,
                                      const PruneBound& b) {
  if (b.state == 1) return m;
  if (b.state == 2) return 0u;
  const double a = g.a_kick[Cl];
  const double a2 = a * a, aN = a * b.N;
  const float xsl = s.xs[t * 4 + Cl];
  uint32_t keep = 0;
  for (uint32_t mm = m; mm; mm &= mm - 1) {
    const uint32_t j = (uint32_t)__builtin_ctz(mm);
    const int o = tile_at(t, Cl, (int)j);
    const double r = (double)(s.tm[o] - xsl);
    const double w = s.tw[o];
    const double e = r * b.S - aN;
    if ((b.S * w) * (e * e) <= (b.S + w * a2) * b.D) keep |= 1u << j;
  }
  return keep;
}

// Window slot of the hit of mask m in layer Cl nearest (weighted) to the two-anchor fit
// (approximate arithmetic: the choice only steers the pruning).
__device__ inline uint32_t nearest_slot(const Geom& g, const GroupScratch& s, int t, int Cl, uint32_t m,
                                        float qab) {
  const float a = g.a_kick[Cl];
  const float xsl = s.xs[t * 4 + Cl];
  float best = 0.0f;
  uint32_t arg = 0;
  bool any = false;
  for (uint32_t mm = m; mm; mm &= mm - 1) {
    const uint32_t j = (uint32_t)__builtin_ctz(mm);
    const int o = tile_at(t, Cl, (int)j);
    const float e = (s.tm[o] - xsl) - a * qab;
    const float sc = s.tw[o] * e * e;
    if (!any || sc < best) { best = sc; arg = j; any = true; }
  }
  return arg;
}

// The slot of mask m in layer Cl whose x is closest to the pair-slope extrapolation from the first
// anchor (the first one in walk order on a tie), as a one-bit mask; 0 for an empty mask.
__device__ inline uint32_t closest_slot_mask(const Geom& g, const GroupScratch& s, int t, int A, int Cl,
                                             uint32_t m, float mA, float slope) {
  const float xt = mA + slope * (g.z_layer[Cl] - g.z_layer[A]);
  uint32_t arg = 0u;
  float bd = 0.0f;
  bool any = false;
  for (uint32_t wm = to_walk_mask(s, t, Cl, m); wm; wm &= wm - 1) {
    const uint32_t j = walk_slot(s, t, Cl, (uint32_t)__builtin_ctz(wm));
    const float dist = fabsf(s.tm[tile_at(t, Cl, (int)j)] - xt);
    if (!any || dist < bd) { arg = j; bd = dist; any = true; }
  }
  return any ? (1u << arg) : 0u;
}

// One batch of at most 64 passing anchor pairs (s.bp, pairs of one track contiguous): completion
// masks, for 4-hit candidates the seed and the pruning, then the candidates flattened over the
// lanes; each candidate's key is folded into its track's minimum.
__device__ inline void run_batch(const Geom& g, const CPar& p, const GroupScratch& s, int A, int B,
                                 int C1, int C2, float inv_dz_ab, int nhits, uint32_t np) {
  const int lane = lane_id();
  uint32_t m1 = 0, m2 = 0;
  int tt = 0, jA = 0, jB = 0;
  if ((uint32_t)lane < np) {
    const uint32_t b = s.bp[lane];
    tt = (int)(b & 0xFFu);
    jA = (int)((b >> 8) & 0xFFu);
    jB = (int)(b >> 16);
    const float mA = s.tm[tile_at(tt, A, jA)];
    const float mB = s.tm[tile_at(tt, B, jB)];
    const float slope = (mB - mA) * inv_dz_ab;
    completion_ranges(g, p, s, tt, A, C1, C2, mA, slope, m1, m2);
    m1 &= s.umask[tt * 4 + C1];
    m2 &= s.umask[tt * 4 + C2];
  }
  if (nhits == 0) {
    // the paper's search: per pair the completion hit closest to the pair-slope extrapolation in
    // each layer (first on a tie); a pair with at least one is a tracklet; only the first
    // max_tracklets tracklets of each track, in pair order, are candidates
    bool is_tl = false;
    if ((uint32_t)lane < np) {
      const float mA = s.tm[tile_at(tt, A, jA)];
      const float slope = (s.tm[tile_at(tt, B, jB)] - mA) * inv_dz_ab;
      m1 = closest_slot_mask(g, s, tt, A, C1, m1, mA, slope);
      m2 = closest_slot_mask(g, s, tt, A, C2, m2, mA, slope);
      is_tl = (m1 | m2) != 0u;
    }
    // rank of this tracklet among its track's tracklets of the batch (pairs of a track are
    // contiguous lanes), plus the track's tracklets of earlier batches
    const uint64_t tl = ballot(is_tl);
    const int prev_tt = __shfl_up(tt, 1, kWave);
    const bool start = (uint32_t)lane < np && (lane == 0 || prev_tt != tt);
    const uint32_t first = wave_inclusive_max(start ? (uint32_t)lane : 0u);
    const uint32_t rank = (uint32_t)__popcll(tl & __lanemask_lt() & ~((1ull << first) - 1ull));
    const bool take = is_tl && (uint32_t)s.lbk[tt] + rank < (uint32_t)p.max_tracklets;
    wave_sync();
    if (is_tl) atomicAdd(&s.lbk[tt], 1ull);
    if (!take) { m1 = 0u; m2 = 0u; }
  }
  // pruning pays for itself only when the batch has many 4-hit candidates
  uint32_t full_tot = 0;
  if (nhits == 4 && p.prune) {
    const uint32_t full = (uint32_t)lane < np ? (uint32_t)(__popc(m1) * __popc(m2)) : 0u;
    full_tot = wave_sum(full);
  }
  if (nhits == 4 && p.prune && full_tot > (uint32_t)kPruneMinCandidates) {
    // the completion hits that can still be in the track's selected candidate, against the best
    // 4-hit chi2 found so far (the track's seed at least, see seed_tracks)
    if ((uint32_t)lane < np && m1 && m2 && __popc(m1) * __popc(m2) > 1) {
      const unsigned long long bk = s.best[tt];
      const float U = __uint_as_float((uint32_t)(bk >> 24));
      const float Z = s.tz[tt];
      if (bk != kNoKey && isfinite(U) && isfinite(Z)) {
        const PruneBound pb = prune_bound(anchor_fit(g, s, tt, A, B, jA, jB), Z, U);
        m1 = prune_mask(g, s, tt, C1, m1, pb);
        m2 = m1 ? prune_mask(g, s, tt, C2, m2, pb) : 0u;
      }
    }
  }
  uint32_t ncand = 0;
  if ((uint32_t)lane < np) {
    s.bm1[lane] = m1;
    s.bm2[lane] = m2;
    const uint32_t n1 = (uint32_t)__popc(m1), n2 = (uint32_t)__popc(m2);
    ncand = nhits == 4 ? n1 * n2 : (nhits == 3 ? n1 + n2 : ((m1 | m2) ? 1u : 0u));
  }
  uint32_t ctot;
  const uint32_t coff = wave_excl_scan(ncand, &ctot);
  s.boff[lane] = coff;
  if (lane == 0) s.boff[kWave] = ctot;
  wave_sync();
  // candidates of the batch, one per lane; the pair of each candidate slot of a chunk is the last
  // pair starting at or before it (markers at the pairs' first slots, then a running maximum)
  const bool has_cand = ncand > 0u;
  for (uint32_t cb = 0; cb < ctot; cb += kWave) {
    s.mk[lane] = 0u;
    wave_sync();
    if (has_cand && coff >= cb && coff < cb + (uint32_t)kWave) s.mk[coff - cb] = (uint32_t)lane + 1u;
    const uint64_t before = ballot(has_cand && coff <= cb);   // pairs starting at or before the chunk
    wave_sync();
    uint32_t m = s.mk[lane];
    if (lane == 0 && before) m = max(m, (uint32_t)(63 - __builtin_clzll(before)) + 1u);
    const uint32_t pi1 = wave_inclusive_max(m);
    const uint32_t ci = cb + (uint32_t)lane;
    if (ci < ctot) {
      const uint32_t pi = pi1 - 1u;
      const uint32_t rr = ci - s.boff[pi];
      const uint32_t c1m = s.bm1[pi], c2m = s.bm2[pi];
      uint32_t k1, k2;  // window slot + 1 of the completion hits, 0 = none
      if (nhits == 0) {
        k1 = c1m ? (uint32_t)__builtin_ctz(c1m) + 1u : 0u;
        k2 = c2m ? (uint32_t)__builtin_ctz(c2m) + 1u : 0u;
      } else if (nhits == 4) {
        const uint32_t n2 = (uint32_t)__popc(c2m);
        const uint32_t i1 = rr / n2;
        k1 = nth_set_bit(c1m, i1) + 1u;
        k2 = nth_set_bit(c2m, rr - i1 * n2) + 1u;
      } else {
        const uint32_t n1 = (uint32_t)__popc(c1m);
        k1 = rr < n1 ? nth_set_bit(c1m, rr) + 1u : 0u;
        k2 = rr < n1 ? 0u : nth_set_bit(c2m, rr - n1) + 1u;
      }
      const uint32_t b = s.bp[pi];
      const int t2 = (int)(b & 0xFFu);
      const uint32_t a1 = (b >> 8) & 0xFFu, b1 = b >> 16;
      uint32_t code[4];
#pragma unroll
      for (int q = 0; q < kLayers; ++q)
        code[q] = q == A ? a1 + 1u : q == B ? b1 + 1u : q == C1 ? k1 : k2;
      float qop, chi2;
      fit_codes(g, s, t2, code, qop, chi2);
      const int nh = nhits != 0 ? nhits : 2 + (k1 != 0u) + (k2 != 0u);
      atomicMin(&s.best[t2], make_key(nh, chi2, code));
    }
  }
  wave_sync();
}

// Seeds of the pruned 4-hit search.  Each work item (track, usable anchor-A slot) with its passing
// anchor-B slots `rem` proposes the pair with the lowest two-anchor chi2 (approximate arithmetic:
// the choice only steers the pruning); per track the lowest proposal is kept in s.lbk.
__device__ inline void propose_seed(const Geom& g, const GroupScratch& s, int tt, int A, int B,
                                    uint32_t jA, uint32_t rem) {
  const int oA = tile_at(tt, A, (int)jA);
  const float aA = g.a_kick[A], aB = g.a_kick[B];
  const float wA = s.tw[oA];
  const float rAaB = (s.tm[oA] - s.xs[tt * 4 + A]) * aB;
  const float kA = wA * aA * aA;
  const float xsB = s.xs[tt * 4 + B];
  uint32_t best = ~0u, arg = 0;   // lowest |chi2| bits, and its slot (the lowest on a tie)
  for (uint32_t mm = rem; mm; mm &= mm - 1u) {
    const uint32_t jB = (uint32_t)__builtin_ctz(mm);
    const int oB = tile_at(tt, B, (int)jB);
    const float wB = s.tw[oB];
    const float d = rAaB - (s.tm[oB] - xsB) * aA;
    const uint32_t c2 = __float_as_uint(fabsf(__fdividef(wA * wB * d * d, kA + wB * aB * aB)));
    if (c2 < best) {
      best = c2;
      arg = jB;
    }
  }
  if (rem) atomicMin(&s.lbk[tt], ((unsigned long long)best << 32) | (jA << 8) | arg);
}

// Completion slots of a passing pair in one layer Cl (one of the two ranges completion_ranges
// searches together).
__device__ inline uint32_t completion_range(const Geom& g, const CPar& p, const GroupScratch& s, int t,
                                            int A, int Cl, float mA, float slope) {
  float lo, hi;
  completion_bounds(g, p, s, t, A, Cl, mA, slope, lo, hi);
  const uint32_t n = (uint32_t)s.nwin[t * 4 + Cl];
  uint32_t a0 = 0, a1 = n, b0 = 0, b1 = n;
  while (a0 < a1 || b0 < b1) {
    const uint32_t am = a0 + ((a1 - a0) >> 1), bm = b0 + ((b1 - b0) >> 1);
    const float xa = a0 < a1 ? s.tm[tile_at(t, Cl, (int)am)] : 0.0f;
    const float xb = b0 < b1 ? s.tm[tile_at(t, Cl, (int)bm)] : 0.0f;
    if (a0 < a1) { if (xa >= lo) a1 = am; else a0 = am + 1; }
    if (b0 < b1) { if (xb > hi) b1 = bm; else b0 = bm + 1; }
  }
  return range_mask(a0, b0);
}

// Each track's proposed seed pair is completed with the compatible hits nearest to its two-anchor
// fit; when both completion layers have one this is a 4-hit candidate of the track, and its key
// goes into the track's minimum, so that its chi2 bounds the rest.  Four lanes per track (lane
// 4t + l): lanes l = 0 and 1 search completion layers C1 and C2, lane l = 0 fits the candidate.
// want_lane is read on the track's lane 4t.  Every lane calls it.
__device__ inline void seed_tracks(const Geom& g, const CPar& p, const GroupScratch& s, int A, int B,
                                   int C1, int C2, float inv_dz_ab, bool want_lane) {
  const int lane = lane_id();
  const int t = lane >> 2, l = lane & 3;
  const unsigned long long key = s.lbk[t];
  const bool go = __shfl((int)want_lane, lane & ~3, kWave) != 0 && key != kNoKey;
  const int jA = (int)((key >> 8) & 0xFFu), jB = (int)(key & 0xFFu);
  uint32_t m = 0, slot = 0;
  if (go && l < 2) {
    const int Cl = l == 0 ? C1 : C2;
    const int oA = tile_at(t, A, jA), oB = tile_at(t, B, jB);
    const float mA = s.tm[oA];
    const float slope = (s.tm[oB] - mA) * inv_dz_ab;
    m = completion_range(g, p, s, t, A, Cl, mA, slope) & s.umask[t * 4 + Cl];
    if (m) {
      // the two-anchor fit's q in binary32 (it only steers the choice of the completion hits)
      const float aA = g.a_kick[A], aB = g.a_kick[B];
      const float wA = s.tw[oA], wB = s.tw[oB];
      const float qab = __fdividef(wA * aA * (mA - s.xs[t * 4 + A]) + wB * aB * (s.tm[oB] - s.xs[t * 4 + B]),
                                   wA * aA * aA + wB * aB * aB);
      slot = nearest_slot(g, s, t, Cl, m, qab);
    }
  }
  const uint32_t m2 = (uint32_t)__shfl((int)m, lane | 1, kWave);      // layer C2, from lane 4t + 1
  const uint32_t slot2 = (uint32_t)__shfl((int)slot, lane | 1, kWave);
  if (go && l == 0 && m && m2) {
    uint32_t code[4];
    code[A] = (uint32_t)jA + 1u;
    code[B] = (uint32_t)jB + 1u;
    code[C1] = slot + 1u;
    code[C2] = slot2 + 1u;
    float qs, cs;
    fit_codes(g, s, t, code, qs, cs);
    s.best[t] = min(s.best[t], make_key(4, cs, code));
  }
}

// Whether anchor pair (jA, jB) of track tt can hold the track's selected 4-hit candidate: not when
// its two-anchor chi2 alone exceeds the bound T of the best 4-hit chi2 found so far (see
// prune_bound).
__device__ inline bool pair_can_win(const Geom& g, const GroupScratch& s, int tt, int A, int B, int jA,
                                    int jB) {
  const unsigned long long bk = s.best[tt];
  const float U = __uint_as_float((uint32_t)(bk >> 24));
  const float Z = s.tz[tt];
  if (bk == kNoKey || !isfinite(U) || !isfinite(Z)) return true;
  return prune_bound(anchor_fit(g, s, tt, A, B, jA, jB), Z, U).state != 2;
}

// The candidates of one direction with `nhits` hits (4: both completion layers; 3: one of them) for
// the tracks with want_lane set (read on their layer-0 lane).  Work items are (track, anchor-A
// hit); each finds its passing anchor-B hits as one slot range, and the passing pairs are handed
// out in batches of at most 64.
__device__ inline void run_direction(const Geom& g, const CPar& p, const GroupScratch& s, int dir,
                                     int nhits, bool want_lane) {
  const int lane = lane_id();
  const int t = lane >> 2, l = lane & 3;
  int A, B, C1, C2;
  dir_layers(dir, A, B, C1, C2);
  const float inv_dz_ab = 1.0f / (g.z_layer[B] - g.z_layer[A]);
  if (nhits == 0 && lane < kGroupTracks) s.lbk[lane] = 0ull;   // tracklets found per track
  // 4-hit search with pruning allowed: the passing anchor-B slots of every work item first; when
  // the group has more than kFilterMinPairs anchor pairs, a seed candidate per track, and then only
  // the pairs whose two-anchor chi2 leaves room under the best chi2 found so far are batched (kept
  // pairs accumulate in s.bp until a batch of 64 is full)
  const bool slots_first = nhits == 4 && p.prune;
  bool pruned = false;
  if (slots_first && lane < kGroupTracks) s.lbk[lane] = kNoKey;     // seed proposal per track
  const uint32_t cnt = (l == 0 && want_lane) ? (uint32_t)s.nwin[t * 4 + A] : 0u;
  uint32_t total;
  const uint32_t off = wave_excl_scan(cnt, &total);
  if (l == 0) s.poff[t] = off;
  if (lane == 0) s.poff[kGroupTracks] = total;
  wave_sync();
  // track of each work item of the chunk at `base`: markers at the tracks' first items, then a
  // running maximum (every lane calls it)
  auto item_track = [&](uint32_t base) -> int {
    s.mk[lane] = 0u;
    wave_sync();
    if (l == 0 && cnt > 0u && off >= base && off < base + (uint32_t)kWave) s.mk[off - base] = (uint32_t)t + 1u;
    const uint64_t before = ballot(l == 0 && cnt > 0u && off <= base);
    wave_sync();
    uint32_t mtr = s.mk[lane];
    if (lane == 0 && before) mtr = max(mtr, (uint32_t)((63 - __builtin_clzll(before)) >> 2) + 1u);
    return (int)wave_inclusive_max(mtr) - 1;
  };
  if (slots_first) {
    uint32_t npairs = 0;
    for (uint32_t base = 0; base < total; base += kWave) {
      const uint32_t it = base + (uint32_t)lane;
      const int tt = item_track(base);
      uint32_t rem = 0;
      if (it < total) {
        const uint32_t jA = it - s.poff[tt];
        if ((s.umask[tt * 4 + A] >> jA) & 1u) {
          const float mA = s.tm[tile_at(tt, A, (int)jA)];
          rem = slope_range(s, tt, B, mA, inv_dz_ab, s.tx[tt], p.slope_tol) & s.umask[tt * 4 + B];
        }
        s.irem[it] = rem;
      }
      npairs += wave_sum((uint32_t)__popc(rem));
    }
    pruned = npairs > kFilterMinPairs;
    wave_sync();
    if (pruned) {
      for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t it = base + (uint32_t)lane;
        const int tt = item_track(base);
        if (it < total) propose_seed(g, s, tt, A, B, it - s.poff[tt], s.irem[it]);
      }
      wave_sync();
      seed_tracks(g, p, s, A, B, C1, C2, inv_dz_ab, want_lane);
      wave_sync();
    }
  }
  uint32_t nkeep = 0;   // pruned search: pairs kept in s.bp[0, nkeep), waiting for a full batch
  for (uint32_t base = 0; base < total; base += kWave) {
    const uint32_t it = base + (uint32_t)lane;
    uint32_t rem = 0;    // anchor-B slots still to be paired with this lane's anchor-A hit
    uint32_t head = 0;   // track | anchor-A slot << 8
    const int tt = item_track(base);
    if (it < total) {
      // the paper's search takes the anchor-A hits in walk order, the exhaustive one in slot order
      const uint32_t jA = nhits == 0 ? walk_slot(s, tt, A, it - s.poff[tt]) : it - s.poff[tt];
      head = (uint32_t)tt | (jA << 8);
      if (slots_first) {
        rem = s.irem[it];
      } else if ((s.umask[tt * 4 + A] >> jA) & 1u) {
        const float mA = s.tm[tile_at(tt, A, (int)jA)];
        rem = slope_range(s, tt, B, mA, inv_dz_ab, s.tx[tt], p.slope_tol) & s.umask[tt * 4 + B];
        if (nhits == 0) rem = to_walk_mask(s, tt, B, rem);   // anchor-B hits in walk order too
      }
    }
    while (wave_any(rem != 0u)) {
      const uint32_t c = (uint32_t)__popc(rem);
      uint32_t tot;
      const uint32_t o = wave_excl_scan(c, &tot);
      // slots left in the batch for this lane, written without a branch: a conditional form
      // (o >= 64 ? 0 : 64 - o) has been folded by the compiler into the wrapping 64 - o
      const uint32_t room = (uint32_t)kWave - min(o, (uint32_t)kWave);
      const uint32_t take = min(c, room);
      for (uint32_t k = 0; k < take; ++k) {
        uint32_t jB = (uint32_t)__builtin_ctz(rem);
        if (nhits == 0) jB = walk_slot(s, (int)(head & 0xFFu), B, jB);
        rem &= rem - 1u;
        s.bp[nkeep + o + k] = head | (jB << 16);
      }
      wave_sync();
      const uint32_t np = min(tot, (uint32_t)kWave);
      if (!pruned) {
        run_batch(g, p, s, A, B, C1, C2, inv_dz_ab, nhits, np);
        continue;
      }
      // the new pairs s.bp[nkeep, nkeep + np): the ones that can hold their track's winner are
      // moved down behind the kept ones
      uint32_t pr = 0u;
      bool kp = false;
      if ((uint32_t)lane < np) {
        pr = s.bp[nkeep + (uint32_t)lane];
        kp = pair_can_win(g, s, (int)(pr & 0xFFu), A, B, (int)((pr >> 8) & 0xFFu), (int)(pr >> 16));
      }
      const uint64_t km = ballot(kp);
      wave_sync();
      if (kp) s.bp[nkeep + lanes_before(km)] = pr;
      nkeep += (uint32_t)__popcll(km);
      wave_sync();
      if (nkeep >= (uint32_t)kWave) {
        run_batch(g, p, s, A, B, C1, C2, inv_dz_ab, nhits, (uint32_t)kWave);
        const uint32_t rest = nkeep - (uint32_t)kWave;
        const uint32_t v = (uint32_t)lane < rest ? s.bp[kWave + lane] : 0u;
        wave_sync();
        if ((uint32_t)lane < rest) s.bp[lane] = v;
        nkeep = rest;
        wave_sync();
      }
    }
  }
  if (nkeep > 0u) run_batch(g, p, s, A, B, C1, C2, inv_dz_ab, nhits, nkeep);
  wave_sync();
}

// One direction: the 4-hit candidates first; a 3-hit candidate can never be selected over a 4-hit
// one, so 3-hit candidates are only searched for the tracks without a 4-hit candidate.
template <bool kGreedy>
__device__ inline void search_direction(const Geom& g, const CPar& p, const GroupScratch& s,
                                        int dir, bool want_lane) {
  const int t = lane_id() >> 2;
  if constexpr (kGreedy) {   // the paper's search: one pass, 3- and 4-hit tracklets together
    run_direction(g, p, s, dir, 0, want_lane);
    return;
  }
  run_direction(g, p, s, dir, 4, want_lane);
  const bool need3 = want_lane && s.best[t] == kNoKey;
  if (wave_any(need3)) run_direction(g, p, s, dir, 3, need3);
}

}  // namespace utc

namespace utc {

struct TrackIO {
  const float* vx;
  const float* vy;
  const float* vtx;
  const float* vty;
  int32_t* hit_idx;
  float* qop;
  float* chi2;
  int32_t* nhits;
  int16_t* windows;
};

// The whole search for tracks [tbase, min(tbase+16, t1)) of one event.
// VELO state of the track of this lane in the group starting at tbase (zeros past t1).
struct LaneState {
  float x0, y0, tx, ty;
};

__device__ inline LaneState load_state(const TrackIO& io, uint32_t tbase, uint32_t t1) {
  const uint32_t trk = tbase + (uint32_t)(lane_id() >> 2);
  LaneState st{0.0f, 0.0f, 0.0f, 0.0f};
  if (trk < t1) {
    st.x0 = io.vx[trk];
    st.y0 = io.vy[trk];
    st.tx = io.vtx[trk];
    st.ty = io.vty[trk];
  }
  return st;
}

template <bool kULds, bool kWLds, bool kGreedy>
__device__ inline void compass_group(const Geom& g, const CPar& p, const EventView& ev,
                                     const GroupScratch& s, uint32_t tbase, uint32_t t1,
                                     const TrackIO& io, const LaneState& st)
{
  const int lane = lane_id();
  const int t = lane >> 2, l = lane & 3;
  const int S = g.S;
  const int M = p.max_hits;
  const uint32_t trk = tbase + (uint32_t)t;
  const bool has = trk < t1;
  const float x0 = st.x0, y0 = st.y0, tx = st.tx, ty = st.ty;
  // straight-line extrapolation of the VELO state to this lane's layer
  const float dz = g.z_layer[l] - g.z_velo;
  const float xs = x0 + tx * dz;
  const float yl = y0 + ty * dz;
  const float up = xs - yl * g.dxdy[l];
  // acceptance: inside the planes at the first and the last layer
  const float u_max = g.u_min + (float)S * g.sector_width;
  bool ok = true;
  if (l == 0 || l == kLayers - 1)
    ok = (g.y_begin <= yl && yl <= g.y_end) && (g.u_min <= up && up <= u_max);
  const uint64_t okm = ballot(ok);
  // inside at the track's layer-0 lane (4t) and layer-3 lane (4t + 3)
  const bool active = has && !ev.overflow && ((okm >> (lane & ~3)) & 9ull) == 9ull;

  // window (Section V-A): central sector and neighbours, [up - W, up + W], nearest max_hits hits
  uint32_t wf = 0;
  int wn = 0;
  int wc = 0, ws_lo = 0, ws_hi = -1;   // central sector and the allowed sector range
  if (active) {
    const float ts = floorf((up - g.u_min) * g.inv_sector_width);
    const int c = ts < 0.0f ? 0 : (ts > (float)(S - 1) ? S - 1 : (int)ts);
    const int s_lo = c - p.half < 0 ? 0 : c - p.half;
    const int s_hi = c + p.half > S - 1 ? S - 1 : c + p.half;
    wc = c;
    ws_lo = s_lo;
    ws_hi = s_hi;
    const uint32_t H0 = ev.hoff[l * S + s_lo], H1 = ev.hoff[l * S + s_hi + 1];
    const float lo = up - p.W, hi = up + p.W;
    // both edges in one loop (two independent searches over [H0, H1), loads issued together);
    // with a coarse index in LDS the searches first narrow each edge to less than one stride
    uint32_t a0 = H0, a1 = H1, b0 = H0, b1 = H1;
    if (!kULds && ev.stride > 1u && H1 > H0) {
      const uint32_t st = ev.stride;
      const uint32_t c_lo = (H0 + st - 1) / st, c_hi = (H1 - 1) / st + 1;   // coarse entries in [H0, H1)
      uint32_t ca0 = c_lo, ca1 = c_hi, cb0 = c_lo, cb1 = c_hi;
      while (ca0 < ca1 || cb0 < cb1) {
        const uint32_t am = ca0 + ((ca1 - ca0) >> 1), bm = cb0 + ((cb1 - cb0) >> 1);
        const float ua = ca0 < ca1 ? ev.u_lds[am] : 0.0f;
        const float ub = cb0 < cb1 ? ev.u_lds[bm] : 0.0f;
        if (ca0 < ca1) {
          if (ua >= lo) ca1 = am; else ca0 = am + 1;
        }
        if (cb0 < cb1) {
          if (ub > hi) cb1 = bm; else cb0 = bm + 1;
        }
      }
      // the first true hit lies after the last false coarse entry and at or before the first true one
      if (ca0 > c_lo) a0 = (ca0 - 1) * st + 1;
      if (ca0 < c_hi) a1 = ca0 * st;
      if (cb0 > c_lo) b0 = (cb0 - 1) * st + 1;
      if (cb0 < c_hi) b1 = cb0 * st;
    }
    while (a0 < a1 || b0 < b1) {
      const uint32_t am = a0 + ((a1 - a0) >> 1), bm = b0 + ((b1 - b0) >> 1);
      const float ua = a0 < a1 ? ev_u<kULds>(ev, am) : 0.0f;
      const float ub = b0 < b1 ? ev_u<kULds>(ev, bm) : 0.0f;
      if (a0 < a1) {
        if (ua >= lo) a1 = am; else a0 = am + 1;
      }
      if (b0 < b1) {
        if (ub > hi) b1 = bm; else b0 = bm + 1;
      }
    }
    uint32_t first = a0;
    uint32_t end = b0 < first ? first : b0;
    if (end - first > (uint32_t)M) {
      // the M nearest hits: the first start f whose left hit is no farther than the hit just past
      // the window (identical to dropping the farther end one hit at a time, the right on a tie)
      first = first_true_u32(first, end - (uint32_t)M, [&](uint32_t f) {
        return (up - ev_u<kULds>(ev, f)) <= (ev_u<kULds>(ev, f + (uint32_t)M) - up);
      });
      end = first + (uint32_t)M;
    }
    wf = first;
    wn = (int)(end - first);
  }
  s.nwin[lane] = wn;
  s.xs[lane] = xs;
  if (l == 0) {
    s.tx[t] = tx;
    s.best[t] = kNoKey;
  }
  // tile: x at the track's y and weight of each window hit; -1 marks a strip that does not cover y.
  // Per-hit strip ranges are read only when the track's y is outside the range that every strip
  // of the event covers; without them (NULL) every strip spans the detector's range.
  const bool per_hit_y = ev.yb_glb && !(ev.y_lo <= yl && yl <= ev.y_hi);
  const float g_yb = ev.yb_glb ? -INFINITY : g.y_begin, g_ye = ev.yb_glb ? INFINITY : g.y_end;
  uint32_t umask = 0;
  float wm = 0.0f;
  float rz = 0.0f;   // largest |x - xs| over the usable window slots
  for (int j0 = 0; j0 < wn; j0 += 8) {
    float uu[8], ww[8], yb[8], ye[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t k = wf + (uint32_t)(j0 + q);
      const bool in = j0 + q < wn;
      uu[q] = 0.0f;
      ww[q] = 0.0f;
      yb[q] = g_yb;
      ye[q] = g_ye;
      if (in) {
        uu[q] = ev_u<kULds>(ev, k);
        ww[q] = ev_w<kWLds>(ev, k);
        if (per_hit_y) {
          yb[q] = ev.yb_glb[ev.first + k];
          ye[q] = ev.ye_glb[ev.first + k];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (j0 + q < wn) {
        const float w = (yb[q] <= yl && yl <= ye[q]) ? ww[q] : -1.0f;
        const float xm = uu[q] + yl * g.dxdy[l];
        s.tm[tile_at(t, l, j0 + q)] = xm;
        s.tw[tile_at(t, l, j0 + q)] = w;
        if (w >= 0.0f) {
          umask |= 1u << (j0 + q);
          wm = fmaxf(wm, w);
          rz = fmaxf(rz, fabsf(xm - xs));
        }
      }
    }
  }
  // per-track bound Z of |q| sqrt(Saa) for the pruning margin: the largest |r| / a over the
  // usable window slots and the sum of the largest usable weight times a^2, over the four layers
  rz *= g.inv_a_up[l];
  float kz = wm * g.a_kick[l] * g.a_kick[l];
  rz = fmaxf(rz, __shfl_xor(rz, 1, kWave));
  rz = fmaxf(rz, __shfl_xor(rz, 2, kWave));
  kz = kz + __shfl_xor(kz, 1, kWave);
  kz = kz + __shfl_xor(kz, 2, kWave);
  if (l == 0) s.tz[t] = p.prune ? rz * __builtin_amdgcn_sqrtf(kz) * 1.001f : INFINITY;
  s.umask[lane] = umask;
  s.wfirst[lane] = wf;
  if constexpr (kGreedy) {
    // walk order of the window (Section V-B: the combined sector ranges with the central sector
    // first, then the neighbours at growing distance, the left one first; ascending x inside a
    // sector).  The window [wf, wf + wn) lies inside the allowed sectors, so every slot is placed
    // by distance p.half; both arrays start as the identity, so that with hit offsets that are not
    // ascending every entry still names a slot of the window.
    for (int j = 0; j < wn; ++j) {
      s.walk[tile_at(t, l, j)] = (uint8_t)j;
      s.iwalk[tile_at(t, l, j)] = (uint8_t)j;
    }
    uint32_t pos = 0;
    const uint32_t wend = wf + (uint32_t)wn;
    for (int d = 0; d <= p.half && pos < (uint32_t)wn; ++d) {
      for (int side = -1; side <= 1; side += 2) {
        if (d == 0 && side == 1) continue;
        const int sec = wc + side * d;
        if (sec < ws_lo || sec > ws_hi) continue;
        const uint32_t lo = max(ev.hoff[l * S + sec], wf);
        const uint32_t hi = min(ev.hoff[l * S + sec + 1], wend);
        for (uint32_t k = lo; k < hi && pos < (uint32_t)wn; ++k, ++pos) {
          s.walk[tile_at(t, l, (int)pos)] = (uint8_t)(k - wf);
          s.iwalk[tile_at(t, l, (int)(k - wf))] = (uint8_t)pos;
        }
      }
    }
  }
  wave_sync();

  // tracklets (Section V-B): forward anchors first; backward only where forward found nothing
  search_direction<kGreedy>(g, p, s, 0, active);
  const bool need_back = active && s.best[t] == kNoKey;
  if (wave_any(need_back)) search_direction<kGreedy>(g, p, s, 1, need_back);

  const unsigned long long key = active ? s.best[t] : kNoKey;
  const bool found = key != kNoKey;
  const uint32_t code = found ? (uint32_t)((key >> (6 * (3 - l))) & 63ull) : 0u;
  wf = s.wfirst[lane];   // read back rather than held in a register across the search
  wn = s.nwin[lane];
  if (has) {
    io.hit_idx[(int64_t)trk * 4 + l] = code ? (int32_t)(ev.first + wf + code - 1) : -1;
    if (io.windows) {
      const int64_t o = ((int64_t)trk * 4 + l) * 2;
      io.windows[o] = active ? (int16_t)(wf - ev.hoff[l * S]) : (int16_t)-1;
      io.windows[o + 1] = (int16_t)wn;
    }
    if (l == 0) {
      float q = 0.0f, c2 = 0.0f;
      int nh = 0;
      if (found) {
        uint32_t codes[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) codes[k] = (uint32_t)((key >> (6 * (3 - k))) & 63ull);
        fit_codes(g, s, t, codes, q, c2);
        nh = (key >> 63) ? 3 : 4;
      }
      io.qop[trk] = q;
      io.chi2[trk] = c2;
      io.nhits[trk] = nh;
    }
  }
  wave_sync();
}

}  // namespace utc
