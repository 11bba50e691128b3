// Decoding of one (event, layer) unit by one wavefront: the device code of the counting and the
// decoding kernels.
#pragma once

#include "common.hpp"

namespace utc {

constexpr uint32_t kMaxBankWords = UTC_MAX_BANK_WORDS;
constexpr int kMinCap = 256;         // smallest chunk of raw words staged in LDS per wavefront
constexpr size_t kWaveLdsDefault = 10 * 1024;   // LDS per wavefront that keeps 16 waves per CU

struct HitsOut {
  uint32_t* lhcbid;
  float* z;
  float* u;
  float* y_begin;
  float* y_end;
  float* weight;
};

// Per-wavefront LDS scratch; cap = raw words staged per chunk.
struct WaveScratch {
  uint32_t* off;    // [S+1] raw word offsets of the unit's banks
  uint32_t* hb;     // [S+1] first hit of each bank inside the current chunk
  float* u0;        // [S] bin-0 position of each sector of the unit's layer
  float* wt;        // [16] weight of each cluster size
  uint16_t* raw;    // [cap] staged raw words; then the arrival slot of each hit in its sort bin;
                    // then the chunk's words in sorted order
  uint16_t* kw;     // [cap] word of each valid word (hit) in bank order
  uint16_t* cbank;  // [cap] bank of each hit
  uint16_t* mark;   // [cap] bank start markers by raw position, then valid words before it; then
                    // the sort's bin counters (two per 4 bytes) and bin starts
  uint16_t* order;  // [cap] hits in bin order
  int cap;
};

__host__ __device__ inline size_t wave_table_bytes(int S) {
  return 2 * sizeof(uint32_t) * (size_t)(S + 1) + sizeof(float) * ((size_t)S + 16);
}

__host__ __device__ inline size_t wave_scratch_bytes(int S, int cap) {
  const size_t b = wave_table_bytes(S) + 5 * sizeof(uint16_t) * (size_t)cap;
  return (b + 15) / 16 * 16;
}

// Largest chunk (a multiple of 64 words, at least kMinCap) whose scratch fits `target` bytes of
// LDS per wavefront.
inline int chunk_words(int S, size_t target) {
  const size_t t = wave_table_bytes(S) + 16;
  int cap = t < target ? (int)((target - t) / (5 * sizeof(uint16_t))) : 0;
  cap = cap / 64 * 64;
  return cap < kMinCap ? kMinCap : (cap > (int)kMaxBankWords ? (int)kMaxBankWords : cap);
}

__device__ inline WaveScratch carve_scratch(char* p, int S, int cap) {
  WaveScratch w;
  w.off = reinterpret_cast<uint32_t*>(p);
  w.hb = w.off + (S + 1);
  w.u0 = reinterpret_cast<float*>(w.hb + (S + 1));
  w.wt = w.u0 + S;
  w.raw = reinterpret_cast<uint16_t*>(w.wt + 16);   // 4-byte aligned, as are all five arrays
  w.kw = w.raw + cap;
  w.cbank = w.kw + cap;
  w.mark = w.cbank + cap;
  w.order = w.mark + cap;
  w.cap = cap;
  return w;
}

__device__ inline bool bank_ok(uint32_t a, uint32_t e) { return e >= a && e - a <= kMaxBankWords; }

struct UnitCount {
  uint32_t T;       // valid words (hits) of the unit
  bool bad;         // some bank is malformed: banks are then handled one by one
  bool staged;      // all of the unit's words are already in ws.raw
};

// Offsets of the unit's banks to LDS, well-formedness checks, hit count; the words are staged in
// LDS on the way when they fit.  Uniform across the wavefront.  With ws.raw == nullptr nothing is
// staged (count only).  With `layer` >= 0 the layer's sector positions and the weight table are
// staged too, their loads issued together with those of the offsets.
__device__ inline UnitCount unit_count(const Geom& g, const uint16_t* __restrict__ words,
                                       const uint32_t* __restrict__ bank_offsets, int64_t b0,
                                       const WaveScratch& ws, uint32_t* flags, int layer = -1)
{
  const int S = g.S;
  const int lane = lane_id();
  const float* __restrict__ u0_row = layer >= 0 ? g.u0 + (size_t)layer * S : nullptr;
  const float wt = (u0_row && lane < 16) ? g.weight_by_size[lane] : 0.f;
  for (int s0 = 0; s0 <= S; s0 += 4 * kWave) {
    uint32_t v[4];
    float t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * kWave + lane;
      v[k] = s <= S ? bank_offsets[b0 + s] : 0u;
      t[k] = (u0_row && s < S) ? u0_row[s] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * kWave + lane;
      if (s <= S) ws.off[s] = v[k];
      if (u0_row && s < S) ws.u0[s] = t[k];
    }
  }
  if (u0_row && lane < 16) ws.wt[lane] = wt;
  wave_sync();
  bool bad = false;
  for (int s = lane; s < S; s += kWave) {
    const uint32_t a = ws.off[s], e = ws.off[s + 1];
    if (e < a) {
      bad = true;
      raise_flag(flags, UTC_FLAG_BANK_ORDER);
    } else if (e - a > kMaxBankWords) {
      bad = true;
      raise_flag(flags, UTC_FLAG_BANK_SIZE);
    }
  }
  UnitCount st;
  st.bad = wave_any(bad);
  st.T = 0;
  st.staged = false;
  if (!st.bad) {
    const uint32_t w0 = ws.off[0];
    const uint32_t nw = ws.off[S] - w0;
    st.staged = ws.raw != nullptr && nw <= (uint32_t)ws.cap;
    // the decoding kernel (ws.raw set) needs the words here only to stage them: a unit that does
    // not fit is read chunk by chunk later, and its hit count comes from the counting kernel
    if (ws.raw != nullptr && !st.staged) return st;
    uint32_t c = 0;
    if ((reinterpret_cast<uintptr_t>(words) & 15u) == 0) {
      // 16-byte loads of 8 words per lane from the aligned word at or before w0
      const uint32_t a0 = w0 & ~7u;
      const uint32_t span = w0 + nw - a0;
      for (uint32_t j0 = 0; j0 < span; j0 += 8 * 2 * kWave) {
        uint4 v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t j = j0 + 8 * (k * kWave + lane);
          v[k] = j < span ? *reinterpret_cast<const uint4*>(words + a0 + j) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t j = j0 + 8 * (k * kWave + lane);
          const uint32_t parts[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
          for (int h = 0; h < 8; ++h) {
            const uint32_t word = (parts[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
            const uint32_t g = a0 + j + (uint32_t)h;   // absolute word index
            if (g >= w0 && g < w0 + nw) {
              if (st.staged) ws.raw[g - w0] = (uint16_t)word;
              c += (word & 0xFu) != 0u;
            }
          }
        }
      }
    } else
    for (uint32_t i0 = 0; i0 < nw; i0 += 8 * kWave) {
      uint16_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t i = i0 + k * kWave + lane;
        v[k] = i < nw ? words[w0 + i] : (uint16_t)0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t i = i0 + k * kWave + lane;
        if (st.staged && i < nw) ws.raw[i] = v[k];
        c += (v[k] & 0xFu) != 0u;
      }
    }
    st.T = wave_sum(c);
  } else {
    uint32_t c = 0;
    for (int s = lane; s < S; s += kWave) {
      const uint32_t a = ws.off[s], e = ws.off[s + 1];
      if (bank_ok(a, e))
        for (uint32_t i = a; i < e; ++i) c += (words[i] & 0xFu) != 0u;
    }
    st.T = wave_sum(c);
  }
  return st;
}

// Decode one raw word of sector s in layer `layer`.
struct DecodedHit {
  uint32_t lhcbid;
  float u, w;
};

__device__ inline DecodedHit decode_word(const Geom& g, int layer, uint32_t s, uint32_t v) {
  const uint32_t size = v & 0xFu, frac = (v >> 4) & 7u, strip = v >> 7;
  DecodedHit d;
  d.lhcbid = ((uint32_t)layer << 28) | (s << 12) | (strip << 3) | frac;
  d.u = fmaf((float)(strip * 8u + frac), g.pitch8, g.u0[layer * g.S + (int)s]);
  d.w = g.weight_by_size[size];
  return d;
}

__device__ inline void store_hit(const Geom& g, float z, const DecodedHit& d, int64_t h,
                                 int64_t capacity, const HitsOut& out, uint32_t* flags) {
  if (h >= capacity) {
    raise_flag(flags, UTC_FLAG_CAPACITY);
    return;
  }
  out.lhcbid[h] = d.lhcbid;
  if (out.z) out.z[h] = z;   // the layer constants are optional outputs
  out.u[h] = d.u;
  if (out.y_begin) out.y_begin[h] = g.y_begin;
  if (out.y_end) out.y_end[h] = g.y_end;
  out.weight[h] = d.w;
}

// A bank too large for the LDS chunk: every hit (64 at a time, in bank order) is ranked against the
// whole bank, whose words pass through LDS a chunk at a time (ws.raw is free here: a unit with such a
// bank is never staged whole).  O(n^2 / 64) LDS compares per wavefront for a bank of n words.
__device__ inline uint32_t big_bank(const Geom& g, const uint16_t* __restrict__ words, int layer,
                                    uint32_t s, uint32_t a, uint32_t n, int64_t first_hit,
                                    int64_t capacity, const WaveScratch& ws, const HitsOut& out,
                                    uint32_t* flags)
{
  const int lane = lane_id();
  const float z_l = g.z_layer[layer];
  const uint32_t cap = (uint32_t)ws.cap & ~3u;
  uint32_t nh = 0;
  for (uint32_t i0 = 0; i0 < n; i0 += kWave) {
    const uint32_t i = i0 + lane;
    const uint32_t v = i < n ? (uint32_t)words[a + i] : 0u;
    const bool valid = (v & 0xFu) != 0u;
    nh += (uint32_t)__popcll(ballot(valid));
    uint32_t rank = 0;
    for (uint32_t t0 = 0; t0 < n; t0 += cap) {
      const uint32_t tn = min(cap, n - t0);
      wave_sync();   // the previous tile is no longer read
      for (uint32_t k = lane; k < tn; k += kWave) ws.raw[k] = words[a + t0 + k];
      for (uint32_t k = tn + lane; k < ((tn + 3u) & ~3u); k += kWave) ws.raw[k] = 0;   // padding
      wave_sync();
      if (valid) {
        // a word o of the bank at position p comes before this hit when it is valid and
        // (o, p) < (v, i); two words per 4-byte LDS read (ws.raw is 4-byte aligned)
        const uint32_t* q = reinterpret_cast<const uint32_t*>(ws.raw);
        for (uint32_t j = 0; j < tn; j += 4) {
          const uint32_t p0 = q[j >> 1], p1 = q[(j >> 1) + 1];
          const uint32_t o[4] = {p0 & 0xFFFFu, p0 >> 16, p1 & 0xFFFFu, p1 >> 16};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const uint32_t pos = t0 + j + (uint32_t)h;
            rank += (uint32_t)(((o[h] & 0xFu) != 0u) & ((o[h] < v) | ((o[h] == v) & (pos < i))));
          }
        }
      }
    }
    if (valid) store_hit(g, z_l, decode_word(g, layer, s, v), first_hit + rank, capacity, out, flags);
  }
  return nh;
}

// Sort bin of hit k (Section IV: hits of a sector are kept in strip order).  Each bank of the chunk
// is cut into as many equal bins of the word's strip and fraction bits (word >> 4, 12 bits) as it
// has hits, numbered from the bank's first hit on: bins of lower banks and lower words come first.
__device__ inline uint32_t hit_bin(const WaveScratch& ws, uint32_t bank, uint32_t word) {
  const uint32_t lo = ws.hb[bank], m = ws.hb[bank + 1] - lo;
  return lo + (((word >> 4) * m) >> 12);
}

// Compaction, sort and store of the unit's hits, first hit `base`.
__device__ inline void unit_write(const Geom& g, const uint16_t* __restrict__ words, int layer,
                                  int64_t b0, uint32_t base, const UnitCount& st,
                                  const WaveScratch& ws, int64_t capacity,
                                  uint32_t* __restrict__ hit_offsets, const HitsOut& out,
                                  uint32_t* flags)
{
  const int S = g.S;
  const int lane = lane_id();
  // read once here: an indexed read of the by-value geometry goes to kernel-argument memory, and
  // inside the store loop it would be repeated (and waited for) after every store
  const float z_l = g.z_layer[layer];
  uint32_t local = 0;
  int c0 = 0;
  while (c0 < S) {
    const uint32_t a0 = ws.off[c0], e0 = ws.off[c0 + 1];
    int c1;
    if (st.bad) {
      if (!bank_ok(a0, e0)) {
        if (lane == 0) hit_offsets[b0 + c0] = base + local;
        ++c0;
        continue;
      }
      c1 = e0 - a0 > (uint32_t)ws.cap ? c0 : c0 + 1;
    } else if (st.staged) {
      c1 = S;   // the whole unit is in LDS already
    } else {
      // the longest run of banks from c0 whose words fit in the staging buffer
      c1 = (int)first_true(c0 + 1, S + 1, [&](int64_t b) { return ws.off[b] - a0 > (uint32_t)ws.cap; }) - 1;
    }
    if (c1 == c0) {
      if (lane == 0) hit_offsets[b0 + c0] = base + local;
      local += big_bank(g, words, layer, (uint32_t)c0, a0, e0 - a0, (int64_t)base + local, capacity, ws,
                        out, flags);
      wave_sync();
      ++c0;
      continue;
    }
    const uint32_t n = ws.off[c1] - a0;
    if (!st.staged && (reinterpret_cast<uintptr_t>(words) & 15u) == 0) {
      // 16-byte loads of 8 words per lane from the aligned word at or before a0
      const uint32_t al = a0 & ~7u;
      const uint32_t span = a0 + n - al;
      for (uint32_t j0 = 0; j0 < span; j0 += 8 * 2 * kWave) {
        uint4 v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t j = j0 + 8 * (k * kWave + lane);
          v[k] = j < span ? *reinterpret_cast<const uint4*>(words + al + j) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t j = j0 + 8 * (k * kWave + lane);
          const uint32_t parts[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
          for (int h = 0; h < 8; ++h) {
            const uint32_t gi = al + j + (uint32_t)h;
            if (gi >= a0 && gi < a0 + n) ws.raw[gi - a0] = (uint16_t)((parts[h >> 1] >> (16 * (h & 1))) & 0xFFFFu);
          }
        }
      }
    } else if (!st.staged) {
      for (uint32_t i0 = 0; i0 < n; i0 += 8 * kWave) {
        uint16_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t i = i0 + k * kWave + lane;
          v[k] = i < n ? words[a0 + i] : (uint16_t)0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t i = i0 + k * kWave + lane;
          if (i < n) ws.raw[i] = v[k];
        }
      }
    }
    // bank start markers (bank + 1 at the first word of every non-empty bank of the chunk)
    for (uint32_t i = lane; i < n; i += kWave) ws.mark[i] = 0;
    wave_sync();
    for (int b = c0 + lane; b < c1; b += kWave)
      if (ws.off[b + 1] > ws.off[b]) ws.mark[ws.off[b] - a0] = (uint16_t)(b + 1);
    wave_sync();

    // stable compaction of the valid words, each with its bank (running maximum of the markers);
    // the marker slot is then reused for the number of valid words before that raw position
    // (four groups of 64 words per pass, their LDS reads and scans independent)
    constexpr int kCompactGroups = 4;
    uint32_t run = 0;
    uint32_t bank_carry = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += kCompactGroups * kWave) {
      uint32_t v[kCompactGroups], bk[kCompactGroups];
#pragma unroll
      for (int k = 0; k < kCompactGroups; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kWave + lane);
        v[k] = i < n ? (uint32_t)ws.raw[i] : 0u;
        bk[k] = i < n ? (uint32_t)ws.mark[i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kCompactGroups; ++k) bk[k] = wave_inclusive_max(bk[k]);
#pragma unroll
      for (int k = 0; k < kCompactGroups; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kWave + lane);
        const bool valid = (v[k] & 0xFu) != 0u;
        const uint32_t b = bk[k] > bank_carry ? bk[k] : bank_carry;
        bank_carry = (uint32_t)__builtin_amdgcn_readlane((int)b, kWave - 1);
        const uint64_t m = ballot(valid);
        const uint32_t pos = run + lanes_before(m);
        if (i < n) ws.mark[i] = (uint16_t)pos;
        if (valid) {
          ws.kw[pos] = (uint16_t)v[k];
          ws.cbank[pos] = (uint16_t)(b - 1);
        }
        run += (uint32_t)__popcll(m);
      }
    }
    const uint32_t nh = run;
    wave_sync();
    for (int b = c0 + lane; b <= c1; b += kWave) {
      const uint32_t r = ws.off[b] - a0;
      ws.hb[b] = r < n ? (uint32_t)ws.mark[r] : nh;
    }
    wave_sync();
    for (int b = c0 + lane; b < c1; b += kWave) hit_offsets[b0 + b] = base + local + ws.hb[b];

    // each hit's rank in its bank by (word, position): a counting sort of the chunk's hits on their
    // bins (hit_bin), then a rank among the few hits of the same bin; the word goes to its sorted
    // slot of the chunk.  Four groups of 64 hits per pass, their LDS reads issued together.
    constexpr int G = 4;
    const uint32_t pad_bank = (uint32_t)c0;   // a valid bank index for lanes past the last hit
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws.mark);   // bin counters, 16 bits each
    for (uint32_t i = lane; i < (nh + 1) / 2; i += kWave) cnt[i] = 0u;
    wave_sync();
    for (uint32_t k0 = 0; k0 < nh; k0 += G * kWave) {
      uint32_t bk[G], w[G], b[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        bk[q] = k < nh ? (uint32_t)ws.cbank[k] : pad_bank;
        w[q] = k < nh ? (uint32_t)ws.kw[k] : 0u;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) b[q] = hit_bin(ws, bk[q], w[q]);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        if (k < nh) {
          const uint32_t sh = 16u * (b[q] & 1u);
          ws.raw[k] = (uint16_t)(atomicAdd(&cnt[b[q] >> 1], 1u << sh) >> sh);
        }
      }
    }
    wave_sync();
    // bin starts, in place: lane l scans the bins [l*L, l*L + L) after a scan of the lane sums
    {
      const uint32_t L = (nh + kWave - 1) / kWave;
      const uint32_t f = (uint32_t)lane * L;
      const uint32_t e = f + L < nh ? f + L : nh;
      uint32_t sum = 0;
      for (uint32_t i = f; i < e; i += 8) {
        uint32_t c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = i + q < e ? (uint32_t)ws.mark[i + q] : 0u;
#pragma unroll
        for (int q = 0; q < 8; ++q) sum += c[q];
      }
      uint32_t tot;
      uint32_t run = wave_excl_scan(sum, &tot);
      for (uint32_t i = f; i < e; i += 8) {
        uint32_t c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = i + q < e ? (uint32_t)ws.mark[i + q] : 0u;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (i + q < e) ws.mark[i + q] = (uint16_t)run;
          run += c[q];
        }
      }
    }
    wave_sync();
    // the hits of each bin in bank order (arrival slots are in no particular order)
    for (uint32_t k0 = 0; k0 < nh; k0 += G * kWave) {
      uint32_t bk[G], w[G], sl[G], b[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        bk[q] = k < nh ? (uint32_t)ws.cbank[k] : pad_bank;
        w[q] = k < nh ? (uint32_t)ws.kw[k] : 0u;
        sl[q] = k < nh ? (uint32_t)ws.raw[k] : 0u;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) b[q] = ws.mark[hit_bin(ws, bk[q], w[q])];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        if (k < nh) ws.order[b[q] + sl[q]] = (uint16_t)k;
      }
    }
    wave_sync();
    uint16_t* sorted = ws.raw;   // the arrival slots are no longer needed
    for (uint32_t k0 = 0; k0 < nh; k0 += G * kWave) {
      uint32_t bk[G], w[G], s0[G], s1[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        bk[q] = k < nh ? (uint32_t)ws.cbank[k] : pad_bank;
        w[q] = k < nh ? (uint32_t)ws.kw[k] : 0u;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t b = hit_bin(ws, bk[q], w[q]);
        s0[q] = ws.mark[b];
        s1[q] = b + 1 < nh ? (uint32_t)ws.mark[b + 1] : nh;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const uint32_t k = k0 + (uint32_t)(q * kWave + lane);
        if (k < nh) {
          // the hits of the bin below (word, position) = (w, k), compared as word << 16 | position,
          // four at a time; a slot past the bin stands for the hit itself, which is not below itself
          const uint32_t mine = (w[q] << 16) | k;
          uint32_t rank = s0[q];
          for (uint32_t j = s0[q]; j < s1[q]; j += 4) {
            uint32_t o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] = j + r < s1[q] ? (uint32_t)ws.order[j + r] : k;
#pragma unroll
            for (int r = 0; r < 4; ++r) rank += (((uint32_t)ws.kw[o[r]] << 16) | o[r]) < mine;
          }
          sorted[rank] = (uint16_t)w[q];
        }
      }
    }
    wave_sync();
    // decode in sorted order and store: the 64 lanes write 64 consecutive hits of each array,
    // four such groups per pass (their LDS reads in flight together).  Sorting stays inside the
    // banks, so sorted slot p belongs to the bank of compacted hit p.
    constexpr int kStoreGroups = 4;
    for (uint32_t p0 = 0; p0 < nh; p0 += kStoreGroups * kWave) {
      uint32_t bk[kStoreGroups], v[kStoreGroups];
      float u0[kStoreGroups], w[kStoreGroups];
#pragma unroll
      for (int k = 0; k < kStoreGroups; ++k) {
        const uint32_t p = p0 + (uint32_t)(k * kWave + lane);
        bk[k] = p < nh ? (uint32_t)ws.cbank[p] : 0u;
        v[k] = p < nh ? (uint32_t)sorted[p] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kStoreGroups; ++k) {
        u0[k] = ws.u0[bk[k]];
        w[k] = ws.wt[v[k] & 0xFu];
      }
#pragma unroll
      for (int k = 0; k < kStoreGroups; ++k) {
        const uint32_t p = p0 + (uint32_t)(k * kWave + lane);
        if (p < nh) {
          const uint32_t frac = (v[k] >> 4) & 7u, strip = v[k] >> 7;
          DecodedHit d;
          d.lhcbid = ((uint32_t)layer << 28) | (bk[k] << 12) | (strip << 3) | frac;
          d.u = fmaf((float)(strip * 8u + frac), g.pitch8, u0[k]);
          d.w = w[k];
          store_hit(g, z_l, d, (int64_t)base + local + p, capacity, out, flags);
        }
      }
    }
    local += nh;
    c0 = c1;
    wave_sync();
  }
}

}  // namespace utc
