// Device helpers shared by the sector, block and H.V kernels: packed state
// labels, sector rank / unrank over digit-sum count tables, successor in
// label order, and the orbit search.
//
// A packed label stores site k's digit a_k = m_k + s in bits [k*b, k*b+b),
// b = ceil(log2(2s+1)).  Comparing packed labels as integers gives the same
// order as comparing the labels n of Eq. (2), so "smallest label in the
// orbit" is the smallest packed word.  Also the start-vector generator of the
// Lanczos chains.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "ftlm.h"

namespace ftlm {
namespace dev {

// Row map of the padded vector layouts: representative i starts at row
// (i / rpl) * rpline + (i % rpl) * dstride (dstride = d_Gamma).  rpl = 1:
// row i * rpline, with rpline = d_Gamma (plain padded rows) or a power of
// two above it (aligned rows); rpl > 1: rpl representatives packed into one
// 128-byte line of rpline rows, counted in 32 bits.
struct PadMap {
  uint32_t dstride, rpl, rpline;
  uint64_t n_reps;
};

__host__ __device__ __forceinline__ uint64_t padded_row(uint32_t dstride, uint32_t rpl, uint32_t rpline, uint64_t i) {
  if (rpl <= 1) return i * (uint64_t)rpline;
  const uint32_t i32 = (uint32_t)i;
  return (uint64_t)(i32 / rpl) * rpline + (uint64_t)(i32 % rpl) * dstride;
}

// The representative i and row k within it that stored row `row` holds;
// false for the rows between packed representatives and past the last one.
__host__ __device__ __forceinline__ bool padded_rep_of(const PadMap& m, uint64_t row, uint64_t& i, int& k) {
  if (m.rpl <= 1) {
    i = row / m.rpline;
    k = (int)(row - i * m.rpline);
    return i < m.n_reps;
  }
  const uint64_t g = row / m.rpline;
  const uint32_t w = (uint32_t)(row - g * m.rpline);
  const uint32_t slot = w / m.dstride;
  k = (int)(w - slot * m.dstride);
  i = g * m.rpl + slot;
  return slot < m.rpl && i < m.n_reps;
}

template <typename W>
__device__ __forceinline__ int digit(W x, int k, int b, W mask) {
  return (int)((x >> (k * b)) & mask);
}

// Number of labels strictly below x in its sector (digits sum to A), in
// ascending label order.  cnt[k * stride + v] = ways for k digits to sum to v.
template <typename W>
__device__ __forceinline__ uint64_t sector_rank(W x, int N, int b, int d, int A, const uint64_t* cnt,
                                                int stride) {
  const W mask = (W(1) << b) - 1;
  uint64_t r = 0;
  int rem = A;
  for (int pos = N - 1; pos >= 0; --pos) {
    int a = digit(x, pos, b, mask);
    for (int t = 0; t < a; ++t) {
      int v = rem - t;
      if (v >= 0) r += cnt[pos * stride + v];
    }
    rem -= a;
  }
  return r;
}

// The label of rank i in the sector.
template <typename W>
__device__ __forceinline__ W sector_unrank(uint64_t i, int N, int b, int d, int A, const uint64_t* cnt,
                                           int stride) {
  W x = 0;
  int rem = A;
  for (int pos = N - 1; pos >= 0; --pos) {
    int a = 0;
    for (; a < d - 1; ++a) {
      int v = rem - a;
      uint64_t c = v >= 0 ? cnt[pos * stride + v] : 0;
      if (i < c) break;
      i -= c;
    }
    x |= W(a) << (pos * b);
    rem -= a;
  }
  return x;
}

// Next larger label with the same digit sum.  For b == 1 the next bit
// permutation with equal popcount; otherwise move one unit up into the
// lowest raisable digit that has a non-zero digit sum below it and refill the
// lower digits with the smallest arrangement (largest digits lowest).
template <typename W>
__device__ __forceinline__ W sector_next(W x, int N, int b, int d) {
  if (b == 1) {
    if (x == 0) return x;
    W t = x | (x - 1);
    int tz = (sizeof(W) == 8) ? __builtin_ctzll((unsigned long long)x) : __builtin_ctz((unsigned)x);
    W nt = ~t;
    W low = nt & (W(0) - nt);
    return (t + 1) | (W((low - 1) >> (tz + 1)));
  }
  const W mask = (W(1) << b) - 1;
  int below = 0;
  for (int k = 0; k < N; ++k) {
    int a = digit(x, k, b, mask);
    if (k > 0 && below >= 1 && a < d - 1) {
      W y = x;
      // clear digits 0..k, set digit k to a + 1, refill 0..k-1 with below - 1
      W clear = (k + 1) * b >= (int)(8 * sizeof(W)) ? ~W(0) : ((W(1) << ((k + 1) * b)) - 1);
      y &= ~clear;
      y |= W(a + 1) << (k * b);
      int rem = below - 1;
      for (int j = 0; j < k && rem > 0; ++j) {
        int v = rem < d - 1 ? rem : d - 1;
        y |= W(v) << (j * b);
        rem -= v;
      }
      return y;
    }
    below += a;
  }
  return x;  // x was the largest label of the sector
}

// Image of x under group element g through 4-bit chunk tables:
// tab[(g * NCH + c) * 16 + v] = packed image of chunk value v at chunk c.
template <typename W, int NCH>
__device__ __forceinline__ W permute(const W* __restrict__ tab, int g, const int* off) {
  const W* t = tab + (size_t)g * (NCH * 16);
  W img = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) img |= t[off[c]];
  return img;
}

template <typename W, int NCH>
__device__ __forceinline__ void chunk_offsets(W a, int* off) {
#pragma unroll
  for (int c = 0; c < NCH; ++c) off[c] = c * 16 + (int)((a >> (4 * c)) & W(15));
}

// Chunk tables of a factored group G = T H (every g = t h exactly once):
// the tables of the |H| elements, then those of the |T| elements, then
// gidx[t * |H| + h] = index of t h (uint16).  With H = {e} the T tables are
// those of every element in index order.
template <typename W, int NCH>
struct OrbitTabs {
  const W* H;
  const W* T;
  const uint16_t* gidx;
  int nH, nT;
};

template <typename W, int NCH>
__device__ __forceinline__ OrbitTabs<W, NCH> orbit_tabs(const W* tab, int nH, int nT) {
  OrbitTabs<W, NCH> o;
  o.H = tab;
  o.T = tab + (size_t)nH * NCH * 16;
  o.gidx = reinterpret_cast<const uint16_t*>(tab + (size_t)(nH + nT) * NCH * 16);
  o.nH = nH;
  o.nT = nT;
  return o;
}

// Orbit minimum and the smallest group index h reaching it (U(h) a = best).
// Every lane of the wave walks the (h, t) pairs in the same order, so the
// table reads of one step hit at most 16 distinct words per chunk; ties on
// the image are broken by the group index, so the result does not depend on
// the walk order.
template <typename W, int NCH>
__device__ __forceinline__ void canon_min(W a, const OrbitTabs<W, NCH>& o, W& best, int& bestg) {
  int offa[NCH];
  chunk_offsets<W, NCH>(a, offa);
  best = a;
  bestg = 0;
  for (int hi = 0; hi < o.nH; ++hi) {
    int off[NCH];
    if (hi == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) off[c] = offa[c];
    } else {
      chunk_offsets<W, NCH>(permute<W, NCH>(o.H, hi, offa), off);
    }
    for (int ti = hi == 0 ? 1 : 0; ti < o.nT; ++ti) {
      const W img = permute<W, NCH>(o.T, ti, off);
      if (img <= best) {
        const int g = o.gidx[ti * o.nH + hi];
        if (img < best || g < bestg) {
          best = img;
          bestg = g;
        }
      }
    }
  }
}

// Orbit minimum over G x Z2 (spin flip F, which reverses label order: F x =
// full - x for packed labels).  The images of the flipped elements (g, 1) are
// F(U(g) a), whose minimum is F of the G-orbit maximum, so one walk keeps the
// minimum and the maximum, each with the smallest index reaching it.  Index
// of (g, f) is f |G| + g, and ties on the label go to the smaller index, so a
// G-element wins a tie with a flipped one.  zf = 0 gives canon_min.
template <typename W, int NCH>
__device__ __forceinline__ void canon_min_z(W a, const OrbitTabs<W, NCH>& o, bool zf, W full, int G, W& best,
                                            int& bestg) {
  if (!zf) {
    canon_min<W, NCH>(a, o, best, bestg);
    return;
  }
  int offa[NCH];
  chunk_offsets<W, NCH>(a, offa);
  best = a;
  bestg = 0;
  W top = a;
  int topg = 0;
  for (int hi = 0; hi < o.nH; ++hi) {
    int off[NCH];
    if (hi == 0) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) off[c] = offa[c];
    } else {
      chunk_offsets<W, NCH>(permute<W, NCH>(o.H, hi, offa), off);
    }
    for (int ti = hi == 0 ? 1 : 0; ti < o.nT; ++ti) {
      const W img = permute<W, NCH>(o.T, ti, off);
      if (img <= best || img >= top) {
        const int g = o.gidx[ti * o.nH + hi];
        if (img < best || (img == best && g < bestg)) {
          best = img;
          bestg = g;
        }
        if (img > top || (img == top && g < topg)) {
          top = img;
          topg = g;
        }
      }
    }
  }
  const W ftop = full - top;
  if (ftop < best) {
    best = ftop;
    bestg = G + topg;
  }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Start-vector element j of the chain keyed by key (SplitMix64, Steele, Lea,
// Flood 2014): Rademacher takes the sign of the top bit of the (j+1)-th output;
// Gaussian draws outputs 2j+1, 2j+2 through the Box-Muller transform.
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__device__ __forceinline__ double start_value(uint64_t key, uint64_t j, int dist) {
  if (dist == FTLM_RADEMACHER) {
    const uint64_t x = mix64(key + (j + 1) * kGamma);
    return (x >> 63) ? -1.0 : 1.0;
  }
  const uint64_t x1 = mix64(key + (2 * j + 1) * kGamma);
  const uint64_t x2 = mix64(key + (2 * j + 2) * kGamma);
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

}  // namespace dev
}  // namespace ftlm
