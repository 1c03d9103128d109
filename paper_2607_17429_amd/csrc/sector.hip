// Irrep-independent preprocessing of one magnetization sector (paper
// Section 3): orbit representatives, stabilizers, the rank lookup, Eq. (16)
// diagonal energies and the per-flip entry table (target representative,
// connecting element, flip), all built by GPU kernels.
//
// Representatives (Section 2.3: the smallest label of each orbit) come from a
// sweep over the sector in rank order: thread t owns ranks [64t, 64t + 64),
// unranks the first label, steps through the next 63 in label order and sets
// bit k of word t when no group element maps the label to a smaller one.  The
// bitmap over sector ranks, with per-word prefix counts, is also the lookup:
// index(r) = base[rank(r) >> 6] + popcount of the lower bits of that word.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "device.h"
#include "dispatch.h"
#include "internal.h"
#include "tune_cache.h"

namespace ftlm {

namespace {

constexpr int kThreads = 256;

template <typename W, bool LDS>
__device__ __forceinline__ const W* stage_table(const W* g_tab, uint32_t n_words, W* smem) {
  if constexpr (!LDS) {
    return g_tab;
  } else {
    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) smem[i] = g_tab[i];
    __syncthreads();
    return smem;
  }
}

struct SecArgs {
  const void* tab;   // factored chunk tables (dev::OrbitTabs layout)
  const uint64_t* cnt;
  int cnt_stride;
  int N, b, d, A, G, nH, nT;
  int zf;          // resolve by the spin flip too (G x Z2)
  uint64_t full;   // packed label with every digit d - 1 (F x = full - x)
  uint64_t D_M, n_words, n_reps;
  uint32_t tab_words;
};

// ---- representative sweep --------------------------------------------------
template <typename W, int NCH, bool LDS>
__global__ void __launch_bounds__(kThreads) k_enum(SecArgs a, uint64_t* __restrict__ bits_out) {
  extern __shared__ uint64_t smem_raw[];
  const W* tab = stage_table<W, LDS>((const W*)a.tab, a.tab_words, (W*)smem_raw);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const dev::OrbitTabs<W, NCH> o = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.n_words; w += stride) {
    W x = dev::sector_unrank<W>(w * 64, a.N, a.b, a.d, a.A, a.cnt, a.cnt_stride);
    uint64_t bits = 0;
    for (int k = 0; k < 64; ++k) {
      const bool valid = w * 64 + k < a.D_M;
      int offx[NCH];
      dev::chunk_offsets<W, NCH>(x, offx);
      const W fx = (W)a.full - x;
      bool smaller = a.zf && fx < x;  // (e, F)
      // walk g = t h; every lane runs the same trip counts, so the vote is uniform
      int step = 0;
      for (int hi = 0; hi < o.nH; ++hi) {
        int off[NCH];
        if (hi == 0) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) off[c] = offx[c];
        } else {
          dev::chunk_offsets<W, NCH>(dev::permute<W, NCH>(o.H, hi, offx), off);
        }
        bool done = false;
        for (int ti = hi == 0 ? 1 : 0; ti < o.nT; ++ti) {
          const W img = dev::permute<W, NCH>(o.T, ti, off);
          smaller |= img < x || (a.zf && img > fx);  // F(img) < x
          if ((++step & 3) == 0 && __all(smaller || !valid)) {
            done = true;
            break;
          }
        }
        if (done) break;
      }
      if (valid && !smaller) bits |= 1ull << k;
      x = dev::sector_next<W>(x, a.N, a.b, a.d);
    }
    bits_out[w] = bits;
  }
}

__global__ void k_popcount(const uint64_t* __restrict__ bits, uint64_t* __restrict__ out, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = __popcll(bits[i]);
}

__global__ void k_to_u32(const uint64_t* __restrict__ in, uint32_t* __restrict__ out, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)in[i];
}

template <typename W>
__global__ void __launch_bounds__(kThreads) k_extract(SecArgs a, const uint64_t* __restrict__ bits,
                                                     const uint32_t* __restrict__ base, uint64_t* __restrict__ reps) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.n_words; w += stride) {
    uint64_t m = bits[w];
    if (!m) continue;
    W x = dev::sector_unrank<W>(w * 64, a.N, a.b, a.d, a.A, a.cnt, a.cnt_stride);
    uint64_t j = base[w];
    const int top = 63 - __clzll(m);
    for (int k = 0; k <= top; ++k) {
      if ((m >> k) & 1) reps[j++] = (uint64_t)x;
      if (k < top) x = dev::sector_next<W>(x, a.N, a.b, a.d);
    }
  }
}

// ---- stabilizers -----------------------------------------------------------
// flag[i] = 1 when some g != e fixes representative i.
template <typename W, int NCH, bool LDS>
__global__ void __launch_bounds__(kThreads) k_stab_flag(SecArgs a, const uint64_t* __restrict__ reps,
                                                       uint64_t* __restrict__ flag) {
  extern __shared__ uint64_t smem_raw[];
  const W* tab = stage_table<W, LDS>((const W*)a.tab, a.tab_words, (W*)smem_raw);
  const dev::OrbitTabs<W, NCH> o = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_reps; i += stride) {
    const W r = (W)reps[i];
    int offr[NCH];
    dev::chunk_offsets<W, NCH>(r, offr);
    const W fr = (W)a.full - r;
    bool fixed = a.zf && fr == r;  // (e, F)
    int step = 0;
    for (int hi = 0; hi < o.nH; ++hi) {
      int off[NCH];
      if (hi == 0) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) off[c] = offr[c];
      } else {
        dev::chunk_offsets<W, NCH>(dev::permute<W, NCH>(o.H, hi, offr), off);
      }
      bool done = false;
      for (int ti = hi == 0 ? 1 : 0; ti < o.nT; ++ti) {
        const W img = dev::permute<W, NCH>(o.T, ti, off);
        fixed |= img == r || (a.zf && img == fr);
        if ((++step & 3) == 0 && __all(fixed)) {
          done = true;
          break;
        }
      }
      if (done) break;
    }
    flag[i] = fixed ? 1 : 0;
  }
}

// Full stabilizer masks of the representatives with a non-trivial stabilizer,
// written compacted (pos = exclusive scan of the flags, pos[n_reps] = count).
template <typename W, int NCH, bool LDS>
__global__ void __launch_bounds__(kThreads) k_stab_mask(SecArgs a, const uint64_t* __restrict__ reps,
                                                       const uint64_t* __restrict__ pos, int mw,
                                                       uint64_t* __restrict__ masks, uint64_t* __restrict__ idx_out) {
  extern __shared__ uint64_t smem_raw[];
  const W* tab = stage_table<W, LDS>((const W*)a.tab, a.tab_words, (W*)smem_raw);
  const dev::OrbitTabs<W, NCH> o = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_reps; i += stride) {
    const uint64_t p = pos[i];
    if (pos[i + 1] == p) continue;
    const W r = (W)reps[i];
    const W fr = (W)a.full - r;
    int offr[NCH];
    dev::chunk_offsets<W, NCH>(r, offr);
    uint64_t* mk = masks + p * mw;
    for (int wq = 0; wq < mw; ++wq) mk[wq] = 0;
    for (int hi = 0; hi < o.nH; ++hi) {
      int off[NCH];
      dev::chunk_offsets<W, NCH>(dev::permute<W, NCH>(o.H, hi, offr), off);
      for (int ti = 0; ti < o.nT; ++ti) {
        const W img = dev::permute<W, NCH>(o.T, ti, off);
        const int g = o.gidx[ti * o.nH + hi];
        if (img == r) mk[g >> 6] |= 1ull << (g & 63);   // this lane's own mask words
        if (a.zf && img == fr) {
          const int gf = a.G + g;                       // (g, F)
          mk[gf >> 6] |= 1ull << (gf & 63);
        }
      }
    }
    idx_out[p] = i;
  }
}

__global__ void __launch_bounds__(kThreads) k_first_trivial(const uint64_t* __restrict__ pos, uint64_t n,
                                                           unsigned long long* out) {
  __shared__ unsigned long long red[kThreads];
  unsigned long long best = ~0ull;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    if (pos[i + 1] == pos[i]) {
      best = i;
      break;  // later i of this lane are larger
    }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != ~0ull) atomicMin(out, red[0]);
}

__global__ void k_assign_stab(const uint64_t* __restrict__ pos, uint64_t n, const uint16_t* __restrict__ ids_nt,
                              uint16_t trivial_id, uint16_t* __restrict__ stab_id) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = pos[i];
    stab_id[i] = (pos[i + 1] != p) ? ids_nt[p] : trivial_id;
  }
}

// ---- flips (Eq. 3) -----------------------------------------------------------
struct FlipArgs {
  const int32_t* bonds;
  const double* J;
  int nbonds;
};

template <typename W>
__device__ __forceinline__ bool admissible(W p, int cand, const FlipArgs& f, int b, int d, W mask) {
  const int bond = cand >> 1;
  const int i = f.bonds[2 * bond], j = f.bonds[2 * bond + 1];
  const int ai = dev::digit(p, i, b, mask), aj = dev::digit(p, j, b, mask);
  return (cand & 1) ? (ai > 0 && aj < d - 1) : (ai < d - 1 && aj > 0);
}

template <typename W>
__device__ __forceinline__ W apply_flip(W p, int cand, const FlipArgs& f, int b) {
  const int bond = cand >> 1;
  const int i = f.bonds[2 * bond], j = f.bonds[2 * bond + 1];
  const W ui = W(1) << (i * b), uj = W(1) << (j * b);
  return (cand & 1) ? (p - ui + uj) : (p + ui - uj);
}

template <typename W>
__device__ __forceinline__ int next_admissible(W p, int cur, int ncand, const FlipArgs& f, int b, int d, W mask) {
  for (int c = cur + 1; c < ncand; ++c)
    if (admissible(p, c, f, b, d, mask)) return c;
  return -1;
}

template <typename W>
__global__ void __launch_bounds__(kThreads) k_entry_count(SecArgs a, FlipArgs f, const uint64_t* __restrict__ reps,
                                                         uint64_t* __restrict__ counts, double* __restrict__ ediag) {
  const W mask = (W(1) << a.b) - 1;
  const double s = 0.5 * (a.d - 1);
  const int ncand = 2 * f.nbonds;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_reps; i += stride) {
    const W p = (W)reps[i];
    uint64_t c = 0;
    for (int q = 0; q < ncand; ++q) c += admissible(p, q, f, a.b, a.d, mask) ? 1 : 0;
    counts[i] = c;
    double e = 0;
    for (int bnd = 0; bnd < f.nbonds; ++bnd) {
      const double mi = dev::digit(p, f.bonds[2 * bnd], a.b, mask) - s;
      const double mj = dev::digit(p, f.bonds[2 * bnd + 1], a.b, mask) - s;
      e += f.J[bnd] * mi * mj;
    }
    ediag[i] = e;
  }
}

template <typename W>
__device__ __forceinline__ bool lookup(W r, const SecArgs& a, const uint64_t* __restrict__ bits,
                                       const uint32_t* __restrict__ base, uint64_t& idx) {
  const uint64_t rk = dev::sector_rank<W>(r, a.N, a.b, a.d, a.A, a.cnt, a.cnt_stride);
  if (rk >= a.D_M) return false;
  const uint64_t w = rk >> 6;
  const uint64_t m = bits[w];
  const int k = (int)(rk & 63);
  idx = base[w] + (uint64_t)__popcll(m & ((1ull << k) - 1));
  return (m >> k) & 1;
}

// One lane per representative; in round t every lane canonicalizes its t-th
// admissible flip, so all lanes walk the group elements together.
template <typename W, int NCH, bool LDS>
__global__ void __launch_bounds__(kThreads) k_entry_fill(SecArgs a, FlipArgs f, const uint64_t* __restrict__ reps,
                                                        const uint64_t* __restrict__ row_ptr,
                                                        const uint64_t* __restrict__ bits,
                                                        const uint32_t* __restrict__ base,
                                                        uint64_t* __restrict__ entries,
                                                        uint32_t* __restrict__ eidx, uint16_t* __restrict__ ehc,
                                                        int hbits, const uint16_t* __restrict__ stab_id,
                                                        uint16_t triv_sid) {
  extern __shared__ uint64_t smem_raw[];
  const W* tab = stage_table<W, LDS>((const W*)a.tab, a.tab_words, (W*)smem_raw);
  const dev::OrbitTabs<W, NCH> o = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  const W mask = (W(1) << a.b) - 1;
  const int ncand = 2 * f.nbonds;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n_iter = (a.n_reps + stride - 1) / stride;  // same trip count on every lane
  for (uint64_t it = 0; it < n_iter; ++it) {
    const uint64_t i = it * stride + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < a.n_reps;
    const W p = live ? (W)reps[i] : W(0);
    uint64_t out = live ? row_ptr[i] : 0;
    int cur = live ? next_admissible<W>(p, -1, ncand, f, a.b, a.d, mask) : -1;
    while (__any(cur >= 0)) {
      const W x = cur >= 0 ? apply_flip<W>(p, cur, f, a.b) : p;
      W r;
      int h;
      dev::canon_min_z<W, NCH>(x, o, a.zf, (W)a.full, a.G, r, h);
      if (cur >= 0) {
        uint64_t idx = 0;
        bool ok = lookup<W>(r, a, bits, base, idx);
        // a canonical label of the sector is always a representative
        // top bit: the target's stabilizer is trivial (its n_Gamma, L and V
        // are then known without reading its stabilizer id)
        const bool triv = ok && stab_id[idx] == triv_sid;
        if (eidx) {
          eidx[out] = ok ? (uint32_t)idx : 0xFFFFFFFFu;
          ehc[out] = (uint16_t)(h | (cur << hbits) | (triv ? 0x8000 : 0));
          ++out;
        } else {
          entries[out++] = (ok ? idx : 0xFFFFFFFFull) | ((uint64_t)h << 32) | ((uint64_t)cur << 48) |
                           (triv ? (1ull << 63) : 0ull);
        }
        cur = next_admissible<W>(p, cur, ncand, f, a.b, a.d, mask);
      }
    }
  }
}

// ---- orbit search for arbitrary labels (test / export entry point) ---------
template <typename W, int NCH, bool LDS>
__global__ void __launch_bounds__(kThreads) k_canon_labels(SecArgs a, const uint64_t* __restrict__ bits,
                                                          const uint32_t* __restrict__ base,
                                                          const uint64_t* __restrict__ labels, int64_t n,
                                                          uint64_t* __restrict__ rep_out, int32_t* __restrict__ h_out,
                                                          int64_t* __restrict__ idx_out) {
  extern __shared__ uint64_t smem_raw[];
  const W* tab = stage_table<W, LDS>((const W*)a.tab, a.tab_words, (W*)smem_raw);
  const dev::OrbitTabs<W, NCH> o = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n_iter = (n + stride - 1) / stride;
  for (int64_t it = 0; it < n_iter; ++it) {
    const int64_t i = it * stride + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    uint64_t lab = live ? labels[i] : 0;
    // Eq. (2) label -> packed digits
    W x = 0;
    int sum = 0;
    bool in_range = true;
    {
      uint64_t y = lab;
      for (int k = 0; k < a.N; ++k) {
        int dg = (int)(y % (uint64_t)a.d);
        y /= (uint64_t)a.d;
        x |= W(dg) << (k * a.b);
        sum += dg;
      }
      in_range = (y == 0) && (sum == a.A);
    }
    W r;
    int h;
    dev::canon_min_z<W, NCH>(x, o, a.zf, (W)a.full, a.G, r, h);
    if (live) {
      uint64_t idx = 0;
      bool ok = in_range && lookup<W>(r, a, bits, base, idx);
      // packed -> Eq. (2)
      uint64_t outlab = 0;
      const W mask = (W(1) << a.b) - 1;
      for (int k = a.N - 1; k >= 0; --k) outlab = outlab * (uint64_t)a.d + (uint64_t)dev::digit(r, k, a.b, mask);
      rep_out[i] = in_range ? outlab : 0;
      h_out[i] = in_range ? h : -1;
      idx_out[i] = ok ? (int64_t)idx : -1;
    }
  }
}

unsigned grid_for(uint64_t n, int threads = kThreads, unsigned cap = 65536u * 4) {
  uint64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

int max_lds_bytes() {
  static int v = -1;
  if (v < 0) {
    int dev = 0, x = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0)
      v = std::min(x, 65536);
    else
      v = 65536;
  }
  return v;
}

}  // namespace

std::shared_ptr<Sector> build_sector(const ftlm_cluster* cl, std::shared_ptr<const Group> G, int two_M,
                                     const ftlm_opts* opts) {
  if (!cl || !G) fail(FTLM_ERR_INVALID_ARG, "null cluster or group");
  auto S = std::make_shared<Sector>();
  Sector& s = *S;
  s.G = G;
  s.N = cl->N;
  s.two_s = cl->two_s;
  s.two_M = two_M;
  if (s.N != G->N) fail(FTLM_ERR_INVALID_ARG, "cluster N differs from the group's N");
  if (s.two_s < 1 || s.two_s > 62) fail(FTLM_ERR_INVALID_ARG, "two_s must be in 1..62");
  if (G->order > 1024) fail(FTLM_ERR_GROUP_TOO_LARGE, "sector tables support |G| <= 1024");
  s.d = s.two_s + 1;
  s.bits = 0;
  while ((1 << s.bits) < s.d) ++s.bits;
  if (s.N * s.bits > 64) fail(FTLM_ERR_UNSUPPORTED, "packed labels need more than 64 bits");
  s.wide = s.N * s.bits > 32;
  s.nch = nch_bucket((s.N * s.bits + 3) / 4);
  // spin flip (G x Z2) at M = 0
  s.zflip = opts && opts->spin_flip;
  if (s.zflip && two_M != 0) fail(FTLM_ERR_INVALID_ARG, "the spin flip resolves only the M = 0 sector");
  s.full = 0;
  for (int k = 0; k < s.N; ++k) s.full |= (uint64_t)(s.d - 1) << (k * s.bits);
  s.gorder = G->order * (s.zflip ? 2 : 1);
  if (cl->nbonds < 0 || (cl->nbonds > 0 && !cl->bonds)) fail(FTLM_ERR_INVALID_ARG, "bad bond list");
  if (cl->nbonds > 16000) fail(FTLM_ERR_INVALID_ARG, "too many bonds");
  s.nbonds = cl->nbonds;
  s.bonds.assign(cl->bonds, cl->bonds + 2 * (size_t)cl->nbonds);
  s.J.resize(s.nbonds);
  std::map<std::pair<int, int>, double> bondmap;
  for (int b = 0; b < s.nbonds; ++b) {
    int i = s.bonds[2 * b], j = s.bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= s.N || j >= s.N || i == j) fail(FTLM_ERR_INVALID_ARG, "bond site out of range");
    s.J[b] = cl->J ? cl->J[b] : 1.0;
    bondmap[{std::min(i, j), std::max(i, j)}] += s.J[b];
  }
  // bond invariance under every group element (weighted, Section 3)
  for (int g = 0; g < G->order; ++g) {
    const int32_t* p = &G->perms[(size_t)g * s.N];
    for (auto& kv : bondmap) {
      int a = p[kv.first.first], c = p[kv.first.second];
      auto it = bondmap.find({std::min(a, c), std::max(a, c)});
      if (it == bondmap.end() || std::fabs(it->second - kv.second) > 1e-12 * std::max(1.0, std::fabs(kv.second)))
        fail(FTLM_ERR_BONDS_NOT_INVARIANT, "bond list is not invariant under the group");
    }
  }
  {
    uint64_t h = fnv1a(&s.N, sizeof(s.N));
    h = fnv1a(&s.two_s, sizeof(s.two_s), h);
    h = fnv1a(s.bonds.data(), s.bonds.size() * sizeof(int32_t), h);
    h = fnv1a(s.J.data(), s.J.size() * sizeof(double), h);
    h = fnv1a(G->perms.data(), G->perms.size() * sizeof(int32_t), h);
    const int zf = s.zflip ? 1 : 0;
    s.cluster_hash = fnv1a(&zf, sizeof(zf), h);
  }
  // digit-sum counts
  const int Amax = s.N * (s.d - 1);
  s.cnt_stride = Amax + 1;
  s.cnt.assign((size_t)(s.N + 1) * s.cnt_stride, 0);
  s.cnt[0] = 1;
  for (int k = 1; k <= s.N; ++k)
    for (int v = 0; v <= Amax; ++v) {
      unsigned __int128 c = 0;
      for (int a = 0; a < s.d && a <= v; ++a) c += s.cnt[(size_t)(k - 1) * s.cnt_stride + v - a];
      s.cnt[(size_t)k * s.cnt_stride + v] = (uint64_t)c;
    }
  const int A2 = s.N * s.two_s + two_M;
  hipStream_t st = tl_alloc_stream;  // the caller's build stream, or the null stream
  if (A2 % 2 != 0 || A2 < 0 || A2 / 2 > Amax) {
    s.A = 0;
    s.D_M = 0;
  } else {
    s.A = A2 / 2;
    s.D_M = s.cnt[(size_t)s.N * s.cnt_stride + s.A];
  }
  s.n_words = (s.D_M + 63) / 64;
  // permutation chunk tables of the factored group (dev::OrbitTabs layout):
  // all |G| elements when their tables take at most 16 KiB, otherwise
  // G = T H with |H| + |T| tables
  const int G_ = G->order;
  const size_t wbytes = s.wide ? 8 : 4;
  std::vector<uint8_t> tab_host;                 // host copies of tables in flight to the device
  std::vector<double> fac(2 * s.d * s.d);
  {
    const int max_plain = (int)std::max<size_t>(1, 16384 / ((size_t)s.nch * 16 * wbytes));
    const Factorization fz = factor_group(*G, max_plain);
    s.fac_nH = (int)fz.H.size();
    s.fac_nT = (int)fz.T.size();
    const size_t rows = (size_t)s.fac_nH + s.fac_nT;
    const size_t tab_bytes = rows * s.nch * 16 * wbytes + fz.gidx.size() * 2;
    s.tab_words = (uint32_t)((tab_bytes + wbytes - 1) / wbytes);
    std::vector<uint8_t> bytes(s.tab_words * wbytes, 0);
    for (size_t row = 0; row < rows; ++row) {
      const int g = row < (size_t)s.fac_nH ? fz.H[row] : fz.T[row - s.fac_nH];
      const int32_t* p = &G->perms[(size_t)g * s.N];
      for (int c = 0; c < s.nch; ++c)
        for (int v = 0; v < 16; ++v) {
          uint64_t img = 0;
          for (int t = 0; t < 4; ++t) {
            if (!((v >> t) & 1)) continue;
            int bit = 4 * c + t;
            if (bit >= s.N * s.bits) continue;
            int site = bit / s.bits, sub = bit % s.bits;
            img |= 1ull << (p[site] * s.bits + sub);
          }
          const size_t at = ((row * s.nch + c) * 16 + v) * wbytes;
          if (s.wide) {
            std::memcpy(&bytes[at], &img, 8);
          } else {
            const uint32_t i32 = (uint32_t)img;
            std::memcpy(&bytes[at], &i32, 4);
          }
        }
    }
    std::memcpy(&bytes[rows * s.nch * 16 * wbytes], fz.gidx.data(), fz.gidx.size() * 2);
    s.d_tab.alloc((bytes.size() + 7) / 8);
    FTLM_HIP(hipMemcpyAsync(s.d_tab.p, bytes.data(), bytes.size(), hipMemcpyHostToDevice, st));
    tab_host.swap(bytes);  // kept until the stream has passed the copy
  }
  // the small tables go up without a wait each; the first synchronization
  // below (after the representative count) covers them
  s.d_cnt.upload_async(s.cnt, st);
  s.d_bonds.upload_async(s.bonds, st);
  s.d_J.upload_async(s.J, st);
  {
    const double sp = 0.5 * s.two_s, ss = sp * (sp + 1);
    for (int ai = 0; ai < s.d; ++ai)
      for (int aj = 0; aj < s.d; ++aj) {
        double mi = ai - sp, mj = aj - sp;
        // sign 0: s_i^+ s_j^-; sign 1: s_i^- s_j^+ (Eq. 3 with J = 1)
        fac[(0 * s.d + ai) * s.d + aj] = 0.5 * std::sqrt(std::max(0.0, ss - mi * (mi + 1))) *
                                         std::sqrt(std::max(0.0, ss - mj * (mj - 1)));
        fac[(1 * s.d + ai) * s.d + aj] = 0.5 * std::sqrt(std::max(0.0, ss - mi * (mi - 1))) *
                                         std::sqrt(std::max(0.0, ss - mj * (mj + 1)));
      }
    s.d_fac.upload_async(fac, st);
  }
  const size_t tab_bytes = (size_t)s.tab_words * wbytes;
  const bool lds = tab_bytes <= (size_t)max_lds_bytes();
  SecArgs a{};
  a.tab = s.d_tab.p;
  a.cnt = s.d_cnt.p;
  a.cnt_stride = s.cnt_stride;
  a.N = s.N;
  a.b = s.bits;
  a.d = s.d;
  a.A = s.A;
  a.G = G_;
  a.zf = s.zflip ? 1 : 0;
  a.full = s.full;
  a.nH = s.fac_nH;
  a.nT = s.fac_nT;
  a.D_M = s.D_M;
  a.n_words = s.n_words;
  a.tab_words = s.tab_words;
  const size_t shm = lds ? tab_bytes : 0;
  FlipArgs f{s.d_bonds.p, s.d_J.p, s.nbonds};

  if (s.D_M == 0) {
    s.n_reps = 0;
    s.d_row_ptr.alloc(1);
    FTLM_HIP(hipMemsetAsync(s.d_row_ptr.p, 0, sizeof(uint64_t), st));
    FTLM_HIP(hipStreamSynchronize(st));
    return S;
  }
  const int64_t limit = opts ? opts->hbm_limit_bytes : 0;
  // representatives
  s.d_rank_bits.alloc(s.n_words);
  FTLM_DISPATCH_NCH(s.nch, {
    if (lds)
      hipLaunchKernelGGL((k_enum<W, NCH, true>), dim3(grid_for(s.n_words)), dim3(kThreads), shm, st, a, s.d_rank_bits.p);
    else
      hipLaunchKernelGGL((k_enum<W, NCH, false>), dim3(grid_for(s.n_words)), dim3(kThreads), 0, st, a, s.d_rank_bits.p);
  });
  FTLM_HIP(hipGetLastError());
  {
    DevBuf<uint64_t> tmp;
    tmp.alloc(s.n_words);
    hipLaunchKernelGGL(k_popcount, dim3(grid_for(s.n_words)), dim3(kThreads), 0, st, s.d_rank_bits.p, tmp.p, s.n_words);
    uint64_t total = 0;
    scan_exclusive_u64(tmp.p, tmp.p, s.n_words, &total, st);
    if (total >= 0xFFFFFFFFull) fail(FTLM_ERR_UNSUPPORTED, "more than 2^32 - 1 representatives");
    s.n_reps = total;
    s.d_rank_base.alloc(s.n_words);
    hipLaunchKernelGGL(k_to_u32, dim3(grid_for(s.n_words)), dim3(kThreads), 0, st, tmp.p, s.d_rank_base.p, s.n_words);
    FTLM_HIP(hipGetLastError());
    FTLM_HIP(hipStreamSynchronize(st));
  }
  a.n_reps = s.n_reps;
  s.d_reps.alloc(s.n_reps);
  FTLM_DISPATCH_NCH(s.nch, {
    hipLaunchKernelGGL((k_extract<W>), dim3(grid_for(s.n_words)), dim3(kThreads), 0, st, a, s.d_rank_bits.p,
                       s.d_rank_base.p, s.d_reps.p);
  });
  FTLM_HIP(hipGetLastError());

  // stabilizers: flags -> compaction -> host interning in first-appearance order
  {
    DevBuf<uint64_t> pos;
    pos.alloc(s.n_reps + 1);
    FTLM_HIP(hipMemsetAsync(pos.p + s.n_reps, 0, sizeof(uint64_t), st));
    FTLM_DISPATCH_NCH(s.nch, {
      if (lds)
        hipLaunchKernelGGL((k_stab_flag<W, NCH, true>), dim3(grid_for(s.n_reps)), dim3(kThreads), shm, st, a, s.d_reps.p, pos.p);
      else
        hipLaunchKernelGGL((k_stab_flag<W, NCH, false>), dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, a, s.d_reps.p, pos.p);
    });
    FTLM_HIP(hipGetLastError());
    uint64_t n_nt = 0;
    scan_exclusive_u64(pos.p, pos.p, s.n_reps + 1, &n_nt, st);
    const int mw = (s.gorder + 63) / 64;
    DevBuf<uint64_t> masks, idx;
    masks.alloc(std::max<uint64_t>(n_nt, 1) * mw);
    idx.alloc(std::max<uint64_t>(n_nt, 1));
    if (n_nt) {
      FTLM_DISPATCH_NCH(s.nch, {
        if (lds)
          hipLaunchKernelGGL((k_stab_mask<W, NCH, true>), dim3(grid_for(s.n_reps)), dim3(kThreads), shm, st, a, s.d_reps.p,
                             pos.p, mw, masks.p, idx.p);
        else
          hipLaunchKernelGGL((k_stab_mask<W, NCH, false>), dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, a, s.d_reps.p,
                             pos.p, mw, masks.p, idx.p);
      });
      FTLM_HIP(hipGetLastError());
    }
    DevBuf<unsigned long long> first;
    first.alloc(1);
    unsigned long long init = ~0ull;
    FTLM_HIP(hipMemcpyAsync(first.p, &init, sizeof(init), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_first_trivial, dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, pos.p, s.n_reps, first.p);
    FTLM_HIP(hipGetLastError());
    std::vector<uint64_t> h_masks(n_nt * mw), h_idx(n_nt);
    if (n_nt) {
      FTLM_HIP(hipMemcpyAsync(h_masks.data(), masks.p, n_nt * mw * 8, hipMemcpyDeviceToHost, st));
      FTLM_HIP(hipMemcpyAsync(h_idx.data(), idx.p, n_nt * 8, hipMemcpyDeviceToHost, st));
    }
    unsigned long long first_trivial = 0;
    FTLM_HIP(hipMemcpyAsync(&first_trivial, first.p, sizeof(first_trivial), hipMemcpyDeviceToHost, st));
    FTLM_HIP(hipStreamSynchronize(st));
    std::map<std::vector<uint64_t>, uint16_t> ids;
    std::vector<uint64_t> trivial_mask(mw, 0);
    trivial_mask[0] = 1;  // identity only
    std::vector<uint16_t> ids_nt(std::max<uint64_t>(n_nt, 1), 0);
    auto intern = [&](const std::vector<uint64_t>& m) -> uint16_t {
      auto it = ids.find(m);
      if (it != ids.end()) return it->second;
      if (ids.size() >= 65535) fail(FTLM_ERR_UNSUPPORTED, "too many distinct stabilizers");
      uint16_t id = (uint16_t)ids.size();
      ids.emplace(m, id);
      std::vector<int32_t> el;
      for (int g = 0; g < s.gorder; ++g)
        if ((m[g / 64] >> (g % 64)) & 1) el.push_back(g);
      s.stab_elems.push_back(el);
      s.stab_size.push_back((uint16_t)el.size());
      return id;
    };
    const bool has_trivial = first_trivial != ~0ull;
    bool trivial_done = !has_trivial;
    uint16_t trivial_id = 0;
    for (uint64_t q = 0; q < n_nt; ++q) {
      if (!trivial_done && h_idx[q] > first_trivial) {
        trivial_id = intern(trivial_mask);
        trivial_done = true;
      }
      std::vector<uint64_t> m(h_masks.begin() + q * mw, h_masks.begin() + (q + 1) * mw);
      ids_nt[q] = intern(m);
    }
    if (!trivial_done) trivial_id = intern(trivial_mask);
    s.trivial_sid = trivial_id;
    s.n_stab = (int32_t)ids.size();
    // representatives per stabilizer id (block dimensions follow from them)
    s.stab_count.assign(s.n_stab, 0);
    s.stab_count[trivial_id] += s.n_reps - n_nt;
    for (uint64_t q = 0; q < n_nt; ++q) s.stab_count[ids_nt[q]] += 1;
    DevBuf<uint16_t> d_ids;
    d_ids.upload_async(ids_nt, st);
    s.d_stab_id.alloc(s.n_reps);
    hipLaunchKernelGGL(k_assign_stab, dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, pos.p, s.n_reps, d_ids.p,
                       trivial_id, s.d_stab_id.p);
    FTLM_HIP(hipGetLastError());
    FTLM_HIP(hipStreamSynchronize(st));  // ids_nt and the temporaries go out of scope
  }

  // diagonal energies and the entry table
  s.d_ediag.alloc(s.n_reps);
  s.d_row_ptr.alloc(s.n_reps + 1);
  FTLM_HIP(hipMemsetAsync(s.d_row_ptr.p + s.n_reps, 0, sizeof(uint64_t), st));
  FTLM_DISPATCH_NCH(s.nch, {
    hipLaunchKernelGGL((k_entry_count<W>), dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, a, f, s.d_reps.p,
                       s.d_row_ptr.p, s.d_ediag.p);
  });
  FTLM_HIP(hipGetLastError());
  uint64_t n_ent = 0;
  scan_exclusive_u64(s.d_row_ptr.p, s.d_row_ptr.p, s.n_reps + 1, &n_ent, st);
  s.n_entries = n_ent;
  // Entry format: 6 bytes (u32 target index + u16 holding h, the flip id and
  // the trivial-target bit) when they fit in 16 bits, 8 bytes (one u64:
  // idx | h << 32 | flip << 48 | trivial << 63) otherwise.
  {
    int hb = 1, cb = 1;
    while ((1 << hb) < s.gorder) ++hb;
    while ((1 << cb) < 2 * s.nbonds) ++cb;
    s.ent_hbits = hb;
    const bool compact_ok = hb + cb <= 15;
    const int fmt = opts ? opts->entry_format : FTLM_ENTRIES_AUTO;
    if (fmt < FTLM_ENTRIES_AUTO || fmt > FTLM_ENTRIES_COMPACT) fail(FTLM_ERR_INVALID_ARG, "bad entry_format");
    if (fmt == FTLM_ENTRIES_COMPACT && !compact_ok)
      fail(FTLM_ERR_UNSUPPORTED, "compact entries need |G| and the flip count to fit 15 bits");
    size_t free_b = 0, total_b = 0;
    FTLM_HIP(hipMemGetInfo(&free_b, &total_b));
    if (fmt == FTLM_ENTRIES_AUTO)
      s.entry_bytes = (compact_ok && (double)n_ent * 8.0 > (double)free_b / 4.0) ? 6 : 8;
    else
      s.entry_bytes = fmt == FTLM_ENTRIES_COMPACT ? 6 : 8;
  }
  int mode = opts ? opts->hv_mode : FTLM_HV_AUTO;
  if (mode == FTLM_HV_AUTO) {
    // the table must leave a third of the free memory for blocks and vectors
    size_t free_b = 0, total_b = 0;
    FTLM_HIP(hipMemGetInfo(&free_b, &total_b));
    mode = ((double)n_ent * s.entry_bytes <= (double)free_b * 2.0 / 3.0) ? FTLM_HV_ENTRIES : FTLM_HV_ONTHEFLY;
  }
  if (limit > 0 && (int64_t)(s.device_bytes() + (mode == FTLM_HV_ENTRIES ? n_ent * s.entry_bytes : 0)) > limit)
    fail(FTLM_ERR_OUT_OF_MEMORY, "sector tables exceed the HBM limit");
  s.hv_mode = mode;
  if (mode == FTLM_HV_ENTRIES && n_ent) {
    if (s.entry_bytes == 6) {
      s.d_eidx.alloc(n_ent);
      s.d_ehc.alloc(n_ent);
    } else {
      s.d_entries.alloc(n_ent);
    }
    FTLM_DISPATCH_NCH(s.nch, {
      if (lds)
        hipLaunchKernelGGL((k_entry_fill<W, NCH, true>), dim3(grid_for(s.n_reps)), dim3(kThreads), shm, st, a, f,
                           s.d_reps.p, s.d_row_ptr.p, s.d_rank_bits.p, s.d_rank_base.p, s.d_entries.p, s.d_eidx.p,
                           s.d_ehc.p, s.ent_hbits, s.d_stab_id.p, (uint16_t)s.trivial_sid);
      else
        hipLaunchKernelGGL((k_entry_fill<W, NCH, false>), dim3(grid_for(s.n_reps)), dim3(kThreads), 0, st, a, f,
                           s.d_reps.p, s.d_row_ptr.p, s.d_rank_bits.p, s.d_rank_base.p, s.d_entries.p, s.d_eidx.p,
                           s.d_ehc.p, s.ent_hbits, s.d_stab_id.p, (uint16_t)s.trivial_sid);
    });
    FTLM_HIP(hipGetLastError());
  }
  FTLM_HIP(hipStreamSynchronize(st));
  return S;
}

void sector_canonicalize(const Sector& s, const uint64_t* labels, int64_t n, uint64_t* rep, int32_t* h,
                         int64_t* index, hipStream_t st) {
  if (n < 0 || (n > 0 && (!labels || !rep || !h || !index))) fail(FTLM_ERR_INVALID_ARG, "bad canonicalize arguments");
  if (n == 0) return;
  SecArgs a{};
  a.tab = s.d_tab.p;
  a.cnt = s.d_cnt.p;
  a.cnt_stride = s.cnt_stride;
  a.N = s.N;
  a.b = s.bits;
  a.d = s.d;
  a.A = s.A;
  a.G = s.G->order;
  a.zf = s.zflip ? 1 : 0;
  a.full = s.full;
  a.nH = s.fac_nH;
  a.nT = s.fac_nT;
  a.D_M = s.D_M;
  a.n_words = s.n_words;
  a.n_reps = s.n_reps;
  a.tab_words = s.tab_words;
  const size_t tab_bytes = (size_t)s.tab_words * (s.wide ? 8 : 4);
  const bool lds = tab_bytes <= (size_t)max_lds_bytes();
  const uint64_t* bits = s.d_rank_bits.p;
  const uint32_t* base = s.d_rank_base.p;
  if (s.D_M == 0) {
    // empty sector: nothing is in range; still run the search for rep/h
    a.D_M = 0;
  }
  FTLM_DISPATCH_NCH(s.nch, {
    if (lds)
      hipLaunchKernelGGL((k_canon_labels<W, NCH, true>), dim3(grid_for((uint64_t)n)), dim3(kThreads), tab_bytes, st, a,
                         bits, base, labels, n, rep, h, index);
    else
      hipLaunchKernelGGL((k_canon_labels<W, NCH, false>), dim3(grid_for((uint64_t)n)), dim3(kThreads), 0, st, a, bits,
                         base, labels, n, rep, h, index);
  });
  FTLM_HIP(hipGetLastError());
}

std::vector<uint64_t> sector_export_labels(const Sector& s) {
  std::vector<uint64_t> packed = s.d_reps.download();
  if (s.d == (1 << s.bits)) return packed;  // packed digits are the Eq. (2) label
  const uint64_t mask = (1ull << s.bits) - 1;
  for (auto& x : packed) {
    uint64_t lab = 0;
    for (int k = s.N - 1; k >= 0; --k) lab = lab * (uint64_t)s.d + ((x >> (k * s.bits)) & mask);
    x = lab;
  }
  return packed;
}

}  // namespace ftlm
