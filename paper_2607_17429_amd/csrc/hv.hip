// Matrix-free H.V in the symmetry-adapted basis (paper Eqs. 15-16).
//
// Gather form used here (derived from Eq. 15 with U(h) a = r for the flipped
// state a = flip_e(p) of output representative p):
//
//   Y[p] = E_diag(p) X[p]
//        + sqrt(L_p) V_p^T  sum_e  c_e(p) / sqrt(L_r)  rho(h)^T  V_r X[r]
//
// with c_e(p) the Eq. (3) coefficient of flip e evaluated on p's digits and
// L = |G| / |Stab|.  One output representative is owned by a group of GL
// lanes (GL = smallest power of two >= nvec, at most 64), lane = vector
// column, so every output element is written by exactly one lane and the sum
// over flips runs in a fixed order (deterministic, no atomics).  Per flip the
// group gathers the n_r contiguous rows of X[r] (n_r * nvec contiguous
// elements), expands them with V_r when the stabilizer is non-trivial,
// contracts with rho(h)^T and accumulates in the d-dimensional irrep space;
// the projection with V_p happens once per output representative.
//
// The flips come either from the sector's entry table (target index, h and
// flip id precomputed once per sector and shared by all irreps) or are found
// on the fly: flip, orbit search over the group, rank lookup.
//
// Lanczos epilogue (EPI): the kernel writes w = s_j (H q_j) - bs_j q_prev
// over q_prev (Y holds q_prev on entry) and per-workgroup FP64 partial sums
// of q_j . w (w as stored), so alpha_j needs no extra pass over the vectors.
#include <algorithm>
#include <cmath>

#include "device.h"
#include "dispatch.h"
#include "internal.h"

namespace ftlm {

namespace {

constexpr int kThreads = 256;
constexpr uint64_t kOffMask = (1ull << 48) - 1;

template <typename T, typename A>
struct HvArgs {
  const uint64_t* reps;
  const uint64_t* row_ptr;
  const uint64_t* entries;
  const uint64_t* meta;
  const double* ediag;
  const A* rhoT;      // [g][beta][gamma]
  const A* V;         // [s][gamma][k]
  const A* stabf;     // [s][4] = n, sqrtL, 1/sqrtL, trivial
  const int32_t* bonds;
  const double* J;
  const double* fac;  // [2][dloc][dloc]
  int b, dloc, nbonds, G, n_stab;
  uint64_t n_reps;
  const T* X;
  T* Y;
  int64_t ld;
  int nvec, GL, log2GL;
  // on-the-fly search
  const void* tab;
  const uint64_t* cnt;
  const uint64_t* rank_bits;
  const uint32_t* rank_base;
  int cnt_stride, N, A_tot;
  uint64_t D_M;
  uint32_t tab_words;
  // Lanczos epilogue
  const double* scal;
  double* partials;
};

template <typename W>
__device__ __forceinline__ bool lookup_rep(W r, int N, int b, int d, int A, const uint64_t* cnt, int stride,
                                           uint64_t D_M, const uint64_t* bits, const uint32_t* base, uint64_t& idx) {
  const uint64_t rk = dev::sector_rank<W>(r, N, b, d, A, cnt, stride);
  if (rk >= D_M) return false;
  const uint64_t m = bits[rk >> 6];
  const int k = (int)(rk & 63);
  idx = base[rk >> 6] + (uint64_t)__popcll(m & ((1ull << k) - 1));
  return (m >> k) & 1;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl((unsigned)(v & 0xffffffffu), src);
  uint32_t hi = __shfl((unsigned)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

template <typename T, typename A, int DG, bool OTF, int NCH, bool LDS_TAB>
__global__ void __launch_bounds__(kThreads) k_hv(HvArgs<T, A> a) {
  const bool EPI = a.partials != nullptr;
  using W = word_t<NCH>;
  extern __shared__ uint64_t smem_raw[];
  const W* tab = nullptr;
  if constexpr (OTF) {
    if constexpr (LDS_TAB) {
      W* s = (W*)smem_raw;
      for (uint32_t i = threadIdx.x; i < a.tab_words; i += blockDim.x) s[i] = ((const W*)a.tab)[i];
      __syncthreads();
      tab = s;
    } else {
      tab = (const W*)a.tab;
    }
  }
  const int lane = threadIdx.x & 63;
  const int GL = a.GL;
  const int lg = lane & (GL - 1);
  const int gbase = lane - lg;
  const int v = blockIdx.y * 64 + lg;
  const bool vok = lg < 64 && v < a.nvec;
  const int slots_per_wave = 64 >> a.log2GL;
  const int waves = blockDim.x >> 6;
  const uint64_t slot = ((uint64_t)blockIdx.x * waves + (threadIdx.x >> 6)) * slots_per_wave + (lane >> a.log2GL);
  const uint64_t slot_stride = (uint64_t)gridDim.x * waves * slots_per_wave;
  const W lmask = (W(1) << a.b) - 1;
  const int ncand = 2 * a.nbonds;
  double dot = 0.0;

  for (uint64_t p = slot; p < a.n_reps; p += slot_stride) {
    const uint64_t mp = a.meta[p];
    const int sp = (int)(mp >> 48);
    const int np_ = (int)a.stabf[4 * sp];
    if (np_ == 0) continue;
    const uint64_t offp = mp & kOffMask;
    const W plab = (W)a.reps[p];
    A acc[DG];
#pragma unroll
    for (int q = 0; q < DG; ++q) acc[q] = A(0);

    const uint64_t e_begin = OTF ? 0 : a.row_ptr[p];
    const uint64_t e_end = OTF ? (uint64_t)ncand : a.row_ptr[p + 1];
    for (uint64_t e = e_begin; e < e_end; e += GL) {
      uint64_t my = ~0ull;
      if constexpr (!OTF) {
        if (e + lg < e_end) my = a.entries[e + lg];
      } else {
        const int cand = (int)e + lg;
        bool ok = false;
        W x = plab;
        if (cand < ncand) {
          const int bond = cand >> 1;
          const int i = a.bonds[2 * bond], j = a.bonds[2 * bond + 1];
          const int ai = dev::digit(plab, i, a.b, lmask), aj = dev::digit(plab, j, a.b, lmask);
          ok = (cand & 1) ? (ai > 0 && aj < a.dloc - 1) : (ai < a.dloc - 1 && aj > 0);
          const W ui = W(1) << (i * a.b), uj = W(1) << (j * a.b);
          if (ok) x = (cand & 1) ? (plab - ui + uj) : (plab + ui - uj);
        }
        W r;
        int h;
        dev::canon_min<W, NCH>(x, tab, a.G, r, h);
        uint64_t idx = 0;
        if (ok && lookup_rep<W>(r, a.N, a.b, a.dloc, a.A_tot, a.cnt, a.cnt_stride, a.D_M, a.rank_bits, a.rank_base, idx))
          my = idx | ((uint64_t)h << 32) | ((uint64_t)cand << 48);
      }
      const int cnt = (int)min((uint64_t)GL, e_end - e);
      for (int jj = 0; jj < cnt; ++jj) {
        const uint64_t ent = shfl64(my, gbase + jj);
        const uint32_t idx = (uint32_t)(ent & 0xffffffffu);
        if (idx == 0xffffffffu) continue;
        const int h = (int)((ent >> 32) & 0xffff);
        const int cand = (int)(ent >> 48);
        const uint64_t mr = a.meta[idx];
        const int sr = (int)(mr >> 48);
        const int nr = (int)a.stabf[4 * sr];
        if (nr == 0) continue;
        const uint64_t offr = mr & kOffMask;
        const int bond = cand >> 1;
        const int bi = a.bonds[2 * bond], bj = a.bonds[2 * bond + 1];
        const int ai = dev::digit(plab, bi, a.b, lmask), aj = dev::digit(plab, bj, a.b, lmask);
        const A c = (A)(a.J[bond] * a.fac[((cand & 1) * a.dloc + ai) * a.dloc + aj]) * a.stabf[4 * sr + 2];
        A t[DG];
        if (a.stabf[4 * sr + 3] != A(0)) {
#pragma unroll
          for (int q = 0; q < DG; ++q) t[q] = vok ? (A)a.X[(offr + q) * a.ld + v] : A(0);
        } else {
          A xk[DG];
#pragma unroll
          for (int k = 0; k < DG; ++k) xk[k] = (vok && k < nr) ? (A)a.X[(offr + k) * a.ld + v] : A(0);
          const A* Vr = a.V + (size_t)sr * DG * DG;
#pragma unroll
          for (int q = 0; q < DG; ++q) {
            A s = A(0);
#pragma unroll
            for (int k = 0; k < DG; ++k) s += Vr[q * DG + k] * xk[k];
            t[q] = s;
          }
        }
        const A* R = a.rhoT + (size_t)h * DG * DG;
#pragma unroll
        for (int be = 0; be < DG; ++be) {
          A s = A(0);
#pragma unroll
          for (int q = 0; q < DG; ++q) s += R[be * DG + q] * t[q];
          acc[be] += c * s;
        }
      }
    }
    // project with V_p, add the diagonal, write
    const A sqL = a.stabf[4 * sp + 1];
    const bool ptriv = a.stabf[4 * sp + 3] != A(0);
    const A* Vp = a.V + (size_t)sp * DG * DG;
    const double ed = a.ediag[p];
#pragma unroll
    for (int k = 0; k < DG; ++k) {
      if (k >= np_) break;
      A y;
      if (ptriv) {
        y = acc[k];
      } else {
        A s = A(0);
#pragma unroll
        for (int be = 0; be < DG; ++be) s += Vp[be * DG + k] * acc[be];
        y = s;
      }
      y *= sqL;
      if (vok) {
        const uint64_t at = (offp + k) * a.ld + v;
        const A xv = (A)a.X[at];
        const A hx = y + (A)ed * xv;
        if (!EPI) {
          a.Y[at] = (T)hx;
        } else {
          const A sj = (A)a.scal[2 * v], bsj = (A)a.scal[2 * v + 1];
          const A w = sj * hx - bsj * (A)a.Y[at];
          const T ws = (T)w;
          a.Y[at] = ws;
          dot += (double)a.X[at] * (double)ws;
        }
      }
    }
  }
  if (EPI) {
    __shared__ double red[kThreads];
    red[threadIdx.x] = vok ? dot : 0.0;
    __syncthreads();
    if ((int)threadIdx.x < GL) {
      double s = 0.0;
      for (int q = 0; q < kThreads / GL; ++q) s += red[q * GL + threadIdx.x];
      const int vv = blockIdx.y * 64 + threadIdx.x;
      if (vv < a.nvec) a.partials[(size_t)blockIdx.x * a.nvec + vv] = s;
    }
  }
}

template <typename T, typename A, int DG, bool OTF, int NCH, bool LDS_TAB>
void launch(const HvArgs<T, A>& a, dim3 grid, size_t shm, hipStream_t st) {
  hipLaunchKernelGGL((k_hv<T, A, DG, OTF, NCH, LDS_TAB>), grid, dim3(kThreads), shm, st, a);
}

template <typename T, typename A, int DG>
void launch_mode(const HvArgs<T, A>& a, const Sector& s, dim3 grid, hipStream_t st, bool otf, size_t tab_bytes,
                 bool lds) {
  if (!otf) {
    // the label word width still matters: flips read p's digits
    if (s.wide)
      launch<T, A, DG, false, 16, false>(a, grid, 0, st);
    else
      launch<T, A, DG, false, 8, false>(a, grid, 0, st);
    return;
  }
  FTLM_DISPATCH_NCH(s.nch, {
    if (lds)
      launch<T, A, DG, true, NCH, true>(a, grid, tab_bytes, st);
    else
      launch<T, A, DG, true, NCH, false>(a, grid, 0, st);
  });
}

template <typename T, typename A>
void dispatch(const Block& b, const HvArgs<T, A>& a, dim3 grid, hipStream_t st, bool otf, size_t tab_bytes,
              bool lds) {
  const Sector& s = *b.sec;
#define FTLM_DG_CASE(n)                                                           \
  case n:                                                                         \
    launch_mode<T, A, n>(a, s, grid, st, otf, tab_bytes, lds);                    \
    break;
  switch (b.dg) {
    FTLM_DG_CASE(1) FTLM_DG_CASE(2) FTLM_DG_CASE(3) FTLM_DG_CASE(4) FTLM_DG_CASE(5) FTLM_DG_CASE(6)
    FTLM_DG_CASE(7) FTLM_DG_CASE(8) FTLM_DG_CASE(9) FTLM_DG_CASE(10) FTLM_DG_CASE(11) FTLM_DG_CASE(12)
    default:
      fail(FTLM_ERR_DIM_GT_12, "irrep dimension above 12");
  }
#undef FTLM_DG_CASE
}

int group_lanes(int nvec) {
  int gl = 1;
  while (gl < nvec && gl < 64) gl <<= 1;
  return gl;
}

dim3 hv_grid(const Block& b, int nvec) {
  const int gl = group_lanes(nvec);
  const uint64_t slots_per_block = (uint64_t)(kThreads / 64) * (64 / gl);
  uint64_t gx = (b.sec->n_reps + slots_per_block - 1) / slots_per_block;
  gx = std::max<uint64_t>(1, std::min<uint64_t>(gx, 8192));
  return dim3((unsigned)gx, (unsigned)((nvec + 63) / 64), 1);
}

}  // namespace

int hv_partial_groups(const Block& b, int nvec) { return (int)hv_grid(b, nvec).x; }

void apply_hv(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, hipStream_t st,
              const LanczosEpilogue* lz) {
  const Sector& s = *b.sec;
  if (nvec <= 0 || ld < nvec) fail(FTLM_ERR_INVALID_ARG, "need 0 < nvec <= ld");
  if (b.D == 0 || s.n_reps == 0) return;
  if (!X || !Y) fail(FTLM_ERR_INVALID_ARG, "null vector");
  const bool otf = s.hv_mode == FTLM_HV_ONTHEFLY;
  const int gl = group_lanes(nvec);
  int log2gl = 0;
  while ((1 << log2gl) < gl) ++log2gl;
  const dim3 grid = hv_grid(b, nvec);
  const size_t tab_words = (size_t)s.G->order * s.nch * 16;
  const size_t tab_bytes = tab_words * (s.wide ? 8 : 4);
  const bool lds = tab_bytes <= 65536;
  auto fill = [&](auto& a) {
    a.reps = s.d_reps.p;
    a.row_ptr = s.d_row_ptr.p;
    a.entries = s.d_entries.p;
    a.meta = b.d_meta.p;
    a.ediag = s.d_ediag.p;
    a.bonds = s.d_bonds.p;
    a.J = s.d_J.p;
    a.fac = s.d_fac.p;
    a.b = s.bits;
    a.dloc = s.d;
    a.nbonds = s.nbonds;
    a.G = s.G->order;
    a.n_stab = s.n_stab;
    a.n_reps = s.n_reps;
    a.ld = ld;
    a.nvec = nvec;
    a.GL = gl;
    a.log2GL = log2gl;
    a.tab = s.d_tab.p;
    a.cnt = s.d_cnt.p;
    a.rank_bits = s.d_rank_bits.p;
    a.rank_base = s.d_rank_base.p;
    a.cnt_stride = s.cnt_stride;
    a.N = s.N;
    a.A_tot = s.A;
    a.D_M = s.D_M;
    a.tab_words = (uint32_t)tab_words;
    a.scal = lz ? lz->scal : nullptr;
    a.partials = lz ? lz->partials : nullptr;
  };
  if (dtype == FTLM_F64) {
    HvArgs<double, double> a{};
    fill(a);
    a.rhoT = b.d_rhoT64.p;
    a.V = b.d_V64.p;
    a.stabf = b.d_stabf64.p;
    a.X = (const double*)X;
    a.Y = (double*)Y;
    dispatch<double, double>(b, a, grid, st, otf, tab_bytes, lds);
  } else if (dtype == FTLM_F32) {
    HvArgs<float, float> a{};
    fill(a);
    a.rhoT = b.d_rhoT32.p;
    a.V = b.d_V32.p;
    a.stabf = b.d_stabf32.p;
    a.X = (const float*)X;
    a.Y = (float*)Y;
    dispatch<float, float>(b, a, grid, st, otf, tab_bytes, lds);
  } else {
    fail(FTLM_ERR_INVALID_ARG, "dtype must be FTLM_F64 or FTLM_F32");
  }
  FTLM_HIP(hipGetLastError());
}

}  // namespace ftlm
