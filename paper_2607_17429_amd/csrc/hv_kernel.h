// H.V kernel template (paper Eqs. 15-16) shared by the per-dimension
// instantiation units hv_dg*.hip.  The host side (table layout, launch shape,
// dispatch) is in hv.hip.
//
// Gather form (from Eq. 15 with U(h) a = r for the flipped state
// a = flip_e(p) of output representative p):
//
//   Y[p] = E_diag(p) X[p]
//        + sqrt(L_p) V_p^T  sum_e  c_e(p) / sqrt(L_r)  rho(h)^T  V_r X[r]
//
// with c_e(p) the Eq. (3) coefficient of flip e evaluated on p's digits and
// L = |G| / |Stab|.
//
// Lane layout: a group of GL lanes owns one output representative; lane g of
// the group holds VPL vector columns (v = tile + g + j * GL, or the adjacent
// v = tile + g * VPL + j in CONTIG launches, see hv_col_lane).  Every output
// element is written by exactly one lane and the sum over flips runs in a
// fixed order, so results are deterministic and do not depend on how many
// vectors share the launch.  Small GL (8) with VPL vectors per lane keeps 64/GL
// representatives per wave in flight, which is what hides the latency of the
// dependent loads (flip -> target metadata -> X rows): a chunk of GL flips is
// fetched with one load per lane and exchanged by lane shuffles, then each
// flip's n_r rows of X[r] are gathered for all VPL vectors.  rho^T, V_S, the
// stabilizer data and the bond coefficients sit in LDS when they fit; when
// only V_S does not (many stabilizer types), the dense-gather kernels keep
// the others in LDS and read V_S, needed only for non-trivial stabilizers,
// through the caches (VG; table-driven H.V only).
// Arithmetic is FP64; FP32 and FP16 storage round once on the store.
//
// Flips come from the sector's entry table (target index, h, flip id; built
// once per sector and shared by all irreps) or are found on the fly (flip,
// orbit search over the group, rank lookup).
//
// Lanczos epilogue (partials != nullptr): the kernel writes
// w = s_j (H q_j) - bs_j q_prev over q_prev (Y holds q_prev on entry) and
// per-workgroup FP64 partial sums of q_j . w (w as stored).  With a shift
// e (eshift) the kernel applies H - e instead of H (the Chebyshev recursion
// of the kernel polynomial method); e = 0 otherwise.
#pragma once

#include <algorithm>
#include <cmath>

#include "device.h"
#include "dispatch.h"
#include "internal.h"

namespace ftlm {
namespace hvk {

constexpr int kThreads = 256;
// occupancy floor handed to the register allocator for kernels whose
// accumulator (DG x VPL doubles) is small enough to meet it without spills
#ifndef FTLM_HV_WAVES_PER_EU
#define FTLM_HV_WAVES_PER_EU 4
#endif
#ifndef FTLM_HV_FLOOR_WIDTH
#define FTLM_HV_FLOOR_WIDTH 10
#endif
constexpr uint64_t kOffMask = (1ull << 48) - 1;
constexpr uint32_t kInvalid = 0xffffffffu;

template <typename T>
struct HvArgs {
  const uint64_t* reps;
  const uint64_t* row_ptr;
  const uint64_t* entries;   // 8-byte entries, or
  const uint32_t* eidx;      // the 6-byte split form (eidx != nullptr)
  const uint16_t* ehc;
  int hbits;
  // vector layout: pad == 0: block rows (representative i at meta offset);
  // pad != 0: padded rows, representative i at dev::padded_row (i * dstride,
  // dstride = d_Gamma, or packed rpl to a line of rpline rows), and a
  // target's stabilizer id comes from the entry's trivial bit or sid[]
  int pad, dstride, triv_sid;
  uint32_t rpl, rpline;
  const uint16_t* sid;
  const uint64_t* meta;
  const double* ediag;
  const double* rhoT;   // [g][beta][gamma], stride DG
  const double* V;      // [s][gamma][k], stride DG
  const double* stabf;  // [s][4] = n, sqrtL, 1/sqrtL, trivial
  const int32_t* bonds;
  const double* J;
  const double* fac;    // [2][dloc][dloc]
  int b, dloc, nbonds, G, n_stab;
  int nH, nT;           // factored group G = T H of the on-the-fly search
  uint64_t n_reps;
  const T* X;
  T* Y;
  int64_t ld;
  int nvec, GL, log2GL, tile_w;
  int zero;  // always 0 (see the non-trivial stabilizer branch)
  // dynamic LDS layout (byte offsets): [perm table][rho^T][V][stab][J][fac][bonds]
  uint32_t o_rho, o_V, o_stab, o_J, o_fac, o_bonds;
  // on-the-fly search
  const void* tab;
  const uint64_t* cnt;
  const uint64_t* rank_bits;
  const uint32_t* rank_base;
  int cnt_stride, N, A_tot;
  int Gbase, zf;        // |G| and the spin flip of the on-the-fly search
  uint64_t full;
  double fpar;          // flip parity: element (g, F) acts as fpar * rho(g)
  uint64_t D_M;
  uint32_t tab_words;
  // Lanczos epilogue
  const double* scal;
  double* partials;
  double eshift;        // H - eshift is applied (0 except for the Chebyshev recursion)
};

struct LaunchCfg {
  dim3 grid;
  size_t shm;
  bool otf, lds_tab, slds, wide;
  bool contig;  // the dense gather holds: adjacent columns per lane
  bool vg;      // all small tables but V_S in LDS (table-driven H.V)
  int nch, vpl;
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

// Swap a value with the other lane of its lane pair (lanes 2i and 2i + 1):
// DPP quad permutation [1, 0, 3, 2], a register move with no LDS traffic.
__device__ __forceinline__ uint32_t pair_swap_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ float pair_swap(float v) { return __uint_as_float(pair_swap_u32(__float_as_uint(v))); }
__device__ __forceinline__ double pair_swap(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t r = (uint64_t)pair_swap_u32((uint32_t)u) | ((uint64_t)pair_swap_u32((uint32_t)(u >> 32)) << 32);
  return __longlong_as_double((long long)r);
}
__device__ __forceinline__ _Float16 pair_swap(_Float16 v) {
  return __builtin_bit_cast(_Float16, (uint16_t)pair_swap_u32(__builtin_bit_cast(uint16_t, v)));
}

// Both columns of one row of a two-column slice, loaded as one aligned word.
template <typename T>
struct alignas(2 * sizeof(T)) RowPair {
  T c0, c1;
};

template <typename E>
__device__ __forceinline__ const E* stage(const E* src, uint32_t count, char* dst_bytes) {
  E* dst = (E*)dst_bytes;
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
  return dst;
}

// Whether a launch may take the dense gather (padded rows with d_Gamma equal
// to the dimension bucket and full column tiles; uniform over the launch).
template <typename T>
__device__ __forceinline__ bool hv_dense(const HvArgs<T>& a, int DG, int VPL, int ntiles) {
  return a.pad && a.dstride == DG && a.nvec == a.tile_w * ntiles && a.tile_w == a.GL * VPL;
}

// Column layout of a lane group.  Default: lane g holds columns g + j*GL (one
// coalesced load per column; gathers with clamped addresses and selects do
// not merge into wide loads).  CONTIG kernels, launched by the host only where
// the dense gather holds: lane g holds the adjacent columns g*VPL + j, so the
// gather of one row is one wide load per lane.
__host__ __device__ constexpr int hv_col_lane(bool contig, int vpl) { return contig ? vpl : 1; }
__host__ __device__ constexpr int hv_col_step(bool contig, int gl) { return contig ? 1 : gl; }

struct HvTabs {
  const double* rhoT;
  const double* Vt;
  const double* stabf;
  const double* Jb;
  const double* fac;
  const int32_t* bonds;
};

// The H.V over the representatives p = slot, slot + slot_stride, ... of one
// column tile: lane group of GL lanes per representative (see the file text).
// dot[j] accumulates q_j . w of this lane's column j in the Lanczos epilogue.
template <typename T, int DG, int VPL, bool OTF, int NCH, bool CONTIG = false>
__device__ __forceinline__ void hv_pass(const HvArgs<T>& a, const HvTabs& tb,
                                        const dev::OrbitTabs<word_t<NCH>, NCH>& otabs, int tile, int ntiles,
                                        uint64_t slot, uint64_t slot_stride, double (&dot)[VPL], bool (&vok)[VPL]) {
  using W = word_t<NCH>;
  const bool EPI = a.partials != nullptr;
  const double* rhoT = tb.rhoT;
  const double* Vt = tb.Vt;
  const double* stabf = tb.stabf;
  const double* Jb = tb.Jb;
  const double* fac = tb.fac;
  const int32_t* bonds = tb.bonds;
  const int lane = threadIdx.x & 63;
  const int GL = a.GL;
  const int lg = lane & (GL - 1);
  const int gbase = lane - lg;
  // uniform: the whole launch may gather without clamps (see the gather below)
  const bool dense = CONTIG || hv_dense(a, DG, VPL, ntiles);
  // uniform: a pair of lanes per representative, one column each, and
  // two-element rows that start on a two-element boundary (see the gather)
  const bool pair_rows = CONTIG && VPL == 1 && GL == 2 && a.ld == 2 &&
                         ((uintptr_t)a.X & (2 * sizeof(T) - 1)) == 0;
  // lane lg of the group owns columns vbase + j * vstep, j < VPL
  const int vbase = tile * a.tile_w + lg * hv_col_lane(CONTIG, VPL);
  const int vstep = hv_col_step(CONTIG, GL);
#pragma unroll
  for (int j = 0; j < VPL; ++j) vok[j] = vbase + j * vstep < a.nvec;
  const W lmask = (W(1) << a.b) - 1;
  const int ncand = 2 * a.nbonds;
#pragma unroll
  for (int j = 0; j < VPL; ++j) dot[j] = 0.0;

  for (uint64_t p = slot; p < a.n_reps; p += slot_stride) {
    const uint64_t mp = a.meta[p];
    const int sp = (int)(mp >> 48);
    const int np_ = (int)stabf[4 * sp];
    if (np_ == 0) continue;
    const uint64_t offp = a.pad ? dev::padded_row((uint32_t)a.dstride, a.rpl, a.rpline, p) : (mp & kOffMask);
    const W plab = (W)a.reps[p];
    double acc[DG][VPL];
#pragma unroll
    for (int q = 0; q < DG; ++q)
#pragma unroll
      for (int j = 0; j < VPL; ++j) acc[q][j] = 0.0;

    const uint64_t e_begin = OTF ? 0 : a.row_ptr[p];
    const uint64_t e_end = OTF ? (uint64_t)ncand : a.row_ptr[p + 1];
    for (uint64_t e = e_begin; e < e_end; e += GL) {
      // ---- one flip per lane: entry and target metadata
      uint64_t my = kInvalid;
      if constexpr (!OTF) {
        if (e + lg < e_end) {
          if (a.eidx) {
            const uint32_t hc = a.ehc[e + lg];
            my = (uint64_t)a.eidx[e + lg] | ((uint64_t)(hc & ((1u << a.hbits) - 1)) << 32) |
                 ((uint64_t)((hc & 0x7fffu) >> a.hbits) << 48) | ((uint64_t)(hc >> 15) << 63);
          } else {
            my = a.entries[e + lg];
          }
        }
      } else {
        const int cand = (int)e + lg;
        bool ok = false;
        W x = plab;
        if (cand < ncand) {
          const int bond = cand >> 1;
          const int i = bonds[2 * bond], j = bonds[2 * bond + 1];
          const int ai = dev::digit(plab, i, a.b, lmask), aj = dev::digit(plab, j, a.b, lmask);
          ok = (cand & 1) ? (ai > 0 && aj < a.dloc - 1) : (ai < a.dloc - 1 && aj > 0);
          const W ui = W(1) << (i * a.b), uj = W(1) << (j * a.b);
          if (ok) x = (cand & 1) ? (plab - ui + uj) : (plab + ui - uj);
        }
        W r;
        int h;
        dev::canon_min_z<W, NCH>(x, otabs, a.zf != 0, (W)a.full, a.Gbase, r, h);
        uint64_t idx = 0;
        if (ok && lookup_rep<W>(r, a.N, a.b, a.dloc, a.A_tot, a.cnt, a.cnt_stride, a.D_M, a.rank_bits, a.rank_base, idx))
          my = idx | ((uint64_t)h << 32) | ((uint64_t)cand << 48);
      }
      const uint32_t myidx = (uint32_t)(my & 0xffffffffu);
      uint64_t mm = 0;
      if (myidx != kInvalid) {
        if (a.pad) {
          const uint64_t sr = (my >> 63) ? (uint64_t)a.triv_sid : (uint64_t)a.sid[myidx];
          mm = dev::padded_row((uint32_t)a.dstride, a.rpl, a.rpline, myidx) | (sr << 48);
        } else {
          mm = a.meta[myidx];
        }
      }
      const int cnt = (int)min((uint64_t)GL, e_end - e);

      // Branch-free gathers: every lane loads from an in-bounds address
      // (row offr and column 0 stand in for rows >= n_r and columns >= nvec)
      // and a select zeroes those values, so all loads of a flip are in
      // flight together instead of each waiting inside its own branch.
      auto gather = [&](uint64_t offr, int nr, T (&xv)[DG][VPL]) {
        if (pair_rows) {
          // two lanes, one column each, rows of two elements: lane 0 loads
          // rows 0 .. H-1 and lane 1 rows H .. DG-1 (H = ceil(DG / 2)), both
          // columns of a row in one load, then each lane hands the other
          // column to its partner.  ceil(DG / 2) loads per flip instead of DG.
          constexpr int H = (DG + 1) / 2;
          const RowPair<T>* xr = reinterpret_cast<const RowPair<T>*>(a.X) + offr;
#pragma unroll
          for (int k = 0; k < H; ++k) {
            const RowPair<T> v = xr[lg ? (k + H < DG ? k + H : DG - 1) : k];
            const T recv = pair_swap(lg ? v.c0 : v.c1);
            const T keep = lg ? v.c1 : v.c0;
            xv[k][0] = lg ? recv : keep;
            if (k + H < DG) xv[k + H][0] = lg ? keep : recv;
          }
        } else if (dense) {
          // padded rows with d_Gamma == DG and every column in range: rows
          // k >= n_r of a target are stored zeros, so no clamp or select
          const T* xr = a.X + offr * (uint64_t)a.ld + vbase;
#pragma unroll
          for (int q = 0; q < DG; ++q)
#pragma unroll
            for (int j = 0; j < VPL; ++j) xv[q][j] = xr[q * a.ld + j * vstep];
        } else {
#pragma unroll
          for (int q = 0; q < DG; ++q)
#pragma unroll
            for (int j = 0; j < VPL; ++j) {
              const bool use = vok[j] && q < nr;
              const uint64_t at = (offr + (q < nr ? q : 0)) * a.ld + (vok[j] ? vbase + j * vstep : 0);
              const T val = a.X[at];
              xv[q][j] = use ? val : T(0);
            }
        }
      };
      // one flip's term: its coefficient times rho(h)^T (after V_r for a
      // target with a non-trivial stabilizer) applied to the gathered rows
      auto accumulate = [&](uint64_t ent, int sr, const T (&xv)[DG][VPL]) {
        int h = (int)((ent >> 32) & 0xffff);
        const int cand = (int)((ent >> 48) & 0x7fff);
        const int bond = cand >> 1;
        const int ai = dev::digit(plab, bonds[2 * bond], a.b, lmask);
        const int aj = dev::digit(plab, bonds[2 * bond + 1], a.b, lmask);
        double c = Jb[bond] * fac[((cand & 1) * a.dloc + ai) * a.dloc + aj] * stabf[4 * sr + 2];
        // G x Z2: (g, F) has index |G| + g and matrix fpar * rho(g)
        const bool flipped = h >= a.Gbase;
        h = flipped ? h - a.Gbase : h;
        c = flipped ? c * a.fpar : c;
        const double* R = rhoT + (size_t)h * DG * DG;
        if (stabf[4 * sr + 3] != 0.0) {
#pragma unroll
          for (int be = 0; be < DG; ++be) {
#pragma unroll
            for (int j = 0; j < VPL; ++j) {
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < DG; ++q) s += R[be * DG + q] * (double)xv[q][j];
              acc[be][j] += c * s;
            }
          }
        } else {
          // Non-trivial stabilizer: expand with V_r first.  The matrices are
          // re-read from LDS for every vector (offset by the runtime zero
          // a.zero) so the compiler cannot keep both d x d matrices live
          // across the vector loop.
#pragma unroll
          for (int j = 0; j < VPL; ++j) {
            const double* Vr = Vt + (size_t)sr * DG * DG + j * a.zero;
            const double* Rj = R + j * a.zero;
            double t[DG];
#pragma unroll
            for (int q = 0; q < DG; ++q) {
              double s = 0.0;
#pragma unroll
              for (int k = 0; k < DG; ++k) s += Vr[q * DG + k] * (double)xv[k][j];
              t[q] = s;
            }
#pragma unroll
            for (int be = 0; be < DG; ++be) {
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < DG; ++q) s += Rj[be * DG + q] * t[q];
              acc[be][j] += c * s;
            }
          }
        }
      };
      // With several vectors per lane and a flip's rows in at most 12
      // elements and 48 bytes the gathers of two flips are in flight
      // together, which doubles the random requests a lane group keeps
      // outstanding; the terms are still added in flip order, so the result
      // is the same bit for bit.  (Measured: the ten-block icosidodecahedron
      // job 1.48 s against 1.53 s; with more registers per flip, one vector
      // per lane or FP64 rows of 3 x 3 doubles it was slower, and FP16 rows
      // of 15 elements took 4.0 ms per icosidodecahedron H_g launch against
      // 3.5 ms with one flip at a time.)
      constexpr bool kTwo = VPL > 1 && DG * VPL <= 12 && DG * VPL * sizeof(T) <= 48;
#pragma unroll 1
      for (int jj = 0; jj < cnt; jj += (kTwo ? 2 : 1)) {
        const uint64_t ent0 = shfl64(my, gbase + jj);
        const uint64_t mr0 = shfl64(mm, gbase + jj);
        const int sr0 = (int)(mr0 >> 48);
        const int nr0 = (int)stabf[4 * sr0];
        const bool ok0 = (uint32_t)(ent0 & 0xffffffffu) != kInvalid && nr0 != 0;
        if constexpr (kTwo) {
          const int j1 = jj + 1 < cnt ? jj + 1 : jj;
          const uint64_t ent1 = shfl64(my, gbase + j1);
          const uint64_t mr1 = shfl64(mm, gbase + j1);
          const int sr1 = (int)(mr1 >> 48);
          const int nr1 = (int)stabf[4 * sr1];
          const bool ok1 = jj + 1 < cnt && (uint32_t)(ent1 & 0xffffffffu) != kInvalid && nr1 != 0;
          // a skipped flip gathers the output representative's own rows
          T xv0[DG][VPL], xv1[DG][VPL];
          gather(ok0 ? (mr0 & kOffMask) : offp, ok0 ? nr0 : 1, xv0);
          gather(ok1 ? (mr1 & kOffMask) : offp, ok1 ? nr1 : 1, xv1);
          if (ok0) accumulate(ent0, sr0, xv0);
          if (ok1) accumulate(ent1, sr1, xv1);
        } else {
          if (!ok0) continue;
          T xv[DG][VPL];
          gather(mr0 & kOffMask, nr0, xv);
          accumulate(ent0, sr0, xv);
        }
      }
    }
    // ---- project with V_p, add the diagonal, write
    const double sqL = stabf[4 * sp + 1];
    const bool ptriv = stabf[4 * sp + 3] != 0.0;
    const double* Vp = Vt + (size_t)sp * DG * DG;
    const double ed = a.ediag[p];
#pragma unroll
    for (int k = 0; k < DG; ++k) {
      if (k >= np_) break;
#pragma unroll
      for (int j = 0; j < VPL; ++j) {
        double y;
        if (ptriv) {
          y = acc[k][j];
        } else {
          double s = 0.0;
#pragma unroll
          for (int be = 0; be < DG; ++be) s += Vp[be * DG + k] * acc[be][j];
          y = s;
        }
        y *= sqL;
        if (vok[j]) {
          const int v = vbase + j * vstep;
          const uint64_t at = (offp + k) * a.ld + v;
          const double xv = (double)a.X[at];
          const double hx = y + (ed - a.eshift) * xv;
          if (!EPI) {
            a.Y[at] = (T)hx;
          } else {
            const double sj = a.scal[2 * v], bsj = a.scal[2 * v + 1];
            const T ws = (T)(sj * hx - bsj * (double)a.Y[at]);
            a.Y[at] = ws;
            dot[j] += xv * (double)ws;
          }
        }
      }
    }
  }
}

template <typename T, int DG, int VPL, bool OTF, int NCH, bool LDS_TAB, bool SLDS, bool CONTIG = false,
          bool VG = false>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(DG * VPL <= FTLM_HV_FLOOR_WIDTH ? FTLM_HV_WAVES_PER_EU : 1)))
k_hv(HvArgs<T> a) {
  using W = word_t<NCH>;
  extern __shared__ uint64_t smem_raw[];
  char* sm = (char*)smem_raw;
  const bool EPI = a.partials != nullptr;
  const W* tab = nullptr;
  if constexpr (OTF) tab = LDS_TAB ? stage<W>((const W*)a.tab, a.tab_words, sm) : (const W*)a.tab;
  const dev::OrbitTabs<W, NCH> otabs = dev::orbit_tabs<W, NCH>(tab, a.nH, a.nT);
  const double* rhoT = a.rhoT;
  const double* Vt = a.V;
  const double* stabf = a.stabf;
  const double* Jb = a.J;
  const double* fac = a.fac;
  const int32_t* bonds = a.bonds;
  if constexpr (SLDS) {
    rhoT = stage<double>(a.rhoT, (uint32_t)a.G * DG * DG, sm + a.o_rho);
    if constexpr (!VG) Vt = stage<double>(a.V, (uint32_t)a.n_stab * DG * DG, sm + a.o_V);
    stabf = stage<double>(a.stabf, (uint32_t)a.n_stab * 4, sm + a.o_stab);
    Jb = stage<double>(a.J, (uint32_t)a.nbonds, sm + a.o_J);
    fac = stage<double>(a.fac, (uint32_t)(2 * a.dloc * a.dloc), sm + a.o_fac);
    bonds = stage<int32_t>(a.bonds, (uint32_t)(2 * a.nbonds), sm + a.o_bonds);
  }
  if constexpr (SLDS || (OTF && LDS_TAB)) __syncthreads();

  const HvTabs tb{rhoT, Vt, stabf, Jb, fac, bonds};
  const int lane = threadIdx.x & 63;
  const int GL = a.GL;
  const int slots_per_wave = 64 >> a.log2GL;
  const int waves = blockDim.x >> 6;
  const uint64_t slot = ((uint64_t)blockIdx.x * waves + (threadIdx.x >> 6)) * slots_per_wave + (lane >> a.log2GL);
  const uint64_t slot_stride = (uint64_t)gridDim.x * waves * slots_per_wave;
  double dot[VPL];
  bool vok[VPL];
  hv_pass<T, DG, VPL, OTF, NCH, CONTIG>(a, tb, otabs, (int)blockIdx.y, (int)gridDim.y, slot, slot_stride, dot, vok);
  if (EPI) {
    __shared__ double red[kThreads];
    // one vector slot j at a time: lanes with equal lg hold the same column
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
      red[threadIdx.x] = vok[j] ? dot[j] : 0.0;
      __syncthreads();
      if ((int)threadIdx.x < GL) {
        double s = 0.0;
        for (int q = 0; q < kThreads / GL; ++q) s += red[q * GL + threadIdx.x];
        const int vv = blockIdx.y * a.tile_w + (int)threadIdx.x * hv_col_lane(CONTIG, VPL) + j * hv_col_step(CONTIG, GL);
        if (vv < a.nvec) a.partials[(size_t)blockIdx.x * a.nvec + vv] = s;
      }
      __syncthreads();
    }
  }
}

template <typename T, int DG, int VPL, bool OTF, int NCH, bool LDS_TAB>
void launch_k(const HvArgs<T>& a, const LaunchCfg& c, hipStream_t st) {
  // adjacent-column kernels for the dimension buckets 1-6 (a dense launch of
  // bucket 8 or 12 needs d_Gamma exactly 8 or 12; it takes the default layout)
  if constexpr (!OTF && DG <= 6) {
    if (c.slds && c.contig) {
      if (c.vg)
        hipLaunchKernelGGL((k_hv<T, DG, VPL, OTF, NCH, LDS_TAB, true, true, true>), c.grid, dim3(kThreads), c.shm, st, a);
      else
        hipLaunchKernelGGL((k_hv<T, DG, VPL, OTF, NCH, LDS_TAB, true, true>), c.grid, dim3(kThreads), c.shm, st, a);
      return;
    }
  }
  if constexpr (!OTF) {
    if (c.slds && c.vg) {
      hipLaunchKernelGGL((k_hv<T, DG, VPL, OTF, NCH, LDS_TAB, true, false, true>), c.grid, dim3(kThreads), c.shm, st, a);
      return;
    }
  }
  if (c.slds)
    hipLaunchKernelGGL((k_hv<T, DG, VPL, OTF, NCH, LDS_TAB, true>), c.grid, dim3(kThreads), c.shm, st, a);
  else if constexpr (!OTF)
    hipLaunchKernelGGL((k_hv<T, DG, VPL, OTF, NCH, LDS_TAB, false>), c.grid, dim3(kThreads), c.shm, st, a);
  else
    fail(FTLM_ERR_UNSUPPORTED, "on-the-fly H.V needs the irrep tables in LDS");
}

template <typename T, int DG, int VPL>
void launch_vpl(const HvArgs<T>& a, const LaunchCfg& c, hipStream_t st) {
  if (!c.otf) {
    // the label word width still matters: flips read p's digits
    if (c.wide)
      launch_k<T, DG, VPL, false, 16, false>(a, c, st);
    else
      launch_k<T, DG, VPL, false, 8, false>(a, c, st);
    return;
  }
  if constexpr (VPL == 1 || VPL == 4) {
    FTLM_DISPATCH_NCH(c.nch, {
      if (c.lds_tab)
        launch_k<T, DG, VPL, true, NCH, true>(a, c, st);
      else
        launch_k<T, DG, VPL, true, NCH, false>(a, c, st);
    });
  } else {
    fail(FTLM_ERR_INVALID_ARG, "on-the-fly H.V uses 1 or 4 vectors per lane");
  }
}

template <typename T, int DG>
void launch_t(const HvArgs<T>& a, const LaunchCfg& c, hipStream_t st) {
  switch (c.vpl) {
    case 1: launch_vpl<T, DG, 1>(a, c, st); break;
    case 2: launch_vpl<T, DG, 2>(a, c, st); break;
    case 3: launch_vpl<T, DG, 3>(a, c, st); break;
    case 4: launch_vpl<T, DG, 4>(a, c, st); break;
    case 6: launch_vpl<T, DG, 6>(a, c, st); break;
    case 8: launch_vpl<T, DG, 8>(a, c, st); break;
    default: fail(FTLM_ERR_INVALID_ARG, "unsupported vectors per lane");
  }
}

// one instantiation unit per irrep dimension bucket
template <int DG>
void launch_dg(const HvArgs<double>* a64, const HvArgs<float>* a32, const HvArgs<_Float16>* a16,
               const LaunchCfg& c, hipStream_t st);

#define FTLM_HV_INSTANTIATE(DGV)                                                                     \
  template <>                                                                                       \
  void launch_dg<DGV>(const HvArgs<double>* a64, const HvArgs<float>* a32,                         \
                      const HvArgs<_Float16>* a16, const LaunchCfg& c, hipStream_t st) {            \
    if (a64)                                                                                        \
      launch_t<double, DGV>(*a64, c, st);                                                           \
    else if (a32)                                                                                   \
      launch_t<float, DGV>(*a32, c, st);                                                            \
    else                                                                                            \
      launch_t<_Float16, DGV>(*a16, c, st);                                                         \
  }

}  // namespace hvk

// Launch shape, LDS layout and kernel arguments (all but X and Y) of one H.V
// over nvec vectors of leading dimension ld with gl lanes per representative
// (0: the default or autotuned layout).
template <typename T>
void hv_setup(const Block& b, int nvec, int64_t ld, int gl, const VecLayout& vl, const LanczosEpilogue* lz,
              hvk::LaunchCfg& c, hvk::HvArgs<T>& a);

}  // namespace ftlm
