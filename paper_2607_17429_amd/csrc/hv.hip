// Host side of the H.V (paper Eqs. 15-16): LDS layout of the small tables,
// lane layout (lanes per representative, vectors per lane) and dispatch to the
// kernel instantiations in hv_dg*.hip.  The kernel itself is in hv_kernel.h.
#include <map>
#include <mutex>
#include <string>

#include "hv_kernel.h"
#include "tune_cache.h"

namespace ftlm {

using namespace hvk;

namespace {

constexpr uint32_t kSmallLdsBudget = 48 * 1024;
constexpr uint32_t kLdsLimit = 65536 - 2048;  // dynamic LDS; 2 KiB stay for the epilogue reduction

struct Layout {
  int GL, log2GL, VPL, tile_w, tiles;
};

int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

int vpl_bucket(int need, bool otf) {
  if (otf) return need <= 1 ? 1 : 4;
  const int opts[] = {1, 2, 3, 4, 6, 8};
  for (int o : opts)
    if (o >= need) return o;
  return 8;
}

// Lanes per output representative (GL) and vectors per lane (VPL).  Default
// (measured on MI355X for the s=1/2 icosidodecahedron H_g block): one lane per
// vector up to 4 vectors, then about 3 vectors per lane, which keeps 64/GL
// representatives in flight per wave.  gl > 0 forces GL (the autotuner's choice).
Layout choose_layout(int nvec, bool otf, int gl = 0) {
  Layout L{};
  if (gl <= 0) {
    if (nvec <= 4)
      gl = pow2_at_least(nvec);
    else
      gl = otf ? std::min(16, pow2_at_least((nvec + 3) / 4)) : pow2_at_least((nvec + 2) / 3);
  }
  L.GL = std::min(64, pow2_at_least(gl));
  L.VPL = vpl_bucket((std::min(nvec, 64 * 8) + L.GL - 1) / L.GL, otf);
  if (L.GL * L.VPL > 64 && L.GL > 1) {
    // keep a tile within 64 vectors
    L.VPL = vpl_bucket(std::max(1, 64 / L.GL), otf);
  }
  L.log2GL = 0;
  while ((1 << L.log2GL) < L.GL) ++L.log2GL;
  L.tile_w = L.GL * L.VPL;
  L.tiles = (nvec + L.tile_w - 1) / L.tile_w;
  return L;
}

dim3 hv_grid(const Block& b, const Layout& L) {
  const uint64_t slots_per_block = (uint64_t)(kThreads / 64) * (64 / L.GL);
  uint64_t gx = (b.sec->n_reps + slots_per_block - 1) / slots_per_block;
  gx = std::max<uint64_t>(1, std::min<uint64_t>(gx, 8192));
  return dim3((unsigned)gx, (unsigned)L.tiles, 1);
}

uint32_t align16(uint64_t x) { return (uint32_t)((x + 15u) & ~uint64_t(15)); }

// Architecture name of the current device (cached per device ordinal): part
// of every autotuner key, so that a cache loaded from a file tuned on other
// hardware is never used here.
std::string current_arch() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  FTLM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop{};
  FTLM_HIP(hipGetDeviceProperties(&prop, dev));
  return names[dev] = std::string(prop.gcnArchName);
}

TuneKey tune_key(const Block& b, int nvec, int dtype, const VecLayout& vl, bool epi) {
  const Sector& s = *b.sec;
  TuneKey k;
  k.arch = current_arch();
  k.cluster = s.cluster_hash;
  k.N = s.N;
  k.two_s = s.two_s;
  k.G = s.gorder;
  k.dgp = b.dgp;
  k.nvec = nvec;
  k.dtype = dtype;
  k.mode = s.hv_mode;
  k.pad = vl.kind();
  k.epi = epi ? 1 : 0;
  return k;
}

int tuned_gl(const Block& b, int nvec, int dtype, const VecLayout& vl, bool epi) {
  return tune_lookup(tune_key(b, nvec, dtype, vl, epi));
}

// Column sums of a (ng x nvec) array of per-workgroup partials, one workgroup
// per column, in a fixed order.
__global__ void __launch_bounds__(256) k_col_sums(const double* __restrict__ partials, int ng, int nvec,
                                                 double* __restrict__ out) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) s += partials[(size_t)g * nvec + v];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

__global__ void k_fill_f64(double* __restrict__ p, int n, double x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = x;
}

}  // namespace

std::string device_arch() { return current_arch(); }

int irrep_dim_bucket(int d) {
  if (d >= 1 && d <= 6) return d;
  if (d <= 8) return 8;
  if (d <= 12) return 12;
  return -1;
}

int hv_layout_lanes(const Block& b, int nvec, int dtype, const VecLayout& vl, bool epi) {
  return choose_layout(nvec, b.sec->hv_mode == FTLM_HV_ONTHEFLY, tuned_gl(b, nvec, dtype, vl, epi)).GL;
}

int hv_partial_groups(const Block& b, int nvec, int gl) {
  return (int)hv_grid(b, choose_layout(nvec, b.sec->hv_mode == FTLM_HV_ONTHEFLY, gl)).x;
}

void apply_hv(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, hipStream_t st,
              const LanczosEpilogue* lz) {
  apply_hv_gl(b, X, Y, nvec, ld, dtype, st, lz, tuned_gl(b, nvec, dtype, VecLayout{}, lz != nullptr));
}

std::vector<std::pair<int, double>> autotune_hv(const Block& b, int nvec, int dtype, hipStream_t st, int reps,
                                                const VecLayout& vl, bool epi) {
  std::vector<std::pair<int, double>> out;
  if (b.D == 0 || b.sec->n_reps == 0) return out;
  const size_t elem = dtype == FTLM_F64 ? 8 : dtype == FTLM_F32 ? 4 : 2;
  const uint64_t rows = vec_rows(b, vl);
  DevBuf<uint8_t> X, Y;
  DevBuf<double> scal, partials;
  X.alloc((size_t)rows * nvec * elem);
  Y.alloc((size_t)rows * nvec * elem);
  FTLM_HIP(hipMemsetAsync(X.p, 0, X.bytes(), st));
  FTLM_HIP(hipMemsetAsync(Y.p, 0, Y.bytes(), st));
  if (epi) {
    // the Lanczos epilogue with s = b = 0 (the work of a step; the values do not matter)
    scal.alloc(2 * (size_t)nvec);
    hipLaunchKernelGGL(k_fill_f64, dim3((2 * nvec + 255) / 256), dim3(256), 0, st, scal.p, 2 * nvec, 0.0);
    size_t most = 0;
    for (int gl = 1; gl <= 64; gl <<= 1) most = std::max<size_t>(most, (size_t)hv_partial_groups(b, nvec, gl));
    partials.alloc(most * nvec);
  }
  hipEvent_t e0, e1;
  FTLM_HIP(hipEventCreate(&e0));
  FTLM_HIP(hipEventCreate(&e1));
  int best = 0;
  double best_ms = 1e300;
  for (int gl = 1; gl <= 64; gl <<= 1) {
    if (gl * 8 < nvec || gl > pow2_at_least(nvec)) continue;  // VPL <= 8, no empty lanes beyond one pow2
    LanczosEpilogue lz{scal.p, partials.p, hv_partial_groups(b, nvec, gl)};
    const LanczosEpilogue* lzp = epi ? &lz : nullptr;
    apply_hv_gl(b, X.p, Y.p, nvec, nvec, dtype, st, lzp, gl, vl);  // warm
    FTLM_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) apply_hv_gl(b, X.p, Y.p, nvec, nvec, dtype, st, lzp, gl, vl);
    FTLM_HIP(hipEventRecord(e1, st));
    FTLM_HIP(hipEventSynchronize(e1));
    float ms = 0;
    FTLM_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double per = ms / reps;
    out.push_back({gl, per});
    if (per < best_ms) {
      best_ms = per;
      best = gl;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best) tune_store(tune_key(b, nvec, dtype, vl, epi), best);
  return out;
}

HvExPlan plan_hv_ex(const Block& b, int nvec, int64_t ld, int dtype, const ftlm_hv_opts* o) {
  HvExPlan p{};
  if (nvec <= 0 || ld < nvec) fail(FTLM_ERR_INVALID_ARG, "need 0 < nvec <= ld");
  const int64_t elem = dtype == FTLM_F64 ? 8 : dtype == FTLM_F32 ? 4 : 2;
  const int layout = o ? o->layout : FTLM_LAYOUT_BLOCK;
  if (layout == FTLM_LAYOUT_AUTO)
    p.vl = run_layout(b, ld * elem);
  else if (layout == FTLM_LAYOUT_BLOCK || layout == FTLM_LAYOUT_PADDED || layout == FTLM_LAYOUT_PACKED ||
           layout == FTLM_LAYOUT_ALIGNED)
    p.vl = vec_layout(b, layout, ld * elem);
  else
    fail(FTLM_ERR_INVALID_ARG, "layout must be FTLM_LAYOUT_AUTO, _BLOCK, _PADDED, _PACKED or _ALIGNED");
  p.rows = vec_rows(b, p.vl);
  p.epi = o && o->scale;
  if (o && o->dots && !o->scale) fail(FTLM_ERR_INVALID_ARG, "dots need scale");
  const int lanes = o ? o->lanes : 0;
  if (lanes != 0 && (lanes < 0 || lanes > 64 || (lanes & (lanes - 1))))
    fail(FTLM_ERR_INVALID_ARG, "lanes must be 0 or a power of two up to 64");
  const bool otf = b.sec->hv_mode == FTLM_HV_ONTHEFLY;
  const Layout L = choose_layout(nvec, otf, lanes ? lanes : tuned_gl(b, nvec, dtype, p.vl, p.epi));
  p.gl = L.GL;
  p.ng = (b.D && b.sec->n_reps) ? hv_partial_groups(b, nvec, p.gl) : 0;
  if (b.D && b.sec->n_reps) {
    LaunchCfg c{};
    HvArgs<double> a{};
    hv_setup(b, nvec, nvec, p.gl, p.vl, nullptr, c, a);
    p.adjacent = c.contig && c.slds && !c.otf && b.dgp <= 6;
  }
  return p;
}

void apply_hv_ex(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, const ftlm_hv_opts* o,
                 const HvExPlan& p, double* partials, hipStream_t st) {
  if (p.epi && p.ng > 0 && !partials) fail(FTLM_ERR_INVALID_ARG, "no scratch for the partial sums");
  if (p.rows == 0 || b.sec->n_reps == 0) {
    if (o && o->dots) hipLaunchKernelGGL(k_fill_f64, dim3((nvec + 255) / 256), dim3(256), 0, st, o->dots, nvec, 0.0);
    FTLM_HIP(hipGetLastError());
    return;
  }
  if (!X || !Y) fail(FTLM_ERR_INVALID_ARG, "null vector");
  LanczosEpilogue lz{p.epi ? o->scale : nullptr, partials, p.ng, o ? o->shift : 0.0};
  if (p.epi) {
    apply_hv_gl(b, X, Y, nvec, ld, dtype, st, &lz, p.gl, p.vl);
    if (o->dots) hipLaunchKernelGGL(k_col_sums, dim3(nvec), dim3(256), 0, st, partials, p.ng, nvec, o->dots);
  } else if (lz.eshift != 0.0) {
    // a shift without the epilogue: the same kernel with scale (1, 0) would
    // need a scale array; the plain pass takes the shift directly
    apply_hv_gl(b, X, Y, nvec, ld, dtype, st, nullptr, p.gl, p.vl, lz.eshift);
  } else {
    apply_hv_gl(b, X, Y, nvec, ld, dtype, st, nullptr, p.gl, p.vl);
  }
  FTLM_HIP(hipGetLastError());
}

template <typename T>
void hv_setup(const Block& b, int nvec, int64_t ld, int gl, const VecLayout& vl, const LanczosEpilogue* lz,
              LaunchCfg& c, HvArgs<T>& a) {
  const bool pad = vl.pad;
  const Sector& s = *b.sec;
  const bool otf = s.hv_mode == FTLM_HV_ONTHEFLY;
  const Layout L = choose_layout(nvec, otf, gl);
  c = LaunchCfg{};
  c.grid = hv_grid(b, L);
  c.otf = otf;
  c.wide = s.wide;
  c.nch = s.nch;
  c.vpl = L.VPL;
  // kernels specialised for the dense gather (table-driven H.V only)
  c.contig = pad && !otf && b.dg == b.dgp && nvec == L.tile_w * L.tiles;
  const uint64_t tab_words = s.tab_words;
  const uint64_t tab_bytes = tab_words * (s.wide ? 8 : 4);
  const uint64_t DG = (uint64_t)b.dgp;
  const uint64_t ns = (uint64_t)std::max(s.n_stab, 1);
  // small tables first priority; the permutation table joins them in LDS when
  // both fit, otherwise it is read through the caches
  uint64_t small = 0;
  small = align16(small + (uint64_t)s.G->order * (uint64_t)b.dgp * b.dgp * 8);
  small = align16(small + (uint64_t)std::max(s.n_stab, 1) * b.dgp * b.dgp * 8);
  small = align16(small + (uint64_t)std::max(s.n_stab, 1) * 4 * 8);
  small = align16(small + (uint64_t)s.nbonds * 8);
  small = align16(small + (uint64_t)(2 * s.d * s.d) * 8);
  small = align16(small + (uint64_t)s.nbonds * 2 * 4);
  c.lds_tab = otf && align16(tab_bytes) + (small <= kSmallLdsBudget ? small : 0) <= kLdsLimit;
  const uint32_t base = c.lds_tab ? align16(tab_bytes) : 0;
  uint64_t o = base;
  const uint32_t o_rho = (uint32_t)o;
  o = align16(o + (uint64_t)s.G->order * DG * DG * 8);
  const uint32_t o_V = (uint32_t)o;
  o = align16(o + ns * DG * DG * 8);
  const uint32_t o_stab = (uint32_t)o;
  o = align16(o + ns * 4 * 8);
  const uint32_t o_J = (uint32_t)o;
  o = align16(o + (uint64_t)s.nbonds * 8);
  const uint32_t o_fac = (uint32_t)o;
  o = align16(o + (uint64_t)(2 * s.d * s.d) * 8);
  const uint32_t o_bonds = (uint32_t)o;
  o = align16(o + (uint64_t)s.nbonds * 2 * 4);
  c.slds = (o - base) <= kSmallLdsBudget && o <= kLdsLimit;
  c.shm = c.slds ? o : base;
  c.vg = false;
  uint32_t vg_stab = 0, vg_J = 0, vg_fac = 0, vg_bonds = 0;
  if (!c.slds && !otf) {
    // the kernels without V_S in LDS (VG): rho^T and the small tables only;
    // V_S, used only for non-trivial stabilizers, is read through the caches
    // (a 6x6-torus sector has up to 324 stabilizer types)
    uint64_t v = align16(base + (uint64_t)s.G->order * DG * DG * 8);
    vg_stab = (uint32_t)v;
    v = align16(v + ns * 4 * 8);
    vg_J = (uint32_t)v;
    v = align16(v + (uint64_t)s.nbonds * 8);
    vg_fac = (uint32_t)v;
    v = align16(v + (uint64_t)(2 * s.d * s.d) * 8);
    vg_bonds = (uint32_t)v;
    v = align16(v + (uint64_t)s.nbonds * 2 * 4);
    if ((v - base) <= kSmallLdsBudget && v <= kLdsLimit) {
      c.slds = c.vg = true;
      c.shm = v;
    }
  }
  {
    a.reps = s.d_reps.p;
    a.row_ptr = s.d_row_ptr.p;
    a.entries = s.d_entries.p;
    a.eidx = s.d_eidx.p;
    a.ehc = s.d_ehc.p;
    a.hbits = s.ent_hbits;
    a.pad = pad ? 1 : 0;
    a.dstride = b.dg;
    a.rpl = vl.rpl;
    a.rpline = vl.rpl > 1 || vl.aligned ? vl.rpline : (uint32_t)b.dg;
    a.triv_sid = s.trivial_sid;
    a.sid = s.d_stab_id.p;
    a.meta = b.d_meta.p;
    a.ediag = s.d_ediag.p;
    a.rhoT = b.d_rhoT64.p;
    a.V = b.d_V64.p;
    a.stabf = b.d_stabf64.p;
    a.bonds = s.d_bonds.p;
    a.J = s.d_J.p;
    a.fac = s.d_fac.p;
    a.b = s.bits;
    a.dloc = s.d;
    a.nbonds = s.nbonds;
    a.G = s.G->order;  // rho^T tables: one per element of G
    a.Gbase = s.G->order;
    a.fpar = b.fpar;
    a.zf = s.zflip ? 1 : 0;
    a.full = s.full;
    a.nH = s.fac_nH;
    a.nT = s.fac_nT;
    a.n_stab = (int)ns;
    a.n_reps = s.n_reps;
    a.ld = ld;
    a.nvec = nvec;
    a.GL = L.GL;
    a.log2GL = L.log2GL;
    a.tile_w = L.tile_w;
    a.zero = 0;
    a.o_rho = o_rho;
    a.o_V = c.vg ? 0 : o_V;
    a.o_stab = c.vg ? vg_stab : o_stab;
    a.o_J = c.vg ? vg_J : o_J;
    a.o_fac = c.vg ? vg_fac : o_fac;
    a.o_bonds = c.vg ? vg_bonds : o_bonds;
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
    a.eshift = lz ? lz->eshift : 0.0;
  }
}

template void hv_setup<double>(const Block&, int, int64_t, int, const VecLayout&, const LanczosEpilogue*,
                               LaunchCfg&, HvArgs<double>&);
template void hv_setup<float>(const Block&, int, int64_t, int, const VecLayout&, const LanczosEpilogue*, LaunchCfg&,
                              HvArgs<float>&);
template void hv_setup<_Float16>(const Block&, int, int64_t, int, const VecLayout&, const LanczosEpilogue*,
                                 LaunchCfg&, HvArgs<_Float16>&);

void apply_hv_gl(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, hipStream_t st,
                 const LanczosEpilogue* lz, int gl, const VecLayout& vl, double shift) {
  const Sector& s = *b.sec;
  if (nvec <= 0 || ld < nvec) fail(FTLM_ERR_INVALID_ARG, "need 0 < nvec <= ld");
  if (b.D == 0 || s.n_reps == 0) return;
  if (!X || !Y) fail(FTLM_ERR_INVALID_ARG, "null vector");
  LaunchCfg c{};
  HvArgs<double> a64{};
  HvArgs<float> a32{};
  HvArgs<_Float16> a16{};
  const HvArgs<double>* p64 = nullptr;
  const HvArgs<float>* p32 = nullptr;
  const HvArgs<_Float16>* p16 = nullptr;
  if (dtype == FTLM_F64) {
    hv_setup(b, nvec, ld, gl, vl, lz, c, a64);
    a64.X = (const double*)X;
    a64.Y = (double*)Y;
    if (!lz) a64.eshift = shift;
    p64 = &a64;
  } else if (dtype == FTLM_F32) {
    hv_setup(b, nvec, ld, gl, vl, lz, c, a32);
    a32.X = (const float*)X;
    a32.Y = (float*)Y;
    if (!lz) a32.eshift = shift;
    p32 = &a32;
  } else if (dtype == FTLM_F16) {
    hv_setup(b, nvec, ld, gl, vl, lz, c, a16);
    a16.X = (const _Float16*)X;
    a16.Y = (_Float16*)Y;
    if (!lz) a16.eshift = shift;
    p16 = &a16;
  } else {
    fail(FTLM_ERR_INVALID_ARG, "dtype must be FTLM_F64, FTLM_F32 or FTLM_F16");
  }
  switch (b.dgp) {
    case 1: launch_dg<1>(p64, p32, p16, c, st); break;
    case 2: launch_dg<2>(p64, p32, p16, c, st); break;
    case 3: launch_dg<3>(p64, p32, p16, c, st); break;
    case 4: launch_dg<4>(p64, p32, p16, c, st); break;
    case 5: launch_dg<5>(p64, p32, p16, c, st); break;
    case 6: launch_dg<6>(p64, p32, p16, c, st); break;
    case 8: launch_dg<8>(p64, p32, p16, c, st); break;
    case 12: launch_dg<12>(p64, p32, p16, c, st); break;
    default: fail(FTLM_ERR_DIM_GT_12, "irrep dimension above 12");
  }
  FTLM_HIP(hipGetLastError());
}

}  // namespace ftlm
