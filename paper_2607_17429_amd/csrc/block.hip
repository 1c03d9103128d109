// One (M, Gamma, row) block on top of a sector (paper Section 2.3, Eqs. 8-13).
//
// Per stabilizer S (host, FP64): P_S = (1/|S|) sum_{h in S} rho(h) (real
// irreps), n_Gamma(S) = (1/|S|) sum_h chi(h), V_S = modified Gram-Schmidt
// over the columns of P_S in index order (a column is dropped when its
// residual norm is below 1e-8; the kept count must equal n_Gamma), and the
// orbit length L_S = |G| / |S|.  Per representative (device): n_Gamma and the
// exclusive prefix sum giving each representative's first block row.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace ftlm {

namespace {

// n_Gamma per representative, and the number of active representatives
// (block-level sum, one atomic per workgroup).
__global__ void __launch_bounds__(256) k_rep_counts(const uint16_t* __restrict__ stab_id, uint64_t n,
                                                   const uint8_t* __restrict__ n_stab, uint64_t* __restrict__ out,
                                                   unsigned long long* __restrict__ n_active) {
  __shared__ unsigned long long red[256];
  unsigned long long act = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint8_t c = n_stab[stab_id[i]];
    out[i] = c;
    act += c ? 1 : 0;
  }
  red[threadIdx.x] = act;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(n_active, red[0]);
}

__global__ void k_meta(const uint64_t* __restrict__ off, const uint16_t* __restrict__ stab_id, uint64_t n,
                       uint64_t* __restrict__ meta) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    meta[i] = off[i] | ((uint64_t)stab_id[i] << 48);
}

unsigned grid1(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 65536ull * 4));
}

double check_user_rho(const Group& G, const double* rho, int d) {
  const int n = G.order;
  double worst = 0;
  for (int a = 0; a < n; ++a) {
    const double* ra = rho + (size_t)a * d * d;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double s = 0;
        for (int k = 0; k < d; ++k) s += ra[k * d + i] * ra[k * d + j];
        worst = std::max(worst, std::fabs(s - (i == j ? 1.0 : 0.0)));
      }
    for (int b = 0; b < n; ++b) {
      const double* rb = rho + (size_t)b * d * d;
      const double* rab = rho + (size_t)G.idx_mul(a, b) * d * d;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          double s = 0;
          for (int k = 0; k < d; ++k) s += ra[i * d + k] * rb[k * d + j];
          worst = std::max(worst, std::fabs(s - rab[i * d + j]));
        }
    }
  }
  return worst;
}

__global__ void __launch_bounds__(256) k_hv_stats(const uint64_t* __restrict__ meta, const uint64_t* __restrict__ row_ptr,
                                                 const uint64_t* __restrict__ entries, const uint32_t* __restrict__ eidx,
                                                 const uint8_t* __restrict__ n_stab, uint64_t n, unsigned triv_sid,
                                                 unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[5][256];
  unsigned long long c = 0, ca = 0, rows = 0, act = 0, nt = 0;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (uint64_t)gridDim.x * blockDim.x) {
    if (n_stab[meta[p] >> 48] == 0) continue;
    ++act;
    for (uint64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
      const uint64_t idx = eidx ? (uint64_t)eidx[e] : (entries[e] & 0xffffffffull);
      ++c;
      if (idx == 0xffffffffull) continue;
      const unsigned sr = (unsigned)(meta[idx] >> 48);
      const unsigned nr = n_stab[sr];
      if (nr) {
        ++ca;
        rows += nr;
        nt += sr != triv_sid ? 1 : 0;
      }
    }
  }
  red[0][threadIdx.x] = act;
  red[1][threadIdx.x] = c;
  red[2][threadIdx.x] = ca;
  red[3][threadIdx.x] = rows;
  red[4][threadIdx.x] = nt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) atomicAdd(&out[threadIdx.x], red[threadIdx.x][0]);
}

}  // namespace

void block_hv_stats(const Block& b, ftlm_hv_stats* res) {
  std::memset(res, 0, sizeof(*res));
  const Sector& s = *b.sec;
  if (!s.n_reps || b.D == 0) return;  // an empty block has no active representative
  if (s.hv_mode != FTLM_HV_ENTRIES) fail(FTLM_ERR_UNSUPPORTED, "work counts need the entry table");
  DevBuf<uint8_t> d_n;
  d_n.upload(b.n_stab);
  DevBuf<unsigned long long> out;
  out.alloc(5);
  hipStream_t st = tl_alloc_stream;
  FTLM_HIP(hipMemsetAsync(out.p, 0, out.bytes(), st));
  hipLaunchKernelGGL(k_hv_stats, dim3(grid1(s.n_reps)), dim3(256), 0, st, b.d_meta.p, s.d_row_ptr.p,
                     s.d_entries.p, s.d_eidx.p, d_n.p, s.n_reps, (unsigned)s.trivial_sid, out.p);
  FTLM_HIP(hipGetLastError());
  unsigned long long h[5];
  FTLM_HIP(hipMemcpyAsync(h, out.p, sizeof(h), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipStreamSynchronize(st));
  res->n_active = h[0];
  res->connections = h[1];
  res->active_connections = h[2];
  res->gathered_rows = h[3];
  res->nontrivial_targets = h[4];
  res->entry_bytes = s.entry_bytes;
}

std::unique_ptr<Block> build_block(std::shared_ptr<Sector> sec, int irrep, int row, const ftlm_opts* opts) {
  if (!sec) fail(FTLM_ERR_INVALID_ARG, "null sector");
  const Group& G = *sec->G;
  auto B = std::make_unique<Block>();
  B->sec = sec;
  B->irrep = irrep;
  B->row = row;
  const int n = G.order;          // |G|
  const int ng = sec->gorder;      // |G|, or 2|G| with the spin flip
  // with the spin flip, irrep 2i + q is Gamma_i with flip parity (-1)^q
  const int base_irrep = sec->zflip ? irrep >> 1 : irrep;
  const double parity = (sec->zflip && (irrep & 1)) ? -1.0 : 1.0;
  if (irrep < 0) fail(FTLM_ERR_IRREP_OUT_OF_RANGE, "irrep index out of range");
  if (opts) {
    if (opts->lanczos_layout < FTLM_LAYOUT_AUTO || opts->lanczos_layout > FTLM_LAYOUT_ALIGNED)
      fail(FTLM_ERR_INVALID_ARG, "lanczos_layout must be AUTO, BLOCK, PADDED, PACKED or ALIGNED");
    B->lanczos_layout = opts->lanczos_layout;
  }
  if (opts && opts->user_rho && opts->user_rho_dim > 0) {
    const int d = opts->user_rho_dim;
    if (d > 12) fail(FTLM_ERR_DIM_GT_12, "irrep dimension above 12");
    B->dg = d;
    B->weight = opts->user_rho_weight > 0 ? opts->user_rho_weight : d;
    if (B->weight > d) fail(FTLM_ERR_INVALID_ARG, "user_rho_weight above user_rho_dim");
    B->rho.assign(opts->user_rho, opts->user_rho + (size_t)n * d * d);
    double res = check_user_rho(G, B->rho.data(), d);
    if (!(res < 1e-9)) fail(FTLM_ERR_BAD_RHO, "user rho is not an orthogonal representation (residual " + std::to_string(res) + ")");
  } else {
    if (!G.irreps_computed) fail(FTLM_ERR_UNSUPPORTED, "group irreps not available (|G| > 1024); pass user_rho");
    if (!G.all_real) fail(FTLM_ERR_COMPLEX_IRREP_UNSUPPORTED, "the group's real irreps are incomplete");
    if (base_irrep >= (int)G.irreps.size()) fail(FTLM_ERR_IRREP_OUT_OF_RANGE, "irrep index out of range");
    const Irrep& ir = G.irreps[base_irrep];
    if (ir.dim > 12) fail(FTLM_ERR_DIM_GT_12, "irrep dimension above 12");
    B->dg = ir.dim;
    B->weight = ir.weight();
    B->rho = ir.rho;
  }
  const int d = B->dg;
  if (row < 0 || row >= d) fail(FTLM_ERR_ROW_OUT_OF_RANGE, "row must be in 0..d-1");
  if (sec->zflip) {
    // rho'(g, f) = parity^f rho(g): the flipped half follows the G half
    B->rho.resize((size_t)ng * d * d);
    for (size_t q = 0; q < (size_t)n * d * d; ++q) B->rho[(size_t)n * d * d + q] = parity * B->rho[q];
  }
  B->dgp = irrep_dim_bucket(d);
  // per stabilizer data
  const int ns = sec->n_stab;
  B->n_stab.assign(std::max(ns, 1), 0);
  B->V_stab.assign((size_t)std::max(ns, 1) * d * d, 0.0);
  B->L_stab.assign(std::max(ns, 1), 1.0);
  B->trivial.assign(std::max(ns, 1), 0);
  for (int s = 0; s < ns; ++s) {
    const auto& S = sec->stab_elems[s];
    const double inv = 1.0 / (double)S.size();
    std::vector<double> P((size_t)d * d, 0.0);
    double chi = 0;
    for (int h : S) {
      const double* r = &B->rho[(size_t)h * d * d];
      for (int q = 0; q < d * d; ++q) P[q] += r[q] * inv;
      for (int q = 0; q < d; ++q) chi += r[q * d + q] * inv;
    }
    const int nG = (int)std::lround(chi);
    if (std::fabs(chi - nG) > 1e-6) fail(FTLM_ERR_BAD_RHO, "stabilizer character sum is not an integer");
    std::vector<std::vector<double>> cols;
    for (int j = 0; j < d; ++j) {
      std::vector<double> v(d);
      for (int i = 0; i < d; ++i) v[i] = P[i * d + j];
      for (const auto& q : cols) {
        double dot = 0;
        for (int i = 0; i < d; ++i) dot += q[i] * v[i];
        for (int i = 0; i < d; ++i) v[i] -= dot * q[i];
      }
      double nrm = 0;
      for (int i = 0; i < d; ++i) nrm += v[i] * v[i];
      nrm = std::sqrt(nrm);
      if (nrm < 1e-8) continue;
      for (int i = 0; i < d; ++i) v[i] /= nrm;
      cols.push_back(v);
    }
    if ((int)cols.size() != nG) fail(FTLM_ERR_BAD_RHO, "Gram-Schmidt rank differs from the character count");
    B->n_stab[s] = (uint8_t)nG;
    for (int k = 0; k < nG; ++k)
      for (int i = 0; i < d; ++i) B->V_stab[((size_t)s * d + i) * d + k] = cols[k][i];
    B->L_stab[s] = (double)ng / (double)S.size();
    B->trivial[s] = (S.size() == 1) ? 1 : 0;
  }
  hipStream_t st = tl_alloc_stream;  // the caller's build stream, or the null stream
  // D and the active count from the sector's representatives per stabilizer
  uint64_t D = 0, n_act = 0;
  for (int s = 0; s < ns; ++s) {
    D += sec->stab_count[s] * (uint64_t)B->n_stab[s];
    n_act += B->n_stab[s] ? sec->stab_count[s] : 0;
  }
  if (D >= (1ull << 48)) fail(FTLM_ERR_UNSUPPORTED, "block dimension above 2^48");
  B->D = D;
  B->n_active = n_act;
  B->D_pad = sec->n_reps * (uint64_t)B->dg;
  if (D == 0) {
    // an empty block never runs an H.V: no device tables, nothing to wait for
    B->fpar = parity;
    return B;
  }
  // device tables: every copy is asynchronous from host arrays that live to
  // the one synchronization at the end
  // rho^T[g][beta][gamma] = rho(g)[gamma][beta], zero-padded to the kernel's dimension bucket
  const int dp = B->dgp;
  // only the |G| matrices of G: the flipped half is parity * rho(g), applied
  // by the kernel as a sign on the coefficient
  B->fpar = parity;
  std::vector<double> rt((size_t)n * dp * dp, 0.0);
  for (int g = 0; g < n; ++g)
    for (int be = 0; be < d; ++be)
      for (int ga = 0; ga < d; ++ga) rt[((size_t)g * dp + be) * dp + ga] = B->rho[((size_t)g * d + ga) * d + be];
  B->d_rhoT64.upload_async(rt, st);
  std::vector<double> vp((size_t)std::max(ns, 1) * dp * dp, 0.0);
  for (int s = 0; s < ns; ++s)
    for (int i = 0; i < d; ++i)
      for (int k = 0; k < d; ++k) vp[((size_t)s * dp + i) * dp + k] = B->V_stab[((size_t)s * d + i) * d + k];
  B->d_V64.upload_async(vp, st);
  std::vector<double> sf((size_t)std::max(ns, 1) * 4, 0.0);
  for (int s = 0; s < ns; ++s) {
    sf[4 * s + 0] = B->n_stab[s];
    sf[4 * s + 1] = std::sqrt(B->L_stab[s]);
    sf[4 * s + 2] = 1.0 / std::sqrt(B->L_stab[s]);
    sf[4 * s + 3] = B->trivial[s];
  }
  B->d_stabf64.upload_async(sf, st);
  DevBuf<uint8_t> d_n;
  DevBuf<unsigned long long> per;
  DevBuf<uint64_t> off;
  if (sec->n_reps) {
    // row offsets = exclusive scan of n_Gamma over the representatives
    d_n.upload_async(B->n_stab, st);
    per.alloc(1);
    FTLM_HIP(hipMemsetAsync(per.p, 0, per.bytes(), st));
    off.alloc(sec->n_reps + 1);
    FTLM_HIP(hipMemsetAsync(off.p + sec->n_reps, 0, sizeof(uint64_t), st));
    hipLaunchKernelGGL(k_rep_counts, dim3(grid1(sec->n_reps)), dim3(256), 0, st, sec->d_stab_id.p, sec->n_reps, d_n.p,
                       off.p, per.p);
    FTLM_HIP(hipGetLastError());
    scan_exclusive_u64(off.p, off.p, sec->n_reps + 1, nullptr, st);
    B->d_meta.alloc(sec->n_reps);
    hipLaunchKernelGGL(k_meta, dim3(grid1(sec->n_reps)), dim3(256), 0, st, off.p, sec->d_stab_id.p, sec->n_reps,
                       B->d_meta.p);
    FTLM_HIP(hipGetLastError());
  }
  FTLM_HIP(hipStreamSynchronize(st));
  if (opts && opts->hbm_limit_bytes > 0 && B->device_bytes() > opts->hbm_limit_bytes)
    fail(FTLM_ERR_OUT_OF_MEMORY, "block tables exceed the HBM limit");
  return B;
}

}  // namespace ftlm
