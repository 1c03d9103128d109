// Kernel polynomial method on one block (the spectral-density route to
// thermodynamics that the paper names next to FTLM, its Ref. [6]), on the
// same symmetry-adapted H.V.
//
// For R start vectors r (the FTLM chains' vectors, same keys and generator)
// the Chebyshev vectors t_0 = r, t_1 = H~ r, t_{n+1} = 2 H~ t_n - t_{n-1} with
// H~ = (H - c) / w are formed by the H.V with its Lanczos epilogue (shift c,
// scales 1/w then 2/w, previous vector subtracted over itself), and
// two moments come from every product (Weisse et al., Rev. Mod. Phys. 78,
// 275 (2006), Eq. (34)):
//   mu_{2n+1} = 2 <t_{n+1}, t_n> - mu_1,   mu_{2n+2} = 2 <t_{n+1}, t_{n+1}> - mu_0,
// divided by <r, r> of the stored start vector.  Dot products are FP64
// partial sums per workgroup reduced in a fixed order (deterministic).
#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"

namespace ftlm {

namespace {

// thread layout (row r0, chain v) as in the Lanczos kernels; D rows of the
// stored vectors.  With meta (padded layouts) stored row r holds row k of
// representative i (dev::padded_rep_of), block row offset(i) + k for
// k < n_Gamma(i); every other stored row is zero.
template <typename T>
__global__ void __launch_bounds__(256) k_kpm_start(const uint64_t* __restrict__ keys, int dist, uint64_t D, int R,
                                                  const double* __restrict__ inv_norm, T* __restrict__ Q,
                                                  T* __restrict__ Qz, double* __restrict__ partials,
                                                  const uint64_t* __restrict__ meta,
                                                  const double* __restrict__ stabf, dev::PadMap pm) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int RB = blockDim.x / R;
  const int v = t % R, r0 = t / R;
  double acc = 0.0;
  if (r0 < RB)
    for (uint64_t row = (uint64_t)blockIdx.x * RB + r0; row < D; row += (uint64_t)gridDim.x * RB) {
      uint64_t brow = row;
      bool live = true;
      if (meta) {
        uint64_t i;
        int k;
        live = dev::padded_rep_of(pm, row, i, k);
        if (live) {
          const uint64_t m = meta[i];
          live = k < (int)stabf[4 * (m >> 48)];
          brow = (m & ((1ull << 48) - 1)) + (uint64_t)k;
        }
      }
      const double x = live ? dev::start_value(keys[v], brow, dist) : 0.0;
      if (inv_norm) {
        const T q = (T)(x * inv_norm[v]);
        Q[row * R + v] = q;
        Qz[row * R + v] = T(0);
        acc += (double)q * (double)q;
      } else {
        acc += x * x;
      }
    }
  red[t] = acc;
  __syncthreads();
  if (t < R) {
    double s = 0.0;
    for (int q = 0; q < RB; ++q) s += red[q * R + t];
    partials[(size_t)blockIdx.x * R + t] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_kpm_norm(uint64_t D, int R, const T* __restrict__ Q,
                                                 double* __restrict__ partials) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int RB = blockDim.x / R;
  const int v = t % R, r0 = t / R;
  double acc = 0.0;
  if (r0 < RB)
    for (uint64_t row = (uint64_t)blockIdx.x * RB + r0; row < D; row += (uint64_t)gridDim.x * RB) {
      const double q = (double)Q[row * R + v];
      acc += q * q;
    }
  red[t] = acc;
  __syncthreads();
  if (t < R) {
    double s = 0.0;
    for (int q = 0; q < RB; ++q) s += red[q * R + t];
    partials[(size_t)blockIdx.x * R + t] = s;
  }
}

// <t, t> per column with NV adjacent columns per thread (one 16-byte load):
// CPR = R / NV column groups per row, blockDim.x / CPR rows per block pass;
// partial sums per column as in k_kpm_norm.
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_kpm_norm_vec(uint64_t D, int R, const T* __restrict__ Q,
                                                     double* __restrict__ partials) {
  typedef T vec_t __attribute__((ext_vector_type(NV)));
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int CPR = R / NV;
  const int RB = blockDim.x / CPR;
  const int cg = t % CPR, r0 = t / CPR;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (r0 < RB)
    for (uint64_t row = (uint64_t)blockIdx.x * RB + r0; row < D; row += (uint64_t)gridDim.x * RB) {
      const vec_t q = *(const vec_t*)(Q + row * R + (uint64_t)cg * NV);
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += (double)q[k] * (double)q[k];
    }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    red[t] = acc[k];
    __syncthreads();
    if (t < CPR) {
      double s = 0.0;
      for (int q = 0; q < RB; ++q) s += red[q * CPR + t];
      partials[(size_t)blockIdx.x * R + t * NV + k] = s;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double group_sum(const double* __restrict__ partials, int ngroups, int R, int v) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < ngroups; b += blockDim.x) s += partials[(size_t)b * R + v];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  return red[0];
}

// one block per chain; mode 0: inv_norm from the draw's norm; mode 1: <r, r>
// of the stored start vector and mu_0 = 1
__global__ void __launch_bounds__(256) k_kpm_init(const double* __restrict__ partials, int ngroups, int R,
                                                 double* __restrict__ inv_norm, double* __restrict__ rr,
                                                 double* __restrict__ mu, int M, int mode) {
  const int v = blockIdx.x;
  const double s = group_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      inv_norm[v] = s > 0 ? 1.0 / sqrt(s) : 0.0;
    } else {
      rr[v] = s;
      mu[(size_t)v * M] = 1.0;
    }
  }
}

// moments 2k+1 and 2k+2 from <t_k, t_{k+1}> (H.V partials) and <t_{k+1}, t_{k+1}>
__global__ void __launch_bounds__(256) k_kpm_moments(const double* __restrict__ pdot, int ng_dot,
                                                    const double* __restrict__ pnrm, int ng_nrm, int R,
                                                    const double* __restrict__ rr, double* __restrict__ mu, int M,
                                                    int k) {
  const int v = blockIdx.x;
  const double d = group_sum(pdot, ng_dot, R, v);
  const double n = group_sum(pnrm, ng_nrm, R, v);
  if (threadIdx.x == 0) {
    const double inv = rr[v] > 0 ? 1.0 / rr[v] : 0.0;
    double* m = mu + (size_t)v * M;
    if (k == 0) {
      if (1 < M) m[1] = d * inv;
    } else if (2 * k + 1 < M) {
      m[2 * k + 1] = 2.0 * d * inv - m[1];
    }
    if (2 * k + 2 < M) m[2 * k + 2] = 2.0 * n * inv - m[0];
  }
}

unsigned groups_for(uint64_t rows, int RB) {
  uint64_t g = (rows + RB - 1) / RB;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 4096));
}

template <typename T>
void kpm_typed(const Block& b, int R, int M, uint64_t seed, int dist, double center, double half_width,
               double* moments, hipStream_t st) {
  // the Lanczos run's row layout: padded rows give the H.V its dense gather
  const VecLayout vl = run_layout(b, (int64_t)R * (int64_t)sizeof(T));
  const uint64_t D = vec_rows(b, vl);
  const uint64_t* meta = vl.pad ? b.d_meta.p : nullptr;
  const dev::PadMap pm = pad_map(b, vl);
  const double* stabf = b.d_stabf64.p;
  const int TB = R * (256 / R);
  const unsigned nb = groups_for(D, TB / R);
  const int dtype = sizeof(T) == 8 ? FTLM_F64 : FTLM_F32;
  const int gl = hv_layout_lanes(b, R, dtype, vl, true);
  const int ng_hv = hv_partial_groups(b, R, gl);
  DevBuf<T> q0, q1;
  q0.alloc(D * R);
  q1.alloc(D * R);
  std::vector<uint64_t> hkeys(R);
  for (int v = 0; v < R; ++v) hkeys[v] = chain_key(seed, b.sec->two_M, b.irrep, b.row, v);
  DevBuf<uint64_t> keys;
  keys.upload(hkeys, st);
  DevBuf<double> pdot, pnrm, inv_norm, rr, mu, scal0, scal1;
  pdot.alloc((size_t)std::max(ng_hv, 1) * R);
  pnrm.alloc((size_t)nb * R);
  inv_norm.alloc(R);
  rr.alloc(R);
  mu.alloc((size_t)R * M);
  // epilogue scales per column: t_1 = (1/w)(H - c) t_0; t_{n+1} = (2/w)(H - c) t_n - t_{n-1}
  std::vector<double> s0(2 * R), s1(2 * R);
  for (int v = 0; v < R; ++v) {
    s0[2 * v] = 1.0 / half_width;
    s0[2 * v + 1] = 0.0;
    s1[2 * v] = 2.0 / half_width;
    s1[2 * v + 1] = 1.0;
  }
  scal0.upload(s0, st);
  scal1.upload(s1, st);
  hipLaunchKernelGGL((k_kpm_start<T>), dim3(nb), dim3(TB), 0, st, keys.p, dist, D, R, (const double*)nullptr, q0.p,
                     q1.p, pnrm.p, meta, stabf, pm);
  hipLaunchKernelGGL(k_kpm_init, dim3(R), dim3(256), 0, st, pnrm.p, (int)nb, R, inv_norm.p, rr.p, mu.p, M, 0);
  hipLaunchKernelGGL((k_kpm_start<T>), dim3(nb), dim3(TB), 0, st, keys.p, dist, D, R, inv_norm.p, q0.p, q1.p,
                     pnrm.p, meta, stabf, pm);
  hipLaunchKernelGGL(k_kpm_init, dim3(R), dim3(256), 0, st, pnrm.p, (int)nb, R, inv_norm.p, rr.p, mu.p, M, 1);
  FTLM_HIP(hipGetLastError());
  const int steps = M > 1 ? M / 2 : 0;  // step k yields moments 2k+1 and 2k+2
  for (int k = 0; k < steps; ++k) {
    T* tk = (k & 1) ? q1.p : q0.p;
    T* tprev = (k & 1) ? q0.p : q1.p;  // t_{k-1} on entry, t_{k+1} on exit
    LanczosEpilogue lz{k == 0 ? scal0.p : scal1.p, pdot.p, ng_hv, center};
    apply_hv_gl(b, tk, tprev, R, R, dtype, st, &lz, gl, vl);
    constexpr int NV = 16 / (int)sizeof(T);
    if (R % NV == 0 && ((uintptr_t)tprev & 15) == 0) {
      // rows of whole 16-byte column groups, every row 16-byte aligned
      const int cpr = R / NV;
      hipLaunchKernelGGL((k_kpm_norm_vec<T, NV>), dim3(nb), dim3(cpr * (256 / cpr)), 0, st, D, R, tprev, pnrm.p);
    } else {
      hipLaunchKernelGGL((k_kpm_norm<T>), dim3(nb), dim3(TB), 0, st, D, R, tprev, pnrm.p);
    }
    hipLaunchKernelGGL(k_kpm_moments, dim3(R), dim3(256), 0, st, pdot.p, ng_hv, pnrm.p, (int)nb, R, rr.p, mu.p, M,
                       k);
    FTLM_HIP(hipGetLastError());
  }
  FTLM_HIP(hipMemcpyAsync(moments, mu.p, mu.bytes(), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipStreamSynchronize(st));
}

}  // namespace

void run_kpm(Block& b, int R, int M, uint64_t seed, int storage, int dist, double center, double half_width,
             double* moments, hipStream_t st) {
  if (!moments) fail(FTLM_ERR_INVALID_ARG, "null output");
  if (R <= 0 || R > 256) fail(FTLM_ERR_INVALID_ARG, "R must be in 1..256");
  if (M <= 0) fail(FTLM_ERR_INVALID_ARG, "n_moments must be positive");
  if (!(half_width > 0) || !std::isfinite(center)) fail(FTLM_ERR_INVALID_ARG, "need a finite centre and half_width > 0");
  if (dist != FTLM_RADEMACHER && dist != FTLM_GAUSSIAN) fail(FTLM_ERR_INVALID_ARG, "bad distribution");
  if (b.D == 0) {
    std::fill(moments, moments + (size_t)R * M, 0.0);
    return;
  }
  AllocStreamScope scope(st ? st : tl_alloc_stream);
  if (storage == FTLM_F64)
    kpm_typed<double>(b, R, M, seed, dist, center, half_width, moments, st);
  else if (storage == FTLM_F32)
    kpm_typed<float>(b, R, M, seed, dist, center, half_width, moments, st);
  else
    fail(FTLM_ERR_INVALID_ARG, "storage must be FTLM_F64 or FTLM_F32");
  // a spectrum outside (c - w, c + w) makes the Chebyshev vectors grow
  for (size_t i = 0; i < (size_t)R * M; ++i)
    if (!(std::fabs(moments[i]) <= 1.0 + 1e-6))
      fail(FTLM_ERR_INVALID_ARG, "moments leave [-1, 1]: the block spectrum is not inside center +- half_width");
}

}  // namespace ftlm
