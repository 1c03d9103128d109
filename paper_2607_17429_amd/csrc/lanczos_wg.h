// Fused Lanczos kernel for small blocks (paper Sections 2.2 and 3): one
// workgroup runs every step of the R chains of one block job (start vectors,
// H.V with the Lanczos epilogue, alpha, update, beta) with workgroup barriers
// between the phases, so a whole campaign of small, uneven blocks is one launch
// per kernel shape instead of four launches per step and block.
//
// The recurrence, the scaling of the stored vectors and the stopping rule are
// those of the per-step kernels in lanczos.hip: w = s_j H q_j - beta_j s_{j-1}
// q_{j-1} written over q_{j-1} by the H.V pass (hv_pass, shared with k_hv),
// alpha_j = s_j <q_j, w>, w -= alpha_j s_j q_j, beta_{j+1} = |w|, q_{j+1} = w,
// s_{j+1} = 1 / beta_{j+1}.  Reductions run over the workgroup in a fixed order
// (deterministic; the order differs from the per-step kernels', so the two
// agree to rounding).  Vectors use the block row layout; the irrep tables and
// the bond data sit in LDS, and so do the two vectors when they fit.
#pragma once

#include "hv_kernel.h"

namespace ftlm {
namespace hvk {

constexpr int kWgMaxR = kWgMaxChains;
// threads per job: 512 (two waves per SIMD, so twice the representatives in
// flight as with 256) for irrep dimension buckets up to 6, whose registers fit
// the 256 per lane this allows; 256 for the 8 and 12 buckets
template <int DG>
constexpr int kWgThreads = DG <= 6 ? 512 : 256;

template <typename T>
struct WgJob {
  HvArgs<T> a;          // tables of the block (X, Y and scal are set by the kernel)
  T* q0;                // D x R, row-major (chain fastest)
  T* q1;                // D x R
  const uint64_t* keys; // R chain keys
  double* alpha;        // R x steps
  double* beta;         // R x steps
  int32_t* nsteps;      // R
  uint64_t D;
  int R, steps, target, dist;
  double sigma;         // storage scale of the stored vectors (1 for FP32 / FP64)
  int lds_vec;          // 1: q0, q1 live in dynamic LDS at byte offset o_q (q0 and q1 unused)
  uint32_t o_q;
};

struct WgChain {
  double s, bs, beta, scale, ca, a;
  int n, done;
};

// Column sums of red[q * W + c], q < n, by pairwise halving (a fixed order,
// log2(n) barrier steps instead of n serial reads); the sum of column c ends
// in red[c].  Called by every thread after red is written and synchronized.
__device__ __forceinline__ void wg_col_sum(double* red, int W, int n) {
  for (int m = n; m > 1;) {
    const int half = (m + 1) >> 1;
    for (int i = threadIdx.x; i < (m - half) * W; i += blockDim.x) {
      const int q = half + i / W, c = i - (i / W) * W;
      red[(q - half) * W + c] += red[q * W + c];
    }
    __syncthreads();
    m = half;
  }
}

// Per-chain sums of one value per thread (thread t holds chain t % R, rows
// t / R + k * RB); out[v] for v < R, in a fixed order.
__device__ __forceinline__ void wg_chain_sum(double x, int R, int RB, double* red, double* out) {
  red[threadIdx.x] = x;
  __syncthreads();
  wg_col_sum(red, R, RB);
  if ((int)threadIdx.x < R) out[threadIdx.x] = red[threadIdx.x];
  __syncthreads();
}

template <typename T, int DG, int VPL, int NCH>
__global__ void __launch_bounds__(kWgThreads<DG>) k_lanczos_wg(const WgJob<T>* __restrict__ jobs) {
  constexpr int NT = kWgThreads<DG>;
  using W = word_t<NCH>;
  extern __shared__ uint64_t smem_raw[];
  char* sm = (char*)smem_raw;
  __shared__ double red[NT];
  __shared__ double scal[2 * kWgMaxR];
  __shared__ double csum[kWgMaxR];
  __shared__ WgChain ch[kWgMaxR];

  const WgJob<T>& J = jobs[blockIdx.x];
  HvArgs<T> a = J.a;
  // the two Lanczos vectors: in LDS when they fit (the H.V gathers and the
  // update then never leave the CU), otherwise in device memory
  T* const q0 = J.lds_vec ? (T*)(sm + J.o_q) : J.q0;
  T* const q1 = J.lds_vec ? q0 + J.D * (uint64_t)J.R : J.q1;
  double* const alpha = J.alpha;
  double* const beta = J.beta;
  const uint64_t D = J.D;
  const int R = J.R, steps = J.steps, target = J.target, dist = J.dist;
  const double sigma = J.sigma;
  const int t = threadIdx.x;

  const HvTabs tb{stage<double>(a.rhoT, (uint32_t)a.G * DG * DG, sm + a.o_rho),
                  stage<double>(a.V, (uint32_t)a.n_stab * DG * DG, sm + a.o_V),
                  stage<double>(a.stabf, (uint32_t)a.n_stab * 4, sm + a.o_stab),
                  stage<double>(a.J, (uint32_t)a.nbonds, sm + a.o_J),
                  stage<double>(a.fac, (uint32_t)(2 * a.dloc * a.dloc), sm + a.o_fac),
                  stage<int32_t>(a.bonds, (uint32_t)(2 * a.nbonds), sm + a.o_bonds)};
  const dev::OrbitTabs<W, NCH> otabs = dev::orbit_tabs<W, NCH>((const W*)nullptr, 1, 1);  // entries: unused
  for (int i = t; i < R * steps; i += NT) {
    alpha[i] = 0.0;
    beta[i] = 0.0;
  }

  // ---- start vectors: FP64 norm of the draw, then the stored q_0 and its norm
  const int RB = NT / R;
  const int v = t % R, r0 = t / R;
  const bool act = r0 < RB;
  const uint64_t key = J.keys[v];
  double acc = 0.0;
  if (act)
    for (uint64_t row = (uint64_t)r0; row < D; row += (uint64_t)RB) {
      const double x = dev::start_value(key, row, dist);
      acc += x * x;
    }
  wg_chain_sum(acc, R, RB, red, csum);  // also the barrier after the table staging
  const double inv = csum[v] > 0 ? sigma / sqrt(csum[v]) : 0.0;  // stored q_0 has norm sigma
  acc = 0.0;
  if (act)
    for (uint64_t row = (uint64_t)r0; row < D; row += (uint64_t)RB) {
      const T q = (T)(dev::start_value(key, row, dist) * inv);
      q0[row * R + v] = q;
      q1[row * R + v] = T(0);
      acc += (double)q * (double)q;
    }
  wg_chain_sum(acc, R, RB, red, csum);
  if (t < R) {
    WgChain c{};
    c.s = csum[t] > 0 ? 1.0 / sqrt(csum[t]) : 0.0;
    ch[t] = c;
  }
  __syncthreads();

  // H.V lane layout: slots of GL lanes over the workgroup, one column tile
  a.scal = scal;
  a.partials = csum;  // non-null: hv_pass applies the Lanczos epilogue (sums are reduced below)
  const int GL = a.GL;
  const int lane = t & 63;
  const uint64_t slot = (uint64_t)(t >> 6) * (uint64_t)(64 >> a.log2GL) + (uint64_t)(lane >> a.log2GL);
  const uint64_t slot_stride = (uint64_t)(NT / 64) * (uint64_t)(64 >> a.log2GL);

  for (int j = 0; j < target; ++j) {
    if (t < R) {
      scal[2 * t] = ch[t].s * sigma;
      scal[2 * t + 1] = ch[t].bs * sigma;
    }
    __syncthreads();
    T* const qj = (j & 1) ? q1 : q0;
    T* const qp = (j & 1) ? q0 : q1;
    a.X = qj;
    a.Y = qp;
    double dot[VPL];
    bool vok[VPL];
    hv_pass<T, DG, VPL, false, NCH>(a, tb, otabs, 0, 1, slot, slot_stride, dot, vok);
    // column sums of q_j . w: lanes with equal (lane mod GL) hold the same column
#pragma unroll
    for (int k = 0; k < VPL; ++k) {
      red[t] = vok[k] ? dot[k] : 0.0;
      __syncthreads();
      wg_col_sum(red, GL, NT / GL);
      if (t < GL && t + k * GL < R) csum[t + k * GL] = red[t];
      __syncthreads();
    }
    if (t < R) {
      WgChain c = ch[t];
      const double al = c.s * csum[t] / sigma;
      c.ca = al * c.s * sigma;
      c.a = al;
      if (!c.done) alpha[(size_t)t * steps + j] = al;
      ch[t] = c;
    }
    __syncthreads();
    // ---- w -= alpha_j s_j q_j, |w|^2
    const double ca = ch[v].ca;
    acc = 0.0;
    if (act)
      for (uint64_t row = (uint64_t)r0; row < D; row += (uint64_t)RB) {
        const uint64_t at = row * R + v;
        const T w = (T)((double)qp[at] - ca * (double)qj[at]);
        qp[at] = w;
        acc += (double)w * (double)w;
      }
    wg_chain_sum(acc, R, RB, red, csum);
    if (t < R) {
      WgChain c = ch[t];
      if (!c.done) {
        const double b = sqrt(csum[t]) / sigma;
        beta[(size_t)t * steps + j] = b;
        c.scale = fmax(c.scale, fabs(c.a) + c.beta + b);
        c.n = j + 1;
        if (j + 1 >= target || b <= 1e-10 * c.scale) {
          c.done = 1;
        } else {
          c.bs = b * c.s;
          c.s = 1.0 / (b * sigma);
          c.beta = b;
        }
      }
      if (c.done) {
        c.s = 0.0;
        c.bs = 0.0;
      }
      ch[t] = c;
    }
    __syncthreads();
    int live = 0;
    for (int c = 0; c < R; ++c) live |= !ch[c].done;
    if (!live) break;  // uniform: every thread reads the same chain states
  }
  if (t < R) J.nsteps[t] = ch[t].n;
}

// One launch: grid = one workgroup per job, all jobs of one kernel shape.
template <int DG>
void wg_launch(int dtype, int vpl, bool wide, const void* jobs, int njobs, size_t shm, hipStream_t st);

template <typename T, int DG, int VPL>
void wg_launch_t(bool wide, const void* jobs, int njobs, size_t shm, hipStream_t st) {
  if (wide)
    hipLaunchKernelGGL((k_lanczos_wg<T, DG, VPL, 16>), dim3(njobs), dim3(kWgThreads<DG>), shm, st,
                       (const WgJob<T>*)jobs);
  else
    hipLaunchKernelGGL((k_lanczos_wg<T, DG, VPL, 8>), dim3(njobs), dim3(kWgThreads<DG>), shm, st,
                       (const WgJob<T>*)jobs);
}

template <typename T, int DG>
void wg_launch_v(int vpl, bool wide, const void* jobs, int njobs, size_t shm, hipStream_t st) {
  switch (vpl) {
    case 1: wg_launch_t<T, DG, 1>(wide, jobs, njobs, shm, st); break;
    case 2: wg_launch_t<T, DG, 2>(wide, jobs, njobs, shm, st); break;
    case 3: wg_launch_t<T, DG, 3>(wide, jobs, njobs, shm, st); break;
    case 4: wg_launch_t<T, DG, 4>(wide, jobs, njobs, shm, st); break;
    default: fail(FTLM_ERR_INVALID_ARG, "fused Lanczos: unsupported vectors per lane");
  }
}

#define FTLM_WG_INSTANTIATE(DGV)                                                                          \
  template <>                                                                                            \
  void wg_launch<DGV>(int dtype, int vpl, bool wide, const void* jobs, int njobs, size_t shm,            \
                      hipStream_t st) {                                                                  \
    if (dtype == FTLM_F64)                                                                               \
      wg_launch_v<double, DGV>(vpl, wide, jobs, njobs, shm, st);                                         \
    else if (dtype == FTLM_F32)                                                                          \
      wg_launch_v<float, DGV>(vpl, wide, jobs, njobs, shm, st);                                          \
    else                                                                                                 \
      fail(FTLM_ERR_INVALID_ARG, "fused Lanczos: storage must be FTLM_F64 or FTLM_F32");                 \
  }

}  // namespace hvk
}  // namespace ftlm
