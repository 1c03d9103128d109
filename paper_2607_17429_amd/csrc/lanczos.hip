// Batched Lanczos chains for the FTLM estimator (paper Sections 2.2 and 3).
//
// All R chains of a block share every H.V launch (vector column = chain).
// Vectors are kept unnormalised as stored (q_j with a per-chain FP64 scale
// s_j, v_j = s_j q_j), so every recursion coefficient comes from the vectors
// exactly as stored:
//   w       = s_j H q_j - beta_j s_{j-1} q_{j-1}   (H.V epilogue, over q_{j-1})
//   alpha_j = s_j <q_j, w>                         (FP64 partials from the same pass)
//   w      -= alpha_j s_j q_j ;  beta_{j+1} = |w|  (one update pass, FP64 partials)
//   q_{j+1} = w, s_{j+1} = 1 / beta_{j+1}
// Reductions over workgroup partials run in a fixed order (deterministic).
// Start vectors: SplitMix64 (Steele, Lea, Flood 2014) stream per chain keyed by
// (seed, 2M, irrep, row, chain); element j uses the (j+1)-th output
// (Rademacher: sign of the top bit) or outputs 2j+1, 2j+2 (Gaussian by the
// Box-Muller transform); normalised in FP64, then rounded to storage.
#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"

namespace ftlm {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

struct Chain {
  double s;       // scale of q_j
  double bs;      // beta_j * s_{j-1}
  double beta;    // beta_j
  double scale;   // max_i (|alpha_i| + beta_i + beta_{i+1})
  double ca;      // alpha_j * s_j (update coefficient)
  int n;          // products done
  int done;
};

__device__ __forceinline__ double start_value(uint64_t key, uint64_t j, int dist) {
  if (dist == FTLM_RADEMACHER) {
    const uint64_t x = dev::mix64(key + (j + 1) * kGamma);
    return (x >> 63) ? -1.0 : 1.0;
  }
  const uint64_t x1 = dev::mix64(key + (2 * j + 1) * kGamma);
  const uint64_t x2 = dev::mix64(key + (2 * j + 2) * kGamma);
  const double u1 = ((double)(x1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

// Threads are laid out as (row-in-block r0, chain v) with TB = R * (256 / R)
// threads per block, so each thread's elements belong to one chain and the
// per-chain block sums are reduced in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_start(const uint64_t* __restrict__ keys, int dist, uint64_t D, int R,
                                              const double* __restrict__ inv_norm, T* __restrict__ Q,
                                              double* __restrict__ partials) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int RB = blockDim.x / R;
  const int v = t % R, r0 = t / R;
  double acc = 0.0;
  for (uint64_t row = (uint64_t)blockIdx.x * RB + r0; row < D; row += (uint64_t)gridDim.x * RB) {
    const double x = start_value(keys[v], row, dist);
    if (inv_norm) {
      const T q = (T)(x * inv_norm[v]);
      Q[row * R + v] = q;
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

// w -= ca_v q_j (stored), partial |w|^2
template <typename T>
__global__ void __launch_bounds__(256) k_update(const Chain* __restrict__ ch, uint64_t D, int R, const T* __restrict__ Qj,
                                               T* __restrict__ Wv, double* __restrict__ partials) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int RB = blockDim.x / R;
  const int v = t % R, r0 = t / R;
  const double ca = ch[v].ca;
  double acc = 0.0;
  for (uint64_t row = (uint64_t)blockIdx.x * RB + r0; row < D; row += (uint64_t)gridDim.x * RB) {
    const uint64_t at = row * R + v;
    const T w = (T)((double)Wv[at] - ca * (double)Qj[at]);
    Wv[at] = w;
    acc += (double)w * (double)w;
  }
  red[t] = acc;
  __syncthreads();
  if (t < R) {
    double s = 0.0;
    for (int q = 0; q < RB; ++q) s += red[q * R + t];
    partials[(size_t)blockIdx.x * R + t] = s;
  }
}

__device__ __forceinline__ double block_sum(const double* __restrict__ partials, int ngroups, int R, int v) {
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

// one block per chain
__global__ void __launch_bounds__(256) k_init_chain(const double* __restrict__ partials, int ngroups, int R,
                                                   double* __restrict__ inv_norm, Chain* __restrict__ ch, int phase) {
  const int v = blockIdx.x;
  const double s = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    if (phase == 0) {
      inv_norm[v] = s > 0 ? 1.0 / sqrt(s) : 0.0;
    } else {
      Chain c{};
      c.s = s > 0 ? 1.0 / sqrt(s) : 0.0;
      c.bs = 0.0;
      c.beta = 0.0;
      c.scale = 0.0;
      c.ca = 0.0;
      c.n = 0;
      c.done = 0;
      ch[v] = c;
    }
  }
}

__global__ void k_scal(const Chain* __restrict__ ch, int R, double* __restrict__ scal) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < R) {
    scal[2 * v] = ch[v].s;
    scal[2 * v + 1] = ch[v].bs;
  }
}

__global__ void __launch_bounds__(256) k_alpha(const double* __restrict__ partials, int ngroups, int R, Chain* __restrict__ ch,
                                              double* __restrict__ alpha, int j, int steps) {
  const int v = blockIdx.x;
  const double s = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    Chain c = ch[v];
    const double a = c.s * s;
    c.ca = a * c.s;
    if (!c.done) alpha[(size_t)v * steps + j] = a;
    ch[v] = c;
  }
}

__global__ void __launch_bounds__(256) k_beta(const double* __restrict__ partials, int ngroups, int R, Chain* __restrict__ ch,
                                             const double* __restrict__ alpha, double* __restrict__ beta,
                                             double* __restrict__ scal, int j, int steps, int target) {
  const int v = blockIdx.x;
  const double s2 = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    Chain c = ch[v];
    if (!c.done) {
      const double b = sqrt(s2);
      beta[(size_t)v * steps + j] = b;
      const double a = alpha[(size_t)v * steps + j];
      c.scale = fmax(c.scale, fabs(a) + c.beta + b);
      c.n = j + 1;
      if (j + 1 >= target || b <= 1e-10 * c.scale) {
        c.done = 1;
      } else {
        c.bs = b * c.s;
        c.s = 1.0 / b;
        c.beta = b;
      }
    }
    if (c.done) {
      c.s = 0.0;
      c.bs = 0.0;
    }
    ch[v] = c;
    scal[2 * v] = c.s;
    scal[2 * v + 1] = c.bs;
  }
}

__global__ void k_nsteps(const Chain* __restrict__ ch, int R, int32_t* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < R) out[v] = ch[v].n;
}

unsigned blocks_for(uint64_t rows, int RB) {
  uint64_t g = (rows + RB - 1) / RB;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 4096));
}

template <typename T>
void run_typed(Block& b, int R, int steps, uint64_t seed, int dist, int storage, double* alpha, double* beta,
               int32_t* nsteps, hipStream_t st) {
  const uint64_t D = b.D;
  const int target = (int)std::min<uint64_t>((uint64_t)steps, D);
  std::fill(alpha, alpha + (size_t)R * steps, 0.0);
  std::fill(beta, beta + (size_t)R * steps, 0.0);
  std::fill(nsteps, nsteps + R, 0);
  if (D == 0 || target == 0) return;
  const int TB = R * (256 / R);
  const int RB = TB / R;
  const unsigned nb_vec = blocks_for(D, RB);
  // one lane layout for the whole run (the partial-sum buffer is sized for it)
  const int gl = hv_layout_lanes(b, R, sizeof(T) == 8 ? FTLM_F64 : FTLM_F32);
  const int ng_hv = hv_partial_groups(b, R, gl);
  const int ng_max = std::max<int>((int)nb_vec, ng_hv);
  DevBuf<T> q0, q1;
  q0.alloc(D * R);
  q1.alloc(D * R);
  DevBuf<uint64_t> keys;
  std::vector<uint64_t> hkeys(R);
  for (int v = 0; v < R; ++v) hkeys[v] = chain_key(seed, b.sec->two_M, b.irrep, b.row, v);
  keys.upload(hkeys, st);
  DevBuf<double> partials, inv_norm, scal, d_alpha, d_beta;
  partials.alloc((size_t)ng_max * R);
  inv_norm.alloc(R);
  scal.alloc(2 * R);
  d_alpha.alloc((size_t)R * steps);
  d_beta.alloc((size_t)R * steps);
  FTLM_HIP(hipMemsetAsync(d_alpha.p, 0, d_alpha.bytes(), st));
  FTLM_HIP(hipMemsetAsync(d_beta.p, 0, d_beta.bytes(), st));
  DevBuf<Chain> ch;
  ch.alloc(R);
  DevBuf<int32_t> d_n;
  d_n.alloc(R);
  // start vectors: norm of the FP64 draw, then the stored, normalised q_0 and its norm
  hipLaunchKernelGGL((k_start<T>), dim3(nb_vec), dim3(TB), 0, st, keys.p, dist, D, R, (const double*)nullptr,
                     q0.p, partials.p);
  hipLaunchKernelGGL(k_init_chain, dim3(R), dim3(256), 0, st, partials.p, (int)nb_vec, R, inv_norm.p, ch.p, 0);
  hipLaunchKernelGGL((k_start<T>), dim3(nb_vec), dim3(TB), 0, st, keys.p, dist, D, R, inv_norm.p, q0.p, partials.p);
  hipLaunchKernelGGL(k_init_chain, dim3(R), dim3(256), 0, st, partials.p, (int)nb_vec, R, inv_norm.p, ch.p, 1);
  FTLM_HIP(hipMemsetAsync(q1.p, 0, q1.bytes(), st));
  hipLaunchKernelGGL(k_scal, dim3((R + 63) / 64), dim3(64), 0, st, ch.p, R, scal.p);
  FTLM_HIP(hipGetLastError());
  T* qj = q0.p;
  T* qprev = q1.p;
  const int dtype = sizeof(T) == 8 ? FTLM_F64 : FTLM_F32;
  for (int j = 0; j < target; ++j) {
    LanczosEpilogue lz{scal.p, partials.p, ng_hv};
    apply_hv_gl(b, qj, qprev, R, R, dtype, st, &lz, gl);  // qprev <- w
    hipLaunchKernelGGL(k_alpha, dim3(R), dim3(256), 0, st, partials.p, ng_hv, R, ch.p, d_alpha.p, j, steps);
    hipLaunchKernelGGL((k_update<T>), dim3(nb_vec), dim3(TB), 0, st, ch.p, D, R, qj, qprev, partials.p);
    hipLaunchKernelGGL(k_beta, dim3(R), dim3(256), 0, st, partials.p, (int)nb_vec, R, ch.p, d_alpha.p, d_beta.p, scal.p, j,
                       steps, target);
    FTLM_HIP(hipGetLastError());
    std::swap(qj, qprev);
  }
  hipLaunchKernelGGL(k_nsteps, dim3((R + 63) / 64), dim3(64), 0, st, ch.p, R, d_n.p);
  FTLM_HIP(hipMemcpyAsync(alpha, d_alpha.p, d_alpha.bytes(), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipMemcpyAsync(beta, d_beta.p, d_beta.bytes(), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipMemcpyAsync(nsteps, d_n.p, R * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipStreamSynchronize(st));
  (void)storage;
}

}  // namespace

uint64_t chain_key(uint64_t seed, int two_M, int irrep, int row, int chain) {
  auto mix = [](uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  uint64_t h = mix(seed + kGamma);
  const int64_t xs[4] = {two_M, irrep, row, chain};
  for (int i = 0; i < 4; ++i) h = mix(h ^ ((uint64_t)xs[i] + (uint64_t)(i + 2) * kGamma));
  return h;
}

void run_lanczos(Block& b, int R, int steps, uint64_t seed, int storage, int dist, double* alpha, double* beta,
                 int32_t* nsteps, hipStream_t st) {
  if (R <= 0 || R > 256) fail(FTLM_ERR_INVALID_ARG, "R must be in 1..256");
  if (steps <= 0) fail(FTLM_ERR_INVALID_ARG, "steps must be positive");
  if (!alpha || !beta || !nsteps) fail(FTLM_ERR_INVALID_ARG, "null output");
  if (dist != FTLM_RADEMACHER && dist != FTLM_GAUSSIAN) fail(FTLM_ERR_INVALID_ARG, "bad distribution");
  if (storage == FTLM_F64)
    run_typed<double>(b, R, steps, seed, dist, storage, alpha, beta, nsteps, st);
  else if (storage == FTLM_F32)
    run_typed<float>(b, R, steps, seed, dist, storage, alpha, beta, nsteps, st);
  else
    fail(FTLM_ERR_INVALID_ARG, "storage must be FTLM_F64 or FTLM_F32");
}

}  // namespace ftlm
