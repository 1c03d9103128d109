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
// FP16 storage keeps every stored vector multiplied by a per-chain power of
// two sigma (~ sqrt(rows)), so its elements are of order one: q_0 is stored
// with norm sigma, the epilogue and update use sigma-scaled coefficients and
// alpha, beta divide it out.  For FP32 and FP64 sigma = 1 and every formula
// reduces exactly to the one above.
// Reductions over workgroup partials run in a fixed order (deterministic).
// Start vectors: SplitMix64 (Steele, Lea, Flood 2014) stream per chain keyed by
// (seed, 2M, irrep, row, chain); element j uses the (j+1)-th output
// (Rademacher: sign of the top bit) or outputs 2j+1, 2j+2 (Gaussian by the
// Box-Muller transform); normalised in FP64, then rounded to storage.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "device.h"
#include "internal.h"

namespace ftlm {

namespace {

using dev::kGamma;
using dev::start_value;

struct Chain {
  double s;       // scale of q_j
  double bs;      // beta_j * s_{j-1}
  double beta;    // beta_j
  double scale;   // max_i (|alpha_i| + beta_i + beta_{i+1})
  double ca;      // alpha_j * s_j (update coefficient)
  int n;          // products done
  int done;
  int step;       // index j of the next step (the kernels of a step read it
                  // here, so one captured graph serves every step)
  double sigma;   // power-of-two storage scale (1 unless FP16)
};

// Threads are laid out as (row-in-block r0, chain v) with TB = R * (256 / R)
// threads per block, so each thread's elements belong to one chain and the
// per-chain block sums are reduced in a fixed order.
template <typename T>
// Padded layout (meta != nullptr): stored row r holds row k of representative
// i (dev::padded_rep_of), which is block row offset(i) + k for k < n_Gamma(i);
// every other stored row is zero.  D counts stored rows.
__global__ void __launch_bounds__(256) k_start(const uint64_t* __restrict__ keys, int dist, uint64_t D, int R,
                                              const double* __restrict__ inv_norm, T* __restrict__ Q,
                                              double* __restrict__ partials, const uint64_t* __restrict__ meta,
                                              const double* __restrict__ stabf, dev::PadMap pm) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int RB = blockDim.x / R;
  const int v = t % R, r0 = t / R;
  double acc = 0.0;
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
    const double x = live ? start_value(keys[v], brow, dist) : 0.0;
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
                                                   double* __restrict__ inv_norm, Chain* __restrict__ ch, int phase,
                                                   double sigma) {
  const int v = blockIdx.x;
  const double s = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    if (phase == 0) {
      inv_norm[v] = s > 0 ? sigma / sqrt(s) : 0.0;  // stored q_0 has norm sigma
    } else {
      Chain c{};
      c.sigma = sigma;
      c.s = s > 0 ? 1.0 / sqrt(s) : 0.0;
      c.bs = 0.0;
      c.beta = 0.0;
      c.scale = 0.0;
      c.ca = 0.0;
      c.n = 0;
      c.done = 0;
      c.step = 0;
      ch[v] = c;
    }
  }
}

__global__ void k_scal(const Chain* __restrict__ ch, int R, double* __restrict__ scal) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < R) {
    scal[2 * v] = ch[v].s * ch[v].sigma;
    scal[2 * v + 1] = ch[v].bs * ch[v].sigma;
  }
}

__global__ void __launch_bounds__(256) k_alpha(const double* __restrict__ partials, int ngroups, int R, Chain* __restrict__ ch,
                                              double* __restrict__ alpha, int steps) {
  const int v = blockIdx.x;
  const double s = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    Chain c = ch[v];
    const int j = c.step;
    const double a = c.s * s / c.sigma;
    c.ca = a * c.s * c.sigma;
    if (!c.done) alpha[(size_t)v * steps + j] = a;
    ch[v] = c;
  }
}

__global__ void __launch_bounds__(256) k_beta(const double* __restrict__ partials, int ngroups, int R, Chain* __restrict__ ch,
                                             const double* __restrict__ alpha, double* __restrict__ beta,
                                             double* __restrict__ scal, int steps, int target) {
  const int v = blockIdx.x;
  const double s2 = block_sum(partials, ngroups, R, v);
  if (threadIdx.x == 0) {
    Chain c = ch[v];
    const int j = c.step;
    c.step = j + 1;
    if (!c.done) {
      const double b = sqrt(s2) / c.sigma;
      beta[(size_t)v * steps + j] = b;
      const double a = alpha[(size_t)v * steps + j];
      c.scale = fmax(c.scale, fabs(a) + c.beta + b);
      c.n = j + 1;
      if (j + 1 >= target || b <= 1e-10 * c.scale) {
        c.done = 1;
      } else {
        c.bs = b * c.s;
        c.s = 1.0 / (b * c.sigma);
        c.beta = b;
      }
    }
    if (c.done) {
      c.s = 0.0;
      c.bs = 0.0;
    }
    ch[v] = c;
    scal[2 * v] = c.s * c.sigma;
    scal[2 * v + 1] = c.bs * c.sigma;
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
void enqueue_begin_typed(LanczosRun& L, hipStream_t st) {
  const int R = L.R;
  const uint64_t D = L.rows;
  T* q0 = (T*)L.q0.p;
  Chain* ch = (Chain*)L.chain.p;
  FTLM_HIP(hipMemsetAsync(L.d_alpha.p, 0, L.d_alpha.bytes(), st));
  FTLM_HIP(hipMemsetAsync(L.d_beta.p, 0, L.d_beta.bytes(), st));
  FTLM_HIP(hipMemsetAsync(L.d_n.p, 0, L.d_n.bytes(), st));
  if (L.target == 0) return;
  // start vectors: norm of the FP64 draw, then the stored, normalised q_0 and its norm
  const uint64_t* meta = L.vl.pad ? L.block->d_meta.p : nullptr;
  const double* stabf = L.block->d_stabf64.p;
  const dev::PadMap pm = pad_map(*L.block, L.vl);
  hipLaunchKernelGGL((k_start<T>), dim3(L.nb_vec), dim3(L.TB), 0, st, L.keys.p, L.dist, D, R, (const double*)nullptr,
                     q0, L.partials.p, meta, stabf, pm);
  hipLaunchKernelGGL(k_init_chain, dim3(R), dim3(256), 0, st, L.partials.p, L.nb_vec, R, L.inv_norm.p, ch, 0,
                     L.sigma);
  hipLaunchKernelGGL((k_start<T>), dim3(L.nb_vec), dim3(L.TB), 0, st, L.keys.p, L.dist, D, R, L.inv_norm.p, q0,
                     L.partials.p, meta, stabf, pm);
  hipLaunchKernelGGL(k_init_chain, dim3(R), dim3(256), 0, st, L.partials.p, L.nb_vec, R, L.inv_norm.p, ch, 1,
                     L.sigma);
  FTLM_HIP(hipMemsetAsync(L.q1.p, 0, L.q1.bytes(), st));
  hipLaunchKernelGGL(k_scal, dim3((R + 63) / 64), dim3(64), 0, st, ch, R, L.scal.p);
  FTLM_HIP(hipGetLastError());
}

// One Lanczos step j: q_j lives in q0 for even j and in q1 for odd j; the
// other buffer holds q_{j-1} and receives w.  The kernels take j from the
// chain state, so the enqueue depends only on the parity of j.
template <typename T>
void enqueue_one_step(LanczosRun& L, hipStream_t st, bool odd, int timed_j) {
  const Block& b = *L.block;
  const int R = L.R, steps = L.steps;
  const uint64_t D = L.rows;
  Chain* ch = (Chain*)L.chain.p;
  const int dtype = sizeof(T) == 8 ? FTLM_F64 : sizeof(T) == 4 ? FTLM_F32 : FTLM_F16;
  T* qj = (T*)(odd ? L.q1.p : L.q0.p);
  T* qprev = (T*)(odd ? L.q0.p : L.q1.p);
  LanczosEpilogue lz{L.scal.p, L.partials.p, L.ng_hv};
  if (timed_j >= 0) FTLM_HIP(hipEventRecord(L.hv_events[2 * timed_j], st));
  apply_hv_gl(b, qj, qprev, R, R, dtype, st, &lz, L.gl, L.vl);  // qprev <- w
  if (timed_j >= 0) FTLM_HIP(hipEventRecord(L.hv_events[2 * timed_j + 1], st));
  hipLaunchKernelGGL(k_alpha, dim3(R), dim3(256), 0, st, L.partials.p, L.ng_hv, R, ch, L.d_alpha.p, steps);
  hipLaunchKernelGGL((k_update<T>), dim3(L.nb_vec), dim3(L.TB), 0, st, ch, D, R, qj, qprev, L.partials.p);
  hipLaunchKernelGGL(k_beta, dim3(R), dim3(256), 0, st, L.partials.p, L.nb_vec, R, ch, L.d_alpha.p, L.d_beta.p,
                     L.scal.p, steps, L.target);
  FTLM_HIP(hipGetLastError());
}

// Steps j0 <= j < j1.  On a capturable stream, pairs of steps starting at an
// even j replay one captured graph of an even and an odd step; otherwise (the
// null stream, timing requested, or a lone step) the kernels are enqueued
// directly.  Both orders are the same kernels with the same arguments.
template <typename T>
void enqueue_steps_typed(LanczosRun& L, hipStream_t st, int j0, int j1) {
  int j = j0;
  const bool graphs = L.use_graphs && st != nullptr && !L.timed;
  if (j < j1 && (j & 1)) enqueue_one_step<T>(L, st, true, L.timed ? j : -1), ++j;
  if (graphs && j + 1 < j1) {
    if (!L.pair_exec) {
      hipGraph_t g = nullptr;
      FTLM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_one_step<T>(L, st, false, -1);
        enqueue_one_step<T>(L, st, true, -1);
      } catch (...) {
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      FTLM_HIP(hipStreamEndCapture(st, &g));
      L.pair_graph = g;
      FTLM_HIP(hipGraphInstantiate(&L.pair_exec, g, nullptr, nullptr, 0));
    }
    for (; j + 1 < j1; j += 2) FTLM_HIP(hipGraphLaunch(L.pair_exec, st));
  }
  for (; j < j1; ++j) enqueue_one_step<T>(L, st, (j & 1) != 0, L.timed ? j : -1);
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

bool padded_vectors(const Block& b) {
  bool pad = false;
  if (b.lanczos_layout == FTLM_LAYOUT_PADDED || b.lanczos_layout == FTLM_LAYOUT_PACKED ||
      b.lanczos_layout == FTLM_LAYOUT_ALIGNED)
    pad = true;
  else if (b.lanczos_layout == FTLM_LAYOUT_AUTO)
    pad = b.D >= (1ull << 20) && (double)b.D_pad <= 1.02 * (double)b.D;
  if (pad && b.D_pad >= (1ull << 48)) fail(FTLM_ERR_UNSUPPORTED, "padded rows above 2^48");
  return pad;
}

VecLayout vec_layout(const Block& b, int kind, int64_t row_bytes) {
  VecLayout v;
  if (kind == FTLM_LAYOUT_BLOCK) return v;
  if (kind != FTLM_LAYOUT_PADDED && kind != FTLM_LAYOUT_PACKED && kind != FTLM_LAYOUT_ALIGNED)
    fail(FTLM_ERR_INVALID_ARG, "bad row layout");
  v.pad = true;
  if (kind == FTLM_LAYOUT_ALIGNED && row_bytes > 0 && (row_bytes & (row_bytes - 1)) == 0 && b.dg > 0) {
    uint32_t S = 1;
    while (S < (uint32_t)b.dg) S <<= 1;
    if (S > (uint32_t)b.dg && (int64_t)S * row_bytes <= 128) {
      v.aligned = true;
      v.rpline = S;
    }
  }
  if (kind == FTLM_LAYOUT_PACKED && row_bytes > 0 && 128 % row_bytes == 0 && b.dg > 0 &&
      b.sec->n_reps < (1ull << 32)) {
    const uint32_t L = (uint32_t)(128 / row_bytes);
    const uint32_t p = L / (uint32_t)b.dg;
    if (p >= 2 && p * (uint32_t)b.dg < L) {
      v.rpl = p;
      v.rpline = L;
    }
  }
  if (vec_rows(b, v) >= (1ull << 48)) fail(FTLM_ERR_UNSUPPORTED, "padded rows above 2^48");
  return v;
}

// AUTO takes plain padded rows: packing measured no faster (the s = 3/2
// dodecahedron H_g block, 2 FP32 chains: 578 ms per H.V packed and padded; the
// gather is bound by the device's rate of random line accesses, one per
// connection either way, not by the bytes of the lines), and it costs rows.
VecLayout run_layout(const Block& b, int64_t row_bytes) {
  if (!padded_vectors(b)) return VecLayout{};
  const int kind = b.lanczos_layout == FTLM_LAYOUT_PACKED || b.lanczos_layout == FTLM_LAYOUT_ALIGNED
                       ? b.lanczos_layout
                       : FTLM_LAYOUT_PADDED;
  return vec_layout(b, kind, row_bytes);
}

uint64_t vec_rows(const Block& b, const VecLayout& v) {
  if (!v.pad) return b.D;
  const uint64_t n = b.sec->n_reps;
  if (v.aligned) return n * (uint64_t)v.rpline;
  if (v.rpl <= 1) return n * (uint64_t)b.dg;
  return (n + v.rpl - 1) / v.rpl * (uint64_t)v.rpline;
}

dev::PadMap pad_map(const Block& b, const VecLayout& v) {
  dev::PadMap m{};
  m.dstride = (uint32_t)std::max(b.dg, 1);
  m.rpl = v.rpl;
  m.rpline = v.rpl > 1 || v.aligned ? v.rpline : m.dstride;
  m.n_reps = b.sec->n_reps;
  return m;
}

LanczosRun::LanczosRun(const Block& b, int R_, int steps_, uint64_t seed_, int storage_, int dist_)
    : block(&b), R(R_), steps(steps_), storage(storage_), dist(dist_), seed(seed_) {
  if (R <= 0 || R > 256) fail(FTLM_ERR_INVALID_ARG, "R must be in 1..256");
  if (steps <= 0) fail(FTLM_ERR_INVALID_ARG, "steps must be positive");
  if (dist != FTLM_RADEMACHER && dist != FTLM_GAUSSIAN) fail(FTLM_ERR_INVALID_ARG, "bad distribution");
  if (storage != FTLM_F64 && storage != FTLM_F32 && storage != FTLM_F16)
    fail(FTLM_ERR_INVALID_ARG, "storage must be FTLM_F64, FTLM_F32 or FTLM_F16");
  const uint64_t D = b.D;
  target = (int)std::min<uint64_t>((uint64_t)steps, D);
  const int64_t elem = storage == FTLM_F64 ? 8 : storage == FTLM_F32 ? 4 : 2;
  vl = run_layout(b, (int64_t)R * elem);
  rows = vec_rows(b, vl);
  // FP16: elements of a unit vector are ~ 1/sqrt(rows); scale them to ~1
  sigma = 1.0;
  if (storage == FTLM_F16 && rows > 1) sigma = std::ldexp(1.0, (int)std::floor(0.5 * std::log2((double)rows)));
  TB = R * (256 / R);
  nb_vec = (int)blocks_for(std::max<uint64_t>(rows, 1), TB / R);
  // one lane layout for the whole run (the partial-sum buffer is sized for it)
  gl = hv_layout_lanes(b, R, storage, vl, true);
  ng_hv = D ? hv_partial_groups(b, R, gl) : 1;
}

size_t LanczosRun::estimate_bytes(const Block& b, int R, int steps, int storage) {
  const size_t elem = storage == FTLM_F64 ? 8 : storage == FTLM_F32 ? 4 : 2;
  // packed rows add at most a third of the padded rows (p >= 2 representatives
  // per line), aligned rows less than double them (S < 2 d_Gamma)
  const uint64_t rows = std::max(b.D, b.lanczos_layout == FTLM_LAYOUT_BLOCK     ? b.D
                                      : b.lanczos_layout == FTLM_LAYOUT_ALIGNED ? 2 * b.D_pad
                                                                                : b.D_pad + b.D_pad / 2);
  return 2 * (size_t)rows * R * elem + (size_t)8192 * R * 8 + (size_t)R * steps * 16 + (size_t)R * 128;
}

void LanczosRun::enable_timing() {
  timed = true;
  hv_events.assign(2 * (size_t)std::max(target, 0), nullptr);
  for (auto& e : hv_events) FTLM_HIP(hipEventCreate(&e));
}

double LanczosRun::hv_ms() const {
  double t = 0.0;
  for (size_t j = 0; j + 1 < hv_events.size(); j += 2) {
    float ms = 0.f;
    FTLM_HIP(hipEventElapsedTime(&ms, hv_events[j], hv_events[j + 1]));
    t += ms;
  }
  return t;
}

LanczosRun::~LanczosRun() {
  for (auto& e : hv_events)
    if (e) (void)hipEventDestroy(e);
  if (pair_exec) (void)hipGraphExecDestroy(pair_exec);
  if (pair_graph) (void)hipGraphDestroy(pair_graph);
}

void LanczosRun::allocate() {
  const size_t elem = storage == FTLM_F64 ? 8 : storage == FTLM_F32 ? 4 : 2;
  q0.alloc(std::max<uint64_t>(rows, 1) * R * elem);
  q1.alloc(std::max<uint64_t>(rows, 1) * R * elem);
  std::vector<uint64_t> hkeys(R);
  for (int v = 0; v < R; ++v)
    hkeys[v] = chain_key(seed, block->sec->two_M, block->irrep, block->row, first_chain + v);
  keys.upload(hkeys);
  partials.alloc((size_t)std::max(nb_vec, ng_hv) * R);
  inv_norm.alloc(R);
  scal.alloc(2 * R);
  d_alpha.alloc((size_t)R * steps);
  d_beta.alloc((size_t)R * steps);
  chain.alloc(sizeof(Chain) * R);
  d_n.alloc(R);
}

void LanczosRun::enqueue_begin(hipStream_t st) {
  if (storage == FTLM_F64)
    enqueue_begin_typed<double>(*this, st);
  else if (storage == FTLM_F32)
    enqueue_begin_typed<float>(*this, st);
  else
    enqueue_begin_typed<_Float16>(*this, st);
}

void LanczosRun::enqueue_steps(hipStream_t st, int j0, int j1) {
  j0 = std::max(j0, 0);
  j1 = std::min(j1, target);
  if (j0 >= j1) return;
  if (storage == FTLM_F64)
    enqueue_steps_typed<double>(*this, st, j0, j1);
  else if (storage == FTLM_F32)
    enqueue_steps_typed<float>(*this, st, j0, j1);
  else
    enqueue_steps_typed<_Float16>(*this, st, j0, j1);
}

void LanczosRun::enqueue_end(hipStream_t st) {
  if (target == 0) return;
  hipLaunchKernelGGL(k_nsteps, dim3((R + 63) / 64), dim3(64), 0, st, (Chain*)chain.p, R, d_n.p);
  FTLM_HIP(hipGetLastError());
}

void LanczosRun::enqueue(hipStream_t st) {
  enqueue_begin(st);
  enqueue_steps(st, 0, target);
  enqueue_end(st);
}

void LanczosRun::download(hipStream_t st, double* alpha, double* beta, int32_t* nsteps) {
  FTLM_HIP(hipMemcpyAsync(alpha, d_alpha.p, d_alpha.bytes(), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipMemcpyAsync(beta, d_beta.p, d_beta.bytes(), hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipMemcpyAsync(nsteps, d_n.p, (size_t)R * sizeof(int32_t), hipMemcpyDeviceToHost, st));
}

namespace {

// Checkpoint file: a fixed header, then the per-chain states, alpha and beta
// (R x steps), and the two stored vectors q0 and q1 (rows x R each).
constexpr char kRunMagic[8] = {'F', 'T', 'L', 'M', 'R', 'U', 'N', '1'};
struct RunFileHeader {
  char magic[8];
  uint32_t version, header_bytes;
  uint64_t cluster_hash;
  int32_t two_M, irrep, row, dg;
  uint64_t D, rows;
  int32_t layout, R, steps, storage, dist, target, next_step, first_chain;
  int32_t chain_bytes, rpl;
  uint64_t seed;
  double sigma;
  uint64_t vec_bytes;
};

constexpr size_t kStageBytes = 64ull << 20;

struct File {
  FILE* f = nullptr;
  File(const char* path, const char* mode) : f(std::fopen(path, mode)) {
    if (!f) fail(FTLM_ERR_INVALID_ARG, std::string("cannot open ") + path);
  }
  ~File() {
    if (f) std::fclose(f);
  }
};

struct Pinned {
  void* p = nullptr;
  explicit Pinned(size_t n) { FTLM_HIP(hipHostMalloc(&p, n, hipHostMallocDefault)); }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

// device -> file and file -> device through a pinned staging buffer
void dev_to_file(FILE* f, const void* dev, size_t bytes, hipStream_t st, Pinned& stage) {
  for (size_t o = 0; o < bytes; o += kStageBytes) {
    const size_t n = std::min(kStageBytes, bytes - o);
    FTLM_HIP(hipMemcpyAsync(stage.p, (const uint8_t*)dev + o, n, hipMemcpyDeviceToHost, st));
    FTLM_HIP(hipStreamSynchronize(st));
    if (std::fwrite(stage.p, 1, n, f) != n) fail(FTLM_ERR_INVALID_ARG, "checkpoint write failed");
  }
}

void file_to_dev(FILE* f, void* dev, size_t bytes, hipStream_t st, Pinned& stage) {
  for (size_t o = 0; o < bytes; o += kStageBytes) {
    const size_t n = std::min(kStageBytes, bytes - o);
    FTLM_HIP(hipStreamSynchronize(st));  // the previous chunk has left the staging buffer
    if (std::fread(stage.p, 1, n, f) != n) fail(FTLM_ERR_INVALID_ARG, "checkpoint file is truncated");
    FTLM_HIP(hipMemcpyAsync((uint8_t*)dev + o, stage.p, n, hipMemcpyHostToDevice, st));
  }
  FTLM_HIP(hipStreamSynchronize(st));
}

}  // namespace

void LanczosRun::save(const char* path, hipStream_t st, int next_step) const {
  if (!path) fail(FTLM_ERR_INVALID_ARG, "null path");
  FTLM_HIP(hipStreamSynchronize(st));
  RunFileHeader h{};
  std::memcpy(h.magic, kRunMagic, 8);
  h.version = 1;
  h.header_bytes = sizeof(RunFileHeader);
  h.cluster_hash = block->sec->cluster_hash;
  h.two_M = block->sec->two_M;
  h.irrep = block->irrep;
  h.row = block->row;
  h.dg = block->dg;
  h.D = block->D;
  h.rows = rows;
  h.layout = vl.kind();
  h.rpl = (int32_t)vl.rpl;
  h.R = R;
  h.steps = steps;
  h.storage = storage;
  h.dist = dist;
  h.target = target;
  h.next_step = next_step;
  h.first_chain = first_chain;
  h.chain_bytes = (int32_t)sizeof(Chain);
  h.seed = seed;
  h.sigma = sigma;
  h.vec_bytes = q0.bytes();
  // written next to the target and renamed into place once complete, so an
  // interrupted save leaves an earlier checkpoint at path intact
  const std::string part = std::string(path) + ".part";
  try {
    File f(part.c_str(), "wb");
    if (std::fwrite(&h, sizeof(h), 1, f.f) != 1) fail(FTLM_ERR_INVALID_ARG, "checkpoint write failed");
    Pinned stage(kStageBytes);
    dev_to_file(f.f, chain.p, chain.bytes(), st, stage);
    dev_to_file(f.f, d_alpha.p, d_alpha.bytes(), st, stage);
    dev_to_file(f.f, d_beta.p, d_beta.bytes(), st, stage);
    dev_to_file(f.f, q0.p, q0.bytes(), st, stage);
    dev_to_file(f.f, q1.p, q1.bytes(), st, stage);
    const int rc = std::fclose(f.f);
    f.f = nullptr;
    if (rc != 0) fail(FTLM_ERR_INVALID_ARG, "checkpoint write failed");
    if (std::rename(part.c_str(), path) != 0) fail(FTLM_ERR_INVALID_ARG, std::string("cannot replace ") + path);
  } catch (...) {
    std::remove(part.c_str());
    throw;
  }
}

std::unique_ptr<LanczosRun> LanczosRun::load(const Block& b, const char* path, hipStream_t st, int& next_step) {
  if (!path) fail(FTLM_ERR_INVALID_ARG, "null path");
  File f(path, "rb");
  RunFileHeader h{};
  if (std::fread(&h, sizeof(h), 1, f.f) != 1 || std::memcmp(h.magic, kRunMagic, 8) != 0 || h.version != 1 ||
      h.header_bytes != sizeof(RunFileHeader) || h.chain_bytes != (int32_t)sizeof(Chain))
    fail(FTLM_ERR_INVALID_ARG, std::string(path) + " is not a Lanczos checkpoint of this library");
  if (h.cluster_hash != b.sec->cluster_hash || h.two_M != b.sec->two_M || h.irrep != b.irrep || h.row != b.row ||
      h.dg != b.dg || h.D != b.D)
    fail(FTLM_ERR_INVALID_ARG, "the checkpoint belongs to another block");
  auto L = std::make_unique<LanczosRun>(b, h.R, h.steps, h.seed, h.storage, h.dist);
  L->first_chain = h.first_chain;
  if (L->rows != h.rows || L->vl.kind() != h.layout || (int32_t)L->vl.rpl != h.rpl || L->target != h.target ||
      L->sigma != h.sigma)
    fail(FTLM_ERR_INVALID_ARG, "the checkpoint's row layout differs from this block's");
  L->allocate();
  if (L->q0.bytes() != h.vec_bytes) fail(FTLM_ERR_INVALID_ARG, "checkpoint vector size mismatch");
  Pinned stage(kStageBytes);
  file_to_dev(f.f, L->chain.p, L->chain.bytes(), st, stage);
  file_to_dev(f.f, L->d_alpha.p, L->d_alpha.bytes(), st, stage);
  file_to_dev(f.f, L->d_beta.p, L->d_beta.bytes(), st, stage);
  file_to_dev(f.f, L->q0.p, L->q0.bytes(), st, stage);
  file_to_dev(f.f, L->q1.p, L->q1.bytes(), st, stage);
  // the H.V epilogue's coefficients follow from the chain states
  hipLaunchKernelGGL(k_scal, dim3((L->R + 63) / 64), dim3(64), 0, st, (const Chain*)L->chain.p, L->R, L->scal.p);
  FTLM_HIP(hipGetLastError());
  next_step = h.next_step;
  return L;
}

void run_lanczos(Block& b, int R, int steps, uint64_t seed, int storage, int dist, double* alpha, double* beta,
                 int32_t* nsteps, hipStream_t st, ftlm_run_info* info) {
  if (!alpha || !beta || !nsteps) fail(FTLM_ERR_INVALID_ARG, "null output");
  LanczosRun L(b, R, steps, seed, storage, dist);
  AllocStreamScope scope(st ? st : tl_alloc_stream);  // stream-ordered scratch: no device-wide sync on free
  if (info) L.enable_timing();
  L.allocate();
  L.enqueue(st);
  L.download(st, alpha, beta, nsteps);
  FTLM_HIP(hipStreamSynchronize(st));
  if (info) {
    info->layout = L.vl.kind();
    info->rows = L.rows;
    info->hv_launches = L.target;
    info->hv_ms = L.hv_ms();
  }
}

}  // namespace ftlm
