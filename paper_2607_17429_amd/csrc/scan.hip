// Exclusive prefix sum over uint64 device arrays (three-phase: per-tile scan
// in LDS, recursive scan of tile totals, add-back).  Deterministic.
#include "internal.h"

namespace ftlm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) scan_tiles(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                          uint64_t n, uint64_t* __restrict__ tile_sums) {
  __shared__ uint64_t sh[kScanThreads];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    sum += v[i];
  }
  sh[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of per-thread sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint64_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  uint64_t run = sh[threadIdx.x] - sum;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void __launch_bounds__(kScanThreads) scan_add(uint64_t* __restrict__ out, uint64_t n,
                                                        const uint64_t* __restrict__ tile_offsets) {
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kScanItems;
  const uint64_t add = tile_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] += add;
}

}  // namespace

void scan_exclusive_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* total, hipStream_t s) {
  if (n == 0) {
    if (total) *total = 0;
    return;
  }
  const uint64_t tiles = (n + kTile - 1) / kTile;
  DevBuf<uint64_t> sums;
  sums.alloc(tiles + 1);
  hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n, sums.p);
  FTLM_HIP(hipGetLastError());
  if (tiles > 1) {
    uint64_t tt = 0;
    scan_exclusive_u64(sums.p, sums.p, tiles, total ? &tt : nullptr, s);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n, sums.p);
    FTLM_HIP(hipGetLastError());
    if (total) *total = tt;
  } else if (total) {
    FTLM_HIP(hipMemcpyAsync(total, sums.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    FTLM_HIP(hipStreamSynchronize(s));
  }
  // `sums` must outlive the adds: a stream-ordered free does; a plain one waits
  if (tiles > 1 && !sums.async) FTLM_HIP(hipStreamSynchronize(s));
}

}  // namespace ftlm
