// ftlm_apply_H_ex_noalloc: ftlm_apply_H_ex for callers that cannot allocate
// device memory (work captured into a HIP graph, tight serving loops).  The
// one scratch buffer of that call, the per-workgroup FP64 partial sums of the
// Lanczos epilogue, lives in a file-scope device array instead of a
// per-call allocation.  Each device gets its own copy of the array; its
// address is looked up once per device with hipGetSymbolAddress, and host
// code only ever passes that address to kernels.
#include <mutex>
#include <unordered_map>

#include "capi_guard.h"
#include "internal.h"

namespace ftlm {

namespace {

// 8192 workgroups (the H.V grid's cap) x 64 vectors of partial sums: 4 MiB
constexpr size_t kNoallocScratchDoubles = (size_t)8192 * 64;

__device__ __align__(256) double scratch[kNoallocScratchDoubles];

std::mutex g_scratch_mu;
std::unordered_map<int, double*> g_scratch_ptr;  // device ordinal -> address of its scratch

// The device address of this device's scratch (looked up on its first call).
double* device_scratch() {
  int dev = 0;
  FTLM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  FTLM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(FTLM_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return static_cast<double*>(p);
}

}  // namespace

}  // namespace ftlm

using namespace ftlm;

extern "C" int ftlm_apply_H_ex_noalloc(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld,
                                       int32_t dtype, ftlm_hv_opts* opts, void* stream) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    if (X == Y && X) fail(FTLM_ERR_INVALID_ARG, "X and Y must not overlap");
    const Block& B = *b->b;
    const HvExPlan p = plan_hv_ex(B, nvec, ld, dtype, opts);
    double* partials = nullptr;
    if (p.epi && p.ng > 0) {
      if ((size_t)p.ng * (size_t)nvec > kNoallocScratchDoubles)
        fail(FTLM_ERR_INVALID_ARG, "nvec x workgroups = " + std::to_string((size_t)p.ng * nvec) +
                                       " partial sums exceed the static scratch of " +
                                       std::to_string(kNoallocScratchDoubles));
      partials = device_scratch();
    }
    apply_hv_ex(B, X, Y, nvec, ld, dtype, opts, p, partials, (hipStream_t)stream);
    if (opts) {
      opts->lanes_used = p.gl;
      opts->adjacent_columns = p.adjacent ? 1 : 0;
    }
  });
}
