// Compile-time dispatch over the number of 4-bit label chunks.  Up to 8
// chunks the packed label fits 32 bits and the kernels use uint32_t words.
#pragma once

#include <cstdint>
#include <type_traits>

namespace ftlm {

template <int NCH>
using word_t = typename std::conditional<(NCH <= 8), uint32_t, uint64_t>::type;

// Chunk counts are rounded up to a few buckets (tables for the extra chunks
// are all zero, so a padded chunk always contributes nothing).
inline int nch_bucket(int nch) {
  const int buckets[] = {3, 5, 8, 10, 12, 16};
  for (int b : buckets)
    if (nch <= b) return b;
  return -1;
}

#define FTLM_NCH_CASE(n, ...)             \
  case n: {                               \
    constexpr int NCH = n;                \
    using W = ::ftlm::word_t<NCH>;        \
    __VA_ARGS__;                          \
  } break;

#define FTLM_DISPATCH_NCH(nch, ...)                                       \
  switch (nch) {                                                          \
    FTLM_NCH_CASE(3, __VA_ARGS__) FTLM_NCH_CASE(5, __VA_ARGS__)           \
    FTLM_NCH_CASE(8, __VA_ARGS__) FTLM_NCH_CASE(10, __VA_ARGS__)          \
    FTLM_NCH_CASE(12, __VA_ARGS__) FTLM_NCH_CASE(16, __VA_ARGS__)         \
    default:                                                              \
      ::ftlm::fail(FTLM_ERR_UNSUPPORTED, "label wider than 64 bits");     \
  }

}  // namespace ftlm
