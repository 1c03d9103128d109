// Host-side check of the row maps of the padded vector layouts: the device
// helpers padded_row (representative -> first stored row) and padded_rep_of
// (stored row -> representative and row within it) are host-callable, so the
// same functions the kernels use are run here over every layout shape the
// library builds (plain padded rows, aligned rows of a power of two above
// d_Gamma, representatives packed into 128-byte lines).  Prints one line per
// shape and "fail ..." for the first violated property.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "device.h"

namespace {

int fails = 0;

void check(bool c, const char* what, uint32_t dg, uint32_t rpl, uint32_t rpline, uint64_t n, uint64_t x) {
  if (!c && fails++ < 5)
    std::printf("fail %s dg=%u rpl=%u rpline=%u n_reps=%llu at %llu\n", what, dg, rpl, rpline,
                (unsigned long long)n, (unsigned long long)x);
}

// rows of the vectors: whole lines for packed layouts, rpline per
// representative otherwise
uint64_t total_rows(uint32_t rpl, uint32_t rpline, uint64_t n) {
  return rpl > 1 ? (n + rpl - 1) / rpl * rpline : n * rpline;
}

void shape(uint32_t dg, uint32_t rpl, uint32_t rpline, uint64_t n) {
  using namespace ftlm::dev;
  const PadMap m{dg, rpl, rpline, n};
  const uint64_t rows = total_rows(rpl, rpline, n);
  std::vector<int> hit(rows, 0);
  uint64_t prev_end = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t r0 = padded_row(dg, rpl, rpline, i);
    // representatives in order, disjoint, inside the vectors
    check(r0 >= prev_end, "order", dg, rpl, rpline, n, i);
    check(r0 + dg <= rows, "inside", dg, rpl, rpline, n, i);
    prev_end = r0 + dg;
    // a packed representative never straddles its line
    if (rpl > 1) check(r0 / rpline == (r0 + dg - 1) / rpline, "line", dg, rpl, rpline, n, i);
    for (uint32_t k = 0; k < dg; ++k) {
      uint64_t ii = ~0ull;
      int kk = -1;
      const bool live = padded_rep_of(m, r0 + k, ii, kk);
      check(live && ii == i && kk == (int)k, "inverse", dg, rpl, rpline, n, r0 + k);
      if (r0 + k < rows) hit[r0 + k] = 1;
    }
  }
  // every other row is a gap: outside any slot (packed) or a row k >= d_Gamma
  // of its representative (aligned), which the kernels treat as zero
  for (uint64_t r = 0; r < rows; ++r) {
    if (hit[r]) continue;
    uint64_t ii = 0;
    int kk = 0;
    const bool live = padded_rep_of(m, r, ii, kk);
    check(!live || kk >= (int)dg, "gap", dg, rpl, rpline, n, r);
    if (live) check(padded_row(dg, rpl, rpline, ii) + (uint64_t)kk == r, "gap-inverse", dg, rpl, rpline, n, r);
  }
  // rows past the vectors belong to no representative
  for (uint64_t r = rows; r < rows + 2 * rpline + 2; ++r) {
    uint64_t ii = 0;
    int kk = 0;
    const bool live = padded_rep_of(m, r, ii, kk);
    check(!live || ii >= n || kk >= (int)dg, "past", dg, rpl, rpline, n, r);
  }
  std::printf("shape dg=%u rpl=%u rpline=%u n_reps=%llu rows=%llu\n", dg, rpl, rpline, (unsigned long long)n,
              (unsigned long long)rows);
}

}  // namespace

int main() {
  const uint64_t ns[] = {1, 2, 3, 7, 64, 1000, 1001};
  const uint32_t row_bytes[] = {8, 16, 32, 64};  // nvec x element bytes of one row
  int shapes = 0;
  for (uint32_t dg = 1; dg <= 12; ++dg) {
    for (uint64_t n : ns) {
      shape(dg, 1, dg, n);  // plain padded rows
      ++shapes;
      for (uint32_t rb : row_bytes) {
        uint32_t S = 1;
        while (S < dg) S <<= 1;
        if (S > dg && S * rb <= 128) {  // aligned rows
          shape(dg, 1, S, n);
          ++shapes;
        }
        const uint32_t L = 128 / rb, p = L / dg;
        if (p >= 2 && p * dg < L) {  // packed lines
          shape(dg, p, L, n);
          ++shapes;
        }
      }
    }
  }
  std::printf("shapes %d\nfails %d\n", shapes, fails);
  return fails == 0 ? 0 : 1;
}
