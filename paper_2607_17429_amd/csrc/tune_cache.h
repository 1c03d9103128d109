// Process-wide autotuner cache of the H.V lane layout, and its text file form.
#pragma once

#include <cstdint>
#include <string>

namespace ftlm {

// What a tuned lane layout depends on: the device architecture, the cluster
// (a hash of its bonds, couplings and group elements, and its sizes), the
// kernel's irrep-dimension bucket, the vector count and storage type, the
// H.V mode, the row layout and whether the Lanczos epilogue runs.
struct TuneKey {
  std::string arch;
  uint64_t cluster = 0;
  int N = 0, two_s = 0, G = 0, dgp = 0, nvec = 0, dtype = 0, mode = 0, pad = 0, epi = 0;
  bool operator<(const TuneKey& o) const;
};

int tune_lookup(const TuneKey& k);            // lanes per representative, 0 if not tuned
void tune_store(const TuneKey& k, int lanes);
void tune_clear();
// One line per entry; arch == nullptr: every architecture.  Return the
// number of entries written / taken in.
int tune_save(const char* path, const char* arch);
int tune_load(const char* path, const char* arch);

// FNV-1a over bytes, chained: the cluster hash of a sector.
uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull);

}  // namespace ftlm
