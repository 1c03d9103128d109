// Autotuner cache (tune_cache.h): a mutex-guarded map in the process, and a
// text file of "arch cluster N two_s G dgp nvec dtype mode pad epi lanes"
// lines so that a tuned layout survives the process.  Host only.
#include "tune_cache.h"

#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#include "common.h"

namespace ftlm {

namespace {
std::mutex g_mu;
std::map<TuneKey, int> g_tune;
}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
  return std::tie(arch, cluster, N, two_s, G, dgp, nvec, dtype, mode, pad, epi) <
         std::tie(o.arch, o.cluster, o.N, o.two_s, o.G, o.dgp, o.nvec, o.dtype, o.mode, o.pad, o.epi);
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

int tune_lookup(const TuneKey& k) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tune.find(k);
  return it == g_tune.end() ? 0 : it->second;
}

void tune_store(const TuneKey& k, int lanes) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune[k] = lanes;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune.clear();
}

int tune_save(const char* path, const char* arch) {
  if (!path) fail(FTLM_ERR_INVALID_ARG, "null path");
  std::ostringstream os;
  int n = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_tune) {
      const TuneKey& k = kv.first;
      if (arch && k.arch != arch) continue;
      os << k.arch << ' ' << k.cluster << ' ' << k.N << ' ' << k.two_s << ' ' << k.G << ' ' << k.dgp << ' '
         << k.nvec << ' ' << k.dtype << ' ' << k.mode << ' ' << k.pad << ' ' << k.epi << ' ' << kv.second << '\n';
      ++n;
    }
  }
  std::ofstream f(path, std::ios::trunc);
  if (!f) fail(FTLM_ERR_INVALID_ARG, std::string("cannot write ") + path);
  f << os.str();
  if (!f) fail(FTLM_ERR_INVALID_ARG, std::string("write failed: ") + path);
  return n;
}

int tune_load(const char* path, const char* arch) {
  if (!path) fail(FTLM_ERR_INVALID_ARG, "null path");
  std::ifstream f(path);
  if (!f) fail(FTLM_ERR_INVALID_ARG, std::string("cannot read ") + path);
  std::string line;
  int n = 0, lineno = 0;
  std::map<TuneKey, int> got;
  while (std::getline(f, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    TuneKey k;
    int lanes = 0;
    if (!(is >> k.arch >> k.cluster >> k.N >> k.two_s >> k.G >> k.dgp >> k.nvec >> k.dtype >> k.mode >> k.pad >> k.epi >>
          lanes))
      fail(FTLM_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(lineno) + ": malformed autotuner entry");
    if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)))
      fail(FTLM_ERR_INVALID_ARG, std::string(path) + ":" + std::to_string(lineno) + ": lanes must be a power of two <= 64");
    if (arch && k.arch != arch) continue;
    got[k] = lanes;
    ++n;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : got) g_tune[kv.first] = kv.second;
  return n;
}

}  // namespace ftlm
