// extern "C" entry points of ftlm.h that run on the host only: groups and
// irreps, tridiagonal Ritz data, the thermal sums (FTLM and KPM), and the
// thread-local last-error message.  These and group.cpp / thermo.cpp make up
// the host-only part of the library, which is also built on its own with the
// address and undefined-behaviour sanitizers (build.py).
#include <cstring>
#include <memory>
#include <string>

#include "capi_guard.h"
#include "group.h"
#include "internal.h"
#include "tune_cache.h"

namespace ftlm {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace ftlm

using namespace ftlm;

extern "C" {

const char* ftlm_last_error(void) { return g_last_error.c_str(); }

int ftlm_group_create(int32_t N, const int32_t* gens, int32_t ngens, ftlm_group** out) {
  return guarded([&] {
    if (!out) fail(FTLM_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    auto G = std::make_shared<Group>(build_group(N, gens, ngens));
    compute_irreps(*G);
    *out = new ftlm_group{G};
  });
}

int ftlm_group_info(const ftlm_group* g, int32_t* order, int32_t* n_irreps, int32_t* n_classes, int32_t* N) {
  return guarded([&] {
    if (!g) fail(FTLM_ERR_INVALID_ARG, "null group");
    if (order) *order = g->G->order;
    if (n_irreps) *n_irreps = (int32_t)g->G->irreps.size();
    if (n_classes) *n_classes = (int32_t)g->G->classes.size();
    if (N) *N = g->G->N;
  });
}

int ftlm_group_elements(const ftlm_group* g, int32_t* perms) {
  return guarded([&] {
    if (!g || !perms) fail(FTLM_ERR_INVALID_ARG, "null argument");
    std::memcpy(perms, g->G->perms.data(), g->G->perms.size() * sizeof(int32_t));
  });
}

int ftlm_group_irreps(const ftlm_group* g, int32_t* dims, int32_t* indicators, int32_t* weights, double* chars,
                      int32_t* class_of, double* max_residual) {
  return guarded([&] {
    if (!g) fail(FTLM_ERR_INVALID_ARG, "null group");
    const Group& G = *g->G;
    const size_t nc = G.classes.size();
    for (size_t i = 0; i < G.irreps.size(); ++i) {
      if (dims) dims[i] = G.irreps[i].dim;
      if (indicators) indicators[i] = G.irreps[i].indicator;
      if (weights) weights[i] = G.irreps[i].weight();
      if (chars)
        for (size_t c = 0; c < nc; ++c) chars[i * nc + c] = G.irreps[i].chars[c];
    }
    if (class_of) std::memcpy(class_of, G.class_of.data(), G.class_of.size() * sizeof(int32_t));
    if (max_residual) *max_residual = G.max_residual;
  });
}

int ftlm_group_rho(const ftlm_group* g, int32_t irrep, double* rho) {
  return guarded([&] {
    if (!g || !rho) fail(FTLM_ERR_INVALID_ARG, "null argument");
    if (irrep < 0 || irrep >= (int)g->G->irreps.size()) fail(FTLM_ERR_IRREP_OUT_OF_RANGE, "irrep index out of range");
    const auto& r = g->G->irreps[irrep].rho;
    std::memcpy(rho, r.data(), r.size() * sizeof(double));
  });
}

void ftlm_group_free(ftlm_group* g) { delete g; }

int ftlm_kpm_observables(const ftlm_kpm_block* blocks, int32_t nblocks, const double* T, int32_t nT, double g,
                         int32_t n_nodes, double* E, double* C, double* chi, double* logZ) {
  return guarded([&] {
    if (nblocks <= 0 || !blocks || nT < 0 || (nT > 0 && !T) || n_nodes < 0) fail(FTLM_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < nT; ++i)
      if (!(T[i] > 0)) fail(FTLM_ERR_INVALID_ARG, "temperatures must be positive");
    kpm_observables(blocks, nblocks, T, nT, g, n_nodes, E, C, chi, logZ);
  });
}

int ftlm_tridiag_ritz(const double* alpha, const double* beta, int32_t n, double* theta, double* weight) {
  return guarded([&] {
    if (n < 0 || n > 4096) fail(FTLM_ERR_INVALID_ARG, "n must be in 0..4096");
    if (n > 0 && (!alpha || !theta || !weight || (n > 1 && !beta))) fail(FTLM_ERR_INVALID_ARG, "null argument");
    tridiag_ritz(alpha, beta, n, theta, weight);
  });
}

int ftlm_observables(const ftlm_ritz* blocks, int32_t nblocks, const double* T, int32_t nT, double g, double* E,
                     double* C, double* chi, double* logZ) {
  return guarded([&] {
    if (nblocks <= 0 || !blocks || nT < 0 || (nT > 0 && !T)) fail(FTLM_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < nT; ++i)
      if (!(T[i] > 0)) fail(FTLM_ERR_INVALID_ARG, "temperatures must be positive");
    observables(blocks, nblocks, T, nT, g, E, C, chi, logZ);
  });
}

int ftlm_autotune_save(const char* path, const char* arch, int32_t* n_saved) {
  return guarded([&] {
    const int n = tune_save(path, arch);
    if (n_saved) *n_saved = n;
  });
}

int ftlm_autotune_load(const char* path, const char* arch, int32_t* n_loaded) {
  return guarded([&] {
    const int n = tune_load(path, arch);
    if (n_loaded) *n_loaded = n;
  });
}

int ftlm_autotune_clear(void) {
  return guarded([&] { tune_clear(); });
}

}  // extern "C"
