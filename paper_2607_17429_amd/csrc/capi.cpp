// extern "C" entry points of ftlm.h that touch the device: argument checks
// and exception -> status translation (the host-only entry points, the
// guard and the thread-local last-error message are in capi_host.cpp).
#include <algorithm>
#include <cstring>
#include <string>

#include "capi_guard.h"
#include "internal.h"

using namespace ftlm;

extern "C" {

int ftlm_sector_create(const ftlm_cluster* cl, const ftlm_group* g, int32_t two_M, const ftlm_opts* opts,
                       ftlm_sector** out) {
  return guarded([&] {
    if (!out || !g) fail(FTLM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto s = build_sector(cl, g->G, two_M, opts);
    *out = new ftlm_sector{s};
  });
}

int ftlm_sector_info_get(const ftlm_sector* s, ftlm_sector_info* info) {
  return guarded([&] {
    if (!s || !info) fail(FTLM_ERR_INVALID_ARG, "null argument");
    const Sector& S = *s->s;
    info->D_M = S.D_M;
    info->n_reps = S.n_reps;
    info->n_entries = S.hv_mode == FTLM_HV_ENTRIES ? S.n_entries : 0;
    info->n_stab = S.n_stab;
    info->label_bits = S.bits;
    info->device_bytes = S.device_bytes();
  });
}

int ftlm_sector_export(const ftlm_sector* s, uint64_t* reps, uint16_t* stab_id, int32_t* stab_size) {
  return guarded([&] {
    if (!s) fail(FTLM_ERR_INVALID_ARG, "null sector");
    const Sector& S = *s->s;
    if (reps && S.n_reps) {
      auto v = sector_export_labels(S);
      std::memcpy(reps, v.data(), v.size() * 8);
    }
    if (stab_id && S.n_reps) {
      auto v = S.d_stab_id.download();
      std::memcpy(stab_id, v.data(), v.size() * 2);
    }
    if (stab_size)
      for (int i = 0; i < S.n_stab; ++i) stab_size[i] = S.stab_size[i];
  });
}

int ftlm_sector_canonicalize(const ftlm_sector* s, const uint64_t* labels, int64_t n, uint64_t* rep, int32_t* h,
                             int64_t* index, void* stream) {
  return guarded([&] {
    if (!s) fail(FTLM_ERR_INVALID_ARG, "null sector");
    sector_canonicalize(*s->s, labels, n, rep, h, index, (hipStream_t)stream);
  });
}

void ftlm_sector_free(ftlm_sector* s) { delete s; }

int ftlm_block_create(ftlm_sector* s, int32_t irrep, int32_t row, const ftlm_opts* opts, ftlm_block** out) {
  return guarded([&] {
    if (!s || !out) fail(FTLM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto b = build_block(s->s, irrep, row, opts);
    *out = new ftlm_block{std::move(b)};
  });
}

int ftlm_build_block(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, int32_t two_M, int32_t irrep,
                     int32_t row, const ftlm_opts* opts, ftlm_block** out) {
  return guarded([&] {
    if (!cl || !out) fail(FTLM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto G = std::make_shared<Group>(build_group(cl->N, gens, ngens));
    if (!(opts && opts->user_rho)) compute_irreps(*G);
    auto sec = build_sector(cl, G, two_M, opts);
    auto b = build_block(sec, irrep, row, opts);
    b->own_group = G;
    *out = new ftlm_block{std::move(b)};
  });
}

int ftlm_block_info_get(const ftlm_block* b, ftlm_block_info* info) {
  return guarded([&] {
    if (!b || !info) fail(FTLM_ERR_INVALID_ARG, "null argument");
    const Block& B = *b->b;
    info->D_M = B.sec->D_M;
    info->n_reps = B.sec->n_reps;
    info->n_active = B.n_active;
    info->D = B.D;
    info->d_gamma = B.dg;
    info->group_order = B.sec->gorder;
    info->two_M = B.sec->two_M;
    info->irrep = B.irrep;
    info->row = B.row;
    info->hv_mode = B.sec->hv_mode;
    info->device_bytes = B.device_bytes();
    info->trace_weight = B.weight;
    info->reserved = 0;
  });
}

int ftlm_block_export(const ftlm_block* b, uint64_t* reps, uint16_t* stab_id, uint8_t* n_gamma, double* norms,
                      uint64_t* offsets) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    const Block& B = *b->b;
    const Sector& S = *B.sec;
    if (!S.n_reps) return;
    if (reps) {
      auto v = sector_export_labels(S);
      std::memcpy(reps, v.data(), v.size() * 8);
    }
    std::vector<uint16_t> sid = S.d_stab_id.download();
    if (stab_id) std::memcpy(stab_id, sid.data(), sid.size() * 2);
    if (n_gamma)
      for (size_t i = 0; i < sid.size(); ++i) n_gamma[i] = B.n_stab[sid[i]];
    if (norms)
      for (size_t i = 0; i < sid.size(); ++i) norms[i] = B.L_stab[sid[i]];
    if (offsets) {
      if (B.D == 0) {  // an empty block keeps no metadata: every offset is 0
        std::fill(offsets, offsets + S.n_reps, (uint64_t)0);
      } else {
        auto m = B.d_meta.download();
        for (size_t i = 0; i < m.size(); ++i) offsets[i] = m[i] & ((1ull << 48) - 1);
      }
    }
  });
}

int ftlm_block_hv_stats(const ftlm_block* b, ftlm_hv_stats* stats) {
  return guarded([&] {
    if (!b || !stats) fail(FTLM_ERR_INVALID_ARG, "null argument");
    block_hv_stats(*b->b, stats);
  });
}

int ftlm_apply_H(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld, int32_t dtype, void* stream) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    if (X == Y && X) fail(FTLM_ERR_INVALID_ARG, "X and Y must not overlap");
    apply_hv(*b->b, X, Y, nvec, ld, dtype, (hipStream_t)stream);
  });
}

int ftlm_apply_H_ex(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld, int32_t dtype,
                    ftlm_hv_opts* opts, void* stream) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    if (X == Y && X) fail(FTLM_ERR_INVALID_ARG, "X and Y must not overlap");
    const Block& B = *b->b;
    const HvExPlan p = plan_hv_ex(B, nvec, ld, dtype, opts);
    hipStream_t st = (hipStream_t)stream;
    AllocStreamScope scope(st ? st : tl_alloc_stream);  // stream-ordered scratch: no device-wide sync on free
    DevBuf<double> partials;
    if (p.epi && p.ng > 0) partials.alloc((size_t)p.ng * nvec);
    apply_hv_ex(B, X, Y, nvec, ld, dtype, opts, p, partials.p, st);
    if (opts) {
      opts->lanes_used = p.gl;
      opts->adjacent_columns = p.adjacent ? 1 : 0;
    }
  });
}

int ftlm_device_arch(char* buf, int32_t len) {
  return guarded([&] {
    if (!buf || len <= 0) fail(FTLM_ERR_INVALID_ARG, "null or empty buffer");
    const std::string a = device_arch();
    if ((int32_t)a.size() >= len) fail(FTLM_ERR_INVALID_ARG, "buffer too small for the architecture name");
    std::memcpy(buf, a.c_str(), a.size() + 1);
  });
}

int ftlm_block_autotune(ftlm_block* b, int32_t nvec, int32_t dtype, void* stream, int32_t* best_lanes,
                        double* best_ms, int32_t* tried, double* tried_ms, int32_t* n_tried) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    if (nvec <= 0 || nvec > 4096) fail(FTLM_ERR_INVALID_ARG, "nvec must be in 1..4096");
    if (dtype != FTLM_F64 && dtype != FTLM_F32 && dtype != FTLM_F16) fail(FTLM_ERR_INVALID_ARG, "bad dtype");
    const Block& B = *b->b;
    // the launch of ftlm_run and ftlm_kpm (their row layout, Lanczos epilogue),
    // whose times are reported, then the plain launch of ftlm_apply_H
    const int64_t elem = dtype == FTLM_F64 ? 8 : dtype == FTLM_F32 ? 4 : 2;
    auto res = autotune_hv(B, nvec, dtype, (hipStream_t)stream, 5, run_layout(B, nvec * elem), true);
    (void)autotune_hv(B, nvec, dtype, (hipStream_t)stream, 5, VecLayout{}, false);
    int bi = -1;
    for (size_t i = 0; i < res.size(); ++i)
      if (bi < 0 || res[i].second < res[bi].second) bi = (int)i;
    if (best_lanes) *best_lanes = bi >= 0 ? res[bi].first : 0;
    if (best_ms) *best_ms = bi >= 0 ? res[bi].second : 0.0;
    const int n = (int)std::min<size_t>(res.size(), 8);
    for (int i = 0; i < n; ++i) {
      if (tried) tried[i] = res[i].first;
      if (tried_ms) tried_ms[i] = res[i].second;
    }
    if (n_tried) *n_tried = n;
  });
}

int ftlm_run(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist, double* alpha,
             double* beta, int32_t* nsteps, void* stream) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    run_lanczos(*b->b, R, steps, seed, storage, dist, alpha, beta, nsteps, (hipStream_t)stream);
  });
}

int ftlm_run_ex(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist, double* alpha,
                double* beta, int32_t* nsteps, void* stream, ftlm_run_info* info) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    if (info) std::memset(info, 0, sizeof(*info));
    run_lanczos(*b->b, R, steps, seed, storage, dist, alpha, beta, nsteps, (hipStream_t)stream, info);
  });
}

int ftlm_run_begin(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist, void* stream,
                   ftlm_run_state** out) {
  return guarded([&] {
    if (!b || !out) fail(FTLM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto s = std::make_unique<ftlm_run_state>();
    s->block = b->b.get();
    s->st = (hipStream_t)stream;
    AllocStreamScope scope(s->st ? s->st : tl_alloc_stream);
    s->run = std::make_unique<LanczosRun>(*s->block, R, steps, seed, storage, dist);
    s->run->allocate();
    s->run->enqueue_begin(s->st);
    s->next_step = 0;
    *out = s.release();
  });
}

int ftlm_run_advance(ftlm_run_state* s, int32_t n, int32_t* done) {
  return guarded([&] {
    if (!s || n < 0) fail(FTLM_ERR_INVALID_ARG, "bad arguments");
    const int j1 = std::min(s->run->target, s->next_step + n);
    s->run->enqueue_steps(s->st, s->next_step, j1);
    s->next_step = std::max(s->next_step, j1);
    if (done) *done = s->next_step;
  });
}

int ftlm_run_save(ftlm_run_state* s, const char* path) {
  return guarded([&] {
    if (!s) fail(FTLM_ERR_INVALID_ARG, "null run");
    s->run->save(path, s->st, s->next_step);
  });
}

int ftlm_run_load(ftlm_block* b, const char* path, void* stream, ftlm_run_state** out) {
  return guarded([&] {
    if (!b || !out) fail(FTLM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto s = std::make_unique<ftlm_run_state>();
    s->block = b->b.get();
    s->st = (hipStream_t)stream;
    AllocStreamScope scope(s->st ? s->st : tl_alloc_stream);
    s->run = LanczosRun::load(*s->block, path, s->st, s->next_step);
    *out = s.release();
  });
}

int ftlm_run_finish(ftlm_run_state* s, double* alpha, double* beta, int32_t* nsteps) {
  return guarded([&] {
    if (!s) fail(FTLM_ERR_INVALID_ARG, "null run");
    if (!alpha || !beta || !nsteps) fail(FTLM_ERR_INVALID_ARG, "null output");
    s->run->enqueue_steps(s->st, s->next_step, s->run->target);
    s->next_step = std::max(s->next_step, s->run->target);
    s->run->enqueue_end(s->st);
    s->run->download(s->st, alpha, beta, nsteps);
    FTLM_HIP(hipStreamSynchronize(s->st));
  });
}

void ftlm_run_state_free(ftlm_run_state* s) {
  if (!s) return;
  AllocStreamScope scope(s->st ? s->st : tl_alloc_stream);
  s->run.reset();
  delete s;
}

int ftlm_run_fused(const ftlm_fused_job* jobs, int32_t n, void* stream) {
  return guarded([&] {
    if (n < 0 || (n > 0 && !jobs)) fail(FTLM_ERR_INVALID_ARG, "bad job list");
    std::vector<WgTask> tasks;
    for (int32_t i = 0; i < n; ++i) {
      const ftlm_fused_job& j = jobs[i];
      if (!j.block) fail(FTLM_ERR_INVALID_ARG, "null block");
      if (j.R < 1 || j.R > 32 || j.steps <= 0) fail(FTLM_ERR_INVALID_ARG, "need 1 <= R <= 32 and steps > 0");
      if (j.first_chain < 0) fail(FTLM_ERR_INVALID_ARG, "first_chain must be >= 0");
      if (j.block->b->D == 0) {  // empty block: no steps
        if (!j.alpha || !j.beta || !j.nsteps) fail(FTLM_ERR_INVALID_ARG, "null output");
        std::memset(j.alpha, 0, sizeof(double) * (size_t)j.R * j.steps);
        std::memset(j.beta, 0, sizeof(double) * (size_t)j.R * j.steps);
        std::memset(j.nsteps, 0, sizeof(int32_t) * (size_t)j.R);
        continue;
      }
      if (!wg_supported(*j.block->b, j.R, j.storage))
        fail(FTLM_ERR_INVALID_ARG, "job " + std::to_string(i) + " does not fit the fused kernel");
      tasks.push_back(WgTask{j.block->b.get(), j.R, j.steps, j.storage, j.dist, j.first_chain, j.seed, j.alpha,
                             j.beta, j.nsteps});
    }
    WgBatch batch(std::move(tasks), (hipStream_t)stream);
    batch.finish();
  });
}

int ftlm_kpm(ftlm_block* b, int32_t R, int32_t n_moments, uint64_t seed, int32_t storage, int32_t dist,
             double center, double half_width, double* moments, void* stream) {
  return guarded([&] {
    if (!b) fail(FTLM_ERR_INVALID_ARG, "null block");
    run_kpm(*b->b, R, n_moments, seed, storage, dist, center, half_width, moments, (hipStream_t)stream);
  });
}

int ftlm_campaign(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, const ftlm_campaign_opts* opts,
                  const double* T, int32_t nT, double* E, double* C, double* chi, double* logZ,
                  ftlm_campaign_stats* stats) {
  return guarded([&] { run_campaign(cl, gens, ngens, opts, T, nT, E, C, chi, logZ, stats); });
}

void ftlm_block_free(ftlm_block* b) { delete b; }

}  // extern "C"
