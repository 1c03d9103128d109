// Whole-cluster FTLM (paper Sections 2.2, 3 and 4): every M >= 0 sector and
// every irrep block (optionally G x Z2 at M = 0), R Lanczos chains per block,
// Ritz data per chain, and the thermal sums of Eqs. (4)-(7), (14) over all of
// them.  Sectors run from the largest 2M down.  Sectors of few
// representatives go to the fused small-block kernel (one workgroup per block
// job, all such jobs in one batch on a stream of their own); the blocks of
// larger sectors run with the per-step kernels (Lanczos steps replay a
// captured graph) over two worker streams, so blocks, the batch and the next
// sector's build overlap.  Runs in flight keep their sector's tables alive
// until they are read back, which happens when their memory passes a quarter
// of the free device memory, and at the end.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ftlm {

namespace {
// worker streams for the per-step blocks; with the build stream and the
// batch stream they fill HIP's default four hardware queues, so the build
// never waits behind a worker's queued steps (measured on the dodecahedron
// campaign: four workers sharing queues with the build made it slower)
constexpr int kStepStreams = 2;

double secs(std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}
}  // namespace

void run_campaign(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, const ftlm_campaign_opts* o,
                  const double* T, int nT, double* E, double* C, double* chi, double* logZ,
                  ftlm_campaign_stats* st) {
  if (!cl || !o || (nT > 0 && !T)) fail(FTLM_ERR_INVALID_ARG, "null argument");
  if (o->R <= 0 || o->steps <= 0) fail(FTLM_ERR_INVALID_ARG, "R and steps must be positive");
  if (o->chains_per_run < 0) fail(FTLM_ERR_INVALID_ARG, "chains_per_run must be >= 0");
  using clk = std::chrono::steady_clock;
  ftlm_campaign_stats S{};
  auto t0 = clk::now();
  auto G = std::make_shared<Group>(build_group(cl->N, gens, ngens));
  compute_irreps(*G);
  if (!G->all_real) fail(FTLM_ERR_COMPLEX_IRREP_UNSUPPORTED, "the group's real irreps are incomplete");
  // sector and block builds on `stream`, per-step Lanczos runs on the worker
  // streams, batches of fused small-block jobs on `wstream`
  hipStream_t stream = nullptr, wstream = nullptr;
  FTLM_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s = nullptr;
    ~StreamGuard() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    }
  } guard{stream};
  FTLM_HIP(hipStreamCreateWithFlags(&wstream, hipStreamNonBlocking));
  StreamGuard wguard{wstream};
  hipStream_t sstreams[kStepStreams] = {};
  StreamGuard sguard[kStepStreams];
  for (int k = 0; k < kStepStreams; ++k) {
    FTLM_HIP(hipStreamCreateWithFlags(&sstreams[k], hipStreamNonBlocking));
    sguard[k].s = sstreams[k];
  }
  AllocStreamScope scope(stream);

  // Ritz data of every block (kept until the sums)
  struct BlockRitz {
    int two_M = 0, d = 0, R = 0, ld = 0;
    uint64_t D = 0;
    std::vector<int32_t> n;
    std::vector<double> alpha, beta, theta, w;
  };
  std::vector<BlockRitz> all;
  const int Ns2 = cl->N * cl->two_s;  // 2 N s
  // largest |M| first: the small sectors fill the fused batch, which then
  // runs while the large sectors' blocks go through the per-step kernels
  std::vector<int> twoMs;
  if (o->all_M)
    for (int m = Ns2; m >= Ns2 % 2; m -= 2) twoMs.push_back(m);
  else
    twoMs.push_back(o->two_M);
  const int per_run = o->chains_per_run == 0 ? o->R : std::min(o->chains_per_run, o->R);
  const uint64_t max_rounds = o->fused_max_rounds > 0 ? (uint64_t)o->fused_max_rounds : kWgAutoMaxRounds;

  // Fused jobs wait in `pending` (their blocks kept alive) and go out as one
  // batch when a sector of large blocks starts, so the two streams overlap,
  // when they hold much memory, or at the end.
  std::vector<WgTask> pending;
  std::vector<std::unique_ptr<Block>> pending_blocks, inflight_blocks;
  std::unique_ptr<WgBatch> inflight;
  int64_t pending_bytes = 0;
  const void* pending_sector = nullptr;
  auto finish_inflight = [&] {
    if (!inflight) return;
    auto tl = clk::now();
    inflight->finish();
    inflight.reset();
    inflight_blocks.clear();
    S.seconds_lanczos += secs(tl, clk::now());
  };
  auto launch_pending = [&] {
    if (pending.empty()) return;
    finish_inflight();
    auto tl = clk::now();
    inflight = std::make_unique<WgBatch>(std::move(pending), wstream);
    inflight_blocks = std::move(pending_blocks);
    pending.clear();
    pending_blocks.clear();
    pending_bytes = 0;
    pending_sector = nullptr;
    S.seconds_lanczos += secs(tl, clk::now());
  };
  size_t free_b = 0, total_b = 0;
  FTLM_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t pending_limit = (int64_t)(free_b / 8);

  // Per-step runs in flight on the worker streams (their blocks kept alive).
  struct StepJob {
    std::unique_ptr<Block> blk;
    std::vector<std::pair<std::unique_ptr<LanczosRun>, int>> runs;  // run, first chain
    size_t ritz = 0;
    int stream = 0;
  };
  std::vector<StepJob> step_jobs;
  struct SyncOnExit {  // an error leaves no run of step_jobs executing when they are destroyed
    hipStream_t* s;
    ~SyncOnExit() {
      for (int k = 0; k < kStepStreams; ++k) (void)hipStreamSynchronize(s[k]);
    }
  } step_sync{sstreams};
  size_t step_bytes = 0;
  const void* step_sector = nullptr;
  const size_t step_limit = free_b / 4;
  int next_stream = 0;
  auto drain_steps = [&] {
    if (step_jobs.empty()) return;
    auto tl = clk::now();
    for (auto& j : step_jobs) {
      BlockRitz& br = all[j.ritz];
      for (auto& [L, r0] : j.runs)
        L->download(sstreams[j.stream], br.alpha.data() + (size_t)r0 * o->steps,
                    br.beta.data() + (size_t)r0 * o->steps, br.n.data() + r0);
    }
    for (int k = 0; k < kStepStreams; ++k) FTLM_HIP(hipStreamSynchronize(sstreams[k]));
    step_jobs.clear();
    step_bytes = 0;
    step_sector = nullptr;
    S.seconds_lanczos += secs(tl, clk::now());
  };

  for (int two_M : twoMs) {
    auto tb = clk::now();
    ftlm_opts so{};
    so.hv_mode = FTLM_HV_AUTO;
    so.spin_flip = (o->spin_flip && two_M == 0) ? 1 : 0;
    std::shared_ptr<Sector> sec = build_sector(cl, G, two_M, &so);
    S.seconds_build += secs(tb, clk::now());
    if (sec->D_M == 0) continue;
    S.sectors += 1;
    // every block of a sector spans the sector's representatives, so the
    // fused kernel's serial length is a property of the sector
    const bool fused_sector = o->engine == FTLM_ENGINE_FUSED ||
                              (o->engine == FTLM_ENGINE_AUTO && wg_rounds(sec->n_reps, per_run) <= max_rounds);
    if (!fused_sector) launch_pending();
    const int nirr = (int)G->irreps.size() * (sec->zflip ? 2 : 1);
    for (int irrep = 0; irrep < nirr; ++irrep) {
      tb = clk::now();
      std::unique_ptr<Block> blk = build_block(sec, irrep, 0, nullptr);
      S.seconds_build += secs(tb, clk::now());
      if (blk->D == 0) {
        S.empty_blocks += 1;
        continue;
      }
      S.blocks += 1;
      S.rows += blk->D;
      BlockRitz br;
      br.two_M = two_M;
      br.d = blk->weight;  // trace weight: d_Gamma, also for a realified complex pair
      br.D = blk->D;
      br.R = o->R;
      br.ld = o->steps;
      br.n.assign(o->R, 0);
      br.alpha.assign((size_t)o->R * o->steps, 0.0);
      br.beta.assign((size_t)o->R * o->steps, 0.0);
      // chains in groups of per_run (all R at once unless a single-vector
      // comparison asks otherwise); chain r keeps its key (seed, 2M, irrep, row, r)
      if (fused_sector && o->engine != FTLM_ENGINE_STEPS && wg_supported(*blk, per_run, o->storage)) {
        S.fused_blocks += 1;
        for (int r0 = 0; r0 < o->R; r0 += per_run) {
          const int rr = std::min(per_run, o->R - r0);
          pending.push_back(WgTask{blk.get(), rr, o->steps, o->storage, o->dist, r0, o->seed,
                                   br.alpha.data() + (size_t)r0 * o->steps, br.beta.data() + (size_t)r0 * o->steps,
                                   br.n.data() + r0});
        }
        pending_bytes += 2 * (int64_t)blk->D * o->R * (o->storage == FTLM_F64 ? 8 : 4) +
                         (pending_sector == sec.get() ? blk->device_bytes() - sec->device_bytes()
                                                      : blk->device_bytes());
        pending_sector = sec.get();
        pending_blocks.push_back(std::move(blk));
      } else {
        // per-step kernels on the next worker stream; results are read back
        // when the sector ends (or memory runs short), so the blocks of a
        // sector overlap on the device
        auto tl = clk::now();
        // vectors of the runs, the block's tables and (once) its sector's tables
        const size_t need = LanczosRun::estimate_bytes(*blk, per_run, o->steps, o->storage) *
                                (size_t)((o->R + per_run - 1) / per_run) +
                            (size_t)(blk->device_bytes() - sec->device_bytes()) +
                            (step_sector == sec.get() ? 0 : (size_t)sec->device_bytes());
        if (!step_jobs.empty() && step_bytes + need > step_limit) drain_steps();
        const int k = next_stream++ % kStepStreams;
        StepJob job;
        for (int r0 = 0; r0 < o->R; r0 += per_run) {
          const int rr = std::min(per_run, o->R - r0);
          auto L = std::make_unique<LanczosRun>(*blk, rr, o->steps, o->seed, o->storage, o->dist);
          L->first_chain = r0;
          {
            AllocStreamScope run_scope(sstreams[k]);  // buffers ordered on the stream that uses them
            L->allocate();
          }
          L->enqueue(sstreams[k]);
          job.runs.push_back({std::move(L), r0});
        }
        job.stream = k;
        job.ritz = all.size();
        job.blk = std::move(blk);
        step_jobs.push_back(std::move(job));
        step_bytes += need;
        step_sector = sec.get();
        S.seconds_lanczos += secs(tl, clk::now());
      }
      all.push_back(std::move(br));
    }
    // runs stay in flight across sectors (the next sector builds meanwhile)
    // until their memory passes the limit
    if (step_bytes > step_limit) drain_steps();
    if (pending_bytes > pending_limit) launch_pending();
  }
  launch_pending();
  drain_steps();
  finish_inflight();
  // blocks in ascending 2M (and irrep) order for the sums
  std::stable_sort(all.begin(), all.end(), [](const BlockRitz& a, const BlockRitz& b) { return a.two_M < b.two_M; });

  auto tt = clk::now();
  for (auto& br : all) {
    for (int r = 0; r < br.R; ++r) {
      const int n = br.n[r];
      S.products += (uint64_t)n;
      S.work += (uint64_t)n * br.D;
    }
  }
  // Ritz data of every chain (independent problems, spread over host threads)
  std::vector<std::pair<size_t, int>> chains;
  for (size_t b = 0; b < all.size(); ++b) {
    all[b].theta.assign((size_t)all[b].R * all[b].ld, 0.0);
    all[b].w.assign((size_t)all[b].R * all[b].ld, 0.0);
    for (int r = 0; r < all[b].R; ++r)
      if (all[b].n[r] > 0) chains.push_back({b, r});
  }
  parallel_for((int64_t)chains.size(), 16, [&](int64_t i) {
    BlockRitz& br = all[chains[i].first];
    const size_t o = (size_t)chains[i].second * br.ld;
    tridiag_ritz(br.alpha.data() + o, br.beta.data() + o, br.n[chains[i].second], br.theta.data() + o,
                 br.w.data() + o);
  });
  S.seconds_thermo += secs(tt, clk::now());
  tt = clk::now();
  std::vector<ftlm_ritz> rz;
  for (auto& b : all)
    rz.push_back(ftlm_ritz{b.two_M, b.d, b.D, b.R, b.ld, b.n.data(), b.theta.data(), b.w.data()});
  if (nT > 0) observables(rz.data(), (int)rz.size(), T, nT, o->g, E, C, chi, logZ);
  S.seconds_thermo += secs(tt, clk::now());
  S.seconds_total = secs(t0, clk::now());
  if (st) *st = S;
}

}  // namespace ftlm
