// Whole-cluster FTLM (paper Sections 2.2, 3 and 4): every M >= 0 sector and
// every irrep block (optionally G x Z2 at M = 0), R Lanczos chains per block,
// Ritz data per chain, and the thermal sums of Eqs. (4)-(7), (14) over all of
// them.  Sectors of few representatives go to the fused small-block kernel
// (one workgroup per block job, all such jobs in one batch launched on a
// second stream); the blocks of larger sectors run one after another with the
// per-step kernels (Lanczos steps replay a captured graph), overlapping the
// batch.  The sector tables of one large M are freed before the next M.
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ftlm {

namespace {
// fused kernel: largest representative rounds per lane group and step for
// which a sector's blocks go to the fused batch under FTLM_ENGINE_AUTO
constexpr uint64_t kFusedMaxRounds = 8;

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
  if (!G->all_real) fail(FTLM_ERR_COMPLEX_IRREP_UNSUPPORTED, "group has irreps that are not of real type");
  // per-step kernels on `stream`; batches of fused small-block jobs on `wstream`
  hipStream_t stream = nullptr, wstream = nullptr;
  FTLM_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    }
  } guard{stream};
  FTLM_HIP(hipStreamCreateWithFlags(&wstream, hipStreamNonBlocking));
  StreamGuard wguard{wstream};
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
  std::vector<int> twoMs;
  if (o->all_M)
    for (int m = Ns2 % 2; m <= Ns2; m += 2) twoMs.push_back(m);
  else
    twoMs.push_back(o->two_M);
  const int per_run = o->chains_per_run == 0 ? o->R : std::min(o->chains_per_run, o->R);
  const uint64_t max_rounds = o->fused_max_rounds > 0 ? (uint64_t)o->fused_max_rounds : kFusedMaxRounds;

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
      br.d = blk->dg;
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
        auto tl = clk::now();
        for (int r0 = 0; r0 < o->R; r0 += per_run) {
          const int rr = std::min(per_run, o->R - r0);
          LanczosRun L(*blk, rr, o->steps, o->seed, o->storage, o->dist);
          L.first_chain = r0;
          L.allocate();
          L.enqueue(stream);
          L.download(stream, br.alpha.data() + (size_t)r0 * o->steps, br.beta.data() + (size_t)r0 * o->steps,
                     br.n.data() + r0);
          FTLM_HIP(hipStreamSynchronize(stream));
        }
        S.seconds_lanczos += secs(tl, clk::now());
      }
      all.push_back(std::move(br));
    }
    if (!fused_sector) finish_inflight();
    if (pending_bytes > pending_limit) launch_pending();
  }
  launch_pending();
  finish_inflight();

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
