// Whole-cluster FTLM (paper Sections 2.2, 3 and 4): every M >= 0 sector and
// every irrep block (optionally G x Z2 at M = 0), R Lanczos chains per block,
// Ritz data per chain, and the thermal sums of Eqs. (4)-(7), (14) over all of
// them.  Blocks run one after another on one non-blocking stream of the
// library (Lanczos steps replay a captured graph); the sector tables of one M
// are shared by its blocks and freed before the next M.
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ftlm {

namespace {
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
  hipStream_t stream = nullptr;
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
  AllocStreamScope scope(stream);

  // Ritz data of every block (kept until the sums)
  struct BlockRitz {
    int two_M = 0, d = 0, R = 0, ld = 0;
    uint64_t D = 0;
    std::vector<int32_t> n;
    std::vector<double> theta, w;
  };
  std::vector<BlockRitz> all;
  const int Ns2 = cl->N * cl->two_s;  // 2 N s
  std::vector<int> twoMs;
  if (o->all_M)
    for (int m = Ns2 % 2; m <= Ns2; m += 2) twoMs.push_back(m);
  else
    twoMs.push_back(o->two_M);
  const int per_run = o->chains_per_run == 0 ? o->R : std::min(o->chains_per_run, o->R);
  for (int two_M : twoMs) {
    auto tb = clk::now();
    ftlm_opts so{};
    so.hv_mode = FTLM_HV_AUTO;
    so.spin_flip = (o->spin_flip && two_M == 0) ? 1 : 0;
    std::shared_ptr<Sector> sec = build_sector(cl, G, two_M, &so);
    S.seconds_build += secs(tb, clk::now());
    if (sec->D_M == 0) continue;
    S.sectors += 1;
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
      br.theta.assign((size_t)o->R * o->steps, 0.0);
      br.w.assign((size_t)o->R * o->steps, 0.0);
      std::vector<double> alpha((size_t)o->R * o->steps), beta((size_t)o->R * o->steps);
      auto tl = clk::now();
      // chains in groups of per_run (all R at once unless a single-vector
      // comparison asks otherwise); chain r keeps its key (seed, 2M, irrep, row, r)
      for (int r0 = 0; r0 < o->R; r0 += per_run) {
        const int rr = std::min(per_run, o->R - r0);
        LanczosRun L(*blk, rr, o->steps, o->seed, o->storage, o->dist);
        L.first_chain = r0;
        L.allocate();
        L.enqueue(stream);
        L.download(stream, alpha.data() + (size_t)r0 * o->steps, beta.data() + (size_t)r0 * o->steps,
                   br.n.data() + r0);
        FTLM_HIP(hipStreamSynchronize(stream));
      }
      S.seconds_lanczos += secs(tl, clk::now());
      auto tt = clk::now();
      for (int r = 0; r < o->R; ++r) {
        const int n = br.n[r];
        S.products += (uint64_t)n;
        S.work += (uint64_t)n * blk->D;
        if (n > 0)
          tridiag_ritz(alpha.data() + (size_t)r * o->steps, beta.data() + (size_t)r * o->steps, n,
                       br.theta.data() + (size_t)r * o->steps, br.w.data() + (size_t)r * o->steps);
      }
      S.seconds_thermo += secs(tt, clk::now());
      all.push_back(std::move(br));
    }
  }
  auto tt = clk::now();
  std::vector<ftlm_ritz> rz;
  for (auto& b : all)
    rz.push_back(ftlm_ritz{b.two_M, b.d, b.D, b.R, b.ld, b.n.data(), b.theta.data(), b.w.data()});
  if (nT > 0) observables(rz.data(), (int)rz.size(), T, nT, o->g, E, C, chi, logZ);
  S.seconds_thermo += secs(tt, clk::now());
  S.seconds_total = secs(t0, clk::now());
  if (st) *st = S;
}

}  // namespace ftlm
