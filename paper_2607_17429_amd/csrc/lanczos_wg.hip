// Host side of the fused small-block Lanczos kernel (lanczos_wg.h): which
// blocks it can run, one device arena per batch of block jobs, jobs grouped by
// kernel shape (storage type, irrep dimension bucket, vectors per lane, label
// width) with one launch per group, and the results copied back per job.
#include <cstring>
#include <map>
#include <tuple>

#include "lanczos_wg.h"

namespace ftlm {

using namespace hvk;

namespace {

// lanes per representative: 4 for up to 4 chains (flip entries of a chunk are
// fetched together), else 8 with up to 4 vectors per lane
int wg_lanes(int R) { return R <= 4 ? 4 : 8; }

// dynamic LDS a job may use for its tables and, when they fit, its two
// vectors (the kernel's static LDS takes another ~4.6 KiB of the 64 KiB)
constexpr size_t kWgLdsBytes = 56 * 1024;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t elem_bytes(int storage) { return storage == FTLM_F64 ? 8 : 4; }

struct Shape {
  int dtype, dgp, vpl;
  bool wide;
  bool operator<(const Shape& o) const {
    return std::tie(dtype, dgp, vpl, wide) < std::tie(o.dtype, o.dgp, o.vpl, o.wide);
  }
};

void launch_shape(const Shape& sh, const void* jobs, int n, size_t shm, hipStream_t st) {
  switch (sh.dgp) {
    case 1: wg_launch<1>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 2: wg_launch<2>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 3: wg_launch<3>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 4: wg_launch<4>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 5: wg_launch<5>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 6: wg_launch<6>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 8: wg_launch<8>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    case 12: wg_launch<12>(sh.dtype, sh.vpl, sh.wide, jobs, n, shm, st); break;
    default: fail(FTLM_ERR_DIM_GT_12, "irrep dimension above 12");
  }
}

}  // namespace

bool wg_supported(const Block& b, int R, int storage) {
  if (R < 1 || R > kWgMaxR || b.D == 0 || b.sec->n_reps == 0) return false;
  if (storage != FTLM_F64 && storage != FTLM_F32) return false;
  if (b.sec->hv_mode != FTLM_HV_ENTRIES || b.lanczos_layout == FTLM_LAYOUT_PADDED ||
      b.lanczos_layout == FTLM_LAYOUT_PACKED || b.lanczos_layout == FTLM_LAYOUT_ALIGNED)
    return false;
  if (irrep_dim_bucket(b.dg) < 0) return false;
  LaunchCfg c{};
  HvArgs<double> a{};
  hv_setup(b, R, R, wg_lanes(R), VecLayout{}, nullptr, c, a);
  return c.slds && !c.vg && a.tile_w >= R && c.vpl <= 4;
}

uint64_t wg_rounds(uint64_t n_reps, int R) {
  // workgroups of 512 threads (irrep dimensions up to 6)
  const uint64_t slots = (uint64_t)kWgThreads<1> / (uint64_t)wg_lanes(R);
  return (n_reps + slots - 1) / slots;
}

WgBatch::WgBatch(std::vector<WgTask> t, hipStream_t st_) : tasks(std::move(t)), st(st_) {
  const size_t n = tasks.size();
  if (n == 0) return;
  for (const WgTask& k : tasks)
    if (!k.block || !wg_supported(*k.block, k.R, k.storage) || k.steps <= 0 || !k.alpha || !k.beta || !k.nsteps ||
        (k.dist != FTLM_RADEMACHER && k.dist != FTLM_GAUSSIAN))
      fail(FTLM_ERR_INVALID_ARG, "fused Lanczos: job not supported by the kernel");
  // kernel shape and arguments of every job
  std::vector<Shape> shape(n);
  std::vector<LaunchCfg> cfg(n);
  std::vector<HvArgs<double>> a64(n);
  std::vector<HvArgs<float>> a32(n);
  std::map<Shape, std::vector<size_t>> groups;
  for (size_t i = 0; i < n; ++i) {
    const WgTask& k = tasks[i];
    const Block& b = *k.block;
    if (k.storage == FTLM_F64)
      hv_setup(b, k.R, k.R, wg_lanes(k.R), VecLayout{}, nullptr, cfg[i], a64[i]);
    else
      hv_setup(b, k.R, k.R, wg_lanes(k.R), VecLayout{}, nullptr, cfg[i], a32[i]);
    shape[i] = Shape{k.storage, b.dgp, cfg[i].vpl, b.sec->wide};
    groups[shape[i]].push_back(i);
  }
  // arena: [job arrays][keys] (uploaded) [alpha][beta][n] (downloaded) [q0 q1 per job]
  size_t off = 0;
  std::map<Shape, size_t> goff;
  for (auto& g : groups) {
    goff[g.first] = off;
    const size_t js = g.first.dtype == FTLM_F64 ? sizeof(WgJob<double>) : sizeof(WgJob<float>);
    off = align256(off + js * g.second.size());
  }
  std::vector<size_t> okey(n), oal(n), obe(n), on(n), oq0(n), oq1(n);
  for (size_t i = 0; i < n; ++i) {
    okey[i] = off;
    off += 8 * (size_t)tasks[i].R;
  }
  up_bytes = off = align256(off);
  out_off = off;
  for (size_t i = 0; i < n; ++i) {
    const size_t rs = (size_t)tasks[i].R * tasks[i].steps;
    oal[i] = off;
    off += 8 * rs;
    obe[i] = off;
    off += 8 * rs;
    on[i] = off;
    off += 4 * (size_t)tasks[i].R;
    off = (off + 7) & ~size_t(7);
  }
  out_bytes = off - out_off;
  off = align256(off);
  // vectors in LDS when the tables and both vectors fit, else in the arena
  std::vector<uint32_t> lds_q(n, 0);  // byte offset of q0 in LDS
  std::vector<char> in_lds(n, 0);
  std::vector<size_t> shm(n);
  for (size_t i = 0; i < n; ++i) {
    const size_t qb = (size_t)tasks[i].block->D * tasks[i].R * elem_bytes(tasks[i].storage);
    const size_t oq = (cfg[i].shm + 15) & ~size_t(15);
    shm[i] = cfg[i].shm;
    oq0[i] = oq1[i] = 0;
    if (oq + 2 * qb <= kWgLdsBytes) {
      in_lds[i] = 1;
      lds_q[i] = (uint32_t)oq;
      shm[i] = oq + 2 * qb;
      continue;
    }
    oq0[i] = off;
    off = align256(off + qb);
    oq1[i] = off;
    off = align256(off + qb);
  }
  {
    AllocStreamScope scope(st);
    arena.alloc(off);
  }
  uint8_t* base = arena.p;
  // pinned, so the upload is asynchronous (a pageable copy can block the host)
  FTLM_HIP(hipHostMalloc(&staging.p, up_bytes, hipHostMallocDefault));
  std::memset(staging.p, 0, up_bytes);
  for (auto& g : groups) {
    size_t pos = goff[g.first];
    for (size_t i : g.second) {
      const WgTask& k = tasks[i];
      const Block& b = *k.block;
      auto fill = [&](auto job) {
        job.q0 = (decltype(job.q0))(base + oq0[i]);
        job.q1 = (decltype(job.q1))(base + oq1[i]);
        job.keys = (const uint64_t*)(base + okey[i]);
        job.alpha = (double*)(base + oal[i]);
        job.beta = (double*)(base + obe[i]);
        job.nsteps = (int32_t*)(base + on[i]);
        job.D = b.D;
        job.R = k.R;
        job.steps = k.steps;
        job.target = (int)std::min<uint64_t>((uint64_t)k.steps, b.D);
        job.dist = k.dist;
        job.sigma = 1.0;
        job.lds_vec = in_lds[i];
        job.o_q = lds_q[i];
        if (job.lds_vec) job.q0 = job.q1 = nullptr;
        std::memcpy((uint8_t*)staging.p + pos, &job, sizeof(job));
        pos += sizeof(job);
      };
      if (k.storage == FTLM_F64) {
        WgJob<double> j{};
        j.a = a64[i];
        fill(j);
      } else {
        WgJob<float> j{};
        j.a = a32[i];
        fill(j);
      }
      uint64_t* keys = (uint64_t*)((uint8_t*)staging.p + okey[i]);
      for (int v = 0; v < k.R; ++v)
        keys[v] = chain_key(k.seed, b.sec->two_M, b.irrep, b.row, k.first_chain + v);
    }
  }
  FTLM_HIP(hipMemcpyAsync(base, staging.p, up_bytes, hipMemcpyHostToDevice, st));
  launched = true;
  launch_groups(groups, goff, shm);
  // where each job's results sit in the downloaded region
  res.resize(n);
  for (size_t i = 0; i < n; ++i) res[i] = {oal[i] - out_off, obe[i] - out_off, on[i] - out_off};
}

// One launch per kernel shape, one after another on st (measured: forking
// the shapes onto streams of their own made them share hardware queues with
// the caller's other streams and stalled those).
template <typename Groups, typename Offsets, typename Shm>
void WgBatch::launch_groups(const Groups& groups, const Offsets& goff, const Shm& shm) {
  for (auto& g : groups) {
    size_t bytes = 0;
    for (size_t i : g.second) bytes = std::max(bytes, (size_t)shm[i]);
    launch_shape(g.first, arena.p + goff.at(g.first), (int)g.second.size(), bytes, st);
  }
  FTLM_HIP(hipGetLastError());
}

void WgBatch::enqueue_download(void* host, size_t bytes) {
  if (!launched) fail(FTLM_ERR_INVALID_ARG, "fused batch: nothing to download");
  if (tasks.size() != 1) fail(FTLM_ERR_INVALID_ARG, "fused batch: asynchronous download is for one job");
  const WgTask& k = tasks[0];
  const size_t need = 16 * (size_t)k.R * k.steps + 4 * (size_t)k.R;  // alpha | beta | nsteps
  if (bytes < need) fail(FTLM_ERR_INVALID_ARG, "fused batch: host buffer too small");
  FTLM_HIP(hipMemcpyAsync(host, arena.p + out_off, need, hipMemcpyDeviceToHost, st));
  launched = false;
}

void WgBatch::enqueue_download_all(void* host, size_t bytes) {
  if (!launched) fail(FTLM_ERR_INVALID_ARG, "fused batch: nothing to download");
  if (bytes < out_bytes) fail(FTLM_ERR_INVALID_ARG, "fused batch: host buffer too small");
  FTLM_HIP(hipMemcpyAsync(host, arena.p + out_off, out_bytes, hipMemcpyDeviceToHost, st));
  launched = false;
}

void WgBatch::finish() {
  if (!launched) return;
  launched = false;
  std::vector<uint8_t> h(out_bytes);
  FTLM_HIP(hipMemcpyAsync(h.data(), arena.p + out_off, out_bytes, hipMemcpyDeviceToHost, st));
  FTLM_HIP(hipStreamSynchronize(st));
  for (size_t i = 0; i < tasks.size(); ++i) {
    const WgTask& k = tasks[i];
    const size_t rs = (size_t)k.R * k.steps;
    std::memcpy(k.alpha, h.data() + res[i][0], 8 * rs);
    std::memcpy(k.beta, h.data() + res[i][1], 8 * rs);
    std::memcpy(k.nsteps, h.data() + res[i][2], 4 * (size_t)k.R);
  }
}

WgBatch::~WgBatch() {
  // the arena is released on st after the kernels, the pinned staging buffer
  // (freed with the members) only once the stream is done with it
  if (launched || staging.p) (void)hipStreamSynchronize(st);
}

}  // namespace ftlm
