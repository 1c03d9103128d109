// Continuous-batching FTLM job server (see ftlm_server.h).
//
// Two threads own all HIP work of a server.  The builder thread builds groups
// (closure and irreps, host) and sector tables (GPU, on its own stream) one at
// a time.  The worker thread loops: (1) take finished builds into the caches,
// (2) retire running jobs and fused batches whose completion events have
// fired, (3) walk the queue in FIFO order: a job whose group or sector is
// missing asks the builder for it (sector memory is reserved against the
// budget first) and waits without holding anyone up; a job whose tables are
// resident is admitted when a slot is free and its block and Lanczos
// footprint fits; a later job may overtake one that does not fit, until that
// one has been overtaken kMaxOvertake times and stops the walk in front of
// it; (4) launch the small jobs admitted in this walk together as one fused
// batch, or alone with the per-step kernels when only one came; (5) sleep
// briefly or until woken.
// Admission builds the block on the worker's stream.  A per-step job gets a
// pooled non-blocking stream; the worker feeds its Lanczos steps in chunks
// (two in flight, each followed by an event) and finally the copy of its
// coefficients and a completion event.  A fused batch is one launch per
// kernel shape of the fused small-block kernel on a pooled stream, one copy
// of all its jobs' coefficients and one event; it takes one slot.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "capi_guard.h"
#include "ftlm_server.h"
#include "internal.h"

namespace ftlm {

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Job {
  int64_t id = 0;
  // copied description
  int N = 0, two_s = 0, ngens = 0, two_M = 0, irrep = 0, row = 0, R = 0, steps = 0, storage = 0, dist = 0;
  uint64_t seed = 0;
  std::vector<int32_t> bonds, gens;
  std::vector<double> J;
  std::string group_key, sector_key;
  // state
  bool done = false, running = false, cancel = false, holds_sector = false;
  int status = FTLM_OK;
  std::string msg;  // error text of a failed job
  double t_submit = 0, t_start = 0, t_end = 0;
  uint64_t D = 0;
  int dg = 0;
  std::unique_ptr<Block> block;
  std::unique_ptr<LanczosRun> run;
  std::unique_ptr<WgBatch> fused;  // the fused small-block kernel instead of run
  int engine = FTLM_ENGINE_AUTO;   // requested, then the one used
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* h_buf = nullptr;  // pinned: alpha | beta | nsteps
  size_t h_bytes = 0;
  double* h_alpha = nullptr;
  double* h_beta = nullptr;
  int32_t* h_n = nullptr;
  int overtaken = 0;
  bool heavy = false;  // a per-step job with an estimated step of at least kHeavyStepSeconds
  bool capped = false; // refused in this walk because the long-step jobs had their slots
  // incremental enqueue: steps [0, next_step) are on the stream, at most two
  // chunks of `chunk` steps are in flight, each followed by an event
  int next_step = 0, chunk = 1;
  bool enqueued_all = false;
  std::deque<hipEvent_t> inflight;
  std::vector<double> alpha, beta;
  std::vector<int32_t> nsteps;
  int64_t footprint = 0;
};

constexpr int kMaxOvertake = 64;
constexpr size_t kMaxBatchJobs = 64;  // jobs of one fused batch
constexpr double kChunkSeconds = 0.01;
constexpr double kHbmBytesPerSecond = 4.0e12;  // sustained gather rate assumed for chunk sizing
// Small jobs are batched into the fused kernel only while no job with steps
// this long runs: its H.V launches fill every compute unit, and the fused
// kernel's one long workgroup per job then waits behind them (measured on the
// serving mix: median latency 110 ms batched against 23 ms with per-step
// kernels, at the same throughput), while short per-step kernels interleave.
constexpr double kHeavyStepSeconds = 1e-3;
// Slots that jobs with long steps leave to the others (when max_active > 2):
// with every slot taken by runs of seconds, a short job waited for one of
// them to finish (measured on the serving mix: queue waits of 1.3-1.6 s with
// 7-8 slots held by 6x6-torus runs).
constexpr int kShortSlots = 2;

// HBM bytes of one Lanczos step (entries, gathered rows, the vector passes)
// at kHbmBytesPerSecond; rows per representative = D / n_reps.
double step_seconds(const Sector& S, double D, int R, int storage) {
  const double elem = storage == FTLM_F64 ? 8.0 : storage == FTLM_F32 ? 4.0 : 2.0;
  const double rows = S.n_reps ? D / (double)S.n_reps : 0.0;
  const double step_bytes = (double)S.n_entries * (rows * R * elem + 8.0) + 6.0 * D * R * elem;
  return step_bytes / kHbmBytesPerSecond;
}

std::string key_of(const void* p, size_t n) { return std::string((const char*)p, n); }

struct BuildReq {
  bool sector = false;  // false: group
  std::string key;
  std::shared_ptr<Job> job;  // source of the cluster description
  std::shared_ptr<Group> G;  // sector builds
};

struct BuildRes {
  bool sector = false;
  std::string key;
  std::shared_ptr<Group> G;
  std::shared_ptr<Sector> S;
  int code = FTLM_OK;
  std::string msg;
};

// Number of labels with digit sum A2/2 (the sector dimension D_M).
long double sector_dim(int N, int two_s, int two_M) {
  const int d = two_s + 1, Amax = N * (d - 1);
  std::vector<long double> c(Amax + 1, 0), n2(Amax + 1, 0);
  c[0] = 1;
  for (int k = 0; k < N; ++k) {
    std::fill(n2.begin(), n2.end(), 0);
    for (int v = 0; v <= Amax; ++v)
      for (int a = 0; a < d && a <= v; ++a) n2[v] += c[v - a];
    c.swap(n2);
  }
  const int A2 = N * two_s + two_M;
  return (A2 % 2 || A2 < 0 || A2 / 2 > Amax) ? 0 : c[A2 / 2];
}

}  // namespace

// Small jobs admitted together and run as one launch of the fused
// small-block kernel per kernel shape.
struct FusedBatch {
  std::vector<std::shared_ptr<Job>> jobs;
  std::unique_ptr<WgBatch> wg;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* h_buf = nullptr;  // pinned: the batch's output region
  size_t h_bytes = 0;
};

struct Server {
  int64_t budget = 0;
  int max_active = 1;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, std::shared_ptr<Job>> jobs;
  int64_t next_id = 0;
  bool stop = false;
  int n_running = 0;
  std::atomic<int64_t> used{0};
  std::thread worker, builder;
  // builder hand-off
  std::mutex bmu;
  std::condition_variable bcv;
  std::deque<BuildReq> breq;
  std::vector<BuildRes> bdone;
  bool bstop = false;
  hipStream_t bstream = nullptr;  // sector tables live on it (stream-ordered frees)
  // worker-only state
  std::map<std::string, std::shared_ptr<Group>> groups;
  std::map<std::string, std::pair<int, std::string>> group_failed;
  std::set<std::string> group_building;
  struct SecEntry {
    std::shared_ptr<Sector> sec;
    int users = 0;
    uint64_t last = 0;
    int64_t bytes = 0;
  };
  std::map<std::string, SecEntry> sectors;
  std::map<std::string, int64_t> sector_building;  // key -> reserved bytes
  uint64_t tick = 0;
  hipStream_t build = nullptr;
  std::vector<std::shared_ptr<Job>> running;    // per-step jobs, one slot each
  std::vector<std::unique_ptr<FusedBatch>> batches;  // one slot each
  std::vector<std::shared_ptr<Job>> forming;    // small jobs admitted in this walk
  int heavy_running = 0;                        // running jobs with Job::heavy
  // Streams, events and pinned result buffers are recycled: creating and
  // freeing them per job would add driver calls that can serialize the device.
  std::vector<std::pair<hipStream_t, hipEvent_t>> free_streams;
  std::vector<hipEvent_t> free_events;
  std::multimap<size_t, void*> free_pinned;

  void loop();
  void feed(Job& j);
  void builder_loop();
  void request(BuildReq r);
  void take_builds();
  // 1: admitted or ended, 0: waits for memory or a slot, -1: waits for a build
  int try_admit(const std::shared_ptr<Job>& j);
  void launch(const std::shared_ptr<Job>& j, SecEntry& se, bool small);
  void start_steps(const std::shared_ptr<Job>& j);
  void flush_forming();
  void finish_batch(FusedBatch& b);
  void take_stream(hipStream_t& s, hipEvent_t& e);
  void* take_pinned(size_t& bytes);
  int slots_in_use() const {
    return (int)running.size() + (int)batches.size() + (forming.empty() ? 0 : 1);
  }
  void retire(const std::shared_ptr<Job>& j, int status);
  int64_t estimate_sector(const Job& j, const Group& G) const;
  int64_t estimate_job(const Job& j, const Group& G, const Sector& S) const;
  void evict_unused(int64_t need, const std::string& keep);
  void dequeue(int64_t id);
};

// Upper bounds: orbits number at most D_M / |G| plus the labels with a
// non-trivial stabilizer (the 1.2 margin and the constant cover those), and
// every bond gives at most one admissible flip per direction.
int64_t Server::estimate_sector(const Job& j, const Group& G) const {
  const long double DM = sector_dim(j.N, j.two_s, j.two_M);
  const long double reps = DM / G.order * 1.2 + 16;
  const long double flips = (long double)j.bonds.size() / 2 * (j.two_s == 1 ? 1.0 : 2.0);
  const long double b = DM / 8 + DM / 64 * 4 + reps * 34 + reps * flips * 8 + (1 << 20);
  return (int64_t)std::min<long double>(b, 9.0e18);
}

int64_t Server::estimate_job(const Job& j, const Group& G, const Sector& S) const {
  const int dg = (G.irreps_computed && j.irrep >= 0 && j.irrep < (int)G.irreps.size()) ? G.irreps[j.irrep].dim : 1;
  const long double D = (long double)S.n_reps * dg;  // >= the block dimension
  const long double b = (long double)S.n_reps * 16 + 2 * D * j.R * (j.storage == FTLM_F64 ? 8 : j.storage == FTLM_F32 ? 4 : 2) +
                        8192.0 * j.R * 8 + (long double)j.R * j.steps * 16 + (1 << 20);
  return (int64_t)std::min<long double>(b, 9.0e18);
}

void Server::evict_unused(int64_t need, const std::string& keep) {
  // evict only when that makes room: a job that cannot fit even with every
  // unused sector gone keeps the caches (other queued jobs may need them)
  int64_t freeable = 0;
  for (auto& kv : sectors)
    if (kv.second.users == 0 && kv.first != keep) freeable += kv.second.bytes;
  if (used - freeable + need > budget) return;
  while (used + need > budget) {
    auto victim = sectors.end();
    for (auto it = sectors.begin(); it != sectors.end(); ++it)
      if (it->second.users == 0 && it->first != keep &&
          (victim == sectors.end() || it->second.last < victim->second.last))
        victim = it;
    if (victim == sectors.end()) return;
    used -= victim->second.bytes;
    sectors.erase(victim);
  }
}

void Server::request(BuildReq r) {
  std::lock_guard<std::mutex> lk(bmu);
  breq.push_back(std::move(r));
  bcv.notify_all();
}

void Server::builder_loop() {
  (void)hipSetDevice(device);
  while (true) {
    BuildReq r;
    {
      std::unique_lock<std::mutex> lk(bmu);
      bcv.wait(lk, [&] { return bstop || !breq.empty(); });
      if (bstop) break;
      r = std::move(breq.front());
      breq.pop_front();
    }
    BuildRes res;
    res.sector = r.sector;
    res.key = r.key;
    try {
      const Job& j = *r.job;
      if (!r.sector) {
        auto g = std::make_shared<Group>(build_group(j.N, j.gens.data(), j.ngens));
        compute_irreps(*g);
        res.G = std::move(g);
      } else {
        AllocStreamScope scope(bstream);
        ftlm_cluster cl{j.N, j.two_s, (int32_t)(j.bonds.size() / 2), j.bonds.data(), j.J.data()};
        // entry tables always: their size is in the sector estimate the
        // budget admitted, and the decision must not depend on what other
        // jobs happen to hold on the device (the free memory AUTO looks at)
        ftlm_opts o{};
        o.hv_mode = FTLM_HV_ENTRIES;
        res.S = build_sector(&cl, r.G, j.two_M, &o);  // synchronizes bstream before returning
      }
    } catch (const Error& e) {
      res.code = e.code;
      res.msg = e.what();
    } catch (const std::exception& e) {
      res.code = FTLM_ERR_INVALID_ARG;
      res.msg = e.what();
    }
    {
      std::lock_guard<std::mutex> lk(bmu);
      bdone.push_back(std::move(res));
    }
    std::lock_guard<std::mutex> lk(mu);
    cv_work.notify_all();
  }
}

void Server::dequeue(int64_t id) {
  std::lock_guard<std::mutex> lk(mu);
  for (auto it = queue.begin(); it != queue.end(); ++it)
    if (*it == id) {
      queue.erase(it);
      break;
    }
}

void Server::take_builds() {
  std::vector<BuildRes> done;
  {
    std::lock_guard<std::mutex> lk(bmu);
    done.swap(bdone);
  }
  for (auto& r : done) {
    if (!r.sector) {
      group_building.erase(r.key);
      if (r.code == FTLM_OK)
        groups[r.key] = r.G;
      else
        group_failed[r.key] = {r.code, r.msg};
      continue;
    }
    auto rit = sector_building.find(r.key);
    if (rit != sector_building.end()) {
      used -= rit->second;
      sector_building.erase(rit);
    }
    if (r.code == FTLM_OK) {
      SecEntry& se = sectors[r.key];
      se.sec = std::move(r.S);
      se.bytes = se.sec->device_bytes();
      se.last = ++tick;
      used += se.bytes;
      continue;
    }
    // the queued jobs that wait for this sector end with the build's error
    std::vector<std::shared_ptr<Job>> failed;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int64_t id : queue) {
        auto& j = jobs[id];
        if (j->sector_key == r.key) failed.push_back(j);
      }
    }
    for (auto& j : failed) {
      j->msg = r.msg;
      retire(j, r.code);
      dequeue(j->id);
    }
  }
}

int Server::try_admit(const std::shared_ptr<Job>& j) {
  j->capped = false;
  auto gf = group_failed.find(j->group_key);
  if (gf != group_failed.end()) {
    j->msg = gf->second.second;
    retire(j, gf->second.first);
    return 1;
  }
  auto git = groups.find(j->group_key);
  if (git == groups.end()) {
    if (group_building.insert(j->group_key).second) request(BuildReq{false, j->group_key, j, nullptr});
    return -1;
  }
  const Group& G = *git->second;
  auto sit = sectors.find(j->sector_key);
  if (sit == sectors.end()) {
    if (sector_building.count(j->sector_key)) return -1;
    const int64_t est = estimate_sector(*j, G);
    if (est > budget) {
      j->msg = "estimated sector tables of " + std::to_string(est) + " bytes exceed the server budget";
      retire(j, FTLM_ERR_OUT_OF_MEMORY);
      return 1;
    }
    if (used + est > budget) evict_unused(est, j->sector_key);
    if (used + est > budget) return 0;
    used += est;
    sector_building[j->sector_key] = est;
    request(BuildReq{true, j->sector_key, j, git->second});
    return -1;
  }
  SecEntry& se = sit->second;
  // a small job under the automatic engine joins the batch of this walk
  // (no slot of its own once the batch has one)
  const bool small = j->engine == FTLM_ENGINE_AUTO && heavy_running == 0 && j->R <= kWgMaxChains &&
                     (j->storage == FTLM_F64 || j->storage == FTLM_F32) &&
                     wg_rounds(se.sec->n_reps, j->R) <= kWgAutoMaxRounds;
  const bool room = forming.size() < kMaxBatchJobs;
  const bool joins = small && room && !forming.empty();
  if (!joins && slots_in_use() >= max_active) return 0;
  // a job with long steps (by an upper bound of the block: d_Gamma rows per
  // representative) does not take the last kShortSlots slots
  if (!small && max_active > kShortSlots && heavy_running >= max_active - kShortSlots) {
    const int dg = (G.irreps_computed && j->irrep >= 0 && j->irrep < (int)G.irreps.size()) ? G.irreps[j->irrep].dim : 1;
    if (step_seconds(*se.sec, (double)se.sec->n_reps * dg, j->R, j->storage) >= kHeavyStepSeconds) {
      j->capped = true;
      return 0;
    }
  }
  const int64_t est = estimate_job(*j, G, *se.sec);
  if (est > budget) {
    j->msg = "estimated job footprint of " + std::to_string(est) + " bytes exceeds the server budget";
    retire(j, FTLM_ERR_OUT_OF_MEMORY);
    return 1;
  }
  if (used + est > budget) evict_unused(est, j->sector_key);
  if (used + est > budget) return 0;
  launch(j, se, small && room);
  return 1;
}

void Server::take_stream(hipStream_t& st, hipEvent_t& ev) {
  if (!free_streams.empty()) {
    std::tie(st, ev) = free_streams.back();
    free_streams.pop_back();
  } else {
    FTLM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    FTLM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
}

void* Server::take_pinned(size_t& bytes) {
  auto pit = free_pinned.lower_bound(bytes);
  if (pit != free_pinned.end() && pit->first <= 2 * bytes) {
    bytes = pit->first;
    void* p = pit->second;
    free_pinned.erase(pit);
    return p;
  }
  void* p = nullptr;
  FTLM_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  return p;
}

void Server::launch(const std::shared_ptr<Job>& j, SecEntry& se, bool small) {
  try {
    AllocStreamScope scope(build);
    se.users++;
    se.last = ++tick;
    j->holds_sector = true;
    j->block = build_block(se.sec, j->irrep, j->row, nullptr);
    j->D = j->block->D;
    j->dg = j->block->dg;
    const int64_t blk = j->block->device_bytes() - se.sec->device_bytes();
    const int64_t lz = (int64_t)LanczosRun::estimate_bytes(*j->block, j->R, j->steps, j->storage);
    j->footprint = blk + lz;
    used += j->footprint;
    FTLM_HIP(hipStreamSynchronize(build));
    const Block& B = *j->block;
    const bool fits = B.D > 0 && wg_supported(B, j->R, j->storage);
    if (j->engine == FTLM_ENGINE_FUSED && !fits)
      fail(FTLM_ERR_INVALID_ARG, "the job does not fit the fused small-block kernel");
    j->running = true;
    j->t_start = now_s(t0);
    {
      std::lock_guard<std::mutex> lk(mu);
      n_running++;
    }
    if (fits && (j->engine == FTLM_ENGINE_FUSED || small)) {
      // launched with the other small jobs of this walk (flush_forming)
      forming.push_back(j);
      return;
    }
    start_steps(j);
  } catch (const Error& e) {
    j->msg = e.what();
    retire(j, e.code);
  } catch (const std::exception& e) {
    j->msg = e.what();
    retire(j, FTLM_ERR_INVALID_ARG);
  }
}

// The per-step kernels on a pooled stream of the job, steps fed in chunks.
void Server::start_steps(const std::shared_ptr<Job>& j) {
  take_stream(j->stream, j->ev);
  const size_t nab = (size_t)j->R * j->steps;
  j->h_bytes = 2 * nab * sizeof(double) + j->R * sizeof(int32_t);
  j->h_buf = take_pinned(j->h_bytes);
  j->h_alpha = static_cast<double*>(j->h_buf);
  j->h_beta = j->h_alpha + nab;
  j->h_n = reinterpret_cast<int32_t*>(j->h_beta + nab);
  j->engine = FTLM_ENGINE_STEPS;
  {
    AllocStreamScope js(j->stream);
    j->run = std::make_unique<LanczosRun>(*j->block, j->R, j->steps, j->seed, j->storage, j->dist);
    j->run->allocate();
    j->run->enqueue_begin(j->stream);
  }
  // Steps go to the stream in chunks of about kChunkSeconds of estimated
  // HBM time, so a long run never holds a shared hardware queue for more
  // than one chunk ahead of other jobs' work.
  {
    const double step_s = step_seconds(*j->block->sec, (double)j->D, j->R, j->storage);
    j->chunk = (int)std::max(1.0, std::min((double)std::max(j->run->target, 1), kChunkSeconds / std::max(step_s, 1e-9)));
    j->heavy = step_s >= kHeavyStepSeconds;
    if (j->heavy) heavy_running++;
  }
  j->next_step = 0;
  j->enqueued_all = false;
  feed(*j);
  running.push_back(j);
}

// The small jobs admitted in one walk (only while no heavy job runs): two or
// more run as one fused batch (one launch per kernel shape), a lone job runs
// the per-step kernels, which are faster for one job (measured on the serving
// mix: 0.7 ms against 1.4 ms fused) unless it asked for the fused engine.
void Server::flush_forming() {
  if (forming.empty()) return;
  std::vector<std::shared_ptr<Job>> js;
  js.swap(forming);
  if (js.size() == 1 && js[0]->engine != FTLM_ENGINE_FUSED) {
    try {
      start_steps(js[0]);
    } catch (const Error& e) {
      js[0]->msg = e.what();
      retire(js[0], e.code);
    }
    return;
  }
  auto b = std::make_unique<FusedBatch>();
  try {
    take_stream(b->stream, b->ev);
    std::vector<WgTask> tasks;
    for (auto& j : js) {
      j->engine = FTLM_ENGINE_FUSED;
      j->alpha.assign((size_t)j->R * j->steps, 0.0);
      j->beta.assign((size_t)j->R * j->steps, 0.0);
      j->nsteps.assign(j->R, 0);
      tasks.push_back(WgTask{j->block.get(), j->R, j->steps, j->storage, j->dist, 0, j->seed, j->alpha.data(),
                             j->beta.data(), j->nsteps.data()});
    }
    {
      AllocStreamScope bs(b->stream);
      b->wg = std::make_unique<WgBatch>(std::move(tasks), b->stream);
    }
    b->h_bytes = std::max<size_t>(b->wg->out_bytes, 8);
    b->h_buf = take_pinned(b->h_bytes);
    b->wg->enqueue_download_all(b->h_buf, b->h_bytes);
    FTLM_HIP(hipEventRecord(b->ev, b->stream));
    b->jobs = std::move(js);
    batches.push_back(std::move(b));
  } catch (const Error& e) {
    for (auto& j : js) {
      j->msg = e.what();
      retire(j, e.code);
    }
    if (b->wg) b->wg.reset();
    if (b->stream) {
      (void)hipStreamSynchronize(b->stream);
      free_streams.emplace_back(b->stream, b->ev);
    }
    if (b->h_buf) free_pinned.emplace(b->h_bytes, b->h_buf);
  }
}

// A batch whose event has fired: every job's coefficients from the pinned
// copy, the jobs retired, the stream, event and buffer back to the pools.
void Server::finish_batch(FusedBatch& b) {
  for (size_t i = 0; i < b.jobs.size(); ++i) {
    auto& j = b.jobs[i];
    const auto& off = b.wg->res[i];
    const size_t rs = (size_t)j->R * j->steps;
    const uint8_t* h = static_cast<const uint8_t*>(b.h_buf);
    std::memcpy(j->alpha.data(), h + off[0], 8 * rs);
    std::memcpy(j->beta.data(), h + off[1], 8 * rs);
    std::memcpy(j->nsteps.data(), h + off[2], 4 * (size_t)j->R);
    bool c;
    {
      std::lock_guard<std::mutex> lk(mu);
      c = j->cancel;
    }
    if (c) j->msg = "cancelled";
    retire(j, c ? FTLM_ERR_CANCELLED : FTLM_OK);
  }
  b.wg.reset();  // stream-ordered free of the arena; waits for the pinned staging buffer
  free_streams.emplace_back(b.stream, b.ev);
  free_pinned.emplace(b.h_bytes, b.h_buf);
  b.stream = nullptr;
  b.ev = nullptr;
  b.h_buf = nullptr;
}

// Keeps up to two chunks of steps in flight; after the last step enqueues the
// step counts, the copy of the coefficients and the completion event.  A
// cancelled running job stops receiving steps.
void Server::feed(Job& j) {
  while (!j.inflight.empty() && hipEventQuery(j.inflight.front()) == hipSuccess) {
    free_events.push_back(j.inflight.front());
    j.inflight.pop_front();
  }
  if (j.enqueued_all) return;
  bool cancel;
  {
    std::lock_guard<std::mutex> lk(mu);
    cancel = j.cancel;
  }
  const int target = j.run->target;
  while (!cancel && j.next_step < target && j.inflight.size() < 2) {
    const int j1 = std::min(target, j.next_step + j.chunk);
    j.run->enqueue_steps(j.stream, j.next_step, j1);
    j.next_step = j1;
    hipEvent_t e;
    if (!free_events.empty()) {
      e = free_events.back();
      free_events.pop_back();
    } else {
      FTLM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    FTLM_HIP(hipEventRecord(e, j.stream));
    j.inflight.push_back(e);
  }
  if (cancel || j.next_step >= target) {
    if (!cancel) {
      j.run->enqueue_end(j.stream);
      j.run->download(j.stream, j.h_alpha, j.h_beta, j.h_n);
    }
    FTLM_HIP(hipEventRecord(j.ev, j.stream));
    j.enqueued_all = true;
  }
}

void Server::retire(const std::shared_ptr<Job>& j, int status) {
  if (j->stream) (void)hipStreamSynchronize(j->stream);
  if (status == FTLM_OK && j->h_alpha) {  // per-step jobs (fused-batch jobs hold theirs already)
    j->alpha.assign(j->h_alpha, j->h_alpha + (size_t)j->R * j->steps);
    j->beta.assign(j->h_beta, j->h_beta + (size_t)j->R * j->steps);
    j->nsteps.assign(j->h_n, j->h_n + j->R);
  }
  j->run.reset();  // stream-ordered frees on the job's stream
  j->fused.reset();
  if (j->stream) (void)hipStreamSynchronize(j->stream);
  j->block.reset();
  if (j->h_buf) free_pinned.emplace(j->h_bytes, j->h_buf);
  j->h_buf = nullptr;
  j->h_alpha = j->h_beta = nullptr;
  j->h_n = nullptr;
  for (hipEvent_t e : j->inflight) free_events.push_back(e);
  j->inflight.clear();
  if (j->stream) free_streams.emplace_back(j->stream, j->ev);
  j->ev = nullptr;
  j->stream = nullptr;
  auto it = sectors.find(j->sector_key);
  if (j->holds_sector && it != sectors.end()) it->second.users--;
  j->holds_sector = false;
  if (j->heavy) heavy_running--;
  j->heavy = false;
  used -= j->footprint;
  j->footprint = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (j->running) n_running--;
  j->running = false;
  j->status = status;
  j->done = true;
  j->t_end = now_s(t0);
  cv_done.notify_all();
}

void Server::loop() {
  (void)hipSetDevice(device);
  (void)hipStreamCreateWithFlags(&build, hipStreamNonBlocking);
  (void)hipStreamCreateWithFlags(&bstream, hipStreamNonBlocking);
  builder = std::thread([this] { builder_loop(); });
  while (true) {
    take_builds();
    // retire finished jobs
    for (size_t i = 0; i < running.size();) {
      auto& j = running[i];
      try {
        feed(*j);
      } catch (const Error& e) {
        auto jj = j;
        running.erase(running.begin() + i);
        jj->msg = e.what();
        retire(jj, e.code);
        continue;
      }
      if (j->enqueued_all && hipEventQuery(j->ev) == hipSuccess) {
        bool c;
        {
          std::lock_guard<std::mutex> lk(mu);
          c = j->cancel;
        }
        auto jj = j;
        running.erase(running.begin() + i);
        if (c) jj->msg = "cancelled";
        retire(jj, c ? FTLM_ERR_CANCELLED : FTLM_OK);
      } else {
        ++i;
      }
    }
    for (size_t i = 0; i < batches.size();) {
      if (hipEventQuery(batches[i]->ev) == hipSuccess) {
        std::unique_ptr<FusedBatch> b = std::move(batches[i]);
        batches.erase(batches.begin() + i);
        finish_batch(*b);
      } else {
        ++i;
      }
    }
    // walk the queue
    std::vector<std::shared_ptr<Job>> pending;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stop && queue.empty() && running.empty() && batches.empty()) break;
      for (int64_t id : queue) pending.push_back(jobs[id]);
    }
    std::vector<Job*> refused;
    for (auto& j : pending) {
      // A job that has been overtaken kMaxOvertake times holds back the
      // queue behind it until it is admitted: nothing behind it is tried, so
      // the memory and slots that running jobs free reach it first and large
      // jobs are not starved.
      if (std::any_of(refused.begin(), refused.end(), [](const Job* q) { return q->overtaken >= kMaxOvertake; }))
        break;
      bool cancelled;
      {
        std::lock_guard<std::mutex> lk(mu);
        cancelled = j->cancel || stop;
      }
      int r;
      if (cancelled) {
        j->msg = "cancelled";
        retire(j, FTLM_ERR_CANCELLED);
        r = 1;
      } else {
        r = try_admit(j);
      }
      if (r == 0) {
        refused.push_back(j.get());
      } else if (r == 1) {
        // a job held back only by the long-step cap is overtaken by other
        // long-step jobs, not by the short ones that use the slots left to them
        if (j->running)
          for (Job* q : refused)
            if (!q->capped || j->heavy) ++q->overtaken;
        dequeue(j->id);
      }
    }
    flush_forming();
    std::unique_lock<std::mutex> lk(mu);
    if (running.empty() && batches.empty() && queue.empty()) {
      if (stop) break;
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    } else {
      cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
  }
  {
    std::lock_guard<std::mutex> lk(bmu);
    bstop = true;
    bcv.notify_all();
  }
  if (builder.joinable()) builder.join();
  {
    std::lock_guard<std::mutex> lk(bmu);
    bdone.clear();
    breq.clear();
  }
  sectors.clear();
  groups.clear();
  if (bstream) (void)hipStreamSynchronize(bstream);
  if (build) (void)hipStreamSynchronize(build);
  for (hipStream_t* sp : {&build, &bstream})
    if (*sp) (void)hipStreamDestroy(*sp);
  for (auto& se : free_streams) {
    (void)hipEventDestroy(se.second);
    (void)hipStreamDestroy(se.first);
  }
  for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
  free_events.clear();
  for (auto& pb : free_pinned) (void)hipHostFree(pb.second);
  free_streams.clear();
  free_pinned.clear();
}

}  // namespace ftlm

struct ftlm_server {
  std::unique_ptr<ftlm::Server> s;
};

using namespace ftlm;

extern "C" {

int ftlm_server_create(int64_t hbm_budget_bytes, int32_t max_active, ftlm_server** out) {
  return guarded([&] {
    if (!out || hbm_budget_bytes <= 0 || max_active <= 0) fail(FTLM_ERR_INVALID_ARG, "bad server arguments");
    auto* h = new ftlm_server{std::make_unique<Server>()};
    Server& S = *h->s;
    S.budget = hbm_budget_bytes;
    S.max_active = max_active;
    S.t0 = std::chrono::steady_clock::now();
    (void)hipGetDevice(&S.device);
    S.worker = std::thread([&S] { S.loop(); });
    *out = h;
  });
}

int ftlm_server_submit(ftlm_server* h, const ftlm_job_desc* d, int64_t* job_id) {
  return guarded([&] {
    if (!h || !d || !job_id) fail(FTLM_ERR_INVALID_ARG, "null argument");
    const ftlm_cluster& c = d->cluster;
    if (c.N <= 0 || c.N > 64 || c.nbonds < 0 || (c.nbonds && !c.bonds) || d->ngens < 0 || (d->ngens && !d->gens))
      fail(FTLM_ERR_INVALID_ARG, "bad cluster or generators");
    if (d->R <= 0 || d->R > 256 || d->steps <= 0) fail(FTLM_ERR_INVALID_ARG, "bad R or steps");
    auto j = std::make_shared<Job>();
    j->N = c.N;
    j->two_s = c.two_s;
    j->bonds.assign(c.bonds, c.bonds + 2 * (size_t)c.nbonds);
    j->J.resize(c.nbonds);
    for (int b = 0; b < c.nbonds; ++b) j->J[b] = c.J ? c.J[b] : 1.0;
    j->ngens = d->ngens;
    j->gens.assign(d->gens, d->gens + (size_t)d->ngens * c.N);
    j->two_M = d->two_M;
    j->irrep = d->irrep;
    j->row = d->row;
    j->R = d->R;
    j->steps = d->steps;
    j->seed = d->seed;
    j->storage = d->storage;
    j->dist = d->dist;
    if (d->engine < FTLM_ENGINE_AUTO || d->engine > FTLM_ENGINE_FUSED) fail(FTLM_ERR_INVALID_ARG, "bad engine");
    j->engine = d->engine;
    j->group_key = key_of(&j->N, 4) + key_of(j->gens.data(), j->gens.size() * 4);
    j->sector_key = key_of(&j->N, 4) + key_of(&j->two_s, 4) + key_of(&j->two_M, 4) +
                    key_of(j->bonds.data(), j->bonds.size() * 4) + key_of(j->J.data(), j->J.size() * 8) +
                    key_of(j->gens.data(), j->gens.size() * 4);
    Server& S = *h->s;
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stop) fail(FTLM_ERR_INVALID_ARG, "server is shutting down");
    j->id = S.next_id++;
    j->t_submit = now_s(S.t0);
    S.jobs[j->id] = j;
    S.queue.push_back(j->id);
    *job_id = j->id;
    S.cv_work.notify_all();
  });
}

int ftlm_server_poll(ftlm_server* h, int64_t id, int32_t* done) {
  return guarded([&] {
    if (!h || !done) fail(FTLM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(h->s->mu);
    auto it = h->s->jobs.find(id);
    if (it == h->s->jobs.end()) fail(FTLM_ERR_INVALID_ARG, "unknown job id");
    *done = it->second->done ? 1 : 0;
  });
}

int ftlm_server_wait(ftlm_server* h, int64_t id, ftlm_job_result* res, double* alpha, double* beta, int32_t* nsteps) {
  int status = FTLM_OK;
  int rc = guarded([&] {
    if (!h) fail(FTLM_ERR_INVALID_ARG, "null server");
    Server& S = *h->s;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.jobs.find(id);
    if (it == S.jobs.end()) fail(FTLM_ERR_INVALID_ARG, "unknown job id");
    auto j = it->second;
    S.cv_done.wait(lk, [&] { return j->done; });
    S.jobs.erase(id);
    lk.unlock();
    status = j->status;
    if (status != FTLM_OK) set_last_error(j->msg);
    if (res) {
      res->status = j->status;
      res->R = j->R;
      res->steps = j->steps;
      res->d_gamma = j->dg;
      res->D = j->D;
      res->submit_s = j->t_submit;
      res->start_s = j->t_start;
      res->end_s = j->t_end;
      res->engine = j->engine;
      res->reserved = 0;
    }
    if (j->status == FTLM_OK) {
      if (alpha) std::memcpy(alpha, j->alpha.data(), j->alpha.size() * 8);
      if (beta) std::memcpy(beta, j->beta.data(), j->beta.size() * 8);
      if (nsteps) std::memcpy(nsteps, j->nsteps.data(), j->nsteps.size() * 4);
    }
  });
  return rc != FTLM_OK ? rc : status;
}

int ftlm_server_cancel(ftlm_server* h, int64_t id) {
  return guarded([&] {
    if (!h) fail(FTLM_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(h->s->mu);
    auto it = h->s->jobs.find(id);
    if (it == h->s->jobs.end()) fail(FTLM_ERR_INVALID_ARG, "unknown job id");
    it->second->cancel = true;
    h->s->cv_work.notify_all();
  });
}

int ftlm_server_stats(ftlm_server* h, int64_t* used_bytes, int32_t* running, int32_t* queued) {
  return guarded([&] {
    if (!h) fail(FTLM_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(h->s->mu);
    if (used_bytes) *used_bytes = h->s->used;
    if (running) *running = h->s->n_running;
    if (queued) *queued = (int32_t)h->s->queue.size();
  });
}

void ftlm_server_free(ftlm_server* h) {
  if (!h) return;
  {
    std::lock_guard<std::mutex> lk(h->s->mu);
    h->s->stop = true;
    h->s->cv_work.notify_all();
  }
  if (h->s->worker.joinable()) h->s->worker.join();
  delete h;
}

}  // extern "C"
