// Continuous-batching FTLM job server (see ftlm_server.h).
//
// One worker thread owns all HIP work.  Each loop it (1) retires running jobs
// whose completion event has fired, (2) admits queued jobs in FIFO order,
// letting a later job overtake one that does not fit, while fewer than
// max_active run and the footprint fits the budget, and (3) sleeps briefly
// or until a submit.  Admission builds (or reuses) the group and the sector
// tables on the server's build stream with stream-ordered allocations, builds
// the block, then enqueues the job's whole Lanczos run and the copy of its
// coefficients on a fresh non-blocking stream, followed by an event.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>

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
  // state
  bool done = false, running = false, cancel = false, holds_sector = false;
  int status = FTLM_OK;
  std::string msg;  // error text of a failed job
  double t_submit = 0, t_start = 0, t_end = 0;
  uint64_t D = 0;
  int dg = 0;
  std::string sector_key;
  std::unique_ptr<Block> block;
  std::unique_ptr<LanczosRun> run;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* h_buf = nullptr;  // pinned: alpha | beta | nsteps
  size_t h_bytes = 0;
  double* h_alpha = nullptr;
  double* h_beta = nullptr;
  int32_t* h_n = nullptr;
  int overtaken = 0;
  std::vector<double> alpha, beta;
  std::vector<int32_t> nsteps;
  size_t footprint = 0;
};

constexpr int kMaxOvertake = 64;

std::string key_of(const void* p, size_t n) { return std::string((const char*)p, n); }

}  // namespace

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
  std::thread worker;
  // worker-only state
  std::map<std::string, std::shared_ptr<Group>> groups;
  struct SecEntry {
    std::shared_ptr<Sector> sec;
    int users = 0;
    uint64_t last = 0;
    int64_t bytes = 0;
  };
  std::map<std::string, SecEntry> sectors;
  uint64_t tick = 0;
  hipStream_t build = nullptr;
  std::vector<std::shared_ptr<Job>> running;
  // Streams, events and pinned result buffers are recycled: creating and
  // freeing them per job would add driver calls that can serialize the device.
  std::vector<std::pair<hipStream_t, hipEvent_t>> free_streams;
  std::multimap<size_t, void*> free_pinned;

  void loop();
  bool try_admit(const std::shared_ptr<Job>& j);
  void retire(const std::shared_ptr<Job>& j, int status);
  int64_t estimate(const Job& j, const Group& G);
  std::shared_ptr<Group> group_of(const Job& j);
  void evict_unused(int64_t need);
};

std::shared_ptr<Group> Server::group_of(const Job& j) {
  const std::string gkey = key_of(j.gens.data(), j.gens.size() * 4) + key_of(&j.N, 4);
  auto git = groups.find(gkey);
  if (git == groups.end()) {
    auto g = std::make_shared<Group>(build_group(j.N, j.gens.data(), j.ngens));
    compute_irreps(*g);
    git = groups.emplace(gkey, std::move(g)).first;
  }
  return git->second;
}

// Device bytes a job will add, from the group and the sector size alone
// (upper bounds: every representative carries a full d_Gamma block, every
// bond a flip), plus the sector tables unless they are resident.
int64_t Server::estimate(const Job& j, const Group& Gr) {
  const int d = j.two_s + 1;
  long double DM = 1;
  {
    // digit-sum count for this M via the same counting recursion as the sector
    const int Amax = j.N * (d - 1);
    std::vector<long double> c(Amax + 1, 0), n2(Amax + 1, 0);
    c[0] = 1;
    for (int k = 0; k < j.N; ++k) {
      std::fill(n2.begin(), n2.end(), 0);
      for (int v = 0; v <= Amax; ++v)
        for (int a = 0; a < d && a <= v; ++a) n2[v] += c[v - a];
      c.swap(n2);
    }
    const int A2 = j.N * j.two_s + j.two_M;
    DM = (A2 % 2 || A2 < 0 || A2 / 2 > Amax) ? 0 : c[A2 / 2];
  }
  const long double G = Gr.order;
  const int dg = (Gr.irreps_computed && j.irrep >= 0 && j.irrep < (int)Gr.irreps.size()) ? Gr.irreps[j.irrep].dim : 1;
  // orbits of a group of order |G| number at most D_M / |G| + (labels with a
  // nontrivial stabilizer); the 1.2 margin and the constant cover the latter
  const long double reps = DM / G * 1.2 + 16;
  const long double D = reps * dg;
  long double sec = 0;
  if (sectors.find(j.sector_key) == sectors.end()) {
    const long double flips = j.bonds.size() / 2.0 * (j.two_s == 1 ? 1.0 : 2.0);
    sec = DM / 8 * 1.5 + reps * 34 + reps * flips * 8;
  }
  const long double vec = 2 * D * j.R * (j.storage == FTLM_F64 ? 8 : 4) + reps * 16 + 8192.0 * j.R * 8;
  return (int64_t)std::min<long double>(sec + vec + (1 << 20), 9.0e18);
}

void Server::evict_unused(int64_t need) {
  while (used + need > budget) {
    auto victim = sectors.end();
    for (auto it = sectors.begin(); it != sectors.end(); ++it)
      if (it->second.users == 0 && (victim == sectors.end() || it->second.last < victim->second.last)) victim = it;
    if (victim == sectors.end()) return;
    used -= victim->second.bytes;
    sectors.erase(victim);
  }
}

bool Server::try_admit(const std::shared_ptr<Job>& j) {
  std::shared_ptr<Group> G;
  try {
    G = group_of(*j);
  } catch (const Error& e) {
    j->msg = e.what();
    retire(j, e.code);
    return true;
  } catch (const std::exception& e) {
    j->msg = e.what();
    retire(j, FTLM_ERR_INVALID_ARG);
    return true;
  }
  const int64_t est = estimate(*j, *G);
  if (est > budget) {
    j->msg = "estimated device footprint " + std::to_string(est) + " bytes exceeds the server budget";
    retire(j, FTLM_ERR_OUT_OF_MEMORY);
    return true;
  }
  if (used + est > budget) evict_unused(est);
  if (used + est > budget) return false;  // wait for memory
  try {
    AllocStreamScope scope(build);
    SecEntry& se = sectors[j->sector_key];
    if (!se.sec) {
      ftlm_cluster cl{j->N, j->two_s, (int32_t)(j->bonds.size() / 2), j->bonds.data(), j->J.data()};
      ftlm_opts o{};
      o.hv_mode = FTLM_HV_AUTO;
      try {
        se.sec = build_sector(&cl, G, j->two_M, &o);
      } catch (...) {
        sectors.erase(j->sector_key);
        throw;
      }
      se.bytes = se.sec->device_bytes();
      used += se.bytes;
    }
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
    if (!free_streams.empty()) {
      std::tie(j->stream, j->ev) = free_streams.back();
      free_streams.pop_back();
    } else {
      FTLM_HIP(hipStreamCreateWithFlags(&j->stream, hipStreamNonBlocking));
      FTLM_HIP(hipEventCreateWithFlags(&j->ev, hipEventDisableTiming));
    }
    const size_t nab = (size_t)j->R * j->steps;
    j->h_bytes = 2 * nab * sizeof(double) + j->R * sizeof(int32_t);
    auto pit = free_pinned.lower_bound(j->h_bytes);
    if (pit != free_pinned.end() && pit->first <= 2 * j->h_bytes) {
      j->h_bytes = pit->first;
      j->h_buf = pit->second;
      free_pinned.erase(pit);
    } else {
      FTLM_HIP(hipHostMalloc(&j->h_buf, j->h_bytes, hipHostMallocDefault));
    }
    j->h_alpha = static_cast<double*>(j->h_buf);
    j->h_beta = j->h_alpha + nab;
    j->h_n = reinterpret_cast<int32_t*>(j->h_beta + nab);
    {
      AllocStreamScope js(j->stream);
      j->run = std::make_unique<LanczosRun>(*j->block, j->R, j->steps, j->seed, j->storage, j->dist);
      j->run->allocate();
      j->run->enqueue(j->stream);
      j->run->download(j->stream, j->h_alpha, j->h_beta, j->h_n);
    }
    FTLM_HIP(hipEventRecord(j->ev, j->stream));
    j->running = true;
    j->t_start = now_s(t0);
    running.push_back(j);
    std::lock_guard<std::mutex> lk(mu);
    n_running++;
  } catch (const Error& e) {
    j->msg = e.what();
    retire(j, e.code);
  } catch (const std::exception& e) {
    j->msg = e.what();
    retire(j, FTLM_ERR_INVALID_ARG);
  }
  return true;
}

void Server::retire(const std::shared_ptr<Job>& j, int status) {
  if (j->stream) (void)hipStreamSynchronize(j->stream);
  if (status == FTLM_OK && j->h_alpha) {
    j->alpha.assign(j->h_alpha, j->h_alpha + (size_t)j->R * j->steps);
    j->beta.assign(j->h_beta, j->h_beta + (size_t)j->R * j->steps);
    j->nsteps.assign(j->h_n, j->h_n + j->R);
  }
  j->run.reset();   // stream-ordered frees on the job's stream
  if (j->stream) (void)hipStreamSynchronize(j->stream);
  j->block.reset();
  if (j->h_buf) free_pinned.emplace(j->h_bytes, j->h_buf);
  j->h_buf = nullptr;
  j->h_alpha = j->h_beta = nullptr;
  j->h_n = nullptr;
  if (j->stream) free_streams.emplace_back(j->stream, j->ev);
  j->ev = nullptr;
  j->stream = nullptr;
  auto it = sectors.find(j->sector_key);
  if (j->holds_sector && it != sectors.end()) it->second.users--;
  j->holds_sector = false;
  used -= (int64_t)j->footprint;
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
  while (true) {
    // retire finished jobs
    for (size_t i = 0; i < running.size();) {
      auto& j = running[i];
      if (hipEventQuery(j->ev) == hipSuccess) {
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
    // admit queued jobs
    std::vector<std::shared_ptr<Job>> pending;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stop && queue.empty() && running.empty()) break;
      for (int64_t id : queue) pending.push_back(jobs[id]);
    }
    bool head_blocked = false;
    std::vector<Job*> refused;
    for (auto& j : pending) {
      if ((int)running.size() >= max_active) break;
      // A job that has been overtaken kMaxOvertake times blocks the queue
      // behind it until it is admitted, so large jobs are not starved.
      if (head_blocked) break;
      bool cancelled;
      {
        std::lock_guard<std::mutex> lk(mu);
        cancelled = j->cancel || stop;
      }
      bool taken;
      if (cancelled) {
        j->msg = "cancelled";
        retire(j, FTLM_ERR_CANCELLED);
        taken = true;
      } else {
        taken = try_admit(j);
      }
      if (!taken) {
        refused.push_back(j.get());
      } else if (j->running) {
        for (Job* r : refused)
          if (++r->overtaken >= kMaxOvertake) head_blocked = true;
      }
      if (taken) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = queue.begin(); it != queue.end(); ++it)
          if (*it == j->id) {
            queue.erase(it);
            break;
          }
      }
    }
    std::unique_lock<std::mutex> lk(mu);
    if (running.empty() && (queue.empty() || stop)) {
      if (stop && queue.empty()) break;
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    } else {
      cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
  }
  sectors.clear();
  if (build) (void)hipStreamSynchronize(build);
  if (build) (void)hipStreamDestroy(build);
  for (auto& se : free_streams) {
    (void)hipEventDestroy(se.second);
    (void)hipStreamDestroy(se.first);
  }
  for (auto& pb : free_pinned) (void)hipHostFree(pb.second);
  free_streams.clear();
  free_pinned.clear();
}

}  // namespace ftlm

struct ftlm_server {
  std::unique_ptr<ftlm::Server> s;
};

using namespace ftlm;

namespace {
template <typename F>
int guarded_s(F&& f) {
  try {
    f();
    return FTLM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return FTLM_ERR_INVALID_ARG;
  }
}
}  // namespace

extern "C" {

int ftlm_server_create(int64_t hbm_budget_bytes, int32_t max_active, ftlm_server** out) {
  return guarded_s([&] {
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
  return guarded_s([&] {
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
  return guarded_s([&] {
    if (!h || !done) fail(FTLM_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(h->s->mu);
    auto it = h->s->jobs.find(id);
    if (it == h->s->jobs.end()) fail(FTLM_ERR_INVALID_ARG, "unknown job id");
    *done = it->second->done ? 1 : 0;
  });
}

int ftlm_server_wait(ftlm_server* h, int64_t id, ftlm_job_result* res, double* alpha, double* beta, int32_t* nsteps) {
  int status = FTLM_OK;
  int rc = guarded_s([&] {
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
  return guarded_s([&] {
    if (!h) fail(FTLM_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(h->s->mu);
    auto it = h->s->jobs.find(id);
    if (it == h->s->jobs.end()) fail(FTLM_ERR_INVALID_ARG, "unknown job id");
    it->second->cancel = true;
    h->s->cv_work.notify_all();
  });
}

int ftlm_server_stats(ftlm_server* h, int64_t* used_bytes, int32_t* running, int32_t* queued) {
  return guarded_s([&] {
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
