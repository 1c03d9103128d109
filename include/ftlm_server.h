/*
 * ftlm_server.h -- continuous-batching FTLM job server on top of ftlm.h.
 *
 * A job is one block run (Section 3 of the paper: R chains, N_L steps, on one
 * (M, Gamma, row) block): cluster, generators, 2M, irrep, row, R, steps, seed,
 * storage and start-vector distribution.  Jobs wait in a FIFO queue and are
 * admitted while a slot is free (max_active slots) and their estimated
 * device footprint (vectors of the run, block tables, and the sector tables
 * unless already resident) fits in hbm_budget_bytes; a later job that fits may
 * overtake one that does not, until that one has been overtaken 64 times and
 * then holds back the queue behind it (nothing behind it is admitted until it
 * is).  Jobs with long steps (about 1 ms or more of estimated device time
 * per Lanczos step) take at most max_active - 2 slots when max_active > 2, so
 * short jobs always find a slot; such a job waiting only for that reason is
 * counted as overtaken by later long-step jobs, not by the short ones.  Small jobs (sectors of a few hundred representatives, R <= 32, FP64
 * or FP32 storage) admitted in the same pass over the queue, while no job
 * with long steps (about 1 ms or more of estimated device time) is running,
 * run together as one batch of the fused small-block kernel
 * (ftlm_run_fused: one launch per kernel shape, one workgroup per job, up to
 * 64 jobs), which takes one slot; a small job admitted alone, or next to a
 * long-step job, runs the per-step kernels, which are faster for one job and
 * interleave with long launches.  Sector tables are built with the entry table (FTLM_HV_ENTRIES),
 * whose size the admission estimate counts.  A job whose estimate alone exceeds
 * hbm_budget_bytes ends with FTLM_ERR_OUT_OF_MEMORY.  Sector tables are cached and shared by all
 * jobs with the same (cluster, generators, 2M); unused ones are evicted when
 * memory is needed.  Groups and sector tables are built by a builder thread
 * of the server, one at a time, while the worker thread keeps admitting and
 * retiring jobs whose tables are resident; a job waiting for a build holds
 * nobody up.  Every admitted job runs on its own non-blocking HIP stream, so
 * work of different jobs overlaps on the device; its Lanczos steps are
 * enqueued in chunks of about 10 ms of estimated device time, so a long job
 * holds a hardware queue shared with other streams for at most one chunk
 * ahead of their work; with at least max_active + 2 hardware queues per
 * process (the HIP runtime's GPU_MAX_HW_QUEUES, read when it starts) no
 * stream shares one, and short jobs do not wait behind long ones at all.  A job may ask for the fused small-block kernel
 * (ftlm_run_fused); it then joins the batch of its pass.  A job's result does
 * not depend on the other jobs (no shared reductions, deterministic kernels,
 * and a job's result in a fused batch does not depend on the batch).  The two server threads own
 * every HIP call of the server; the calls below are thread-safe.
 */
#ifndef FTLM_SERVER_H
#define FTLM_SERVER_H

#include "ftlm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftlm_server ftlm_server;

typedef struct ftlm_job_desc {
  ftlm_cluster cluster;
  const int32_t* gens;   /* ngens x N site permutations */
  int32_t ngens;
  int32_t two_M;
  int32_t irrep;         /* index in the library's irrep order */
  int32_t row;
  int32_t R;             /* chains, 1..256 */
  int32_t steps;         /* Lanczos steps per chain */
  uint64_t seed;
  int32_t storage;       /* FTLM_F64 or FTLM_F32 */
  int32_t dist;          /* FTLM_RADEMACHER or FTLM_GAUSSIAN */
  int32_t engine;        /* enum ftlm_engine: AUTO batches small jobs admitted together into the
                            fused small-block kernel and runs every other job with the per-step
                            kernels; STEPS always runs the per-step kernels; FUSED always runs
                            the fused kernel, batched with the small jobs of its pass
                            (INVALID_ARG where it does not apply, see ftlm_run_fused) */
  int32_t reserved;
} ftlm_job_desc;

typedef struct ftlm_job_result {
  int32_t status;        /* FTLM_OK or the job's error */
  int32_t R;
  int32_t steps;
  int32_t d_gamma;
  uint64_t D;            /* block dimension */
  double submit_s;       /* seconds since the server started */
  double start_s;        /* admission */
  double end_s;          /* results on the host */
  int32_t engine;        /* FTLM_ENGINE_STEPS or FTLM_ENGINE_FUSED: the path the job took.  Its
                            coefficients equal, bit for bit, those of ftlm_run (STEPS) or
                            ftlm_run_fused (FUSED) on the same block */
  int32_t reserved;
} ftlm_job_result;

/* Starts the worker thread on the current device.  Errors: INVALID_ARG. */
int ftlm_server_create(int64_t hbm_budget_bytes, int32_t max_active, ftlm_server** out);
/* Copies the job description and its arrays; returns a job id >= 0. */
int ftlm_server_submit(ftlm_server* s, const ftlm_job_desc* job, int64_t* job_id);
/* Blocks until the job has ended and releases it; alpha and beta (R x steps,
 * beta[r][j] = beta_{j+1}) and nsteps (R) may be NULL.  Returns the job's
 * status (also in res->status); for a failed job ftlm_last_error() on the
 * calling thread returns its message.  Errors: INVALID_ARG for an unknown id. */
int ftlm_server_wait(ftlm_server* s, int64_t job_id, ftlm_job_result* res, double* alpha, double* beta,
                     int32_t* nsteps);
/* Non-blocking: 1 when the job has ended, 0 otherwise. */
int ftlm_server_poll(ftlm_server* s, int64_t job_id, int32_t* done);
/* A queued job ends with FTLM_ERR_CANCELLED; a running one is released as
 * soon as its kernels finish and also ends CANCELLED. */
int ftlm_server_cancel(ftlm_server* s, int64_t job_id);
/* Device bytes held by running jobs and cached sectors, running jobs,
 * queued jobs. */
int ftlm_server_stats(ftlm_server* s, int64_t* used_bytes, int32_t* running, int32_t* queued);
/* Cancels queued jobs, waits for running ones, frees everything. */
void ftlm_server_free(ftlm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* FTLM_SERVER_H */
