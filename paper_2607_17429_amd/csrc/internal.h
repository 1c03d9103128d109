// Internal objects behind the opaque C handles.
#pragma once

#include <array>
#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "group.h"

struct ftlm_group {
  std::shared_ptr<ftlm::Group> G;
};

namespace ftlm {

// Irreducible-representation-independent tables of one M sector.
struct Sector {
  std::shared_ptr<const Group> G;
  // cluster
  int N = 0, two_s = 0, d = 0, bits = 0, two_M = 0, A = 0;
  std::vector<int32_t> bonds;   // 2 * nbonds
  std::vector<double> J;
  int nbonds = 0;
  bool wide = false;            // labels need 64 bits (N * bits > 32)
  int nch = 0;                  // 4-bit chunks of a packed label
  bool zflip = false;           // M = 0 resolved by G x Z2 (global spin flip)
  uint64_t full = 0;            // packed label with every digit d - 1
  int gorder = 0;               // |G|, or 2|G| with the spin flip (element (g, f) = f|G| + g)
  uint64_t D_M = 0, n_reps = 0, n_words = 0;
  int hv_mode = FTLM_HV_ENTRIES;
  uint64_t cluster_hash = 0;    // sizes, bonds, couplings, group elements, spin flip (autotuner key)
  // host copies of small tables
  std::vector<uint64_t> cnt;    // (N+1) x (Amax+1) digit-sum counts
  int cnt_stride = 0;
  std::vector<uint16_t> stab_size;               // per stabilizer id
  std::vector<uint64_t> stab_count;              // representatives per stabilizer id
  std::vector<std::vector<int32_t>> stab_elems;  // per stabilizer id
  int32_t n_stab = 0;
  // device tables
  // chunk tables of the factored group G = T H: (|H| + |T|) x nch x 16 words
  // (uint32 or uint64 payload), then |T| x |H| uint16 element indices
  DevBuf<uint64_t> d_tab;
  int fac_nH = 1, fac_nT = 1;
  uint32_t tab_words = 0;       // in payload words
  DevBuf<uint64_t> d_cnt;
  DevBuf<uint64_t> d_rank_bits; // bitmap over sector ranks
  DevBuf<uint32_t> d_rank_base; // representatives before each word
  DevBuf<uint64_t> d_reps;      // packed labels, ascending
  DevBuf<uint16_t> d_stab_id;
  DevBuf<double> d_ediag;       // Eq. (16) per representative
  DevBuf<uint64_t> d_row_ptr;   // entries of representative i: [row_ptr[i], row_ptr[i+1])
  // entries of a flip: target index, connecting element h, flip id 2*bond + sign,
  // and a bit set when the target's stabilizer is trivial; 8-byte form
  // idx | h << 32 | flip << 48 | trivial << 63, or the 6-byte split form
  // (eidx = idx, ehc = h | flip << ent_hbits | trivial << 15) when h and flip fit 15 bits
  DevBuf<uint64_t> d_entries;
  DevBuf<uint32_t> d_eidx;
  DevBuf<uint16_t> d_ehc;
  int entry_bytes = 8, ent_hbits = 16;
  int trivial_sid = 0;          // stabilizer id of the trivial stabilizer {e}
  uint64_t n_entries = 0;
  DevBuf<int32_t> d_bonds;
  DevBuf<double> d_J;
  DevBuf<double> d_fac;         // [2][d][d] ladder products (J = 1)
  int64_t device_bytes() const {
    return (int64_t)(d_tab.bytes() + d_cnt.bytes() + d_rank_bits.bytes() + d_rank_base.bytes() +
                     d_reps.bytes() + d_stab_id.bytes() + d_ediag.bytes() + d_row_ptr.bytes() +
                     d_entries.bytes() + d_eidx.bytes() + d_ehc.bytes() + d_bonds.bytes() + d_J.bytes() +
                     d_fac.bytes());
  }
};

struct Block {
  std::shared_ptr<Sector> sec;  // shared with other blocks of the sector
  std::shared_ptr<Group> own_group;
  int irrep = 0, row = 0, dg = 0;
  int weight = 0;               // trace weight in the thermal sums (dg, or dg / 2 for a realified pair)
  int dgp = 0;                  // kernel dimension bucket (tables zero-padded to it)
  uint64_t D = 0, n_active = 0;
  uint64_t D_pad = 0;           // n_reps * dg: rows of the padded vector layout
  double fpar = 1.0;            // spin-flip parity of the irrep (G x Z2 sectors)
  int lanczos_layout = FTLM_LAYOUT_AUTO;
  std::vector<double> rho;      // |G| x d x d (the irrep used)
  std::vector<uint8_t> n_stab;  // n_Gamma per stabilizer id
  std::vector<double> V_stab;   // per stabilizer: d x d (columns k < n valid, rest 0)
  std::vector<double> L_stab;   // orbit length per stabilizer id
  std::vector<uint8_t> trivial; // V = identity and n = d
  // device
  DevBuf<uint64_t> d_meta;      // per representative: offset | stab_id << 48
  DevBuf<double> d_rhoT64;      // [g][beta][gamma] = rho(g)[gamma][beta]
  DevBuf<double> d_V64;         // [s][gamma][k]
  DevBuf<double> d_stabf64;     // [s]: {n, sqrtL, 1/sqrtL, trivial}
  int64_t device_bytes() const {
    return (int64_t)(d_meta.bytes() + d_rhoT64.bytes() + d_V64.bytes() + d_stabf64.bytes()) +
           sec->device_bytes();
  }
};

std::shared_ptr<Sector> build_sector(const ftlm_cluster* cl, std::shared_ptr<const Group> G, int two_M,
                                     const ftlm_opts* opts);
void sector_canonicalize(const Sector& s, const uint64_t* labels, int64_t n, uint64_t* rep, int32_t* h,
                         int64_t* index, hipStream_t stream);
std::vector<uint64_t> sector_export_labels(const Sector& s);

std::unique_ptr<Block> build_block(std::shared_ptr<Sector> sec, int irrep, int row, const ftlm_opts* opts);
void block_hv_stats(const Block& b, ftlm_hv_stats* st);

// H.V (Eq. 15 in gather form + Eq. 16).  Optional Lanczos epilogue: when
// lz != nullptr the output is w = s_j H q_j - bs_j q_prev written over q_prev
// (== Y) and per-workgroup FP64 partial sums of q_j . w are produced.
struct LanczosEpilogue {
  const double* scal;   // per vector: [s_j, beta_j * s_{j-1}] pairs
  double* partials;     // n_groups x nvec
  int n_groups;
  double eshift = 0.0;  // the pass applies H - eshift (Chebyshev recursion); 0 for Lanczos
};
void apply_hv(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, hipStream_t stream,
              const LanczosEpilogue* lz = nullptr);

// Row layout of stored vectors: the block's rows, or d_Gamma rows per
// representative (padded), optionally packed p = rpl representatives to a
// 128-byte line of rpline rows (enum ftlm_layout).
struct VecLayout {
  bool pad = false;
  bool aligned = false; // rpline (a power of two > d_Gamma) rows per representative
  uint32_t rpl = 1;     // representatives per line (1: plain padded)
  uint32_t rpline = 0;  // rows per line when rpl > 1, rows per representative when aligned
  int kind() const {
    return !pad ? FTLM_LAYOUT_BLOCK : aligned ? FTLM_LAYOUT_ALIGNED : rpl > 1 ? FTLM_LAYOUT_PACKED : FTLM_LAYOUT_PADDED;
  }
};
// kind BLOCK, PADDED, PACKED or ALIGNED (PACKED and ALIGNED fall back to
// PADDED where they do not apply) for rows of row_bytes bytes
VecLayout vec_layout(const Block& b, int kind, int64_t row_bytes);
// the layout ftlm_run and ftlm_kpm take for this block and row size
VecLayout run_layout(const Block& b, int64_t row_bytes);
uint64_t vec_rows(const Block& b, const VecLayout& v);
namespace dev {
struct PadMap;
}
// the device row map of a padded layout
dev::PadMap pad_map(const Block& b, const VecLayout& v);

// Lane layout: lanes per output representative for (nvec, dtype) (autotuned
// or default), the partial-sum groups of that layout, and H.V with it fixed.
// The autotuner keys its choice by the row layout (pad) and by whether the
// Lanczos epilogue runs (epi).
int hv_layout_lanes(const Block& b, int nvec, int dtype, const VecLayout& vl, bool epi);
int hv_partial_groups(const Block& b, int nvec, int gl);
// vl: row layout of X and Y (default: block rows).
// shift: the plain pass (lz == nullptr) applies H - shift.
void apply_hv_gl(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, hipStream_t stream,
                 const LanczosEpilogue* lz, int gl, const VecLayout& vl = VecLayout{}, double shift = 0.0);

// ftlm_apply_H_ex: the launch decided on the host (row layout, lane layout,
// partial-sum groups of the epilogue, whether the adjacent-column kernel runs)
// and the enqueue with caller-provided scratch for the partials (p.ng * nvec
// doubles when p.epi).
struct HvExPlan {
  VecLayout vl;
  bool epi = false, adjacent = false;
  int gl = 0, ng = 0;
  uint64_t rows = 0;
};
HvExPlan plan_hv_ex(const Block& b, int nvec, int64_t ld, int dtype, const ftlm_hv_opts* o);
void apply_hv_ex(const Block& b, const void* X, void* Y, int nvec, int64_t ld, int dtype, const ftlm_hv_opts* o,
                 const HvExPlan& p, double* partials, hipStream_t st);

// Whether vectors of the block take the padded row layout (d_Gamma rows per
// representative, zeros beyond n_Gamma): the block's lanczos_layout, or for
// FTLM_LAYOUT_AUTO blocks of at least 2^20 rows that pad by at most 2%.
bool padded_vectors(const Block& b);
// Times every lane layout for (nvec, dtype) on this block, caches the fastest
// process-wide and returns (lanes per representative, ms per launch) pairs.
std::vector<std::pair<int, double>> autotune_hv(const Block& b, int nvec, int dtype, hipStream_t st, int reps,
                                                const VecLayout& vl, bool epi);
int irrep_dim_bucket(int d);
// gcnArchName of the current device
std::string device_arch();

// One batched Lanczos run of R chains on a block: device state, an enqueue of
// every kernel on one stream (no host synchronisation) and an asynchronous
// copy of alpha, beta and the per-chain step counts.
struct LanczosRun {
  const Block* block;
  int R, steps, storage, dist;
  uint64_t seed;
  int target = 0, TB = 0, nb_vec = 0, gl = 0, ng_hv = 0;
  int first_chain = 0;           // chain keys start at this chain index
  VecLayout vl;                  // row layout of the stored vectors
  double sigma = 1.0;            // power-of-two storage scale of the vectors (FP16)
  uint64_t rows = 0;             // rows of each stored vector
  // optional timing of the H.V launches (two events per step)
  std::vector<hipEvent_t> hv_events;
  bool timed = false;
  // replayable graph of an even and an odd step (captured on first use)
  bool use_graphs = true;
  hipGraph_t pair_graph = nullptr;
  hipGraphExec_t pair_exec = nullptr;
  DevBuf<uint8_t> q0, q1, chain;
  DevBuf<uint64_t> keys;
  DevBuf<double> partials, inv_norm, scal, d_alpha, d_beta;
  DevBuf<int32_t> d_n;
  LanczosRun(const Block& b, int R, int steps, uint64_t seed, int storage, int dist);
  static size_t estimate_bytes(const Block& b, int R, int steps, int storage);
  void allocate();                 // device buffers (stream-ordered if an allocation stream is set)
  void enqueue(hipStream_t st);    // begin + all steps + end
  void enqueue_begin(hipStream_t st);                  // clear outputs, start vectors
  void enqueue_steps(hipStream_t st, int j0, int j1);  // Lanczos steps j0 <= j < min(j1, target)
  void enqueue_end(hipStream_t st);                    // per-chain step counts
  void enable_timing();
  double hv_ms() const;          // after the stream has finished
  ~LanczosRun();
  void download(hipStream_t st, double* alpha, double* beta, int32_t* nsteps);
  // Checkpoint: the whole device state after `next_step` steps (both vectors,
  // per-chain state, coefficients so far) to a file, and a run rebuilt from
  // one on a block that must be the same (cluster, sector, irrep, row, rows).
  void save(const char* path, hipStream_t st, int next_step) const;
  static std::unique_ptr<LanczosRun> load(const Block& b, const char* path, hipStream_t st, int& next_step);
};

void run_lanczos(Block& b, int R, int steps, uint64_t seed, int storage, int dist, double* alpha,
                 double* beta, int32_t* nsteps, hipStream_t stream, ftlm_run_info* info = nullptr);

// Fused small-block Lanczos: one workgroup runs every step of one block job.
// wg_supported: the kernel can run R chains of this block in this storage
// (FP64 or FP32, entry-table H.V, irrep tables in LDS, R <= 32); wg_rounds:
// representatives per lane group and step in a sector of n_reps
// representatives, the job's serial length.
bool wg_supported(const Block& b, int R, int storage);
uint64_t wg_rounds(uint64_t n_reps, int R);
// automatic engine choice: blocks whose sector needs at most this many
// representative rounds per lane group and step go to the fused kernel
constexpr uint64_t kWgAutoMaxRounds = 8;
// chains one fused job can hold (one column per lane group slot)
constexpr int kWgMaxChains = 32;
struct WgTask {
  const Block* block;            // must outlive the batch
  int R, steps, storage, dist, first_chain;
  uint64_t seed;
  double* alpha;                 // host outputs: R x steps, R x steps, R
  double* beta;
  int32_t* nsteps;
};
// A batch of jobs enqueued on one stream at construction (one launch per
// kernel shape); finish() waits and fills every task's outputs.
struct WgBatch {
  std::vector<WgTask> tasks;
  hipStream_t st = nullptr;
  DevBuf<uint8_t> arena;
  struct Pinned {                   // pinned upload buffer (job structs, keys)
    void* p = nullptr;
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } staging;
  std::vector<std::array<size_t, 3>> res;
  size_t up_bytes = 0, out_off = 0, out_bytes = 0;
  bool launched = false;
  WgBatch(std::vector<WgTask> tasks, hipStream_t st);
  WgBatch(const WgBatch&) = delete;
  WgBatch& operator=(const WgBatch&) = delete;
  void finish();
  // One job only: enqueue the copy of its alpha | beta | nsteps (the layout
  // of contiguous host arrays R x steps, R x steps, R) into host memory
  // (pinned for an asynchronous copy); the caller synchronizes st.
  void enqueue_download(void* host, size_t bytes);
  // Any number of jobs: enqueue the copy of the whole output region
  // (out_bytes) into host memory; job i's alpha, beta and nsteps then sit at
  // byte offsets res[i][0..2] of it once st has passed the copy.
  void enqueue_download_all(void* host, size_t bytes);
  template <typename Groups, typename Offsets, typename Shm>
  void launch_groups(const Groups& groups, const Offsets& goff, const Shm& shm);
  ~WgBatch();
};

void run_kpm(Block& b, int R, int M, uint64_t seed, int storage, int dist, double center, double half_width,
             double* moments, hipStream_t st);
void kpm_observables(const ftlm_kpm_block* blocks, int nb, const double* T, int nT, double g, int n_nodes, double* E,
                     double* C, double* chi, double* logZ);

void tridiag_ritz(const double* alpha, const double* beta, int n, double* theta, double* weight);
void observables(const ftlm_ritz* blocks, int nb, const double* T, int nT, double g, double* E, double* C,
                 double* chi, double* logZ);

uint64_t chain_key(uint64_t seed, int two_M, int irrep, int row, int chain);

void run_campaign(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, const ftlm_campaign_opts* o,
                  const double* T, int nT, double* E, double* C, double* chi, double* logZ,
                  ftlm_campaign_stats* st);

// exclusive prefix sum over n values of a device array (uint64 in/out, in-place allowed)
void scan_exclusive_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* total, hipStream_t s);

}  // namespace ftlm

struct ftlm_sector {
  std::shared_ptr<ftlm::Sector> s;
};

struct ftlm_block {
  std::unique_ptr<ftlm::Block> b;
};

struct ftlm_run_state {
  ftlm::Block* block = nullptr;               // the caller's block (must outlive the state)
  std::unique_ptr<ftlm::LanczosRun> run;
  hipStream_t st = nullptr;
  int next_step = 0;
};
