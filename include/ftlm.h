/*
 * ftlm.h -- C ABI of the MI355X symmetry-adapted finite-temperature Lanczos
 * library (spin-s Heisenberg clusters with site-permutation symmetry).
 *
 * The operations follow the paper "GPU-accelerated finite-temperature Lanczos
 * method for Heisenberg spin systems with non-Abelian permutation symmetries":
 *   - H of Eq. (1) with the spin-flip coefficients of Eq. (3); states are the
 *     integer labels n = sum_k (m_k + s) d^k of Eq. (2), d = 2s + 1.
 *   - One (M, Gamma, row) block of the symmetry-adapted basis of Eq. (12):
 *     orbit representatives (smallest label of each orbit, Section 2.3),
 *     stabilizers (Eq. 8), n_Gamma and V_r (Eqs. 10-11), D = sum n_Gamma (Eq. 13).
 *   - Matrix-free H action through the matrix element of Eq. (15) in gather
 *     form, diagonal of Eq. (16).
 *   - Batched Lanczos chains with start vectors per chain (Section 2.2, 3),
 *     host FP64 tridiagonal Ritz data, thermal sums of Eqs. (4)-(7), (14).
 *
 * Conventions shared by every call
 *   status: 0 = FTLM_OK, negative = error; ftlm_last_error() returns a
 *           thread-local description of the last error on the calling thread.
 *   group elements: the closure of the generators sorted lexicographically by
 *           permutation image array (identity = element 0).  A permutation
 *           array p means: the spin on site k moves to site p[k]; products
 *           compose as (gh)[k] = g[h[k]].
 *   irreps: ordered by dimension, then by the character vector (classes in
 *           the order element order, class size, smallest member) descending.
 *   block rows: representatives in ascending label order, then k = 0..n-1.
 *   vectors: row-major D x ld arrays on the device, column v = chain / vector
 *           (the fastest index), v < nvec <= ld.
 *   streams: hipStream_t passed as void*; NULL = the null stream.
 *   ownership: the library owns groups, sectors and blocks (device tables
 *           included) until the matching *_free; the caller owns every
 *           pointer it passes in.  Objects are not thread-safe; a built block
 *           may be read concurrently by apply calls on several streams.
 */
#ifndef FTLM_H
#define FTLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ftlm_status {
  FTLM_OK = 0,
  FTLM_ERR_INVALID_ARG = -1,
  FTLM_ERR_NOT_A_PERMUTATION = -2,
  FTLM_ERR_GROUP_TOO_LARGE = -3,
  FTLM_ERR_BONDS_NOT_INVARIANT = -4,
  FTLM_ERR_IRREP_OUT_OF_RANGE = -5,
  FTLM_ERR_ROW_OUT_OF_RANGE = -6,
  FTLM_ERR_DIM_GT_12 = -7,
  FTLM_ERR_COMPLEX_IRREP_UNSUPPORTED = -8, /* the group's real irreps do not cover all of its irreps */
  FTLM_ERR_OUT_OF_MEMORY = -9,
  FTLM_ERR_HIP = -10,
  FTLM_ERR_BAD_RHO = -11,
  FTLM_ERR_UNSUPPORTED = -12,
  FTLM_ERR_IRREPS_FAILED = -13,
  FTLM_ERR_CANCELLED = -14,
  FTLM_ERR_QUEUE_FULL = -15
};

/* Storage type of vectors.  Arithmetic is FP64 for every storage type: F32
 * and F16 values are widened when read and rounded once when stored.  In
 * ftlm_run, F16 vectors carry a per-chain power-of-two scale that keeps their
 * elements of order one (FP16 normals start at 6.1e-5). */
enum ftlm_dtype { FTLM_F64 = 0, FTLM_F32 = 1, FTLM_F16 = 2 };
enum ftlm_dist { FTLM_RADEMACHER = 0, FTLM_GAUSSIAN = 1 };
enum ftlm_hv_mode { FTLM_HV_AUTO = 0, FTLM_HV_ENTRIES = 1, FTLM_HV_ONTHEFLY = 2 };

/* Cluster graph of Eq. (1): N sites of spin s = two_s/2, nbonds bonds
 * (bonds[2b], bonds[2b+1]) with couplings J[b] (J == NULL: all 1). */
typedef struct ftlm_cluster {
  int32_t N;
  int32_t two_s;
  int32_t nbonds;
  const int32_t* bonds;
  const double* J;
} ftlm_cluster;

/* Build options (every field 0 / NULL = default). */
/* Row layout of the Lanczos vectors that ftlm_run keeps on the device.
 * BLOCK: the block's own rows (representative i at its offset, n_Gamma(i)
 * rows).  PADDED: d_Gamma rows per representative (representative i at
 * i * d_Gamma, rows k >= n_Gamma(i) held at zero), so the H.V finds a
 * target's rows without reading its offset.  PACKED: PADDED with the
 * representatives packed into 128-byte lines so that none straddles two:
 * with rows of b bytes (b divides 128) and L = 128 / b rows per line, p =
 * floor(L / d_Gamma) representatives share a line, representative i starts
 * at row (i / p) L + (i % p) d_Gamma, and the L - p d_Gamma rows left in a
 * line are held at zero (it applies when 2 <= p and p d_Gamma < L; otherwise
 * it is PADDED).  A random gather of a representative's rows then reads one
 * 128-byte line instead of 1.25 on average for 40-byte slices: fewer bytes,
 * the same number of random accesses.  ALIGNED: PADDED with S rows per
 * representative, S the smallest power of two >= d_Gamma (representative i
 * at row i * S, rows k >= n_Gamma(i) held at zero); it applies when the row
 * size b is a power of two, S > d_Gamma and S b <= 128 (otherwise it is
 * PADDED).  Each representative's rows then fill one naturally aligned block
 * of S b bytes, for S / d_Gamma times the rows.  Neither PACKED nor ALIGNED
 * measured faster than PADDED (s = 3/2 dodecahedron H_g block, 2 FP32
 * vectors), so AUTO takes neither.  AUTO: PADDED when
 * D >= 2^20 and the padding adds at most 2% rows, BLOCK otherwise.  The
 * layout changes only the summation order of the FP64 reductions, not what
 * is computed. */
enum ftlm_layout {
  FTLM_LAYOUT_AUTO = 0,
  FTLM_LAYOUT_BLOCK = 1,
  FTLM_LAYOUT_PADDED = 2,
  FTLM_LAYOUT_PACKED = 3,
  FTLM_LAYOUT_ALIGNED = 4
};

/* Storage of the sector's entry table (one entry per flip: target index,
 * connecting element, flip id, trivial-target bit).  WIDE: 8 bytes.
 * COMPACT: 6 bytes (u32 target + u16 rest), needs |G| and the flip count to
 * fit 15 bits together; it saves memory but costs a second load per entry.
 * AUTO: WIDE unless the wide table would take more than a quarter of the
 * free device memory and COMPACT is possible. */
enum ftlm_entry_format { FTLM_ENTRIES_AUTO = 0, FTLM_ENTRIES_WIDE = 1, FTLM_ENTRIES_COMPACT = 2 };

typedef struct ftlm_opts {
  int32_t hv_mode;          /* enum ftlm_hv_mode; AUTO keeps an entry table when it fits */
  int32_t lanczos_layout;   /* enum ftlm_layout: rows of the Lanczos vectors inside ftlm_run
                               (block options; ignored by sector creation) */
  const double* user_rho;   /* optional irrep matrices, |G| x d x d row-major, element
                               order as above; replaces the library's own irrep */
  int32_t user_rho_dim;     /* d of user_rho (0 = none) */
  int32_t entry_format;     /* enum ftlm_entry_format (sector creation) */
  int64_t hbm_limit_bytes;  /* 0 = no limit; builds that would exceed it fail with
                               FTLM_ERR_OUT_OF_MEMORY before allocating */
  int32_t spin_flip;        /* sector creation: 1 = resolve the M = 0 sector by the global
                               spin flip F (every digit a -> d-1-a) as well, i.e. by
                               G x Z2.  Its element (g, f) acts as U(g) F^f and has index
                               f|G| + g (connecting elements h reach 2|G| - 1); the irreps
                               of its blocks are Gamma_i^+ and Gamma_i^- at indices 2i and
                               2i + 1, rho'(g, f) = (+-1)^f rho_i(g) (user_rho then gives
                               rho_i on G).  INVALID_ARG unless 2M = 0. */
  int32_t user_rho_weight;  /* block creation with user_rho: trace weight of the block in
                               the thermal sums (0 = user_rho_dim; user_rho_dim / 2 for the
                               real form of a complex pair) */
  int64_t reserved[5];
} ftlm_opts;

typedef struct ftlm_group ftlm_group;
typedef struct ftlm_sector ftlm_sector;
typedef struct ftlm_block ftlm_block;

/* ---------------------------------------------------------------- group ---
 * Closure of ngens site permutations (ngens x N int32, row-major) into the
 * full group (Section 3: closure, irreps from the regular representation,
 * real orthogonal form for Frobenius-Schur indicator +1, verification of
 * unitarity, character orthogonality and sum d^2 = |G|).  Host only.
 * Errors: NOT_A_PERMUTATION, GROUP_TOO_LARGE (|G| > 65535), IRREPS_FAILED.
 *
 * The library's irreps are real: an irrep of complex type (indicator 0) and
 * its conjugate are listed once, together, as a real orthogonal
 * representation of dimension 2d (indicator reported as 0), irreducible over
 * the reals.  Its row block (any row) is the real form of the complex block
 * of either member of the pair: twice its dimension, every level twice; in
 * the thermal sums it carries the trace weight d = dim / 2 (ftlm_ritz.d_gamma).
 * An irrep of quaternionic type (indicator -1, d even) is listed as its
 * realification, a real orthogonal representation of dimension 2d
 * (indicator reported as -1), irreducible over the reals; its row block is
 * again the real form of the complex block and carries the trace weight
 * d / 2 = dim / 4.  This replaces the paper's complex-arithmetic path.
 * Irreps are computed for |G| <= 1024. */
int ftlm_group_create(int32_t N, const int32_t* gens, int32_t ngens, ftlm_group** out);
/* |G|, number of irreps, number of conjugacy classes, number of sites (the
 * group and its irreps generated and verified as Section 3 describes). */
int ftlm_group_info(const ftlm_group* g, int32_t* order, int32_t* n_irreps, int32_t* n_classes,
                    int32_t* N);
/* Permutation table, |G| x N int32 (host array owned by the caller): the
 * site-permutation table through which the group enters (Section 3). */
int ftlm_group_elements(const ftlm_group* g, int32_t* perms);
/* Per irrep: dimension, Frobenius-Schur indicator (0 marks a realified
 * complex pair, -1 a realified quaternionic irrep, +1 a real-type irrep),
 * trace weight in the thermal sums of Eq. (14) (the d_Gamma factor: dim for
 * a real-type irrep, dim / 2 for a realified complex pair, dim / 4 for a
 * realified quaternionic irrep; the block's ftlm_block_info.trace_weight),
 * characters of the real form by class (n_irreps x n_classes, row-major) and
 * the class of every element (|G|).  Any pointer may be NULL.  Also the
 * largest verification residual. */
int ftlm_group_irreps(const ftlm_group* g, int32_t* dims, int32_t* indicators, int32_t* weights,
                      double* chars, int32_t* class_of, double* max_residual);
/* Irrep matrices rho(g), |G| x d x d row-major (host array owned by the
 * caller): the rho_Gamma(g) of Eqs. (10) and (15), in real orthogonal form. */
int ftlm_group_rho(const ftlm_group* g, int32_t irrep, double* rho);
void ftlm_group_free(ftlm_group* g);

/* --------------------------------------------------------------- sector ---
 * Irreducible-representation-independent part of one magnetization sector
 * (Section 3: built once per magnetization sector, shared by its irreps): all orbit
 * representatives of the M = two_M/2 sector (ascending), their stabilizers,
 * the rank lookup (sector rank of Ref. [36] + a bitmap over ranks), the
 * diagonal energies of Eq. (16) and, in entry mode, the table of one entry
 * per admissible (representative, bond, sign) flip: target representative,
 * connecting element h with U(h) a = min O(a) (smallest index among
 * minimisers) and the flip.  Built on the device with the GPU kernels.
 * Errors: INVALID_ARG (N*bits > 64, bad bonds/spin), BONDS_NOT_INVARIANT,
 * OUT_OF_MEMORY, HIP.  A sector with no states is legal (n_reps = 0). */
int ftlm_sector_create(const ftlm_cluster* cl, const ftlm_group* g, int32_t two_M,
                       const ftlm_opts* opts, ftlm_sector** out);

typedef struct ftlm_sector_info {
  uint64_t D_M;          /* sector dimension */
  uint64_t n_reps;       /* number of orbits */
  uint64_t n_entries;    /* entry-table length (0 when not kept) */
  int32_t n_stab;        /* number of distinct stabilizers */
  int32_t label_bits;    /* packed bits per site */
  int64_t device_bytes;  /* device memory held by the sector */
} ftlm_sector_info;
int ftlm_sector_info_get(const ftlm_sector* s, ftlm_sector_info* info);
/* Host copies: representative labels of Eq. (2) (n_reps), stabilizer id per
 * representative (ids in order of first appearance), and per stabilizer its
 * size.  Any pointer may be NULL. */
int ftlm_sector_export(const ftlm_sector* s, uint64_t* reps, uint16_t* stab_id, int32_t* stab_size);
/* Device-side orbit search and lookup for n labels of Eq. (2) (device arrays):
 * rep = min O(a), h = smallest element index with U(h) a = rep, index = the
 * representative's position (-1 if a is not in the sector).  Enqueued on
 * stream. */
int ftlm_sector_canonicalize(const ftlm_sector* s, const uint64_t* labels, int64_t n, uint64_t* rep,
                             int32_t* h, int64_t* index, void* stream);
void ftlm_sector_free(ftlm_sector* s);

/* ---------------------------------------------------------------- block ---
 * One (M, Gamma, row) block on top of a sector (Section 2.3): n_Gamma and
 * V_S per stabilizer (V_S by modified Gram-Schmidt over the columns of
 * (1/|S|) sum_{h in S} rho(h), columns with residual < 1e-8 dropped), row
 * offsets, and device copies of rho and V_S.  The row never changes H (the
 * per-row blocks are identical, Section 2.3); it is recorded and checked.
 * The sector must outlive the block.  Errors: IRREP_OUT_OF_RANGE,
 * ROW_OUT_OF_RANGE, DIM_GT_12, COMPLEX_IRREP_UNSUPPORTED, BAD_RHO (user_rho
 * not a unitary homomorphism), OUT_OF_MEMORY, HIP.  D = 0 is legal. */
int ftlm_block_create(ftlm_sector* s, int32_t irrep, int32_t row, const ftlm_opts* opts,
                      ftlm_block** out);
/* One call: group + sector + block of Eqs. (8)-(13) (the block owns the
 * private group and sector).  gens: ngens x N int32. */
int ftlm_build_block(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, int32_t two_M,
                     int32_t irrep, int32_t row, const ftlm_opts* opts, ftlm_block** out);

typedef struct ftlm_block_info {
  uint64_t D_M;          /* sector dimension */
  uint64_t n_reps;       /* orbits in the sector */
  uint64_t n_active;     /* representatives with n_Gamma > 0 */
  uint64_t D;            /* block dimension, Eq. (13) */
  int32_t d_gamma;       /* irrep dimension */
  int32_t group_order;
  int32_t two_M;
  int32_t irrep;
  int32_t row;
  int32_t hv_mode;       /* mode actually used by apply */
  int64_t device_bytes;  /* device memory of block + sector */
  int32_t trace_weight;  /* d_Gamma in the thermal sums: d_gamma, or d_gamma / 2 for a
                            realified complex pair (library irreps) or as given by
                            ftlm_opts.user_rho_weight */
  int32_t reserved;
} ftlm_block_info;
int ftlm_block_info_get(const ftlm_block* b, ftlm_block_info* info);
/* Host copies (n_reps each, any may be NULL): labels of Eq. (2), stabilizer
 * ids, n_Gamma, orbit lengths L_r (as double), row offsets. */
int ftlm_block_export(const ftlm_block* b, uint64_t* reps, uint16_t* stab_id, uint8_t* n_gamma,
                      double* norms, uint64_t* offsets);

/* Work counts of one H.V on this block, for the algorithmic byte model:
 * connections of active output representatives (entries read), those whose
 * target representative is active in this irrep, the rows gathered for
 * them (sum of n_Gamma(target)), how many of those targets have a
 * non-trivial stabilizer, and the size of a stored entry.  Entry mode only
 * (UNSUPPORTED otherwise).  Device reduction, synchronous. */
typedef struct ftlm_hv_stats {
  uint64_t n_active;          /* output representatives with n_Gamma > 0 */
  uint64_t connections;       /* flips of active output representatives */
  uint64_t active_connections;
  uint64_t gathered_rows;
  uint64_t nontrivial_targets; /* active connections whose target has a non-trivial stabilizer */
  int32_t entry_bytes;        /* bytes per stored flip entry (6 or 8) */
  int32_t reserved;
} ftlm_hv_stats;
int ftlm_block_hv_stats(const ftlm_block* b, ftlm_hv_stats* stats);

/* Y = H X (the block matrix of Eq. 15 in gather form, diagonal of Eq. 16)
 * for nvec columns of D x ld device arrays of dtype (F64 or F32;
 * F32 is storage only: products and sums are formed in FP64 and rounded once
 * when Y is stored).  X and Y must not overlap.  Enqueued on stream
 * (asynchronous).  Errors: INVALID_ARG, HIP. */
int ftlm_apply_H(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld, int32_t dtype,
                 void* stream);

/* Options of ftlm_apply_H_ex: the row layout and the fused Lanczos step of
 * the H.V that ftlm_run launches (Eqs. 15-16; the recurrence of Section 2.2).
 * A zeroed struct asks for the row layout ftlm_run takes on this block, the
 * tuned or default lane layout, no epilogue and no shift. */
typedef struct ftlm_hv_opts {
  int32_t layout;         /* enum ftlm_layout of X and Y.  BLOCK: D rows in block order.
                             PADDED: n_reps * d_Gamma rows, representative i at row
                             i * d_Gamma; rows k >= n_Gamma(i) of X must hold zeros, and
                             those rows of Y are not written.  PACKED: as described at
                             enum ftlm_layout with row size ld * element bytes
                             (ceil(n_reps / p) * L rows; the rows between
                             representatives hold zeros in X and are not written in Y).
                             ALIGNED: as described at enum ftlm_layout with row size
                             ld * element bytes (n_reps * S rows; rows k >= n_Gamma(i)
                             hold zeros in X and are not written in Y).
                             AUTO: the layout ftlm_run takes for this block and nvec
                             (ftlm_run_info.layout). */
  int32_t lanes;          /* lanes per output representative: a power of two 1..64, or 0
                             for the autotuned or default choice of ftlm_run */
  const double* scale;    /* device, nvec pairs (s_v, b_v), or NULL.  With it the call is
                             the first half of a Lanczos step: Y[:, v] <- s_v (H - shift)
                             X[:, v] - b_v Y[:, v] (Y read, then overwritten; FP64
                             arithmetic, one rounding to storage) */
  double* dots;           /* device, nvec doubles, or NULL (needs scale): sum over rows of
                             X[:, v] Y[:, v], Y as stored by this call, summed in FP64 in
                             a fixed order (bitwise reproducible) */
  double shift;           /* the call applies H - shift (0: H) */
  int32_t lanes_used;     /* out: lanes per representative of the launch */
  int32_t adjacent_columns; /* out: 1 when the launch ran the kernel whose lanes hold
                             adjacent columns (padded rows, d_Gamma equal to its kernel
                             bucket 1..6, nvec a whole number of column tiles): the
                             kernel of ftlm_run's large blocks */
  int64_t reserved[4];
} ftlm_hv_opts;

/* ftlm_apply_H (Eqs. 15-16) with the options above (opts == NULL: exactly
 * ftlm_apply_H); the scale/dots epilogue is one three-term Lanczos update
 * (Section 3) fused into the product.
 * dtype F64, F32 or F16 (storage; FP64 arithmetic).  X and Y must not
 * overlap.  With scale, device scratch of one FP64 partial sum per workgroup
 * and vector is allocated (stream-ordered) for the call.  Enqueued on stream
 * (asynchronous).  Errors: INVALID_ARG (bad layout, lanes, nvec or ld, dots
 * without scale), UNSUPPORTED (padded rows above 2^48), HIP. */
int ftlm_apply_H_ex(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld, int32_t dtype,
                    ftlm_hv_opts* opts, void* stream);

/* ftlm_apply_H_ex that allocates nothing, for callers that cannot allocate
 * device memory: work captured into a HIP graph, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, results bit for bit
 * equal to ftlm_apply_H_ex.  Its one scratch buffer (the per-workgroup FP64
 * partial sums behind scale/dots) is a static device array of 4 MiB per GPU
 * (8192 x 64 doubles), held until the process ends; INVALID_ARG when a call
 * would need more (nvec x workgroups above that).  The first call on a
 * device looks up the array's device address (hipGetSymbolAddress): make it
 * outside stream capture.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (several streams or host threads)
 * race on it and must be serialized by the caller; each call writes every
 * partial it reads, so nothing needs clearing between calls. */
int ftlm_apply_H_ex_noalloc(ftlm_block* b, const void* X, void* Y, int32_t nvec, int64_t ld, int32_t dtype,
                            ftlm_hv_opts* opts, void* stream);

/* Autotuner: times every lane layout of the H.V kernel (lanes per output
 * representative 1..64, vectors per lane) for nvec columns of dtype on this
 * block, on stream, first for the launch ftlm_run and ftlm_kpm make on this
 * block (its row layout, with the Lanczos epilogue), then for the plain
 * launch of ftlm_apply_H (block rows), and keeps the fastest of each in a
 * process-wide cache keyed by (N, 2s, |G|, irrep dimension, nvec, dtype, H.V
 * mode, row layout, epilogue); later calls with that key use it.  Outputs
 * (may be NULL) describe the first: the chosen lanes per representative and
 * its time per launch in ms; up to 8 (lanes, ms) pairs in tried/tried_ms
 * with their count in n_tried.  Allocates two rows x nvec scratch arrays for
 * the duration of the call.  Synchronous. */
int ftlm_block_autotune(ftlm_block* b, int32_t nvec, int32_t dtype, void* stream, int32_t* best_lanes,
                        double* best_ms, int32_t* tried, double* tried_ms, int32_t* n_tried);

/* The autotuner's choices outlive the process through a text file (one line
 * per choice: architecture, cluster hash, sizes, kernel bucket, vectors,
 * storage, mode, layout, epilogue, lanes).  Every key carries the device
 * architecture (ftlm_device_arch, e.g. "gfx950:sramecc+:xnack-") and a hash
 * of the cluster (sizes, bonds, couplings, group elements, spin flip), so a
 * choice is used only for the hardware and cluster it was timed on.
 * ftlm_autotune_save writes the cached choices of `arch` (NULL: all) to path
 * (replacing the file); ftlm_autotune_load adds those of `arch` (NULL: all)
 * from path to the cache; ftlm_autotune_clear empties the cache.  Host only.
 * Errors: INVALID_ARG (unreadable or unwritable file, malformed line). */
int ftlm_device_arch(char* buf, int32_t len);
int ftlm_autotune_save(const char* path, const char* arch, int32_t* n_saved);
int ftlm_autotune_load(const char* path, const char* arch, int32_t* n_loaded);
int ftlm_autotune_clear(void);

/* R independent Lanczos chains batched into one H.V launch per step
 * (Sections 2.2, 3).  Chain r starts from a SplitMix64 vector keyed by
 * (seed, two_M, irrep, row, r), Rademacher or Gaussian, normalised in FP64,
 * stored in `storage` precision; the recurrence w = H v_j - beta_j v_{j-1},
 * alpha_j = <v_j, w>, w -= alpha_j v_j, beta_{j+1} = |w| runs with
 * FP64 reductions, n = min(steps, D) products, early stop per chain when
 * beta_{j+1} <= 1e-10 max_{i<=j}(|alpha_i| + beta_i + beta_{i+1}).
 * Host outputs: alpha, beta (R x steps, row-major; beta[r][j] = beta_{j+1}),
 * nsteps (R).  Synchronous.  Device scratch is allocated per call. */
int ftlm_run(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist,
             double* alpha, double* beta, int32_t* nsteps, void* stream);

/* What one ftlm_run_ex call did: the vector layout (enum ftlm_layout, never
 * AUTO), the rows of each stored vector, and the number and total duration
 * of its H.V launches, measured with HIP events on the run's stream. */
typedef struct ftlm_run_info {
  int32_t layout;
  int32_t hv_launches;
  uint64_t rows;
  double hv_ms;
} ftlm_run_info;

/* ftlm_run (Sections 2.2 and 3) that also fills *info (may be NULL; then it
 * is ftlm_run).
 * Timing adds two event records per step. */
int ftlm_run_ex(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist,
                double* alpha, double* beta, int32_t* nsteps, void* stream, ftlm_run_info* info);

/* ftlm_run in stages, with a checkpoint of the whole run state in between
 * (for long runs that must survive an interruption, as the paper's
 * multi-hour blocks of Section 4.3).  ftlm_run_begin draws the start vectors
 * of R chains exactly as ftlm_run does; ftlm_run_advance enqueues the next n
 * Lanczos steps on the run's stream (asynchronous; *done = steps enqueued so
 * far, at most min(steps, D)); ftlm_run_save waits for the stream and writes
 * the run's device state (per-chain state, alpha and beta so far, both
 * stored vectors: 2 x rows x R elements) to a file (written as path.part
 * and renamed to path when complete, so an interrupted save leaves an
 * earlier checkpoint at path intact); ftlm_run_load rebuilds a
 * saved run on a block built the same way (same cluster, group, sector,
 * irrep, row and row layout; INVALID_ARG otherwise), ready to advance;
 * ftlm_run_finish runs the remaining steps and returns alpha, beta and
 * nsteps as ftlm_run.  The coefficients of a run interrupted by save and
 * load equal those of one ftlm_run call bit for bit.  The block must outlive
 * the run state; device memory of the state is freed by
 * ftlm_run_state_free.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP. */
typedef struct ftlm_run_state ftlm_run_state;
int ftlm_run_begin(ftlm_block* b, int32_t R, int32_t steps, uint64_t seed, int32_t storage, int32_t dist,
                   void* stream, ftlm_run_state** out);
int ftlm_run_advance(ftlm_run_state* s, int32_t n, int32_t* done);
int ftlm_run_save(ftlm_run_state* s, const char* path);
int ftlm_run_load(ftlm_block* b, const char* path, void* stream, ftlm_run_state** out);
int ftlm_run_finish(ftlm_run_state* s, double* alpha, double* beta, int32_t* nsteps);
void ftlm_run_state_free(ftlm_run_state* s);

/* One job of ftlm_run_fused: R chains of `steps` Lanczos steps on a block. */
typedef struct ftlm_fused_job {
  ftlm_block* block;
  int32_t R;               /* 1..32 */
  int32_t steps;
  uint64_t seed;
  int32_t storage;         /* FTLM_F64 or FTLM_F32 */
  int32_t dist;            /* enum ftlm_dist */
  int32_t first_chain;     /* chain r of the job has the key of chain first_chain + r of
                              ftlm_run on the same block (0: the keys of ftlm_run) */
  int32_t reserved;
  double* alpha;           /* host outputs as in ftlm_run: R x steps */
  double* beta;            /* R x steps */
  int32_t* nsteps;         /* R */
} ftlm_fused_job;

/* Fused small-block Lanczos (Sections 2.2 and 3; the persistent form of the
 * batched recurrence for many small blocks): one workgroup of the device runs
 * every step of one job, i.e. the start vectors, the H.V with the Lanczos
 * epilogue, alpha, the update and beta, with workgroup barriers between the
 * phases, and one launch per kernel shape covers all n jobs.  The recurrence,
 * the keys of the start vectors and the stopping rule are those of ftlm_run;
 * the FP64 sums run over one workgroup in a fixed order (deterministic, equal
 * to ftlm_run's results up to rounding).  Each job's block must use the entry
 * table (FTLM_HV_ENTRIES or AUTO resolved to it), have its irrep tables fit in
 * LDS and not force the padded layout; otherwise FTLM_ERR_INVALID_ARG.  A job
 * works through all of its block's representatives with one workgroup, so it
 * pays only for blocks of up to a few thousand representatives: larger ones
 * belong to ftlm_run.  Blocks may repeat across jobs.  Device scratch
 * (2 D R vectors per job) is allocated per call.  Synchronous. */
int ftlm_run_fused(const ftlm_fused_job* jobs, int32_t n, void* stream);

/* ----------------------------------------------------------------- KPM ---
 * Kernel polynomial method (thermodynamics from a Chebyshev expansion of the
 * density of states, the alternative to FTLM the paper cites as Ref. [6]) on the same
 * symmetry-adapted H.V: Chebyshev moments mu_n = <r|T_n(H~)|r> / <r|r> of
 * H~ = (H - center) / half_width for R start vectors r (the vectors of
 * ftlm_run's chains 0..R-1: same keys, generator and normalisation), from
 * t_0 = r, t_1 = H~ r, t_{n+1} = 2 H~ t_n - t_{n-1}, two moments per H.V
 * (mu_{2n+1} = 2<t_{n+1},t_n> - mu_1, mu_{2n+2} = 2<t_{n+1},t_{n+1}> - mu_0;
 * Weisse et al., Rev. Mod. Phys. 78, 275 (2006)).  Vectors in FTLM_F64 or
 * FTLM_F32 storage (block row layout), FP64 products and reductions in a
 * fixed order.  The block spectrum must lie inside center +- half_width (for
 * example the extreme Ritz values of a short ftlm_run, widened by a few
 * percent); moments that leave [-1, 1] report INVALID_ARG.  Host output
 * moments: R x n_moments (row-major).  ceil((n_moments - 1) / 2) H.V
 * products.  Synchronous; device scratch allocated per call. */
int ftlm_kpm(ftlm_block* b, int32_t R, int32_t n_moments, uint64_t seed, int32_t storage, int32_t dist,
             double center, double half_width, double* moments, void* stream);

/* KPM moments of one block for the thermal sums. */
typedef struct ftlm_kpm_block {
  int32_t two_M;
  int32_t d_gamma;         /* trace weight (as in ftlm_ritz) */
  uint64_t D;
  int32_t R;
  int32_t n_moments;
  double center, half_width;
  const double* moments;   /* R x n_moments */
} ftlm_kpm_block;

/* Host FP64 thermal sums from KPM moments: per block the chain-averaged
 * moments with the Jackson kernel give quadrature weights W_k on the n_nodes
 * Chebyshev nodes x_k = cos(pi (k + 1/2) / n_nodes) (0: twice the largest
 * n_moments), W_k = (1/K)[g_0 mu_0 + 2 sum_n g_n mu_n cos(n theta_k)], at
 * energies center + half_width x_k; then Z, E, C, chi as in ftlm_observables
 * with Boltzmann factors shifted by the lowest node energy.  Errors:
 * INVALID_ARG. */
int ftlm_kpm_observables(const ftlm_kpm_block* blocks, int32_t nblocks, const double* T, int32_t nT, double g,
                         int32_t n_nodes, double* E, double* C, double* chi, double* logZ);

/* Host FP64: eigenvalues theta (ascending) and weights w_k = (first
 * eigenvector component)^2 of the n x n tridiagonal with diagonal alpha and
 * off-diagonal beta[0..n-2] (Section 2.2).  n <= 4096. */
int ftlm_tridiag_ritz(const double* alpha, const double* beta, int32_t n, double* theta,
                      double* weight);

/* Ritz data of one block for the thermal sums. */
typedef struct ftlm_ritz {
  int32_t two_M;
  int32_t d_gamma;         /* trace weight of the block's irrep: its dimension, or
                              dim / 2 for a realified complex pair */
  uint64_t D;
  int32_t R;
  int32_t ld;              /* stride of theta/weight rows (>= max nsteps) */
  const int32_t* nsteps;   /* R */
  const double* theta;     /* R x ld */
  const double* weight;    /* R x ld */
} ftlm_ritz;

/* Host FP64 thermal sums (Eqs. 4-7, 14): E, C (per cluster, k_B = 1) and the
 * zero-field susceptibility chi = g^2 beta <(S^z)^2> on nT temperatures,
 * Boltzmann factors shifted by the lowest Ritz value over all blocks;
 * logZ = ln Z_FTLM.  Output pointers may be NULL.  Errors: INVALID_ARG. */
int ftlm_observables(const ftlm_ritz* blocks, int32_t nblocks, const double* T, int32_t nT, double g,
                     double* E, double* C, double* chi, double* logZ);

/* ------------------------------------------------------------- campaign ---
 * The whole method on one cluster (Sections 2.2, 3, 4): every M >= 0 sector
 * (or one), every irrep block of it (row 0; with spin_flip, G x Z2 at M = 0),
 * R chains per block, Ritz data per chain, and E, C, chi, ln Z on T[0..nT) by
 * ftlm_observables over all blocks.  Uses the library's own irreps (real type
 * required).  Chain r of block (2M, irrep) has the key of ftlm_run, so a
 * block's coefficients equal those of ftlm_run on that block with the same
 * chains per run (to rounding where the fused engine runs the block: its
 * reductions sum in another fixed order).
 *
 * Engines: sectors with few representatives (at most fused_max_rounds
 * representatives per lane group of one workgroup; 0 = the library default
 * of 8) run in the fused small-block kernel: one workgroup does every
 * Lanczos step of one block job (R chains, or chains_per_run of them), and
 * all such jobs of the campaign go out as one batch on a stream of the
 * library.  The blocks of larger sectors run with the per-step kernels (the
 * steps replay a captured graph), spread over two worker streams so that
 * blocks, the batch and the next sector's build overlap; their results are
 * read back when the runs in flight pass a quarter of the free device memory
 * or at the end.  Sectors run from the largest 2M down.  FTLM_ENGINE_STEPS forces the per-step kernels everywhere,
 * FTLM_ENGINE_FUSED the fused kernel wherever it applies (FP64 or FP32
 * storage, entry-table H.V, irrep tables within LDS, at most 32 chains per
 * job).  The sector tables of a large M are freed before the next M.
 * Synchronous. */
enum ftlm_engine { FTLM_ENGINE_AUTO = 0, FTLM_ENGINE_STEPS = 1, FTLM_ENGINE_FUSED = 2 };

typedef struct ftlm_campaign_opts {
  int32_t R;               /* chains per block */
  int32_t steps;           /* Lanczos steps per chain */
  uint64_t seed;
  int32_t storage;         /* enum ftlm_dtype */
  int32_t dist;            /* enum ftlm_dist */
  int32_t all_M;           /* 1: all 2M = (2Ns mod 2) .. 2Ns; 0: only two_M */
  int32_t two_M;
  int32_t spin_flip;       /* resolve M = 0 by G x Z2 */
  int32_t chains_per_run;  /* 0: all R chains share one H.V launch per step; k: runs of k chains
                              (1 = the plain single-vector path) */
  double g;                /* g factor of chi */
  int32_t engine;          /* enum ftlm_engine */
  int32_t fused_max_rounds;/* automatic engine choice (0: default) */
} ftlm_campaign_opts;

typedef struct ftlm_campaign_stats {
  int32_t sectors, blocks, empty_blocks;
  int32_t fused_blocks;    /* blocks run by the fused small-block kernel */
  uint64_t rows;           /* sum of block dimensions */
  uint64_t products;       /* H.v products over all chains */
  uint64_t work;           /* sum over chains of D x products: basis elements x vectors */
  double seconds_build, seconds_lanczos, seconds_thermo, seconds_total;
} ftlm_campaign_stats;

int ftlm_campaign(const ftlm_cluster* cl, const int32_t* gens, int32_t ngens, const ftlm_campaign_opts* opts,
                  const double* T, int32_t nT, double* E, double* C, double* chi, double* logZ,
                  ftlm_campaign_stats* stats);

void ftlm_block_free(ftlm_block* b);
const char* ftlm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FTLM_H */
