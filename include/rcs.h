/*
 * rcs.h -- C ABI of librcs: build the output state of a Sycamore-style grid
 * random circuit as a matrix-product state on one MI355X (gfx950), draw
 * bitstring shots from it, evaluate amplitudes, and score shots by linear
 * cross-entropy benchmarking (XEB).
 *
 * The paper's pipeline (Section 3.2) has four stages: state construction on
 * one GPU, persistence, distributed measurement sampling, and post-processing
 * that computes the linear XEB score (Section 5.1).  This library is the
 * data-parallel core of stages 1, 3 and 4 on one device; the state
 * representation (snake-ordered MPS with SVD truncation) is this library's
 * own choice since the paper does not describe its engine.
 *
 * Conventions for every entry point
 *  - Return value: RCS_OK (0) on success, another rcs_status on failure.  On
 *    failure nothing is written to outputs, handle outputs stay NULL, and
 *    rcs_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses the ABI.
 *  - Bitstrings are uint64 with bit q = measured value of qubit q; qubits are
 *    the present grid sites numbered in row-major order (n <= 64).
 *  - Pointers named *_dev are device pointers owned by the caller (e.g. the
 *    storage of a torch tensor on the same device).  Work on them is ordered
 *    on the state's stream (rcs_build_opts.stream, or rcs_state_set_stream).
 *    Calls that return host scalars synchronise that stream.
 *  - Pointers named *_host are host memory owned by the caller.
 *  - Handles are not thread-safe: one call at a time per handle.
 *  - Complex numbers are two consecutive doubles (re, im), i.e. the layout of
 *    C99 double _Complex and numpy complex128.
 */
#ifndef RCS_H
#define RCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rcs_circuit_s* rcs_circuit;
typedef struct rcs_state_s* rcs_state;

typedef enum {
  RCS_OK = 0,
  RCS_ERR_INVALID_ARG = 1,
  RCS_ERR_UNSUPPORTED = 2,
  RCS_ERR_OUT_OF_MEMORY = 3,
  RCS_ERR_DEVICE = 4,
  RCS_ERR_NUMERIC = 5, /* NaN/Inf, or an SVD that did not converge */
  RCS_ERR_STATE = 6    /* handle in the wrong state for the call */
} rcs_status;

/* ------------------------------------------------------------------ circuits
 * Section 3.1: 53-qubit random circuits, single-qubit gates drawn from
 * {sqrt(X), sqrt(Y), sqrt(W)}, fSim two-qubit gates on coupler pattern
 * sequence ABCDCDAB.  Generated here on a rectangular grid:
 *   W = min(rows, cols) columns, H = max(rows, cols) rows, site r*W + c;
 *   pattern A = horizontal couplers (r,c)-(r,c+1) with c even, B with c odd,
 *   C = vertical (r,c)-(r+1,c) with r even, D with r odd;
 *   cycle t: one single-qubit gate per qubit (never the previous one on that
 *   qubit), then fSim(theta, phi) on every coupler of pattern[t mod len];
 *   optional final single-qubit layer.
 * All draws come from Philox4x32-10 keyed by the seed (counter layout in
 * the library's design notes); the same desc always gives the same circuit.
 * Rotated lattice (lattice = 1), the stand-in for Sycamore's rotated square
 * lattice and its patterns A-H (Google's layout files are not available, so
 * this is a reading): couplers only between adjacent rows, down-left
 * (r,c)-(r+1,c) and down-right (r,c)-(r+1,c+s), s = +1 on even rows and -1
 * on odd rows; A/B = down-left with r even/odd, C/D = down-right with r
 * even/odd, E/F = down-left with r-c even/odd, G/H = down-right with r-ch
 * even/odd (ch = c on even rows, c-1 on odd rows).  Each pattern is a
 * matching; A-D and E-H each cover every coupler once.
 */
typedef struct {
  int32_t rows, cols;             /* grid, 2 <= rows, cols; rows*cols <= 4096 */
  int32_t n_cycles;               /* >= 0 */
  uint64_t seed;
  int32_t n_removed;              /* explicit absent sites ...               */
  const int32_t* removed_sites;   /* ... site indices r*W + c (host, nullable) */
  int32_t n_removed_random;       /* 0 or 1 extra seed-chosen absent site     */
  const char* pattern;            /* letters from "ABCD"; NULL -> "ABCDCDAB"  */
  double theta, phi;              /* fSim angles (pi/2, pi/6 for Sycamore)    */
  int32_t final_1q_layer;         /* 1: one more single-qubit layer at end    */
  int32_t swap_network;           /* MPS order and swap network (0 or 1):     */
                                  /* 0 snake, 1 interleaved row pairs         */
  int32_t lattice;                /* 0 rectangular (patterns A-D above);      */
                                  /* 1 rotated, patterns A-H (below)          */
} rcs_circuit_desc;

/* Validates and generates the circuit and its MPS schedule (host only, no
 * device work).  Errors: INVALID_ARG for null pointers, a grid below 2x2,
 * more than 64 present qubits, bad pattern letters or out-of-range sites. */
rcs_status rcs_circuit_create(const rcs_circuit_desc* desc, rcs_circuit* out);
void rcs_circuit_destroy(rcs_circuit c);

/* Sizes: qubits, single-qubit layers, schedule ops, two-site updates
 * (gates plus SWAPs of the swap network).  Any output may be NULL. */
rcs_status rcs_circuit_info(rcs_circuit c, int32_t* n_qubits, int32_t* n_layers_1q,
                            int32_t* n_ops, int32_t* n_updates);

/* Single-qubit gate indices (0 sqrtX, 1 sqrtY, 2 sqrtW) of every layer:
 * gates_host[layer * n_qubits + q]; capacity n_layers_1q * n_qubits. */
rcs_status rcs_circuit_one_qubit_gates(rcs_circuit c, int32_t* gates_host);

/* The compiled MPS schedule.  snake_host[pos] = qubit at MPS position pos
 * before the first op.  ops_host[4*o + 0..3] = {kind, arg, gate, cycle}:
 * kind 0 = single-qubit layer (arg = layer index), kind 1 = two-site update
 * at positions (arg, arg+1) with gate 0 = fSim, 1 = SWAP (a SWAP update also
 * exchanges the two positions' qubits).  Networks (rcs_circuit_desc.
 * swap_network; rows run along the short side in both):
 *   0 snake: boustrophedon order; a vertical coupler at positions i < j is a
 *     SWAP chain j-1..i+1, the fSim at i, and the chain back i+1..j-1;
 *   1 interleaved: row-major order (qubit q at position q between layers);
 *     each row pair of a vertical layer is sorted into column-interleaved
 *     order by insertion (keys 2c top / 2c+1 bottom; the column's fSim
 *     follows each walk), then the SWAPs are replayed in reverse.  Even
 *     cycles run left to right (bottom qubits walk left), odd cycles right
 *     to left (top qubits walk right).  W^2 updates per full row pair
 *     instead of 2W(W-1) + W.
 * Capacities: n_qubits and 4 * n_ops. */
rcs_status rcs_circuit_schedule(rcs_circuit c, int32_t* snake_host, int32_t* ops_host);

/* ------------------------------------------------------------------- build */
typedef enum { RCS_PREC_C128 = 0, RCS_PREC_C64 = 1, RCS_PREC_SPLIT_BF16 = 2 } rcs_precision;
typedef enum {
  RCS_RANK_FULL_SVD = 0,  /* fp64 one-sided Jacobi SVD + threshold rank rule   */
  RCS_RANK_LEARNED = 1,   /* network-predicted rank, fp32 randomized SVD, judge */
  RCS_RANK_RSVD_AT_CAP = 2 /* fp32 randomized SVD at rank min(chi, m), judge    */
} rcs_rank_mode;

typedef struct {
  int32_t contraction;     /* rcs_precision of the two-site contraction      */
  int32_t rank_mode;       /* rcs_rank_mode                                   */
  double fallback_tau;     /* judge slack; < 0 forces the fp64 fall-back      */
  const float* mlp_weights_host; /* packed fp32 weights (learned mode)        */
  int64_t mlp_count;       /* number of floats in mlp_weights_host            */
  int32_t rsvd_oversample; /* p (default 16)                                  */
  int32_t rsvd_power_iters;/* q (default 2)                                   */
  uint64_t rsvd_seed;      /* sketch seed                                     */
  void* stream;            /* hipStream_t for all work; NULL = null stream    */
  int32_t log_spectra;     /* 1: keep every update's singular spectrum        */
  int32_t max_ops;         /* < 0: whole schedule; else stop after max_ops    */
  int32_t canonicalize;    /* 1 (default): end right-canonical, unit norm     */
  int32_t svd_precision;   /* rcs_svd_precision of the full SVD (default F64) */
} rcs_build_opts;

/* Precision of the full SVD of a truncation step (Section 3.2, stage 1).
 * RCS_SVD_F32: splits whose rank is set by the bond cap (the discarded
 * weight exceeds the eps threshold by more than 1e-4 of the total) run the
 * one-sided Jacobi of the Cholesky-preconditioned matrix in fp32; the kept
 * right singular vectors are made orthonormal in fp64 by two Newton-Schulz
 * steps and the other factor is the fp64 projection, so the stored state is
 * the fp64 projection onto a subspace within fp32 accuracy of the optimal
 * one.  Splits whose rank the eps threshold decides, or whose last kept
 * squared singular value is below 1e-7 of the weight, are redone in fp64
 * from the same preconditioned matrix.  In RCS_RANK_LEARNED mode a cut the
 * network predicts to be cap-limited skips the randomized SVD (whose
 * sketch cannot resolve the spectrum at the cap more cheaply) and goes to
 * this split; a cut it predicts to be eps-limited tries the randomized SVD
 * and, if the judge rejects it, the fp64 split directly. */
typedef enum { RCS_SVD_F64 = 0, RCS_SVD_F32 = 1 } rcs_svd_precision;

/* Fills *opts with defaults: C128, FULL_SVD, tau 1e-6, p 16, q 2, null
 * stream, no logging, whole schedule, canonicalize, fp64 SVD. */
void rcs_build_opts_default(rcs_build_opts* opts);

/* Builds the MPS output state of the circuit with bond cap chi >= 1 and
 * per-step relative discarded-weight threshold 0 <= trunc_eps < 1, in fp64
 * with the full SVD (rcs_build_state_ex with default options).  The state
 * owns its device memory and does not borrow the circuit.  Errors:
 * INVALID_ARG, OUT_OF_MEMORY, DEVICE, NUMERIC (SVD not converged / NaN). */
rcs_status rcs_build_state(rcs_circuit circuit, int32_t chi, double trunc_eps, rcs_state* out);
rcs_status rcs_build_state_ex(rcs_circuit circuit, int32_t chi, double trunc_eps,
                              const rcs_build_opts* opts, rcs_state* out);

/* Builds n states, one per circuit, sharing one set of workspaces, each with
 * its own chi[i] and eps[i].  out[0..n-1] receive handles (all or none). */
rcs_status rcs_build_batch(const rcs_circuit* circuits, const int32_t* chi, const double* eps,
                           int32_t n, const rcs_build_opts* opts, rcs_state* out);

/* ---------------------------------------------------------------- sampling
 * Section 3.2 stage 3: n_shots measurement shots from a right-canonical,
 * unit-norm state.  Shot i, site k (MPS order): w_s = v A_k^s, p_s = |w_s|^2
 * in fp64, u = uniform from Philox(seed; shot i, site k), bit = (u*(p0+p1)
 * >= p0), v <- w_bit.  Past the first site, where dl*dr >= 1024 and not at
 * the last site, p0 + p1 is taken as |v|^2 (equal for a right-canonical
 * state up to its canonical residual) and w_1 is computed only for the
 * shots that chose 1.  bits_dev[i] receives the bitstring of shot
 * first_shot + i, log2p_dev[i] (nullable) log2 |psi(b)|^2.  Shots depend
 * only on (state, seed, shot index), so ranges computed separately and
 * concatenated equal one call.  Errors: INVALID_ARG (null bits_dev), STATE
 * (state not canonical). */
rcs_status rcs_sample(rcs_state s, uint64_t n_shots, uint64_t seed, uint64_t* bits_dev,
                      double* log2p_dev);
rcs_status rcs_sample_range(rcs_state s, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                            uint64_t* bits_dev, double* log2p_dev);

/* Allocation-free form of rcs_sample_range, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same shots, bit
 * for bit.  The sampler's workspace (two W row buffers, per-shot partial
 * norms and chosen branches) lives in a static 64 MiB device array that the
 * library holds on every GPU it runs on until the process ends; no device
 * memory is allocated or freed by the call, and no library routine that
 * allocates is called.  Shots run in passes of the largest multiple of 64
 * (at most 65,536) whose workspace fits the array: 960 shots at maximum
 * bond 1024, 448 at 2048.  All calls on one GPU share the array, so calls
 * that overlap on one GPU (other streams or threads) race; calls on one
 * stream are ordered and safe.  Errors: as rcs_sample_range, plus
 * INVALID_ARG when the state's maximum bond needs more than the array for a
 * 64-shot pass (bond above 16,319), DEVICE when the array's address cannot
 * be obtained. */
rcs_status rcs_sample_range_noalloc(rcs_state s, uint64_t first_shot, uint64_t n_shots, uint64_t seed,
                                    uint64_t* bits_dev, double* log2p_dev);

/* Shots from n states in one launch sequence: shot j of state i goes to
 * bits_dev[i * n_shots + j] (and log2p_dev likewise, nullable); identical to
 * rcs_sample on each state.  Per site index one grouped GEMM launch covers
 * every state that has that site; the whole sequence is captured into one
 * HIP graph on a private stream and replayed (synchronous; orders after
 * work already submitted to the first state's stream). */
rcs_status rcs_sample_batch(const rcs_state* states, int32_t n, uint64_t n_shots, uint64_t seed,
                            uint64_t* bits_dev, double* log2p_dev);

/* psi(b) for m bitstrings: amps_dev[2i], amps_dev[2i+1] = re, im. */
rcs_status rcs_amplitudes(rcs_state s, const uint64_t* bits_dev, uint64_t m, double* amps_dev);

/* Section 5.1 linear XEB: F = 2^n mean_i p_ref_i - 1 and its standard error
 * std(2^n p_ref) / sqrt(m) (m - 1 denominator), from m >= 2 reference
 * probabilities on the device; fixed-order fp64 reduction.  Host outputs. */
rcs_status rcs_xeb(int32_t n_qubits, const double* p_ref_dev, uint64_t m, double* xeb_host,
                   double* stderr_host);
/* The same from log2 probabilities (as written by rcs_sample). */
rcs_status rcs_xeb_log2(int32_t n_qubits, const double* log2p_dev, uint64_t m, double* xeb_host,
                        double* stderr_host);
/* Scores m bitstrings with ref's |psi|^2. */
rcs_status rcs_xeb_state(rcs_state ref, const uint64_t* bits_dev, uint64_t m, double* xeb_host,
                         double* stderr_host);

/* ------------------------------------------------------------ state access */
typedef struct {
  int32_t n_qubits;
  int32_t max_bond;
  int32_t center;          /* orthogonality centre position               */
  int32_t canonical;       /* 1 when right-canonical with unit norm       */
  int32_t n_truncations;   /* two-site updates performed                  */
  int32_t n_fallbacks;     /* learned/rsvd steps redone with the full SVD  */
  int32_t n_rsvd_accepted;
  int32_t jacobi_sweeps_max;
  double log_fidelity_est; /* sum log(1 - eps_step)                       */
  double sum_eps;
  double build_seconds;    /* device time from first kernel to last       */
  double svd_seconds;      /* part spent in SVD/RSVD kernels (if timed)   */
  int64_t device_bytes;    /* MPS + workspace bytes held                  */
  int32_t n_center_moves;  /* single-site orthogonalisations (centre moves) */
  double nominal_svd_flops;/* sum over full SVDs of 4 (14 m n^2 + 8 n^3),    */
                           /* m >= n the two-site matrix shape              */
  double nominal_qr_flops; /* sum over centre moves of 4 (2 m n^2 - 2n^3/3) */
  int32_t n_precond;       /* full SVDs done on the Cholesky-preconditioned */
                           /* matrix (Jacobi on R^H, R^H R = X^H X)         */
  int32_t n_precond_fallback; /* preconditioned attempts redone on X itself */
  int32_t n_center_moves_cholqr; /* centre moves done by CholeskyQR (the   */
                           /* others by the Jacobi orthogonalisation)       */
  int32_t n_svd_f32;       /* splits whose Jacobi ran in fp32 (RCS_SVD_F32) */
  int32_t n_svd_f32_redone;/* fp32 attempts redone in fp64                  */
} rcs_state_info;

rcs_status rcs_state_info_get(rcs_state s, rcs_state_info* out);
/* bond_dims_host[k] = dimension between positions k and k+1 (n-1 values);
 * snake_host[pos] = qubit at position pos (n values).  Either may be NULL. */
rcs_status rcs_state_layout(rcs_state s, int32_t* bond_dims_host, int32_t* snake_host);
rcs_status rcs_state_set_stream(rcs_state s, void* stream);

/* Copies the site tensors to the host: tensors_host receives, for positions
 * 0..n-1 in order, A_k with shape (dim_k, 2, dim_{k+1}) in row-major complex
 * (2 doubles per entry); count_doubles is the capacity in doubles (query
 * the needed size with tensors_host = NULL: *needed_doubles is set). */
rcs_status rcs_state_export(rcs_state s, double* tensors_host, int64_t count_doubles,
                            int64_t* needed_doubles);
/* Creates a state from host site tensors in the export layout.  dims_host
 * has n+1 entries (dims[0] = dims[n] = 1), snake_host n entries (a
 * permutation of 0..n-1).  canonical = 1 asserts the tensors are
 * right-canonical with unit norm (required by rcs_sample).  Errors:
 * INVALID_ARG for bad dims or permutation. */
rcs_status rcs_state_import(int32_t n, const int32_t* dims_host, const int32_t* snake_host,
                            const double* tensors_host, int32_t canonical, void* stream,
                            rcs_state* out);

/* Section 3.2, stage 2: the built state is persisted once and loaded by
 * every independent sampling job.  rcs_state_save writes the state's
 * layout, estimated fidelity and site tensors to `path` (written to
 * path + ".tmp" and renamed, so a reader never sees a partial file);
 * rcs_state_load creates a state from such a file on the calling thread's
 * current device, with its work on `stream` (NULL = null stream).  File
 * layout, little-endian: magic "RCSMPS1\n"; int32 version (1), n,
 * canonical, 0; float64 log F_est; int32 dims[n+1]; int32 snake[n]; the
 * site tensors in the rcs_state_export layout; uint64 FNV-1a checksum of
 * everything before it (64-bit words, then trailing bytes).  Loading a
 * canonical state and sampling a shot range gives the same bits as the
 * saving process would (shots depend only on state, seed and shot index).
 * Errors: INVALID_ARG for unreadable, truncated or corrupt files (bad
 * magic, version, sizes or checksum), DEVICE when writing fails. */
rcs_status rcs_state_save(rcs_state s, const char* path);
rcs_status rcs_state_load(const char* path, void* stream, rcs_state* out);
void rcs_state_destroy(rcs_state s);

/* Per-update record of a build with log_spectra = 1: count, then for record
 * r: meta_host[6r..6r+5] = {position, cycle, m (singular values), kept rank,
 * chi_l, chi_r} and the m singular values (descending) appended to
 * values_host in record order.  Query sizes with NULL outputs. */
rcs_status rcs_state_spectra(rcs_state s, int32_t* n_records, int64_t* n_values,
                             int32_t* meta_host, double* values_host);

/* One record per two-site update of the build, in schedule order (always
 * kept): records_host[7u..7u+6] = {position, cycle, chi_l, chi_m (middle
 * bond before the update), chi_r, kept rank, path}, path 0 = full fp64 SVD,
 * 1 = randomized split accepted, 2 = randomized split rejected by the judge
 * and redone with the full SVD.  Capacity 7 * n_updates (query with NULL). */
rcs_status rcs_state_updates(rcs_state s, int32_t* n_updates, int32_t* records_host);

/* Decisions of every randomized split of a learned or rsvd-at-cap build, in
 * order (the task's learned part: predicted rank, randomized truncated SVD,
 * full-SVD judge).  Per record r:
 *   ints_host[10r..10r+9] = {update index, position, cycle, m = min(rows,
 *     cols) of the two-site matrix, k_hat, sketch width l, kept rank k (the
 *     forced rank min(l, cap) for an early rejection, -1 when l >= m and the
 *     plain split ran), accepted, early (rejected before the projected SVD
 *     because the weight outside the sketched subspace already fails the
 *     judge), number of logged projected singular values};
 *   doubles_host[4r..4r+3] = {eps_pred at k, eps_rand (discarded fraction
 *     incurred), weight outside span(Q), total weight ||M||_F^2};
 *   net_host[98r..98r+97] = the 66 network inputs then its 32 outputs
 *     (learned mode; zeros otherwise);
 *   values_host: the projected singular values (descending, logging builds
 *     only), concatenated in record order.
 * Any output may be NULL; counts come back through n_records / n_values. */
rcs_status rcs_state_rsvd_log(rcs_state s, int32_t* n_records, int64_t* n_values, int32_t* ints_host,
                              double* doubles_host, float* net_host, double* values_host);

/* ------------------------------------------------------------ dense vector
 * Section 5.1 scores samples by linear XEB against the circuit's exact
 * output probabilities.  rcs_dense_simulate writes the exact output state
 * of the circuit (same gates and order as the MPS build, no truncation) to
 * psi_dev: 2^n complex128 amplitudes (n_amps = 2^n, caller-owned device
 * memory, 256 GiB at 34 qubits), index i = sum_q b_q 2^q.  Work is ordered
 * on `stream`.  Errors: INVALID_ARG for a null circuit or pointer, n above
 * 36, n_amps != 2^n, or a coupler spanning 8 or more qubit numbers (grids
 * up to 8 columns).
 * rcs_dense_gather reads entries of such a vector at bitstrings bits_dev[0..m)
 * (masked to n bits): out_dev[i] = psi[b_i] as complex128 (probabilities = 0)
 * or |psi[b_i]|^2 as float64 (probabilities = 1), the reference for rcs_xeb. */
rcs_status rcs_dense_simulate(rcs_circuit c, double* psi_dev, int64_t n_amps, void* stream);
rcs_status rcs_dense_gather(const double* psi_dev, int32_t n_qubits, const uint64_t* bits_dev, uint64_t m,
                            int32_t probabilities, double* out_dev, void* stream);

/* -------------------------------------------------------- kernel-level calls
 * Exposed for parity tests of individual stages and for the training driver.
 * All device pointers, all ordered on `stream`. */

/* Thin SVD of a complex len x cnt matrix given column-major in x_dev
 * (column j at x_dev + 2*len*j) by one-sided block Jacobi in fp64:
 * s_dev[cnt] = singular values in descending order, u_dev (len x cnt,
 * column-major) = left singular vectors (zero columns where s = 0).
 * x_dev is overwritten.  Errors: NUMERIC if not converged. */
rcs_status rcs_svd_jacobi(int32_t len, int32_t cnt, double* x_dev, double* s_dev, double* u_dev,
                          void* stream);

/* The same SVD with the one-sided Jacobi in fp32 (the matrix is rounded to
 * complex64 after the fp64 column sort; Gram blocks and rotations on the
 * fp32 matrix cores; orthogonality tolerance 16 u32 sqrt(len)): singular
 * values with absolute errors of a few u32 ||X||_2, s_dev and u_dev as
 * above (u_dev columns orthonormal to about 1e-5).  x_dev is not modified.
 * Used by RCS_SVD_F32 builds (Section 3.2, stage 1, at reduced precision).
 * Errors: NUMERIC if not converged. */
rcs_status rcs_svd_jacobi_f32(int32_t len, int32_t cnt, const double* x_dev, double* s_dev, double* u_dev,
                              void* stream);

/* Thin QR of a complex len x cnt matrix (cnt <= len, 64 <= cnt <= 4096),
 * column-major in x_dev, as the build's centre moves compute it
 * (CholeskyQR: R from the Cholesky factor of X^H X, Q = X R^{-1}, then three
 * Newton-Schulz steps Q <- Q (3I - Q^H Q)/2): q_dev (len x cnt,
 * column-major) has orthonormal columns spanning range(X), r_dev (cnt x cnt,
 * column-major) = Q^H X, upper triangular up to the Newton-Schulz
 * correction (about u cond(X)^2 relative), and X = Q R.  x_dev is not
 * modified.  Errors: NUMERIC when X is numerically rank deficient or its
 * condition number exceeds about 1e6 (the Cholesky breaks down or
 * |I - Q^H Q| exceeds 1e-4 after the first pass); the build then uses the
 * Jacobi orthogonalisation instead. */
rcs_status rcs_cholqr(int32_t len, int32_t cnt, const double* x_dev, double* q_dev, double* r_dev, void* stream);

/* Two-site contraction: theta'[(s1,a),(s2,c)] = sum_{s1',s2'} G[(s1,s2),(s1',s2')]
 * sum_b A[a,s1',b] B[b,s2',c] with A (dl,2,dm), B (dm,2,dr) in export
 * layout, G 4x4 row-major complex; out_dev receives the (2dl) x (2dr)
 * matrix column-major.  precision = rcs_precision. */
rcs_status rcs_two_site(int32_t dl, int32_t dm, int32_t dr, const double* a_dev,
                        const double* b_dev, const double* gate_host, int32_t precision,
                        double* out_dev, void* stream);

/* Randomized SVD (fp32): len x cnt column-major complex fp64 input, sketch
 * width l, q power iterations, sketch entries {1,i,-1,-i} from Philox(seed;
 * (row, col, step, 4)).  s_dev[l] receives singular values (descending).
 * fro2_host receives ||M||_F^2 (fp64). */
rcs_status rcs_rsvd(int32_t len, int32_t cnt, const double* x_dev, int32_t l, int32_t q,
                    uint64_t seed, uint64_t step, double* s_dev, double* fro2_host, void* stream);

/* The orthonormal basis Q of the same range finder (len x l, column-major
 * complex, column j at q_dev + 2*len*j): the span whose projection
 * rcs_rsvd decomposes.  Same arguments and errors as rcs_rsvd. */
rcs_status rcs_rsvd_basis(int32_t len, int32_t cnt, const double* x_dev, int32_t l, int32_t q,
                          uint64_t seed, uint64_t step, double* q_dev, void* stream);

/* Spectrum features: 64-bin histogram of log10(s^2/sum s^2) (0.25 decade
 * bins over [-16,0), clamped) of s_dev[0..k-1], normalised to sum 1, then
 * bond/(n-2), cycle/n_cycles: 66 floats to feat_dev. */
rcs_status rcs_spectrum_features(const double* s_dev, int32_t k, int32_t bond, int32_t n_sites,
                                 int32_t cycle, int32_t n_cycles, float* feat_dev, void* stream);

/* Training targets of the rank network: 32 floats y_j = log10(max(tail(k_j)
 * / w, 1e-20)), k_j = ceil(m j / 32), j = 1..32, for the full descending
 * spectrum s_dev[0..m-1] (tail and w as in the rank rule, with the 1e-24
 * zero floor). */
rcs_status rcs_spectrum_targets(const double* s_dev, int32_t m, float* y_dev, void* stream);

/* Rank network 66-128-128-32 (ReLU), fp32, packed weights W1,b1,W2,b2,W3,b3
 * (row-major W[out][in]).  Forward: out_dev[batch*32]. */
#define RCS_MLP_PARAMS (66 * 128 + 128 + 128 * 128 + 128 + 128 * 32 + 32)
rcs_status rcs_mlp_forward(const float* w_dev, const float* x_dev, int32_t batch, float* out_dev,
                           void* stream);
/* Mean-squared-error loss and its gradient for every parameter. */
rcs_status rcs_mlp_backward(const float* w_dev, const float* x_dev, const float* y_dev,
                            int32_t batch, float* grad_dev, float* loss_dev, void* stream);
/* Adam step (bias-corrected, step >= 1) on count parameters in place. */
rcs_status rcs_mlp_adam(float* w_dev, const float* grad_dev, float* m_dev, float* v_dev,
                        int32_t count, int32_t step, float lr, float beta1, float beta2,
                        float eps, void* stream);

/* ------------------------------------------------------------ measurement
 * Sampled kernel timing for roofline reporting.  With every > 0, every
 * every-th launch of each timed kernel class is timed by start/stop events
 * attached to the launch (hipExtLaunchKernelGGL) on the stream it runs on,
 * together with the algorithmic flops and HBM bytes of that launch;
 * every = 0 disables probing.  Both calls clear the counters.  Classes:
 * 0 shot GEMM (sampler/amplitudes), 1 Jacobi Gram, 2 Jacobi rotation,
 * 3 two-site contraction, 4 randomized range finder, 5 the other fp64
 * factorisation kernels (Gram and Cholesky preconditioner, CholeskyQR,
 * triangular inverse, projections, Newton-Schulz, ranks); classes 0 and 5
 * time every launch (their launches differ in size in a repeating pattern,
 * with which a fixed stride could alias); class 5 records no flops or
 * bytes. */
rcs_status rcs_profile_enable(int32_t every);
/* Median event interval (seconds, host output) of back-to-back launches of
 * an empty one-workgroup kernel on the null stream, timed the same way: the
 * floor of any probed launch time (dispatch and event overhead). */
rcs_status rcs_profile_event_floor(double* seconds);
/* Per class: launches seen, launches timed, summed seconds / flops / bytes of
 * the timed launches.  Synchronises the pending events. */
rcs_status rcs_profile_read(int32_t kclass, int64_t* launches, int64_t* timed, double* seconds,
                            double* flops, double* bytes);
const char* rcs_profile_class_name(int32_t kclass);

/* --------------------------------------------------------------- tuning
 * Launch parameters of the Jacobi SVD (fp64 and fp32) per column-count bucket: the
 * first entry with cnt <= cnt_max applies (block = 16 or 32 columns per
 * block, inner_sweeps in [1, 8] two-sided sweeps per block-pair meeting).
 * Process-wide; written by the autotuner (paper_2512_07311_amd/autotune.py)
 * from device timings.  Without entries: block 16, one inner sweep. */
rcs_status rcs_tuning_set(int32_t cnt_max, int32_t block, int32_t inner_sweeps);
void rcs_tuning_clear(void);

/* ---------------------------------------------------------------- misc */
const char* rcs_last_error(void);
/* Library version string. */
const char* rcs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RCS_H */
