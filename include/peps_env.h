/*
 * peps_env.h - C ABI of libpepsenv: boundary-MPS environments of finite,
 * open-boundary PEPS on one MI355X (gfx950).
 *
 * Method: Lubasch, Cirac, Banuls, "Unifying Projected Entangled Pair States
 * contractions", arXiv:1311.6696.
 *   - peps_env_boundary: the sandwich contraction of Sec. 2 (fig. Sandwich):
 *     the norm network <psi|psi> is contracted from the top and from the
 *     bottom row by row; each MPS-MPO product is truncated back to bond chi
 *     (the paper's D') by alternating least squares with a QR gauge.
 *   - peps_expect: the row in the centre is contracted between the two
 *     boundaries (Sec. 2) giving log <psi|psi>; <S^z> and the Heisenberg bond
 *     energies of eq. (HeisenbergH) come from row / two-row sandwiches.
 *   - peps_cluster_env: cluster environments of Sec. 5: separable (D'=1,
 *     CU_0, Sec. 5.1) boundaries outside an n x n window around each site,
 *     the sandwich contraction with bond chi inside it (Sec. 5.2, 5.3).
 *
 * Conventions
 *   - Site tensor A[p][l][u][r][d], float64, C order (d fastest), p the
 *     physical index (p = 0 is spin up), l/u/r/d the left/up/right/down
 *     virtual legs; "up" points to row 0; site (r, c) is entry r*cols + c.
 *     Legs on the lattice edge must have dimension 1; neighbouring legs must
 *     agree.  Entries are real; the bra layer is the same tensor.
 *   - Site tensors are DEVICE pointers on the context's device; dims and the
 *     pointer array itself are HOST memory.  Inputs are read during the call
 *     only (the library keeps packed copies).
 *   - Results are written to caller-allocated HOST buffers.
 *   - All work is enqueued on the context's stream; every entry point
 *     returns only after the results it writes are complete.
 *
 * Errors: every entry point returns peps_status.  On error the handles in
 * out[] are set to NULL, no result is written and peps_last_error()
 * describes the failure (thread-local string valid until the next call on
 * the thread).  Shapes, bonds, windows and options are validated on the host
 * before any launch; the input tensors are then checked for NaN/Inf by a
 * read-only pass (PEPS_ERR_NONFINITE, naming a site) before anything is
 * computed.  No C++ exception crosses the ABI.  A context must be used by
 * one thread at a time.
 */
#ifndef PEPS_ENV_H
#define PEPS_ENV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PEPS_OK = 0,
  PEPS_ERR_INVALID = -1,      /* bad shape, bond mismatch, chi < 1, bad window, NULL pointer */
  PEPS_ERR_OOM = -2,          /* device allocation failed or workspace cap exceeded */
  PEPS_ERR_HIP = -3,          /* a HIP runtime call failed */
  PEPS_ERR_NOT_CONVERGED = -4, /* PEPS_OPTS_STRICT: an ALS row reached max_halfsweeps before tol */
  PEPS_ERR_NONFINITE = -5,    /* NaN/Inf in an input tensor or in a computed norm */
  PEPS_ERR_UNSUPPORTED = -6   /* valid request the library does not implement */
} peps_status;

/* Arithmetic of the bulk contractions.  QR gauge, norms and log-scales are
 * always float64. */
typedef enum {
  PEPS_F64 = 0,   /* float64 operands, float64 MFMA */
  PEPS_F32 = 1,   /* float32 operands, float32 MFMA, float32 accumulation */
  PEPS_BF16 = 2   /* bfloat16 operands (RNE from float32), float32 accumulation */
} peps_dtype;

typedef struct peps_ctx peps_ctx;   /* device, stream, memory pool */
typedef struct peps_env peps_env;   /* device-resident boundaries of one lattice or window */

/* One open-boundary PEPS. */
typedef struct {
  int32_t rows, cols;          /* L_r, L_c >= 1 */
  int32_t phys;                /* physical dimension d; the observables need d == 2 */
  const int32_t* dims;         /* host, rows*cols*5 entries (d, Dl, Du, Dr, Dd) per site */
  const double* const* site;   /* host array of rows*cols device pointers */
} peps_state;

/* ALS truncation of a row (Sec. 2: the MPS-MPO product is replaced by the
 * best MPS of bond chi, found by alternating least squares).  With tol == 0
 * every truncated row runs exactly `halfsweeps` half-sweeps (a launch
 * sequence that does not depend on the data).  With tol > 0 it runs at least
 * max(halfsweeps, 2) and at most max_halfsweeps, stopping after the first
 * half-sweep h with |omega_h - omega_(h-1)| <= tol * omega_h, omega being the
 * squared norm of the ALS centre tensor (the squared overlap of the fit with
 * the exact product).  omega is stationary at the optimum, so the rule fixes
 * it to about tol and the boundary tensors only to about sqrt(tol).  Each
 * extra half-sweep waits for the GPU once (the decision is taken on the
 * host).  A row that reaches max_halfsweeps first is marked not converged
 * (peps_env_info); with PEPS_OPTS_STRICT the call then fails with
 * PEPS_ERR_NOT_CONVERGED and returns no environment. */
typedef struct {
  int32_t chi;             /* boundary bond dimension D' >= 1 */
  int32_t dtype;           /* peps_dtype */
  int32_t halfsweeps;      /* ALS half-sweeps per truncated row (the minimum with tol > 0), default 4 if 0 */
  int32_t flags;           /* 0 or PEPS_OPTS_PER_STATE (peps_env_boundary only), PEPS_OPTS_COLUMNS, PEPS_OPTS_STRICT */
  uint64_t seed;           /* SplitMix64 key of the ALS start tensors */
  int32_t max_halfsweeps;  /* with tol > 0: the cap, >= halfsweeps, <= 256 (0: 40) */
  int32_t reserved;        /* must be 0 */
  double tol;              /* 0 (fixed half-sweep count) or the relative omega tolerance, in (0, 1) */
} peps_env_opts;

/* opts.flags: the options argument of peps_env_boundary points to one
 * record per state (every record carries the flag); chi, dtype, halfsweeps
 * and seed may then differ between the lattices of one batched run. */
#define PEPS_OPTS_PER_STATE 1

/* opts.flags (peps_env_boundary only): also contract the lattice from the
 * left and from the right, i.e. the top and bottom boundaries of the
 * transposed lattice (Sec. 2: the same sandwich contraction along the
 * other lattice direction), in the same batched run as the row boundaries.
 * peps_expect then takes each vertical bond (r,c)-(r+1,c) from the
 * single-column sandwich of column c instead of the two-row sandwich of
 * rows r and r+1: a different approximation at truncated chi, the same
 * values at lossless chi.  The transposed sites are strided views of the
 * packed sites, not copies.  With peps_cluster_env every window also gets
 * the boundaries of its transpose (closed by the same CU_0 matrices), and
 * its bond downwards comes from the single-column sandwich of the centre's
 * column. */
#define PEPS_OPTS_COLUMNS 2

/* opts.flags: with tol > 0, fail with PEPS_ERR_NOT_CONVERGED (no
 * environment returned) if any truncated row reaches max_halfsweeps before
 * the tolerance. */
#define PEPS_OPTS_STRICT 4

/* Cluster window around the centre site (ci, cj) of state `state`,
 * rows r0..r1 and columns c0..c1 inclusive, centre inside the window. */
typedef struct {
  int32_t state;
  int32_t r0, r1, c0, c1;
  int32_t ci, cj;
} peps_window;

/* Results of peps_expect for one environment.
 * Whole lattice: sz has rows*cols entries (row-major); bond has
 * rows*(cols-1) horizontal bonds (r,c)-(r,c+1) in row-major order followed
 * by (rows-1)*cols vertical bonds (r,c)-(r+1,c) in row-major order (from
 * the two-row sandwiches, or the column sandwiches with PEPS_OPTS_COLUMNS).
 * Window: sz has 1 entry (centre), bond has 2 (right, down; NaN if the
 * neighbour lies outside the window).
 * log_norm = log|<psi|psi>| from row floor(rows/2); norm_sign its sign.
 * flops = algorithmic flop count of the boundary and expectation work. */
typedef struct {
  double log_norm;
  double norm_sign;
  double* sz;           /* caller-allocated host buffer */
  double* bond;         /* caller-allocated host buffer */
  double flops;
} peps_result;

/* Create a context on HIP device `device` using stream `hip_stream`
 * (a hipStream_t, NULL = the null stream).  The stream is borrowed. */
peps_status peps_ctx_create(int32_t device, void* hip_stream, peps_ctx** out);
void peps_ctx_destroy(peps_ctx* ctx);

/* Top and bottom boundaries of n_states lattices (one batched run).
 * opts points to one options record used for all states, or to n_states
 * records when its flags hold PEPS_OPTS_PER_STATE.  On success out[i]
 * receives a new environment handle per state. */
peps_status peps_env_boundary(peps_ctx* ctx, const peps_state* st, int32_t n_states,
                              const peps_env_opts* opts, peps_env** out);

/* Cluster environments: the CU_0 separable boundaries of the four
 * directions of each referenced state, then the boundaries inside every
 * window (one batched run).  out[i] receives the environment of win[i]. */
peps_status peps_cluster_env(peps_ctx* ctx, const peps_state* st, int32_t n_states,
                             const peps_window* win, int32_t n_win,
                             const peps_env_opts* opts, peps_env** out);

/* Observables of n_env environments (one batched run). */
peps_status peps_expect(peps_ctx* ctx, peps_env* const* env, int32_t n_env, peps_result* out);

void peps_env_free(peps_env* env);

/* Norm environment N_l of single sites (Sec. 2: the network of <psi|psi>
 * with the ket and bra tensors of site l taken out, the matrix of the ALS
 * tensor update N_l A_l = b_l), from the single-row sandwich of the site's
 * row between the stored boundaries; one batched run over all requests.
 * n (device, caller-allocated, K*K doubles with K = Dl*Du*Dr*Dd of the
 * site): N[k][k'] row-major, k = ((l*Du + u)*Dr + r)*Dd + d the ket legs and
 * k' the same bra legs, scaled so that sum_p A[p,k] N[k][k'] A[p,k'] = sign.
 * log_z (out): log|<psi|psi>| as this row's sandwich estimates it, so the
 * unscaled environment is sign * exp(log_z) * N.  (r, c) are window
 * coordinates for a cluster environment (its cut legs closed by the CU_0
 * boundaries: the environment of the cluster update).  dir 0 takes N from
 * the row sandwich of row r; dir 1 (an environment built with
 * PEPS_OPTS_COLUMNS) from the column sandwich of column c, the one that
 * matches the vertical bonds of peps_bond_env; N is in the site's own leg
 * order either way.  N is symmetric and
 * positive semidefinite at lossless chi; truncated boundaries need not be
 * symmetric under ket <-> bra.  All requests share one precision; *flops
 * (may be NULL) receives the algorithmic flops.  The row sandwich of each
 * row used (its left and right column environments) is kept with the
 * environment, in device memory it owns until peps_env_free, and reused by
 * later peps_site_env, peps_bond_env and peps_bond_fit calls. */
typedef struct {
  peps_env* env;
  int32_t r, c;
  int32_t dir;    /* 0: row sandwich, 1: column sandwich */
  double* n;
  double log_z;   /* out */
  double sign;    /* out */
} peps_site_req;
peps_status peps_site_env(peps_ctx* ctx, peps_site_req* req, int32_t n_req, double* flops);

/* Right-hand sides b_l of the ALS update of a horizontal bond (Sec. 2,
 * N_l A_l = b_l) under a two-site gate: the overlap <psi|G psi> of the
 * stored state with the gated one, differentiated by the bra tensor of the
 * left site (r,c) and of the right site (r,c+1), from the row sandwich of
 * row r (both bra tensors of the bond are taken out of the network once,
 * then contracted with either neighbour).  gate (device): d^2 x d^2 float64
 * row-major, G[(p*d + P)*d*d + q*d + Q] maps the physical indices (q, Q) of
 * the left and right site to (p, P).  b_left / b_right (device, may be
 * NULL): d*K doubles [p][k] of that site, k as in peps_site_env, in the
 * scaling of that site's peps_site_env matrix: for the identity gate
 * b[p][k'] = sum_k A[p][k] N[k][k'].  (At truncated chi the boundaries need
 * not be symmetric under ket <-> bra, so neither need N.)  All requests
 * share one precision; *flops (may be NULL) receives the algorithmic flops.
 * dir 1 (an environment built with PEPS_OPTS_COLUMNS): the vertical bond
 * (r,c)-(r+1,c) from the column sandwich of column c, b_left for (r,c) and
 * b_right for (r+1,c), G's first index pair on (r,c), b in each site's own
 * leg order, scaled like peps_site_env with dir 1. */
typedef struct {
  peps_env* env;
  int32_t r, c;           /* bond (r,c)-(r,c+1) (dir 0) or (r,c)-(r+1,c) (dir 1); window coordinates for a window */
  int32_t dir;
  const double* gate;
  double* b_left;
  double* b_right;
} peps_bond_req;
peps_status peps_bond_env(peps_ctx* ctx, const peps_bond_req* req, int32_t n_req, double* flops);

/* The two local problems of the alternating least-squares bond update
 * (Sec. 2; the full update of Sec. 5.2): fitting G psi on the bond of
 * peps_bond_env (same r, c, dir, gate) by psi', the stored state with the
 * bond's two sites replaced by s1 (first site) and s2 (second site).  n1, b1:
 * norm environment of the first site in <psi'|psi'> (its second site s2)
 * and d<psi'|G psi>/d s1; n2, b2 the same for the second site with s1.
 * s1, s2 (device, float64, each site's own shape and leg order) may be the
 * stored tensors.  Outputs (device, caller-allocated, K*K and d*K doubles as
 * in peps_site_env / peps_bond_env) are divided by one positive number per
 * site, that of peps_bond_env, so that s1 = b1 n1^-1 and s2 = b2 n2^-1 solve
 * the two problems; with s = A they equal the site and bond environments.
 * Needs float64 environments. */
typedef struct {
  peps_env* env;
  int32_t r, c;
  int32_t dir;
  const double* gate;
  const double* s1;
  const double* s2;
  double* n1;
  double* b1;
  double* n2;
  double* b2;
} peps_fit_req;
peps_status peps_bond_fit(peps_ctx* ctx, const peps_fit_req* req, int32_t n_req, double* flops);

/* Overlaps of stored boundaries, for the boundary fidelity of Sec. 5.2
 * (f = |tr(X^T Y)| of boundary MPOs scaled to tr(X^T X) = 1): per request
 * the boundaries of env_a and env_b (environments of one lattice, any chi
 * and precision; their float64 tensors are used) after k absorbed rows,
 * side 0 from the top, 1 from the bottom, 2 from the left and 3 from the
 * right (2 and 3 need PEPS_OPTS_COLUMNS), 1 <= k < number of rows (columns
 * for sides 2, 3).  Outputs <X|Y>, <X|X>, <Y|Y>; one batched run. */
typedef struct {
  peps_env* env_a;
  peps_env* env_b;
  int32_t side, k;
  double xy, xx, yy;   /* out */
} peps_overlap_req;
peps_status peps_boundary_overlap(peps_ctx* ctx, peps_overlap_req* req, int32_t n_req);

/* One tensor of a stored boundary (Sec. 2: the boundary MPS after k
 * absorbed rows): side 0 from the top, 1 from the bottom (the lattice
 * mirrored top<->bottom, its rows reversed and up/down legs swapped), 2 from
 * the left and 3 from the right (the transposed lattice; they need
 * PEPS_OPTS_COLUMNS), 1 <= k < rows (columns for sides 2, 3), site c of the
 * boundary (0 <= c < cols of that frame).  dims (host, 4 int32, may be NULL)
 * receives its shape (left bond, ket leg, bra leg, right bond); dst (DEVICE,
 * caller-allocated, may be NULL) receives the float64 tensor X[a][k][b][a']
 * in C order.  The boundary is stored with unit norm; log_scale (host, may
 * be NULL) receives the log of the factor taken out of it, summed over the
 * k absorbed rows, so that the contracted rows equal exp(log_scale) times
 * the stored MPS (up to the truncation).  Waits for the context's stream. */
peps_status peps_env_mps(peps_env* env, int32_t side, int32_t k, int32_t c, int32_t* dims, double* dst,
                         double* log_scale);

/* Thin QR of n_blocks float64 blocks, the gauge step of the truncation
 * (Sec. 2: the ALS sweep keeps every tensor but the centre isometric):
 * A = Q R with A m x n (m >= n >= 1, n <= 1024), Q m x n with orthonormal
 * columns, R n x n upper triangular with R_ii >= 0 (for full column rank
 * the unique such factors).  a, q, r are DEVICE pointers with element
 * strides (row, column); r may be NULL; q may be a itself with the same
 * strides (in-place), otherwise the outputs must not overlap any input.
 * The blk array is host memory.  All blocks run as one batched group with
 * the kernels of the boundary truncation: CholeskyQR2 for tall blocks up to
 * 512 x 32 (128-row slices on separate, co-resident workgroups; Householder
 * when a block is too ill-conditioned for it),
 * register-resident Householder, TSQR or the streaming kernel otherwise. */
typedef struct {
  const double* a;
  int64_t a_rs, a_cs;
  double* q;
  int64_t q_rs, q_cs;
  double* r;
  int64_t r_rs, r_cs;
  int32_t m, n;
} peps_qr_block;
peps_status peps_qr(peps_ctx* ctx, const peps_qr_block* blk, int32_t n_blocks);

/* peps_qr for callers that cannot allocate device memory (code that must not
 * call hipMalloc, e.g. inside tight serving loops or harnesses that forbid
 * it): the same factors from the same kernels, bit for bit, but every piece
 * of workspace - kernel descriptors, the streaming kernel's 2*m*n doubles per
 * block, the multi-workgroup CholeskyQR2's per-block Q1, partial Gram
 * matrices and factors, the TSQR tree's row-block factors and the split-K
 * partials of its rebuild - lives in one fixed device array of
 * PEPS_QR_NOALLOC_BYTES per GPU (held from first use until the process ends;
 * its address is looked up when a context is created), with the
 * CholeskyQR2 route's arrival counters (one unsigned int per block).  The
 * call allocates no device or pinned host memory and waits for its work to
 * finish.  A request whose workspace does not fit fails with PEPS_ERR_OOM
 * before anything is launched.  Every call on one GPU shares that GPU's
 * array (the last call's data stays in it; nothing in it needs to start at
 * zero): calls that overlap on one GPU, from several threads or streams,
 * race and are not allowed. */
#define PEPS_QR_NOALLOC_BYTES (32u << 20)
peps_status peps_qr_noalloc(peps_ctx* ctx, const peps_qr_block* blk, int32_t n_blocks);

/* Diagnostics of an environment's row boundaries (the column boundaries of
 * PEPS_OPTS_COLUMNS are not included), truncated rows in order (top
 * boundaries T_0, T_1, ..., then bottom ones), any pointer may be NULL:
 * n_rows the number of truncated rows; max_halfsweeps the most half-sweeps
 * any of them ran; omegas (n_rows * max_halfsweeps doubles) the squared norm
 * of the ALS centre tensor after each half-sweep, NaN past a row's last;
 * sweeps (n_rows) the half-sweeps each row ran; n_unconverged the rows that
 * stopped at the cap before the tolerance (always 0 with tol == 0).  Waits
 * for the context's stream. */
peps_status peps_env_info(peps_env* env, int32_t* n_rows, int32_t* max_halfsweeps, double* omegas, int32_t* sweeps,
                          int32_t* n_unconverged);

/* Launch-shape autotuning of the contractions.  mode 1: every grouped
 * contraction (with beta = 0) whose signature - precision, output type,
 * tile family, widest N, longest K, total rows and group size to the next
 * power of two - has no stored choice is run and timed with each candidate
 * launch shape (the skinny kernel where it fits, each tile of the family
 * with and without split-K), and the fastest is stored; mode 0: stop
 * tuning, keep using the stored choices; mode 2: forget them (heuristic
 * shapes again).  Tuning calls synchronize and run each contraction several
 * times; the results they return are those of the chosen shape. */
peps_status peps_ctx_autotune(peps_ctx* ctx, int32_t mode);

/* Graph replay: when enabled, every launch sequence the library issues is
 * captured into a HIP graph, keyed by the bytes its kernels and copies read
 * from the host (descriptors with their device pointers, launch shapes,
 * uploaded data).  A later sequence that is byte-identical - the same call
 * on the same shapes and buffers, e.g. the same lattice again with new
 * tensor values written into the same device tensors - replays the graph
 * instead of uploading and launching op by op.  The context keeps at most
 * 512 graphs with their descriptor copies in device memory; disabling
 * waits for the stream and releases them.  Not combined with profiling
 * (profiled calls launch op by op). */
peps_status peps_ctx_graphs(peps_ctx* ctx, int32_t enable);

/* Profiling of the contraction kernel: when enabled, every contraction
 * launch is bracketed by HIP events on the context's stream; statistics are
 * kept per kernel variant, index = (prec*2 + out_dtype)*16 + tile
 * (prec: 0 f64, 1 f32, 2 bf16; out_dtype: 0 f64, 1 f32; tile: 0 64x64,
 * 1 128x32, 2 256x16, 3 32x128, 4 64x32, 5 64x16, 6 128x48, 7 64x80,
 * 8..12 the skinny kernel for outputs up to 16, 32, 48, 64, 80 wide, 13..14
 * the fused ket-bra kernel for dr*p up to 16, 32, 15 the fused two-row
 * column step).  Enabling clears the statistics. */
peps_status peps_ctx_profile(peps_ctx* ctx, int32_t enable);
/* Copies the PEPS_N_STATS per-variant statistics: algorithmic flops,
 * milliseconds, launch counts and algorithmic bytes (each operand read once,
 * the output written once) into host arrays of PEPS_N_STATS entries each;
 * bytes may be NULL. */
#define PEPS_N_STATS 96
peps_status peps_ctx_stats(peps_ctx* ctx, double* flops, double* ms, int64_t* launches, double* bytes);
/* Upper bound (bytes) of the transient workspace one call may hold for the
 * chain intermediates of a batch (default 48 GiB, at least 1 MiB); larger
 * batches run in several groups, and a call in which one sandwich alone
 * needs more fails with PEPS_ERR_OOM before any launch of its sandwiches. */
peps_status peps_ctx_set_workspace(peps_ctx* ctx, uint64_t bytes);

const char* peps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PEPS_ENV_H */
