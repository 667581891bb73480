/*
 * spamm.h - C ABI of the MI355X (gfx950) library for sparse approximate
 * matrix-matrix multiplication with error control, driven inside SP2
 * density-matrix purification (Artemov & Rubensson, "Sparse approximate
 * matrix-matrix multiplication for density matrix purification with error
 * control").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every pointer marked "device" is HIP device memory owned by the caller.
 *   The library never allocates, frees or retains caller memory; scratch
 *   space is the caller's workspace (ws, ws_bytes), sized with the matching
 *   *_workspace_bytes query.
 * - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *   the call returns before it finishes, except where a function says it
 *   reads results back to the host (it then synchronises `stream`).
 * - Return value: SPAMM_OK (0) on success, a negative SPAMM_E* code on
 *   error (nothing was enqueued, or the device results are invalid), or a
 *   positive SPAMM_W* warning (results valid).  spamm_last_error() returns
 *   a message for the last non-zero code of the calling thread.  No C++
 *   exception crosses this boundary.
 *
 * Block-sparse matrix (spamm_bsm)
 * -------------------------------
 * The quadtree of eq. (2) is stored linearised at the leaf level: an n x n
 * matrix with leaf size b has nb = ceil(n/b) block rows; each present leaf
 * block occupies one "slot" holding b*b doubles, column-major inside the
 * block (element (r, c) at offset c*b + r).  Rows/columns past n are zero
 * padding.  Absent blocks are identically zero quadrants.  A slot whose
 * brow is -1 is a hole (a block that was removed); every kernel skips it.
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SPAMM_OK 0
#define SPAMM_EINVAL (-1)     /* bad argument (message says which) */
#define SPAMM_ECAPACITY (-2)  /* an output capacity was too small */
#define SPAMM_EWORKSPACE (-3) /* workspace smaller than the query said */
#define SPAMM_EHIP (-4)       /* a HIP runtime call failed */
#define SPAMM_ENOTSUP (-5)    /* combination not supported */
#define SPAMM_WNOCONV 1       /* purification hit n_max before the stop rule */
#define SPAMM_WTAUFALLBACK 2  /* no candidate met the budget: tau = 0 (exact) */

/* flags */
#define SPAMM_SYMMETRIC 1u   /* A = B = X symmetric: outputs i <= j, C_ji = C_ij^T */
#define SPAMM_B_TRANSPOSED 2u /* B is given as its transpose Bt (Bt_jk = B_kj^T) */
#define SPAMM_SYNC 4u        /* synchronise the stream before returning */
#define SPAMM_BOUND_FLAT 16u  /* spamm_sweep_tau: B_flat = sqrt(sum_ij (sum_{k skipped} p_ikj)^2) (eq. (6) at the
                                 leaves) instead of Algorithm 3's recursive bound */
#define SPAMM_BOUND_SUM 32u   /* spamm_sweep_tau: B_sum = sum of the skipped p_ikj */
#define SPAMM_TIER_BF16 8u   /* spamm_multiply_tiered: low-tier pairs as split-BF16 products (needs
                                SPAMM_B_TRANSPOSED); default: FP32 products */

typedef void* spamm_stream_t; /* hipStream_t */

typedef struct spamm_bsm {
    int64_t n;       /* matrix order */
    int32_t b;       /* leaf size: 32, 64 or 128 */
    int32_t nb;      /* ceil(n / b) */
    int64_t cap;     /* capacity in slots of brow/bcol/val/norm/sq/sqlo */
    int32_t* nslot;  /* device [1]: slots in use (slots 0..nslot-1) */
    int32_t* brow;   /* device [cap]: block row of each slot, -1 = hole */
    int32_t* bcol;   /* device [cap]: block column of each slot */
    int32_t* map;    /* device [nb*nb]: slot of block (r, c) or -1 */
    double* val;     /* device [cap*b*b]: block values, column-major */
    double* norm;    /* device [cap]: Frobenius norm nu of each slot */
    double* sq;      /* device [cap]: RN(exact sum of squares) of each slot */
    double* sqlo;    /* device [cap]: sum of squares minus sq (double-double tail) */
} spamm_bsm;

/*
 * Block norms (the ||A||_F of the skip test of Algorithm 2 and the leaf
 * values of Algorithm 3).
 * For every live slot: sq = RN(sum of x^2) rounded once from the exact sum,
 * norm = correctly rounded sqrt(sq), sqlo = the double-double tail of the
 * sum (for traces).  Deterministic and independent of element order.
 * X: in/out (val read; norm, sq, sqlo written).  No workspace.
 */
int spamm_build_norms(spamm_bsm* X, spamm_stream_t stream);

/*
 * Error-bound sweep over candidate thresholds (Algorithm 3, CSE) followed by
 * the selection rule (the candidate whose bound is the largest one below
 * the budget).
 *   A, B      : inputs with norms built; B transposed when SPAMM_B_TRANSPOSED.
 *   tau       : device [N], strictly decreasing, > 0, 1 <= N <= 1024.
 *   budget    : device [1] (the product error budget delta), or NULL to use
 *               budget_host.
 *   mode      : 0 = the paper's leaf errors; 1 = precision tiers (tau is the
 *               list of low-precision limits sigma, tau0_dev[0] the fixed skip
 *               threshold, c_low the per-pair rounding factor of the low tier).
 *   flags     : SPAMM_B_TRANSPOSED, SPAMM_SYNC, and at most one of
 *               SPAMM_BOUND_FLAT / SPAMM_BOUND_SUM to replace Algorithm 3's
 *               recursive bound by a leaf-level one with the same leaf values
 *               (both modes; both flags -> SPAMM_EINVAL).  B_flat <= B_tree <= B_sum, and all three
 *               bound the product error, so FLAT admits the largest threshold.
 *               The leaf-level bounds add their per-output sums in a fixed
 *               order and are deterministic; they need nb <= 2048
 *               (SPAMM_ENOTSUP otherwise).
 *   bound_out : device [N] bound of ||SpAMM(A,B,tau_k) - AB||_F per candidate.
 *   idx_out   : device [1] selected index (N when none qualifies).
 *   tau_out   : device [1] selected threshold (0 when none qualifies).
 * With SPAMM_SYNC the call reads idx back and returns SPAMM_WTAUFALLBACK
 * (results valid) when no candidate qualified.
 * Workspace: spamm_sweep_workspace_bytes(nb, N).  Its size does not depend
 * on the occupancy: the octree's cube level is held densely, two arrays of
 * T^3 * N doubles with T = 2^(L - l0) cubes per side, L = ceil(log2 nb),
 * l0 = max(3, L - 7) (T <= 128): 17 MB at nb = 256 and N = 32, 11.7 GB at
 * nb = 2048 and N = 350, 34 GB at nb = 2048 and N = 1024.
 */
size_t spamm_sweep_workspace_bytes(int32_t nb, int32_t N);
int spamm_sweep_tau(const spamm_bsm* A, const spamm_bsm* B, const double* tau, int32_t N,
                    const double* budget, double budget_host, int32_t mode, const double* tau0_dev,
                    double c_low, uint32_t flags, double* bound_out, int32_t* idx_out, double* tau_out,
                    void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * SpAMM product at threshold tau (Algorithm 2 with the skip test applied to
 * leaf pairs; identical kept set to the recursive form because a leaf norm
 * never exceeds its ancestors').
 *   C~_ij = sum over k ascending with RN(nu(A_ik) nu(B_kj)) >= tau of A_ik B_kj
 * on the output pattern {(i,j): some kept k}; SPAMM_SYMMETRIC computes i <= j
 * and writes C_ji = C_ij^T.  tau_dev: device [1]; tau = 0 keeps every present
 * pair (the exact product).  C: output with its own capacity; its map is
 * rewritten, nslot set.  kept_out: device [2] = {kept pairs executed, output
 * blocks}; may be NULL.  SPAMM_ECAPACITY when C->cap or the workspace pair
 * capacity is too small (C->nslot then holds the required slot count).
 * Workspace: spamm_multiply_workspace_bytes(nb, max_pairs).
 */
size_t spamm_multiply_workspace_bytes(int32_t nb, int64_t max_pairs);
int spamm_multiply(const spamm_bsm* A, const spamm_bsm* B, const double* tau_dev, uint32_t flags,
                   spamm_bsm* C, int64_t* kept_out, void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * Truncation ||E||_F < delta (the truncation lines of Algorithms 1 and 5),
 * in place on a symmetric matrix with norms built.  Units are diagonal
 * blocks and symmetric off-diagonal pairs; with T = RN(delta^2) and
 * Q = 2^(floor(log2 T) - 40), each unit gets the integer key
 * k = ceil(w*sq/Q) (w = 1 diagonal, 2 pair; saturated at 2^41).  Units are
 * taken in ascending (k, r*nb + c) order and the longest prefix whose key
 * sum stays below K_T = floor(T/Q) is removed, which guarantees the exact
 * removed Frobenius norm is < delta (the key sum is then at most K_T - 1,
 * a margin of Q > 2^-41 T over the rounding of sq and of T).
 * Removed slots become holes.  removed_out: device [2] = {removed units,
 * removed sum of w*sq}; may be NULL.
 * Workspace: spamm_truncate_workspace_bytes(cap).
 */
/*
 * SpAMM product with a low-precision tier (mixed-precision leaf products;
 * not in the paper): kept pairs with tau <= p < sigma run in low precision,
 * each pair's product added into the FP64 accumulator, with
 * ||fl(A_ik B_kj) - A_ik B_kj||_F <= c_t p (spamm_tier_constant):
 *   FP32 tier (default): FP32 copies on the FP32 MFMA,
 *     c_32 = 2u + u^2 + gamma_b(2u)(1+u)^2 + 2^-31, u = 2^-24 (the last
 *     term covers entries and partial results below FP32's normal range);
 *     a pair whose A or B block has a norm below 2^-40 stays FP64;
 *   split-BF16 tier (SPAMM_TIER_BF16, needs SPAMM_B_TRANSPOSED): each block
 *     scaled by a power of two and split x = hi + lo (BF16), the products
 *     hi*hi + hi*lo + lo*hi on the BF16 MFMA with FP32 accumulation, rescaled
 *     exactly; c_bf16 = kappa + gamma_3b(2^-23)(1 + 2u)(1+u)^2 + 2^-100,
 *     kappa = u^2 ((1+u)^2 + 2(1+u)^3 + u^2 (1+u)^2), u = 2^-8.
 * Both rounded up by 1 + 2^-40.  Pairs with p >= sigma are FP64.  Leaf 32 or
 * 64.  kept_out: device [3] = {kept pairs, output blocks, low-tier pairs};
 * may be NULL.
 * Workspace: spamm_multiply_tiered_workspace_bytes(nb, capA, capB, b, max_pairs).
 */
size_t spamm_multiply_tiered_workspace_bytes(int32_t nb, int64_t capA, int64_t capB, int32_t b, int64_t max_pairs);
int spamm_multiply_tiered(const spamm_bsm* A, const spamm_bsm* B, const double* tau_dev, const double* sigma_dev,
                          uint32_t flags, spamm_bsm* C, int64_t* kept_out, void* ws, size_t ws_bytes,
                          spamm_stream_t stream);
/* c_t of a precision tier (1 = FP32, 2 = split BF16) for leaf size b: the per-pair factor of
 * the rounding bound ||fl(A B) - A B||_F <= c_t ||A||_F ||B||_F. */
double spamm_tier_constant(int32_t precision, int32_t b);

size_t spamm_truncate_workspace_bytes(int64_t cap);
int spamm_truncate(spamm_bsm* X, double delta, uint32_t flags, double* removed_out, void* ws,
                   size_t ws_bytes, spamm_stream_t stream);

/*
 * Allocation-free truncation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same operation, kernels and results as spamm_truncate, with
 * its scratch in a fixed device array of the library instead of a workspace:
 * the call allocates nothing (no hipMalloc/hipFree, no allocating library
 * routine).  The array holds the temporaries of X->cap <= 2^20 slots
 * (spamm_truncate_noalloc_max_cap(); about 16 MiB, one copy per GPU the
 * library runs on, held until the process ends); a larger X->cap is
 * rejected with SPAMM_EINVAL.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or host threads at once)
 * race and must be serialised by the caller.
 *   X, delta, flags, removed_out: as spamm_truncate.
 */
int64_t spamm_truncate_noalloc_max_cap(void);
int spamm_truncate_noalloc(spamm_bsm* X, double delta, uint32_t flags, double* removed_out,
                           spamm_stream_t stream);

/* Parameters of purify_sp2 (Algorithms 1, 4 and 5 with SP2 polynomials). */
typedef struct sp2_params {
    int64_t n_occ;       /* occupied count: the trace the iteration converges to */
    double eps;          /* target ||D - D~||_F */
    int32_t n_max;       /* iteration limit (SPAMM_WNOCONV when reached) */
    int32_t variant;     /* 0 hybrid (Alg. 5), 1 SpAMM only (Alg. 4), 2 truncmul (Alg. 1) */
    const double* tau;   /* device [N] candidate thresholds (see spamm_sweep_tau) */
    int32_t N;
    double homo, lumo;   /* eigenvalue bounds of F around the gap (homo < lumo), or NaN */
    double delta_const;  /* explicit per-step delta when homo/lumo are NaN (else NaN) */
    double e_tol;        /* stop when |tr X - ||X||_F^2| <= e_tol (0: noise-floor rule only) */
    int32_t keep_tape;   /* 0: none; 1: keep every X~_i in the workspace; k > 1: keep X~_0, X~_k,
                            X~_2k, ... (checkpoints for the adjoint) */
    int32_t precision;   /* 0 FP64 leaf products; for pairs with tau <= p < sigma (leaf 32/64):
                            1 FP32 tier, 2 split-BF16 tier (hi*hi + hi*lo + lo*hi on the BF16 MFMA) */
    double tier_split;   /* share of the product budget given to skipping when precision != 0 (e.g. 0.5) */
    int32_t graph_steps; /* 0: host-driven loop (per-iteration phase timings); K > 0: the step is
                            captured once as a HIP graph with its decisions taken on the device
                            and replayed, the host polling the stop flag every K iterations
                            (requires keep_tape == 0; phase timings are 0) */
    int32_t bound_kind;  /* threshold selection: 0 Algorithm 3 (B_tree), 1 B_flat, 2 B_sum (see
                            SPAMM_BOUND_FLAT / SPAMM_BOUND_SUM); with a precision tier the
                            same bound selects sigma */
} sp2_params;

/* Per-iteration record written by purify_sp2 (host memory). */
typedef struct sp2_iter_log {
    int32_t i, branch, idx, stop; /* branch 0: x^2, 1: 2x - x^2; stop != 0 on the final record */
    double delta, tau, t1, t2, e;
    int64_t npairs, nout, nslot_hat, nslot_kept, removed_units; /* kept pairs, output blocks of the product,
                                                                   blocks of X^_i, blocks of X~_i (X^_i's minus
                                                                   the truncated ones), truncated units */
    double removed_fro2;
    /* stream-event times in ms: threshold sweep (and the precision tier's copies), kept pairs
       and output pattern, the leaf-product kernel alone (which also forms
       the block norms of its outputs), pass-through blocks and the norms the
       product could not certify, truncation, whole iteration */
    float ms_sweep, ms_pairs, ms_gemm, ms_norms, ms_trunc, ms_total;
    int64_t npairs_low;  /* pairs evaluated in the low-precision tier */
    double sigma;        /* low-precision limit of the step (0: none) */
    int32_t sidx, pad;
} sp2_iter_log;

/*
 * Purification: X_0 = (lmax I - F)/(lmax - lmin) with Gerschgorin bounds,
 * X~_0 truncated with delta_0, then X~_i = trunc(SpAMM-evaluated f_i(X~_{i-1}))
 * with f_i = x^2 or 2x - x^2 (the trace closer to n_occ), the SpAMM
 * threshold chosen by the sweep with budget delta_i/2 and the truncation
 * with delta_i/2 (Algorithm 5), delta_i = eps*g_i/(2*sqrt(2)*(n_max + 1))
 * from the mapped gap g_i (the occupied projector then drifts by at most
 * eps/2 over the run, Davis-Kahan), until the stop rule fires: |e| <= e_tol
 * or, with e = tr X~ - ||X~||_F^2, |e_{i-2}| <= 1/8 and
 * |e_i| > 4 e_{i-2}^2 / (1 - 2|e_{i-2}|)^2 (no quadratic convergence).
 *   F     : symmetric input with norms NOT required (computed internally).
 *   D     : output, capacity D->cap slots (SPAMM_ECAPACITY otherwise), with
 *           its block norms (as spamm_build_norms computes them).
 *   Returns SPAMM_WNOCONV when n_max was reached first, else
 *   SPAMM_WTAUFALLBACK when some step (Algorithms 5 and 4) found no candidate
 *   threshold below its budget and used the exact product (results valid).
 *   log   : host [n_max + 2] records; nlog_out: records written.
 * Workspace: purify_sp2_workspace_bytes(nb, b, N, cap_blocks, max_pairs, tape_steps, precision) with
 * tape_steps = n_max (keep_tape = 1), n_max / keep_tape (keep_tape > 1) or 0.
 * Host-driven loop: reads the spectral bounds back once, then scalars every
 * iteration (synchronises the stream; the read-back goes through a small
 * pinned host buffer allocated for the call).  Graph mode (graph_steps > 0):
 * same decisions, same kernels and bit-identical results; nothing is read
 * back before the loop (a kernel sets the control block up from the bounds
 * on the device; only a D->cap below nb^2 makes the call read F's slot count
 * first), the graph is captured on a stream kept per host thread and device
 * (created on first use, never destroyed), and the stream is synchronised
 * once per graph_steps iterations.  With the split-BF16 tier (precision 2)
 * the host-driven loop forks the BF16 copies of X~_i onto a second kept
 * stream (same lifetime, default priority) beside the threshold sweeps and
 * joins it back before the leaf products; the graph keeps them on its one
 * stream.  Either way the call's work is complete when `stream` is.
 */
size_t purify_sp2_workspace_bytes(int32_t nb, int32_t b, int32_t N, int64_t cap_blocks, int64_t max_pairs,
                                  int32_t tape_steps, int32_t precision);
int purify_sp2(const spamm_bsm* F, const sp2_params* p, spamm_bsm* D, sp2_iter_log* log, int32_t* nlog_out,
               void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * View of tape entry `step` (X~_step, 0 <= step <= tape_steps) inside a
 * purify_sp2 workspace that was run with keep_tape: fills *out with device
 * pointers into ws (no copy).  Arguments must equal those of the
 * purify_sp2_workspace_bytes query the workspace was sized with.
 */
int purify_sp2_tape_view(void* ws, int32_t nb, int32_t b, int32_t N, int64_t cap_blocks, int64_t max_pairs,
                         int32_t tape_steps, int32_t step, spamm_bsm* out);

/*
 * Reverse mode (not in the paper).  With the decisions of a forward run held
 * fixed -- the kept set K_t of every step (leaf-level skip test of
 * Algorithm 2 at tau_t), the truncation pattern S_t of every iterate, the
 * branch f_t and the Gerschgorin bounds of the starting matrix -- the
 * purification of Algorithms 1/4/5 is a polynomial map F -> D~.  These
 * entry points evaluate its gradient for symmetric perturbations: for a
 * loss L(D~), Fbar satisfies <Fbar, H> = dL[H] for every symmetric H, and
 * Fbar is symmetric.
 *
 * One frozen step X~' = mask_{S'}(f(C(X))), C(X)_ij = sum over (i,k,j) in K
 * of X_ik X_kj, K = {(i,k,j): RN(nu(X_ik) nu(X_kj)) >= tau}, f = x^2
 * (branch 0) or 2x - x^2 (branch 1):
 *   X        : X~_{t-1}, norms valid (spamm_build_norms, or a tape entry).
 *   G        : gradient with respect to X~' on its pattern (the pattern of
 *              X~_t), symmetric in pattern and values; only its pattern
 *              arrays and val are read.
 *   xbar_val : output, device [X->cap * b * b] doubles in X's slot layout:
 *              the gradient with respect to X~_{t-1} on its pattern,
 *              Xbar = A + A^T (branch 0) or 2G - (A + A^T) (branch 1),
 *              A_ik = sum_{j: (i,k,j) in K} G_ij X_kj^T.  Slots that are
 *              holes (brow = -1) are not written.
 *   counts_out : optional device int64[2]: output blocks (i <= k) and block
 *              pairs of the step's product launch.
 * Workspace: spamm_adjoint_step_workspace_bytes(nb, X->cap, max_pairs);
 * SPAMM_ECAPACITY when the pair list needs more than max_pairs.
 * Synchronises the stream (it reads the overflow flag back).
 */
size_t spamm_adjoint_step_workspace_bytes(int32_t nb, int64_t cap_blocks, int64_t max_pairs);
int spamm_adjoint_step(const spamm_bsm* X, const spamm_bsm* G, double tau, int32_t branch, double* xbar_val,
                       int64_t* counts_out, void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * Gradient of a loss with respect to F through a whole recorded purification.
 *   F        : the input of the forward run (pattern arrays, n, b).
 *   p        : the forward run's parameters (variant, precision).
 *   tape, ntape, tape_every : host array of handles (purify_sp2_tape_view
 *              of a run with keep_tape = tape_every):
 *              tape_every = 1: every iterate X~_0 .. X~_T (T = nlog - 1
 *                steps), ntape = nlog;
 *              tape_every = k > 1: checkpoints X~_0, X~_k, X~_2k, ...; each
 *                segment is recomputed from its checkpoint with the recorded
 *                thresholds, branches and deltas by the forward's own
 *                kernels (bit-identical iterates), FP64 runs only.
 *              The forward workspace must be unchanged.
 *   D        : the run's result D~ = X~_T (required with checkpoints, may be
 *              NULL with a full tape).
 *   log      : the forward run's records: record t-1 holds tau, delta and
 *              the branch of step t; the last record is the stop.
 *   dbar_val : device [cap * b * b]: dL/dD~ in the slot layout of D~ (only
 *              its symmetric part is used).
 *   fbar_val : output, device [F->cap * b * b] in F's slot layout:
 *              Fbar = -Xbar_0 / (lmax - lmin) on the blocks of F that the
 *              first truncation kept, zero on those it removed.
 * Workspace: purify_sp2_adjoint_workspace_bytes(nb, b, cap, max_pairs,
 * tape_every) with cap the tape entries' capacity; with checkpoints it also
 * holds tape_every - 1 matrices of that capacity and the recomputation's
 * own pair list (of the same max_pairs).  SPAMM_ECAPACITY when a pair list
 * needs more than max_pairs (a bound: nb^2 (nb + 1)).  Synchronises.
 */
size_t purify_sp2_adjoint_workspace_bytes(int32_t nb, int32_t b, int64_t cap_blocks, int64_t max_pairs,
                                          int32_t tape_every);
int purify_sp2_adjoint(const spamm_bsm* F, const sp2_params* p, const spamm_bsm* tape, int32_t ntape,
                       int32_t tape_every, const spamm_bsm* D, const sp2_iter_log* log, int32_t nlog,
                       const double* dbar_val, double* fbar_val, void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * Batched purification of nsys independent systems (not in the paper; each
 * system is Algorithm 5/4/1 exactly as purify_sp2 runs it).  The step of
 * every system is captured once in a HIP graph with the decisions on the
 * device (as purify_sp2 with graph_steps > 0) and replayed until every
 * system has stopped; systems that stop early drop out of the later steps.
 * Per step there is ONE persistent launch of the leaf-product kernel for
 * all systems of a leaf size and tier: it walks the concatenation of their
 * output lists, balanced by kept-pair count over the 8 XCDs.  Each system's
 * result, records and status are bit-identical to its own purify_sp2 run.
 *   F, p, D    : host arrays [nsys] (same contracts as purify_sp2; keep_tape
 *                must be 0; capacities D[q].cap).  D[q] also serves as the
 *                second iterate buffer of system q during the run (the
 *                workspace holds one matrix of that capacity per system, not
 *                two); on return it holds D~ of system q, or scratch contents
 *                when that system failed.  D[q] must not overlap F or the
 *                workspace.
 *   max_pairs  : host [nsys] kept-pair capacity per system.
 *   log        : host [nsys * log_stride], log_stride >= n_max + 2 of every
 *                system; nlog_out, status_out: host [nsys].
 *   graph_steps: the largest of the systems' values is the poll interval.
 * Returns the worst status (negative if any system failed; the others
 * still carry their results).  Synchronises the stream.
 */
size_t purify_sp2_batched_workspace_bytes(int32_t nsys, const spamm_bsm* F, const sp2_params* p,
                                          const int64_t* cap_blocks, const int64_t* max_pairs);
int purify_sp2_batched(int32_t nsys, const spamm_bsm* F, const sp2_params* p, spamm_bsm* D,
                       const int64_t* max_pairs, sp2_iter_log* log, int32_t log_stride, int32_t* nlog_out,
                       int32_t* status_out, void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * Re-blocking (not in the paper): Y = X on another leaf size (Y->b any of
 * 32, 64, 128; Y->n == X->n).  A block of Y is present when a block of X it
 * overlaps is present; values are copied (0 where X has no block or past
 * n); slots of Y in 2D Morton order; norms of Y computed.  Y->cap must hold
 * the blocks (SPAMM_ECAPACITY otherwise; nb_Y^2 always suffices).
 * Workspace: spamm_reblock_workspace_bytes(Y->nb).  Synchronises.
 */
size_t spamm_reblock_workspace_bytes(int32_t nb_to);
int spamm_reblock(const spamm_bsm* X, spamm_bsm* Y, void* ws, size_t ws_bytes, spamm_stream_t stream);

/*
 * Schedule of the leaf-product kernels: workgroups per CU of the persistent
 * grid for leaf size b (0 restores the default: 4, 3, 2 for b = 32, 64,
 * 128).  Process-wide; results do not depend on it (every output block is
 * computed by one workgroup in the same order whatever the grid).
 * spamm_get_gemm_schedule returns the current value.
 */
int spamm_set_gemm_schedule(int32_t b, int32_t workgroups_per_cu);
int spamm_get_gemm_schedule(int32_t b);

/*
 * Small-system passes (not in the paper): for nb <= 64 the occupancy and
 * sweep-list pass, the kept-pair and output-pattern passes of a product and
 * the truncation (iterates of at most 4096 slots) each run in one workgroup
 * instead of a chain of device-wide launches.  Same lists in the same order,
 * so every result is bit-identical either way; only the number of dependent
 * launches per purification step changes.  on: 1 (default) or 0;
 * process-wide, read when work is enqueued (a captured graph keeps the
 * passes it was captured with).  SPAMM_EINVAL for other values.
 * spamm_get_small_path returns the current setting.
 */
int spamm_set_small_path(int32_t on);
int spamm_get_small_path(void);

/*
 * Leaf-size and schedule autotuner (not in the paper).  For each leaf size
 * (32, 64, 128; 32 and 64 with a precision tier) F is re-blocked and the first
 * trial_steps steps of its purification with parameters p are timed (the
 * delta schedule is the one of the full run); the mean time of the steps
 * after the first decides the leaf size.  Then every workgroups-per-CU
 * setting up to the default is timed on the leaf products of the chosen
 * size, and the fastest is installed (spamm_set_gemm_schedule).
 *   best_b, best_per_cu : outputs; ms_per_step: host [3] mean step times for
 *   b = 32, 64, 128 (-1 where not tried).
 * Workspace: purify_sp2_autotune_workspace_bytes(F->n, p->N, p->precision).
 * Synchronises.
 */
size_t purify_sp2_autotune_workspace_bytes(int64_t n, int32_t N, int32_t precision);
int purify_sp2_autotune(const spamm_bsm* F, const sp2_params* p, int32_t trial_steps, int32_t* best_b,
                        int32_t* best_per_cu, float* ms_per_step, void* ws, size_t ws_bytes, spamm_stream_t stream);

const char* spamm_status_str(int code);
const char* spamm_last_error(void);
int spamm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPAMM_H */
