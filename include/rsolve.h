/*
 * rsolve.h -- C-ABI of the recycled GMRES(m) solver for sequences of sparse
 * non-symmetric systems A_i x_i = b_i (one system per time step), built for
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Pitton & Heltai, "Accelerating the iterative solution of
 * convection-diffusion problems using singular value decomposition"):
 *   - the systems form a sequence whose matrix and right-hand side may depend
 *     on the previous solution, and arrive one at a time (section 2, the
 *     closing paragraph of the problem statement); n is fixed per sequence
 *     (section 4, opening of the initial-guess discussion);
 *   - each solve is restarted GMRES(m) (section 3, minimal-residual choice
 *     C_k = A S_k) accelerated by a recycle basis W (the paper's V_s): the
 *     Krylov operator is P A with the oblique projector
 *     P = I - A W (W^T A W)^{-1} W^T (section 3.2, eq. (left_deflation);
 *     section 3.3, Table 1 rows "augmented oblique" / "deflated oblique"),
 *     and the initial guess is the Galerkin projection onto span(W)
 *     (section 4.2, eqs. (projection_guess), (projection_t_s));
 *   - after each solve the solution is stored in a ring of the s most recent
 *     solutions and every `svd_interval` solves W is replaced by the k
 *     dominant left singular vectors of the ring (section 5.2, Algorithm 1).
 *
 * Conventions for every entry point:
 *   - All matrix / vector pointers are DEVICE pointers (HIP, the GPU the
 *     sequence was created on) unless the argument says "host".
 *   - Dense vectors are float64, length n.  CSR matrices are 0-based with
 *     int32 row pointers and column indices, columns sorted strictly
 *     increasing within each row, and an explicitly stored diagonal entry in
 *     every row (required by the Jacobi preconditioner).
 *   - The caller owns every buffer it passes.  The library never allocates
 *     device memory: all of a sequence's state lives in the caller-provided
 *     workspace, which must stay allocated until rsolve_destroy_sequence.
 *   - Entry points return an int status (RSOLVE_OK = 0, RSOLVE_NOT_CONVERGED
 *     = 1, negative = error); no entry point aborts, throws or exits.
 *   - A sequence handle is not thread-safe; distinct handles are independent
 *     and may be used from different host threads on different streams.
 */
#ifndef RSOLVE_H
#define RSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define RSOLVE_OK             0
#define RSOLVE_NOT_CONVERGED  1   /* max_iters reached; x holds the last iterate, stats filled */
#define RSOLVE_E_INVALID     -1   /* bad argument: null handle/pointer, n/nnz mismatch, tol <= 0,
                                     config out of range, corrupt CSR (found on the device) */
#define RSOLVE_E_NONFINITE   -2   /* NaN/Inf met in a norm (b, A or the iteration) */
#define RSOLVE_E_WORKSPACE   -3   /* workspace too small or misaligned (256-byte alignment) */
#define RSOLVE_E_DEVICE      -4   /* a HIP runtime call failed */
#define RSOLVE_E_STATE       -5   /* call out of order (e.g. update before any solve) */
#define RSOLVE_E_BUDGET      -6   /* serving loop: not enough free pool memory or no free slot */

/* ---- configuration values ---- */
#define RSOLVE_PLAIN          0   /* GMRES(m) without recycling */
#define RSOLVE_AUG_OBLIQUE    1   /* Table 1, augmented oblique */
#define RSOLVE_DEFL_OBLIQUE   2   /* Table 1, deflated oblique (same iteration under right
                                     preconditioning with the projected initial guess) */
#define RSOLVE_AUG_ORTHO      3   /* Table 1, augmented orthogonal: Krylov operator (I - W W^T) A D^{-1};
                                     GMRES minimises the projected residual, the cycle-end correction
                                     x += W E^{-1} W^T r makes W^T r = 0 (multi-kernel path only) */
#define RSOLVE_DEFL_ORTHO     4   /* Table 1, deflated orthogonal: also the initial vector projected
                                     (the same iteration once the projected guess leaves W^T r = 0) */
#define RSOLVE_GUESS_PROJECT  5   /* section 4.2: the projection guess x0 + W E^{-1} W^T (b - A x0) onto
                                     the recycle space, then GMRES(m) with the unmodified operator
                                     A D^{-1} and no cycle-end correction (eq. (iteration_projection)) */
#define RSOLVE_GUESS_EXTRAP2  6   /* section 4.1, eq. (ext2): x0 = 2 x_{i-1} - x_{i-2} from the ring of
                                     previous solutions, then plain GMRES(m) */
#define RSOLVE_GUESS_EXTRAP3  7   /* eq. (ext3): x0 = 3 x_{i-1} - 3 x_{i-2} + x_{i-3} */
#define RSOLVE_GUESS_EXTRAP4  8   /* eq. (ext4): x0 = 4 x_{i-1} - 6 x_{i-2} + 4 x_{i-3} - x_{i-4}.
                                     The extrapolation methods keep the ring only (recycle_k = 0,
                                     snapshots_s >= the order, no SVD); with fewer stored solutions
                                     than the order the highest order they allow is used (the last
                                     solution alone once one is stored), and x0 is used only while
                                     the ring is empty.  None of 5..8 runs on the one-block path. */
#define RSOLVE_AUG_LS         9   /* Table 1, augmented LS (section 3.3, the third projector): Krylov
                                     operator P_LS A D^{-1} with P_LS = I - A W (W^T A^T A W)^{-1} W^T A^T,
                                     the orthogonal projector onto the complement of range(A W); the
                                     Krylov initial vector is r itself.  Projected guess as for the
                                     oblique rows; every cycle ends with the least-squares correction
                                     x += W c, r -= A W c, c = (W^T A^T A W)^{-1} W^T A^T r, after which
                                     the true residual is the minimised one (multi-kernel path only) */
#define RSOLVE_DEFL_LS       10   /* Table 1, deflated LS: the Krylov initial vector is P_LS r (the inner
                                     iteration of GCRO); applied as a least-squares correction of x
                                     and r before the first cycle, which leaves the same iterates */
#define RSOLVE_PRECOND_NONE   0
#define RSOLVE_PRECOND_JACOBI 1   /* right Jacobi: operator P A D^{-1}, x = x0 + D^{-1} V y */
#define RSOLVE_PRECOND_SSOR   2   /* right multicolour SSOR (the paper's SSOR of section 6.1 on a
                                     colour ordering): M = (D + w L) D^{-1} (D + w U) / (w (2 - w)) with
                                     L, U the couplings of each row to rows of lower / higher colour,
                                     the colouring first fit in natural row order over the symmetrised
                                     pattern (computed on the host when the pattern is validated, so
                                     pass RSOLVE_SAME_PATTERN for a repeated pattern); operator
                                     P A M^{-1}, x = x0 + M^{-1} V y.  FP64 only, CSR product, not with
                                     the Ritz selections, not on the one-block path, no graphs */
#define RSOLVE_FP64           0   /* everything in float64 */
#define RSOLVE_FP32_IR        1   /* float32 Arnoldi cycles inside float64 iterative refinement */
#define RSOLVE_SELECT_LARGEST 0   /* W = leading left singular vectors (Algorithm 1) */
#define RSOLVE_SELECT_SMALLEST 1  /* W = left singular vectors of the k smallest singular values above
                                     the numerical rank cut (section 5.2, the other choice) */
#define RSOLVE_SELECT_RITZ     2  /* W = Ritz vectors of A (section 5.1, eqs. (def_Ritz_pair),
                                     (eigenvalues_hessenberg)) over the search space of the last
                                     solve, span(W) + span(D^{-1} V_j) with V_j the basis of its last
                                     cycle: the k pairs of smallest |theta|, a complex pair as the real
                                     and imaginary parts of its vector and only whole, orthonormalised
                                     (rank cut as for the ring).  Prepared at the end of each solve,
                                     installed by rsolve_update_recycle (whose x is then not stored; no
                                     snapshot ring is kept).  Needs recycle_k >= 1 and recycle_k +
                                     restart_m <= 64; not on the one-block path */
#define RSOLVE_SELECT_HARMONIC 3  /* the same with harmonic Ritz vectors, (A U)^T (A U) z = theta (A U)^T U z
                                     (eq. (eigenvalues_harmonic)) */
#define RSOLVE_ORTHO_CGS2     0   /* classical Gram-Schmidt applied twice: three basis sweeps per step */
#define RSOLVE_ORTHO_DCGS2    1   /* the same Arnoldi process with the second pass of each basis vector
                                     merged into the next step: two basis sweeps per step, the
                                     Hessenberg column and its rotation one step later */

/* ---- limits ---- */
#define RSOLVE_MAX_RESTART    128
#define RSOLVE_MAX_RECYCLE    64
#define RSOLVE_MAX_SNAPSHOTS  64

/* ---- solve flags (rsolve_stats.flags) ---- */
#define RSOLVE_FLAG_RECYCLE_DROPPED 1u  /* cond_1(W^T A W) > 1e13: this solve ran without W */
#define RSOLVE_FLAG_BREAKDOWN_LUCKY 2u  /* h_{j+1,j} <= 1e-14 ||h_j||: Krylov space invariant */
#define RSOLVE_FLAG_NONFINITE       4u

/* ---- rsolve_csr.flags ---- */
#define RSOLVE_SAME_PATTERN 1u  /* row_ptr/col_idx are those of the previous solve of this
                                   sequence (same content): skip validation and pattern setup */

typedef struct rsolve_seq rsolve_seq;

typedef struct {
    int32_t restart_m;     /* GMRES restart length m, 1..RSOLVE_MAX_RESTART */
    int32_t recycle_k;     /* recycle dimension k, 0..RSOLVE_MAX_RECYCLE (0 = plain) */
    int32_t snapshots_s;   /* snapshot ring size s, k <= s <= RSOLVE_MAX_SNAPSHOTS (0 if k = 0; unused by
                              the Ritz selections);
                              for RSOLVE_GUESS_EXTRAPq: q <= s (the ring of previous solutions) */
    int32_t svd_interval;  /* ell >= 1: recompute W every ell updates (Algorithm 1) */
    int32_t method;        /* RSOLVE_PLAIN / _AUG_OBLIQUE / _DEFL_OBLIQUE / _AUG_ORTHO / _DEFL_ORTHO /
                              _GUESS_PROJECT / _GUESS_EXTRAP2 / _GUESS_EXTRAP3 / _GUESS_EXTRAP4 /
                              _AUG_LS / _DEFL_LS */
    int32_t precond;       /* RSOLVE_PRECOND_NONE / RSOLVE_PRECOND_JACOBI / RSOLVE_PRECOND_SSOR */
    int32_t precision;     /* RSOLVE_FP64 / RSOLVE_FP32_IR */
    int32_t max_iters;     /* cap on Arnoldi steps per solve (>= 1) */
    int32_t select;        /* RSOLVE_SELECT_LARGEST / _SMALLEST (SVD of the ring) / _RITZ / _HARMONIC */
    int32_t ortho;         /* RSOLVE_ORTHO_CGS2 (0) / RSOLVE_ORTHO_DCGS2 (1): Arnoldi orthogonalisation
                              of the multi-kernel path (the one-block path always uses CGS2) */
    double  inner_tol;     /* FP32_IR only: an FP32 cycle stops once its residual estimate has
                              dropped by this factor (0 < inner_tol < 1); ignored for FP64 */
    double  ssor_omega;    /* RSOLVE_PRECOND_SSOR: relaxation factor w, 0 < w < 2 (0 selects 1, symmetric
                              Gauss-Seidel); ignored otherwise */
} rsolve_config;

typedef struct {
    int64_t n;             /* rows = columns */
    int64_t nnz;           /* stored entries, n <= nnz <= nnz_max of the sequence */
    const int32_t* row_ptr;  /* device, n + 1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t* col_idx;  /* device, nnz entries */
    const double*  val;      /* device, nnz entries */
    uint32_t flags;        /* RSOLVE_SAME_PATTERN or 0 */
    uint32_t reserved;     /* must be 0 */
} rsolve_csr;

typedef struct {
    int32_t iterations;    /* Arnoldi steps (one SpMV each) over all cycles of this solve */
    int32_t cycles;        /* GMRES cycles (restarts + 1); FP32_IR: refinement steps */
    int32_t k_eff;         /* recycle columns used by this solve */
    int32_t converged;     /* 1 if ||b - A x||_2 <= tol ||b||_2 (checked explicitly in FP64) */
    uint32_t flags;        /* RSOLVE_FLAG_* */
    int32_t its_estimate_met; /* Arnoldi steps taken when a cycle first ended with its residual estimate
                              |g_{j+1}| <= tol ||b||_2 (the projected residual for the orthogonal and
                              least-squares rows): the count of a solver that stops on that estimate,
                              as a left-preconditioned GMRES stopping on its own residual does; 0 when
                              the initial guess already meets tol, -1 when no cycle met it.  The
                              one-block path reports the step count of a converged solve */
    double rel_res_true;   /* ||b - A x||_2 / ||b||_2 of the returned x (FP64) */
    double rel_res_implicit; /* last Givens residual estimate / ||b||_2 */
    double t_setup_ms;     /* validation, Jacobi scaling, A W, W^T A W, LU, initial guess */
    double t_cycles_ms;    /* Arnoldi cycles and end-of-cycle corrections */
    double t_total_ms;     /* wall time of the call (host clock, call entry to return) */
} rsolve_stats;

/*
 * Bytes of device workspace a sequence needs for systems of size n with at
 * most nnz_max stored entries.  Returns 0 if the configuration is invalid.
 * Layout (all 256-byte aligned, column-major tall blocks with leading
 * dimension ld = n rounded up to 64): Krylov basis V (m+1 columns), recycle
 * basis W and A W (k columns each), snapshot ring (s columns), work vectors,
 * scaled matrix values (nnz_max), float32 shadows in FP32_IR mode, TSQR
 * levels, per-block reduction partials and a control block.
 */
size_t rsolve_workspace_bytes(const rsolve_config* cfg, int64_t n, int64_t nnz_max);

/*
 * Create a sequence.  `hip_stream` is a hipStream_t (NULL = the null stream)
 * on which every kernel of this sequence is enqueued; `workspace` is a device
 * buffer of at least rsolve_workspace_bytes(cfg, n, nnz_max) bytes, 256-byte
 * aligned, owned by the caller.  The HIP device current on the calling thread
 * must be the one that owns the workspace.  Errors: E_INVALID (cfg, n, out),
 * E_WORKSPACE, E_DEVICE.
 */
int rsolve_create_sequence(const rsolve_config* cfg, int64_t n, int64_t nnz_max,
                           void* hip_stream, void* workspace, size_t ws_bytes,
                           rsolve_seq** out);

/*
 * Solve A x = b until ||b - A x||_2 <= tol ||b||_2 (stopping rule of
 * section 6.1; the check is an explicit FP64 residual).  x0 may be NULL
 * (zero start) and x may alias x0.  The initial guess is
 * x0 + W E^{-1} W^T (b - A x0) when the sequence holds a recycle basis; with
 * x0 = NULL this is the projection guess W E^{-1} W^T b of section 4.2.  For
 * the extrapolation methods the guess is the extrapolation of the stored
 * solutions (x0 only while none is stored).
 * Synchronous: returns after x and *st are final.  A's buffers need only stay
 * valid for the duration of the call.  b = 0 gives x = 0 and 0 iterations.
 * Returns OK, NOT_CONVERGED (x = last iterate), E_INVALID (bad pointers, n
 * mismatch, nnz out of range, tol <= 0, corrupt CSR), E_NONFINITE, E_DEVICE.
 */
int rsolve_solve(rsolve_seq* s, const rsolve_csr* A, const double* b, const double* x0,
                 double* x, double tol, rsolve_stats* st);

/*
 * Algorithm 1 of section 5.2: store x (device, n entries; NULL = the last
 * solution returned by rsolve_solve) in the ring of the s most recent
 * solutions; when the number of stored solutions is a multiple of
 * svd_interval, replace W by the min(k, numerical rank) leading left singular
 * vectors of the ring (numerical rank: sigma_i > sigma_1 * max(n, c) * 2^-52
 * with c the number of stored columns).  The extrapolation methods only store
 * x (no SVD; W stays empty; a non-finite x surfaces in the next solve).
 * Synchronous.  Errors: E_STATE (x =
 * NULL before any solve), E_INVALID, E_NONFINITE (non-finite snapshot),
 * E_DEVICE.
 */
int rsolve_update_recycle(rsolve_seq* s, const double* x);

/*
 * Read the recycle state: *k_eff = current number of columns of W, *rank =
 * numerical rank of the ring at the last SVD, sigma_host (host, may be NULL)
 * receives min(cap, c) singular values in descending order.  If W_out
 * (device, may be NULL) is given, W is copied there column-major with leading
 * dimension ld_out >= n.  Synchronous.
 */
int rsolve_get_recycle(rsolve_seq* s, int32_t* k_eff, int32_t* rank, double* sigma_host,
                       int32_t cap, double* W_out, int64_t ld_out);

/* ---- checkpoint and resume ----
 *
 * The state a sequence carries from one solve to the next: Algorithm 1's snapshot ring and
 * counter (section 5.2), the recycle basis W with its singular values and rank, the last
 * solution, a Ritz basis prepared by the last solve and not yet taken by an update (section
 * 5.1), and an SpMV shape set with rsolve_set_spmv_shape.  For callers that must stop a sequence
 * and resume it later or elsewhere (an evicted serving slot, a process restart): a sequence that
 * imports the state of another with the same configuration and size, and then sees the same
 * systems, gives bitwise the same results as the original would have.
 */

/* Bytes of the state of s as it is now (0 for a null handle).  It changes with every solve and
 * update: query it right before rsolve_export_state. */
size_t rsolve_state_bytes(rsolve_seq* s);

/*
 * Copy the state of s into `buf` (host memory, any alignment, `bytes` long): a header (format
 * version, the configuration fields the state depends on, n, the counters, a checksum of the
 * header and the columns) followed by float64 columns of n values (W, the ring by slot, the last
 * solution, a pending Ritz basis), in native byte order.  *written (nullable) receives the bytes used.  Synchronous; s is
 * unchanged.  Errors: E_INVALID (null pointer, bytes < rsolve_state_bytes(s)), E_DEVICE.
 */
int rsolve_export_state(rsolve_seq* s, void* buf, size_t bytes, size_t* written);

/*
 * Replace the state of s with one written by rsolve_export_state.  s must have the same n and
 * the same recycle_k, snapshots_s, svd_interval, method, select and precision as the exporting
 * sequence (restart length, tolerances, preconditioner and orthogonalisation may differ, at the
 * price of bitwise equality).  The pattern caches of s are kept: its next solve checks the
 * pattern as usual.  Synchronous.  Errors: E_INVALID (null pointer, not a state of this format
 * version, another configuration or size, inconsistent counters, truncated buffer, checksum
 * mismatch: s is then unchanged), E_DEVICE.
 */
int rsolve_import_state(rsolve_seq* s, const void* buf, size_t bytes);

/* ---- batched solves of many sequences in one launch ---- */

/* One-block limits: an item whose sequence is FP64 with method RSOLVE_PLAIN, _AUG_OBLIQUE or
 * _DEFL_OBLIQUE, restart_m, recycle_k (and, for the update, snapshots_s <= restart_m + 1)
 * within these limits and n <= RSOLVE_SMALL_MAX_N runs
 * as one workgroup of a shared persistent launch; any other item runs through the
 * multi-kernel path of rsolve_solve / rsolve_update_recycle, one after the other, while that
 * launch is in flight. */
#define RSOLVE_SMALL_MAX_RESTART   64
#define RSOLVE_SMALL_MAX_RECYCLE   32
#define RSOLVE_SMALL_MAX_SNAPSHOTS 32
#define RSOLVE_SMALL_MAX_N         65536

typedef struct {
    rsolve_seq* seq;       /* in: distinct sequences, all on the current HIP device */
    rsolve_csr A;          /* in: this step's matrix (device pointers, as for rsolve_solve) */
    const double* b;       /* in: device, n */
    const double* x0;      /* in: device, n, nullable (zero start) */
    double* x;             /* out: device, n (may alias x0) */
    double tol;            /* in: stop when ||b - A x||_2 <= tol ||b||_2 */
    int32_t status;        /* out: as rsolve_solve returns for this item */
    int32_t reserved;
    rsolve_stats stats;    /* out: t_setup_ms = 0 and t_cycles_ms = t_total_ms = wall time of the
                              whole batch call for the one-block items */
} rsolve_batch_solve_item;

/*
 * Solve one system for each item; each item is exactly the computation of rsolve_solve
 * (section 3.2 oblique projector, section 4.2 projection guess and correction, stop rule of
 * section 6.1), taken by one workgroup that keeps every Arnoldi step, reduction, Givens
 * rotation and restart decision on the device.  `hip_stream` (NULL = the stream of the first
 * one-block item's sequence) carries the launch.  Synchronous.  Returns RSOLVE_OK when the
 * batch ran (per-item outcome in items[i].status: E_INVALID for bad arguments, a sequence on
 * another device or a sequence listed twice, E_STATE never), E_INVALID for a bad array,
 * E_DEVICE on a HIP failure.  A corrupt CSR gives that item E_INVALID without touching the
 * others.
 */
int rsolve_solve_batch(rsolve_batch_solve_item* items, int32_t count, void* hip_stream);

typedef struct {
    rsolve_seq* seq;       /* in: distinct sequences on the current device */
    const double* x;       /* in: device, n; NULL = the last solution of this sequence */
    int32_t status;        /* out: as rsolve_update_recycle returns for this item */
    int32_t reserved;
} rsolve_batch_update_item;

/*
 * Algorithm 1 of section 5.2 for each item, as rsolve_update_recycle.  One-block items take
 * the SVD of the snapshot ring through a Householder QR of the ring (the sequence's Krylov
 * basis is the scratch), a one-sided Jacobi SVD of R and W = Q U_R[:, :k_eff], with the same
 * rank rule.  Synchronous; status conventions as rsolve_solve_batch.
 */
int rsolve_update_recycle_batch(rsolve_batch_update_item* items, int32_t count, void* hip_stream);

/* ---- per-kernel timing (HIP events) ---- */
#define RSOLVE_PROF_SPMV        0   /* Arnoldi product w = A D^{-1} v (plus basis normalisation) */
#define RSOLVE_PROF_DOTS        1   /* CGS2 pass 1: dots with V, W and the A W row F (one sweep) */
#define RSOLVE_PROF_UPDATE_DOTS 2   /* pass-1 update w -= V h1 + A W c fused with pass-2 dots */
#define RSOLVE_PROF_UPDATE_NORM 3   /* pass-2 update fused with ||w||^2 */

typedef struct {
    int32_t kernel;     /* RSOLVE_PROF_* */
    int32_t variant;    /* columns the kernel instance keeps in registers = 8 << variant
                           (dot kernels; 0 for the others) */
    int64_t launches;   /* launches that did work (Arnoldi steps actually taken) */
    double ms;          /* summed HIP-event time of those launches */
    double bytes;       /* summed algorithmic bytes of those launches (each operand read or
                           written once: values, indices, basis columns, vectors) */
} rsolve_prof_entry;

#define RSOLVE_PROF_ALL         0xF /* every kind below: (1 << RSOLVE_PROF_SPMV) | ... */
/* sampling: time only the steps j with j % stride == stride / 2 (stride 1..256, default 1) */
#define RSOLVE_PROF_STRIDE(stride) ((int32_t)(((stride) - 1) & 0xFF) << 8)

/*
 * Per-kernel timing for this sequence: `kinds` is a bit set (bit RSOLVE_PROF_x times that
 * kernel kind, RSOLVE_PROF_ALL all of them, 0 switches timing off).  A timed Arnoldi-step
 * kernel gets two HIP events stamped by its own dispatch on the sequence's stream; durations of
 * the launches that did work are summed after each cycle.  Each timed launch costs a few
 * microseconds of host and queue work, so time only the kinds you need, or OR in
 * RSOLVE_PROF_STRIDE(s) to time every s-th step of a cycle only (the averages stay those of
 * the sampled launches).  Errors: E_INVALID, E_DEVICE (event creation).
 */
int rsolve_profile_enable(rsolve_seq* s, int32_t kinds);

/*
 * Copy up to `cap` non-empty entries (host array) and their number to *count;
 * reset != 0 clears the accumulators afterwards.
 */
int rsolve_profile_read(rsolve_seq* s, rsolve_prof_entry* out, int32_t cap, int32_t* count, int32_t reset);

/* ---- captured Arnoldi steps (hipGraph) ---- */

/*
 * on = 1: rsolve_solve replays the Arnoldi steps of each cycle as captured graphs, one graph
 * per chunk of four steps, captured on first use and kept while the chunk's kernel arguments
 * stay the same (matrix pointers, recycle dimension, precision, SpMV shape); the kernels of a
 * chunk still return at once after the step that ends the cycle.  Ignored while per-kernel
 * timing is on.  on = 0 (default): kernels are enqueued one by one.  Results are the same
 * either way.
 */
int rsolve_enable_graphs(rsolve_seq* s, int32_t on);

/* Graphs captured and graph launches so far (either pointer may be NULL). */
int rsolve_graph_counts(rsolve_seq* s, int64_t* captures, int64_t* launches);

/* ---- SpMV shape of the Arnoldi product, and its autotuner ---- */

#define RSOLVE_SPMV_CSR    0   /* the caller's CSR pattern with the sequence's values */
#define RSOLVE_SPMV_BANDED 1   /* the sequence's banded padded copy: every row padded to whole
                                  chunks of `vec` entries, columns stored as 16-bit offsets
                                  col - row, the entries of each round of `lanes_per_row` chunks
                                  dealt round-robin over the row's lanes.  Needs |col - row| <=
                                  32767 for every entry; built once per pattern, values copied
                                  into it once per solve; (w + 2) bytes per entry instead of
                                  (w + 4) (w = 4 in FP32_IR mode, else 8).  Rows whose offset
                                  lists are equal (the node classes of a structured mesh) share
                                  one list when the pattern has at most 4096 such classes: the
                                  product then reads w bytes per entry and 2 per row */

typedef struct {
    int32_t lanes_per_row;  /* lanes of a wavefront that share one row: 2, 4, 8, 16 or 32 for CSR;
                               2, 4 or 8 for BANDED */
    int32_t vec;            /* CSR: entries a lane loads at once: 4 or 8 (one 16/32-byte load of
                               indices and one of values), or 1 (four strided scalar loads);
                               BANDED: entries per chunk, 4 or 8 */
    int32_t xcd_remap;      /* 1: consecutive row blocks go to the same accelerator die */
    int32_t user_set;       /* rsolve_get_spmv_shape: 1 if set by rsolve_set_spmv_shape */
    int32_t format;         /* RSOLVE_SPMV_CSR or RSOLVE_SPMV_BANDED */
    int32_t reserved;       /* must be 0 */
    double  us;             /* rsolve_tune_spmv: mean time of one product, microseconds */
} rsolve_spmv_shape;

/*
 * Time the Arnoldi product w = A D^{-1} v of this sequence (the kernel of section 3, in the
 * sequence's precision: float32 values for FP32_IR, else float64) for every shape: CSR with
 * lanes per row {2, 4, 8, 16, 32} x entries per lane {1, 4, 8}, and, when the pattern fits it,
 * BANDED with lanes {2, 4, 8} x chunk {4, 8}; each with block order {plain, XCD-aware}.  `reps`
 * timed launches each (HIP events) after one warm-up launch, on the sequence's own stream and
 * buffers.  Writes up to `cap` results in ascending time to `out` (host) and the number of
 * candidates to *count; does not change the sequence's shape.  A's pattern is checked first
 * (E_INVALID if corrupt).  Synchronous.  Errors: E_INVALID, E_DEVICE.
 */
int rsolve_tune_spmv(rsolve_seq* s, const rsolve_csr* A, int32_t reps, rsolve_spmv_shape* out, int32_t cap,
                     int32_t* count);

/* Use `shape` (format, lanes_per_row, vec, xcd_remap; user_set and us are ignored) for this
 * sequence's Arnoldi products from now on.  E_INVALID for a value outside the sets above; a
 * solve with BANDED on a pattern that does not fit it fails with E_INVALID. */
int rsolve_set_spmv_shape(rsolve_seq* s, const rsolve_spmv_shape* shape);

/* The shape in use.  Unless set, it is chosen when a pattern is checked: BANDED with 8-entry
 * chunks and 4 lanes per row when the pattern fits it and has 12 or more entries per row on
 * average, else CSR with 4 entries per lane and lanes from the mean row length. */
int rsolve_get_spmv_shape(rsolve_seq* s, rsolve_spmv_shape* shape);

/* Destroy the handle.  Does not free the workspace (the caller owns it). */
int rsolve_destroy_sequence(rsolve_seq* s);

/* Static, human-readable text for a status code. */
const char* rsolve_status_string(int status);

/* Static text describing the last error seen by this host thread (may be ""). */
const char* rsolve_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RSOLVE_H */
