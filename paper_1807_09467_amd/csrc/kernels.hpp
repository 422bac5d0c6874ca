// Host-side launch wrappers of the rsolve kernels (one translation unit per kernel family).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

namespace rs {

// ---- sparse (k_sparse.hip) ----
// Pattern validation: err[0..3] receive nonzero on (row_ptr range, column range, unsorted or
// duplicate columns, missing diagonal); diag_pos[i] = CSR index of A_ii.
// Banded padded CSR for the Arnoldi product (rows in chunks of E entries, 16-bit column offsets
// col - row, entries dealt round-robin over the LPR lanes of a row in every round of chunks).
// bp_setup: chunk offsets p (n + 1), offsets of every entry and zeros at the padding; returns -1
// for an unsupported (E, LPR) or a scratch buffer (int32, device) shorter than
// bp_scratch_ints(n).  Requires |col - row| <= BP_MAX_OFFSET for every entry.
int64_t bp_scratch_ints(int64_t n);
int bp_setup(int64_t n, const int32_t* rp, const int32_t* ci, int E, int LPR, int32_t* p, int16_t* off, void* val,
             bool f32, int32_t* scratch, int64_t scratch_ints, hipStream_t st);
template <typename T>
void launch_bp_values(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* dinv,
                      const int32_t* p, int E, int LPR, T* out, hipStream_t st);
template <typename T>
void launch_spmv_bp(int E, int LPR, int remap, int64_t n, const int32_t* p, const int16_t* off, const T* val,
                    const T* win, T* vout, T* y, const Ctl* ctl, hipStream_t st, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
// the same product with the offsets of row r read from dict + first[r] E (rows of equal offsets
// share one list)
template <typename T>
void launch_spmv_bc(int E, int LPR, int remap, int64_t n, const int32_t* p, const uint16_t* first,
                    const int16_t* dict, const T* val, const T* win, T* vout, T* y, const Ctl* ctl, hipStream_t st,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// a = b + s c (n doubles, 16-byte aligned arrays): the streaming reference kernel.
void launch_triad(int64_t n, double* a, const double* b, const double* c, double s, int cus, hipStream_t st);

// ---- multicolour SSOR (k_ssor.hip) ----
// The colouring and grouping of one pattern: rows[coff[c] .. coff[c + 1]) are the rows of colour c
// (no two of them couple).  `single`: the whole application in one workgroup that walks the
// colours (small systems, or many colours of few rows); otherwise one launch per colour and sweep.
struct SsorPlan {
    int64_t n = 0;
    int ncol = 0;
    int lpr = 4;                          // lanes per row: 4, 16 or 64
    bool single = true;
    double omega = 1.0;
    const int32_t* colour = nullptr;      // device, n
    const int32_t* rows = nullptr;        // device, n
    const int32_t* coff_dev = nullptr;    // device, ncol + 1
    const int32_t* coff_host = nullptr;   // host, ncol + 1
};
// Lanes per row of the sweeps for a pattern of nnz entries over n rows.
int ssor_lanes(int64_t n, int64_t nnz);
// t = M^{-1} r (r and t distinct, n entries); when vout is given the forward sweep also writes
// vout = ctl->inv_h r.  With ctl given every kernel returns at once once ctl->done is set.
void launch_ssor_apply(const SsorPlan& p, const int32_t* rp, const int32_t* ci, const double* val,
                       const int32_t* dpos, const double* r, double* t, double* vout, const Ctl* ctl,
                       hipStream_t st);
void launch_fill(int64_t n, double* x, double v, hipStream_t st);
void launch_axpy(int64_t n, const double* t, double* x, hipStream_t st);   // x += t
// First-fit colouring of the symmetrised pattern (host arrays) in natural row order: colour[i] is
// the smallest colour held by no neighbour j < i; rows grouped by colour into rows / coff.
// Returns the number of colours.
int colour_first_fit(int64_t n, const int32_t* rp, const int32_t* ci, int32_t* colour, std::vector<int32_t>& rows,
                     std::vector<int32_t>& coff);

// ---- Ritz and harmonic Ritz pairs (k_eig.hip) ----
// The k pairs of smallest modulus of Ga z = theta z (harmonic = 0) or Ga z = theta Gb z (harmonic =
// 1), Ga, Gb r x r column-major (r <= SMAX), written as the r x kk coefficients ctl->T of the
// recycle basis, kk in ctl->k_eff, |theta| in ctl->sigma; scratch of 9 SMAX^2 doubles; one
// wavefront.  ctl->lu_fail = 1 (kk = 0) for a singular Gb or QR steps that do not converge.
void launch_small_eig(const double* Ga, const double* Gb, int r, int k, int harmonic, double* scratch, Ctl* ctl,
                      hipStream_t st);
// out[:, c] = dinv .* V[:, c] in float64, c < cols (dinv nullable: a plain conversion)
template <typename T>
void launch_scale_cols(int64_t n, int64_t ld, const T* V, int cols, const double* dinv, double* out, int64_t ldo,
                       hipStream_t st);

void launch_validate(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, int32_t* diag_pos,
                     int32_t* err, hipStream_t st);
void launch_diag_inv(int64_t n, const int32_t* diag_pos, const double* val, double* dinv, hipStream_t st);
// out64 / out32 (nullable) = val[k] * dinv[col[k]] (dinv nullable: plain copy / conversion)
void launch_scale_values(int64_t nnz, const int32_t* ci, const double* val, const double* dinv, double* out64,
                         float* out32, hipStream_t st);
// Arnoldi product: vout[i] = s * win[i]; y[i] = s * sum_k val[k] win[col[k]], s = ctl->inv_h.
// Shape: lpr lanes per row (2..32), vec entries per lane and load (4 or 8; 1 = four strided
// scalar loads), remap = XCD-aware block order.  ev0 / ev1 (nullable): events stamped with the
// start and end of the kernel's own dispatch (hipExtLaunchKernelGGL), for per-kernel timing
// without extra queue packets.
template <typename T>
void launch_spmv_arnoldi(int lpr, int vec, int remap, int64_t n, const int32_t* rp, const int32_t* ci, const T* val,
                         const T* win, T* vout, T* y, const Ctl* ctl, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// r = b - A x (float64)
void launch_residual(int lpr, int64_t n, const int32_t* rp, const int32_t* ci, const double* val,
                     const double* x, const double* b, double* r, hipStream_t st);
// y = A x (float64)
void launch_spmv(int lpr, int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* x,
                 double* y, hipStream_t st);
// elementwise float64 -> float32 (count entries)
void launch_to_f32(int64_t count, const double* in, float* out, hipStream_t st);

// ---- Krylov cycle (k_krylov.hip) ----
// Multi-dot sweep over up to 3 column groups: group q = columns bases[q][:, 0..counts[q]) dotted
// with vecs[q]; partial[c * nblk + b] for the concatenated column index c.
// pass1_nv > 0: then turn the partials into the pass-1 coefficients of a step with pass1_nv basis
// vectors and pass1_k recycle columns (one-block reduction kernel).
template <typename T>
void launch_dots(int64_t npad, int64_t ld, const T* const* bases, const T* const* vecs, const int* counts,
                 int ngroups, double* partial, int nblk, Ctl* ctl, hipStream_t st, int pass1_nv = 0,
                 int pass1_k = 0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool pass1_orth = false);
// fixed-order sum of the partials into dst[0..ncol); if lu_solve, also ctl->cw = E^{-1} dst[nv..nv+nw)
void launch_reduce(const double* partial, int nblk, int ncol, double* dst, Ctl* ctl, int nv, int nw,
                   bool lu_solve, bool check_done, hipStream_t st);
// w -= V[:, :nv] coefV + Z[:, :nz] coefZ; ctl->h2 = V^T w (new)   (nv <= 128; 8 columns per wavefront;
// a one-block kernel sums the per-block partials)
template <typename T>
void launch_update_dots(int64_t npad, const T* V, int64_t ld, int nv, const T* Z, int nz, T* w,
                        const double* coefV, const double* coefZ, double* partial, int nblk, Ctl* ctl,
                        hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// w -= V[:, :nv] coef; partial[b] = sum over block b of w^2; givens_j >= 0: then form column
// givens_j of H and apply the Givens update (as launch_givens)
template <typename T>
void launch_update_norm(int64_t npad, const T* V, int64_t ld, int nv, T* w, const double* coef,
                        double* partial, int nblk, Ctl* ctl, hipStream_t st, int givens_j, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
// column j of H: reduce ||w||^2, Givens update, stop test, next scale
void launch_givens(const double* partial, int nblk, int j, Ctl* ctl, hipStream_t st);
// start of a cycle: g = beta e1 with beta = ctl->rnorm, done/steps reset; the first Arnoldi
// product scales its input by 1/beta, or by 1 with unit_scale (delayed reorthogonalisation)
void launch_cycle_init(Ctl* ctl, int max_steps, double stop_abs, hipStream_t st, bool unit_scale = false);
// Delayed reorthogonalisation, step j: the sweep over [V_j (nq = j columns), W, A W, u] dotted
// with u and z; the one-block reduction (completes and rotates column j-1, sets done, prepares
// step j; has_z = false on the closing step); the update sweep (v_j and the next candidate u).
// zskip = kz leaves the A W columns out (their dots with u come from the previous update).
template <typename T>
void launch_dots2(int64_t npad, int64_t ld, const T* V, int nq, const T* W, const T* Z, int k, int kz, int zskip,
                  const T* u, const T* z, double* partial, int nblk, Ctl* ctl, hipStream_t st,
                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// the sweep's column sums (written after the partials: partial needs 2 ncol (nblk + 1) doubles),
// then the one-block reduction of the delayed scheme; with zpart, the A W dots with u are the sums
// of the previous update's per-block partials (nblk_z of them per column) minus G cw / nu, with
// G = (A W)^T A W in gz (kz x kz, row-major)
void launch_dcgs2_reduce(double* partial, int nblk, int j, int k, int kz, bool orth, bool has_z, Ctl* ctl,
                         hipStream_t st, const double* zpart = nullptr, int nblk_z = 0, const double* gz = nullptr);
// with zpart (k <= DCGS2_ZD_KMAX), also the per-block dots of the k columns of Z with
// z / nu - V dq - v_j dq_j (the new candidate u plus (A W) cw / nu): zpart[c * nblk + b]
// Blocks of the update sweep for npad rows of elem_bytes-byte values (at most max_blocks): one
// 32-byte slice of every column per thread.  The A W partials it writes number the same.
int dcgs2_update_blocks(int64_t npad, int elem_bytes, int max_blocks);
template <typename T>
void launch_dcgs2_update(int64_t npad, T* V, int64_t ld, int j, const T* Z, int k, T* u, const T* z, int nblk,
                         const Ctl* ctl, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                         double* zpart = nullptr);
// y = R^{-1} g (ctl->steps unknowns)
void launch_cycle_solve(Ctl* ctl, hipStream_t st);
// x[i] += dinv[i] * sum_{c < steps} V[i, c] y[c]   (dinv nullable)
template <typename T>
void launch_x_update(int64_t n, const T* V, int64_t ld, const double* dinv, double* x, const Ctl* ctl,
                     hipStream_t st);
// x += W cw; r -= Z cw; partial = ||r||^2 per block (k may be 0: norm only)
void launch_correct(int64_t npad, const double* W, const double* Z, int64_t ld, int k, double* x, double* r,
                    const Ctl* ctl, double* partial, int nblk, hipStream_t st);
// ctl->rnorm = sqrt(sum partial); ctl->nonfinite on NaN/Inf
void launch_finish_norm(const double* partial, int nblk, Ctl* ctl, int which, hipStream_t st);
// partial = ||v||^2 per block over n entries (caller vector, exact length)
void launch_norm2(int64_t n, const double* v, double* partial, int nblk, hipStream_t st);
// out[i] = in[i] for i < n, 0 for n <= i < npad
void launch_copy_pad(int64_t n, int64_t npad, const double* in, double* out, hipStream_t st);
// out[i] = sum_{j<q} w[j] x[j][i] for i < n, 0 for n <= i < npad (1 <= q <= 4)
struct Extrap {
    const double* x[4];
    double w[4];
    int q;
};
void launch_extrapolate(int64_t n, int64_t npad, const Extrap& e, double* out, hipStream_t st);

// ---- dense (k_dense.hip) ----
// partial[e * nblk + b] = block b's share of (A^T B)[e] (MFMA f64, e = i + p j); rows >= n read
// as zero.  partial holds GRAM_PARTIAL doubles; returns nblk (<= max_blocks) for the reduction.
int launch_gram_tn(int64_t n, const double* A, int64_t lda, int p, const double* B, int64_t ldb, int q,
                   double* partial, int max_blocks, hipStream_t st);
// dst[p*q] (column-major) = fixed-order sum over blocks
void launch_gram_reduce(const double* partial, int nblk, int pq, double* dst, hipStream_t st);
// LU with partial pivoting of E (k x k, column-major in src) into ctl->E/piv, ctl->cond1
void launch_small_lu(const double* src, int k, Ctl* ctl, hipStream_t st);
// one TSQR level: panels of tsqr_panel_rows(c) rows of M (rows x c) -> stacked R factors S
// ((P*c) x c, ld_s), P = ceil(rows / tsqr_panel_rows(c)) = npanels
constexpr int TSQR_MIN_PANEL = 128;   // the smallest panel of any c (sizes the level buffers)
int tsqr_panel_rows(int c);
void launch_tsqr_level(int64_t rows, const double* M, int64_t ldm, int c, double* S, int64_t lds, int npanels,
                       hipStream_t st);
// one-sided Jacobi SVD of the c x c matrix R (column-major, ld); writes ctl->sigma, ctl->rank,
// ctl->k_eff = min(k, rank), ctl->T = V_k Sigma_k^{-1} (the k_eff leading modes, or with smallest the
// k_eff trailing ones above the rank cut)
void launch_jacobi_svd(const double* R, int64_t ld, int c, int k, int64_t n, Ctl* ctl, hipStream_t st,
                       bool smallest = false);
// W[:, :k] = X[:, :c] T (T from ctl); rows >= n get zero
void launch_form_w(int64_t n, int64_t npad, const double* X, int64_t ldx, int c, int k, const Ctl* ctl,
                   double* W, int64_t ldw, hipStream_t st);
// ctl->L = chol(G) for G = ctl->red (k x k column-major)
void launch_cholesky(int k, Ctl* ctl, hipStream_t st);
// W[r, :k] <- L^{-1} W[r, :k]^T (rows < npad)
// W <- W L^{-T} row by row; also writes the result row-major to Wr (row r at Wr + r ldr) when
// Wr is not null, and rounded to float into W32 (same layout as W) when W32 is not null.
void launch_trsm_rows(int64_t npad, double* W, int64_t ldw, int k, const Ctl* ctl, hipStream_t st,
                      double* Wr = nullptr, int ldr = 0, float* W32 = nullptr);
// Z = A W for W kept row-major (ldr a multiple of 16, 128-byte aligned rows); Z column-major (ld),
// and rounded to float into Z32 (same layout) when Z32 is not null.
void launch_spmm_rows(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* Wr, int ldr,
                      int k, double* Z, int64_t ld, hipStream_t st, float* Z32 = nullptr);
// Wr (row-major, ldr) = W (column-major, ld), n rows, k columns.
void launch_to_rows(int64_t n, const double* W, int64_t ld, int k, double* Wr, int ldr, hipStream_t st);

// ---- one-block persistent path for small systems (k_small.hip) ----
constexpr int SMALL_MMAX = 64;     // restart limit of the one-block solver
constexpr int SMALL_KMAX = 32;     // recycle limit
constexpr int SMALL_SMAX = 32;     // snapshot-ring limit of the one-block recycle update
constexpr int SMALL_BATCH = 256;   // jobs per launch (one block each)

// One solve, read by its block from pinned host memory at the start and completed (results)
// by the block at the end.  All pointers are device pointers.
struct SmallJob {
    int64_t n, nnz, ld;
    const int32_t* rp;
    const int32_t* ci;
    const double* val;
    const double* b;
    const double* x0;  // nullable: zero start
    double* x;
    double tol;
    int32_t m, k, max_iters, jacobi;
    int32_t validate, pad0;
    // sequence storage: W, Z = A W (k columns, ld), V (m + 1 columns), two work vectors, the
    // iterate, D^{-1}, the scaled values (nnz) and F (SMALL_MMAX x SMALL_KMAX)
    const double* W;
    double* Z;
    double* V;
    double* w;
    double* r;
    double* xw;
    double* dinv;
    double* vals;
    double* F;
    // results
    int32_t status, iterations, cycles, converged;
    uint32_t flags;
    int32_t k_used;
    double rnorm, bnorm, gimp;
};

// One recycle update (ring push and, when svd != 0, the new W), same conventions.
struct SmallUpd {
    int64_t n, ld;
    const double* src;  // solution to store (n)
    double* X;          // snapshot ring (ld, s columns)
    double* Q;          // scratch, c columns of ld (the sequence's Krylov basis)
    double* W;          // output basis (k_eff columns of ld)
    int32_t slot, c, k, svd;
    // results
    int32_t status, rank, k_eff, smallest;   // smallest: keep the trailing modes above the rank cut
    double sigma[SMALL_SMAX];
};

struct SmallBatch {
    SmallJob* job[SMALL_BATCH];
};
struct SmallUpdBatch {
    SmallUpd* job[SMALL_BATCH];
};

// Block b solves batch.job[b] (count <= SMALL_BATCH): validation, Jacobi scaling, A W, E and its
// LU, projection guess, restarted GMRES(m) cycles with the oblique projector, all on the device.
void launch_small_solve(const SmallBatch& batch, int count, hipStream_t st);
// Block b stores job[b].src in the ring and, if requested, replaces W (Householder QR of the
// ring, Jacobi SVD of R, W = Q U_k).
void launch_small_update(const SmallUpdBatch& batch, int count, hipStream_t st);

}  // namespace rs
