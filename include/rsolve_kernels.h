/*
 * rsolve_kernels.h -- kernel-level entry points of the rsolve library, for
 * callers that compose their own solvers and for unit tests of the building
 * blocks the sequence solver (rsolve.h) is made of.  Same conventions as
 * rsolve.h: device pointers unless marked "host", float64, column-major tall
 * matrices with an explicit leading dimension, int status returns
 * (RSOLVE_OK / RSOLVE_E_*), no allocation by the library.
 */
#ifndef RSOLVE_KERNELS_H
#define RSOLVE_KERNELS_H

#include "rsolve.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * y = A x for a CSR matrix (the sparse product every Krylov step is built on;
 * section 6.2 prices it at O(n b) for bandwidth b).  The CSR must satisfy the
 * rsolve.h conventions; it is NOT validated here (corrupt indices are the
 * caller's responsibility).  Asynchronous on `hip_stream`.
 */
int rsolve_spmv(const rsolve_csr* A, const double* x, double* y, void* hip_stream);

/* Bytes of scratch workspace the kernel-level entry points below need for n rows and
 * at most `cols` (<= 64) columns. */
size_t rsolve_kernel_workspace_bytes(int64_t n, int32_t cols);

/*
 * C = A^T B for tall A (n x p) and B (n x q), p, q <= 64, computed on the
 * float64 matrix cores (MFMA) with a fixed-order split-n reduction; used for
 * E = W^T A W (section 3.2).  C_host (host) receives p x q values,
 * column-major (C[i + p j]).  Synchronous.
 */
int rsolve_gram_tn(int64_t n, const double* A, int64_t lda, int32_t p,
                   const double* B, int64_t ldb, int32_t q, double* C_host,
                   void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * rsolve_gram_tn without a workspace argument, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, result and kernels as rsolve_gram_tn; the split-n partial sums and the reduced
 * p x q result live in a static array of RSOLVE_GRAM_NOALLOC_SCRATCH_BYTES inside the library,
 * one per GPU, held from the first call on that GPU until the process ends.  Nothing in it must
 * start at zero (every launch writes each slot it reads).  Calls on one GPU share that array:
 * calls that overlap on one GPU (from several threads, or on several streams without ordering)
 * race and give wrong results; calls on different GPUs do not interact.  Allocates nothing (no
 * hipMalloc, no library allocator).  Synchronous.  Errors: E_INVALID (null pointer, n < 1,
 * lda or ldb < n, p or q outside 1..RSOLVE_GRAM_NOALLOC_MAX_COLS), E_DEVICE.
 */
#define RSOLVE_GRAM_NOALLOC_MAX_COLS     64
#define RSOLVE_GRAM_NOALLOC_SCRATCH_BYTES ((size_t)(256 * 64 * 64 + 64 * 64) * 8)   /* 8,421,376 */
int rsolve_gram_tn_noalloc(int64_t n, const double* A, int64_t lda, int32_t p, const double* B, int64_t ldb,
                           int32_t q, double* C_host, void* hip_stream);

/*
 * a = b + s c over n float64 values (a, b, c device arrays, 16-byte aligned, a not overlapping b
 * or c): a streaming kernel with 16-byte loads and stores, the measured reference for the HBM
 * roofline of the hot kernels (24 n bytes per call).  Asynchronous on `hip_stream`.  Errors:
 * E_INVALID (null or misaligned pointer, n < 1).
 */
int rsolve_triad(int64_t n, double* a, const double* b, const double* c, double s, void* hip_stream);

/*
 * The colouring behind RSOLVE_PRECOND_SSOR (the multicolour form of the SSOR preconditioner of
 * section 6.1): first fit in natural row order over the symmetrised pattern of an n x n CSR
 * pattern (row i takes the smallest colour held by no row j < i with a_ij or a_ji stored), so
 * rows of one colour never couple.  Host code on host arrays: row_ptr (n + 1 entries, from 0,
 * nondecreasing), col_idx (row_ptr[n] entries in 0..n-1); colour (host, n entries) receives
 * colours 0..*ncolours-1.  Does not use the GPU.  Errors: E_INVALID (null pointer, n < 1, a
 * row pointer or column out of range).
 */
int rsolve_colour_first_fit(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* colour,
                            int32_t* ncolours);

/*
 * The SVD step of Algorithm 1 (section 5.2) on an arbitrary snapshot matrix
 * X (n x c, c <= 64): R from a Householder TSQR of X, one-sided Jacobi SVD of
 * R, then W = X V_k Sigma_k^{-1} re-orthonormalised, with
 * k_eff = min(k, rank), rank = #{sigma_i > sigma_1 max(n, c) 2^-52}.
 * W_out (device, n x k_eff, leading dimension ldw >= n), sigma_host (host,
 * c values, descending), *k_eff and *rank are written.  Synchronous.
 */
int rsolve_snapshot_svd(int64_t n, const double* X, int64_t ldx, int32_t c, int32_t k,
                        double* W_out, int64_t ldw, double* sigma_host,
                        int32_t* k_eff, int32_t* rank,
                        void* workspace, size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RSOLVE_KERNELS_H */
