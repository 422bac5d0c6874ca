// Shared device-side definitions of the rsolve library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int WAVE = 64;
constexpr int MMAX = 128;        // largest restart length
constexpr int KMAX = 64;         // largest recycle dimension
constexpr int SMAX = 64;         // largest snapshot ring
constexpr int BLOCK = 256;       // threads per block of the streaming kernels
constexpr int BP_MAX_OFFSET = 32767;   // largest |col - row| of the banded padded format
constexpr int NBLK_MAX = 2048;   // largest grid of the split-n reductions
constexpr int DCGS2_ZD_KMAX = 16;   // largest recycle dimension whose A W dots ride in the update
constexpr bool CLS_ON = true;          // shared offset lists for the banded product
constexpr int CLS_MAX = 4096;          // most offset classes of a banded copy
constexpr int CLS_DICT_CHUNKS = 65536; // most chunks of their shared offset lists
constexpr int TSQR_PANEL = 256;  // rows per Householder panel
constexpr int64_t GRAM_PARTIAL = 256LL * KMAX * KMAX;  // doubles of a Gram partial buffer

// Control block living in the sequence workspace.  Kernels of one Arnoldi
// cycle read `done` and return at once when it is set, so the host can enqueue
// a whole cycle without a synchronisation per step.
struct Ctl {
    int done;          // the current cycle must stop
    int steps;         // Arnoldi steps taken in the current cycle
    int lucky;         // h_{j+1,j} negligible: invariant Krylov space
    int nonfinite;     // NaN/Inf met
    int max_steps;     // steps allowed in this cycle (restart / remaining budget)
    int k_eff;         // recycle columns (written by the SVD kernel)
    int rank;          // numerical rank of the snapshot ring
    int lu_fail;       // E singular (zero pivot) or cholesky failure
    double stop_abs;   // cycle stops when |g_{j+1}| <= stop_abs
    double inv_h;      // scale of the next basis vector (1/beta, then 1/h_{j+1,j})
    double beta;       // ||r|| at cycle start
    double rnorm;      // ||r|| after the end-of-cycle correction
    double bnorm;      // ||b||
    double gimp;       // |g_{steps}|: implicit residual of the cycle
    double cond1;      // 1-norm condition number of E = W^T A W
    double pad0;
    double g[MMAX + 1];
    double cs[MMAX];
    double sn[MMAX];
    double R[(MMAX + 1) * MMAX];   // rotated Hessenberg, column-major, ld MMAX+1
    double h1[MMAX + KMAX];        // pass-1 coefficients: V part then W part
    double cw[KMAX];               // E^{-1} (W^T w)
    double h2[MMAX];               // pass-2 coefficients
    double y[MMAX];                // cycle least-squares solution
    double E[KMAX * KMAX];         // LU factors of E, row-major
    int piv[KMAX];
    double sigma[SMAX];            // singular values of the ring, descending
    double T[SMAX * KMAX];         // V_k Sigma_k^{-1}, row-major c x k
    double L[KMAX * KMAX];         // cholesky factor of W^T W, row-major
    double red[SMAX * SMAX];       // small reduction results (Gram matrices)
    double F[MMAX * KMAX];         // F[i][c] = v_i^T (A W)_c, row-major with ld KMAX
    // delayed reorthogonalisation (RSOLVE_ORTHO_DCGS2)
    double Hs[(MMAX + 1) * MMAX];  // unrotated Hessenberg, column-major, ld MMAX+1
    double hp[MMAX + 1];           // first-pass coefficients of the column completed next step
    double hr[MMAX];               // reorthogonalisation coefficients of the current candidate
    double dq[MMAX + 1];           // update coefficients of the next candidate
    double inv_nu;                 // 1 / norm of the current candidate after reorthogonalisation
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Sum of one value over a 256-thread block in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* lds4) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) lds4[wv] = v;
    __syncthreads();
    double s = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    return s;
}

// Transposed wave reduction of NT (power of two) per-lane values: afterwards the
// wave-wide sum of column c sits in the lanes selected by `wave_tr_col`.  Costs
// about NT shuffles instead of 6 NT for independent butterflies.  Each halving
// step is a separate template instance so every array index is a constant.
template <int NT, int CNT, int O>
__device__ __forceinline__ void wave_tr_step(double (&a)[NT]) {
    if constexpr (CNT >= 2 && O >= 1) {
        constexpr int H = CNT / 2;
        const bool hi = (threadIdx.x & O) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double keep = hi ? a[i + H] : a[i];
            const double send = hi ? a[i] : a[i + H];
            a[i] = keep + __shfl_xor(send, O, WAVE);
        }
        wave_tr_step<NT, H, O / 2>(a);
    } else if constexpr (CNT == 1 && O >= 1) {
        // one value per lane left: finish over the remaining lane bits
        a[0] += __shfl_xor(a[0], O, WAVE);
        wave_tr_step<NT, 1, O / 2>(a);
    }
}

template <int NT>
__device__ __forceinline__ void wave_tr_reduce(double (&a)[NT]) {
    wave_tr_step<NT, NT, 32>(a);
}

// Column held in a[i] by this lane after wave_tr_reduce<NT>.
template <int NT>
__device__ __forceinline__ int wave_tr_col(int i) {
    const int lane = threadIdx.x & (WAVE - 1);
    int base = 0;
    int cnt = NT;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        if (cnt >= 2) {
            const int half = cnt >> 1;
            if (lane & o) base += half;
            cnt = half;
        }
    }
    return base + i;
}

// Number of values each lane still holds after wave_tr_reduce<NT>.
template <int NT>
constexpr int wave_tr_left() { return NT >= WAVE ? NT / WAVE : 1; }

// True for the lanes that should publish their values after wave_tr_reduce<NT>.
template <int NT>
__device__ __forceinline__ bool wave_tr_owner() {
    if constexpr (NT >= WAVE) return true;
    const int lane = threadIdx.x & (WAVE - 1);
    return (lane & ((WAVE / NT) - 1)) == 0;
}

template <typename T>
__device__ __forceinline__ double to_d(T v) { return static_cast<double>(v); }

constexpr int NXCD = 8;   // accelerator complex dies; blocks are dealt to them round-robin

// Logical block index such that the blocks resident on one XCD cover one contiguous range of
// logical blocks (a bijection of [0, nb)): work with locality between neighbouring blocks (the x
// gathers of a sparse product) then stays within one XCD's L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned x = b % NXCD, i = b / NXCD;
    const unsigned q = nb / NXCD, r = nb % NXCD;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace rs
