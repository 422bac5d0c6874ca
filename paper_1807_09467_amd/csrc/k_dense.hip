// Dense kernels of the recycle space (section 5.2, Algorithm 1) and of the
// projector setup (section 3.2, E = W^T A W):
//   * tall-skinny C = A^T B on the float64 matrix cores (v_mfma_f64_16x16x4f64);
//   * LU with partial pivoting of E and its 1-norm condition number;
//   * one level of a Householder TSQR (panels of 256 rows, R factors stacked);
//   * one-sided (Hestenes) Jacobi SVD of the final small R;
//   * W = X V_k Sigma_k^{-1}, then W <- W L^{-T} with L L^T = W^T W.
#include "kernels.hpp"
#include "svd_dev.hpp"

#include <algorithm>

namespace rs {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// C = A^T B on MFMA for tall A (n x p) and B (n x q), p, q <= 64.  A block walks slabs of R
// rows: both slabs are staged in LDS with coalesced column loads (consecutive threads read
// consecutive rows of one column), then each wavefront feeds R / 4 of the slab's rows to
// v_mfma_f64_16x16x4f64, 4 rows per instruction: the A operand is the 16 x 4 block
// (A^T)[i][row] (lane = i + 16 * row), the B operand the 4 x 16 block B[row][j]; the 16 x 16
// result block holds C[lane / 16 + 4 r][lane % 16] in element r of each lane.  The LDS row
// stride R + 4 puts the 16 columns x 4 rows of an operand read in distinct banks.
// partial[e * nblk + b] = block b's share of entry e = i + p j.
// ---------------------------------------------------------------------------
template <int TP, int TQ, int R>
__global__ __launch_bounds__(BLOCK) void k_gram_tn(int64_t n, const double* __restrict__ A, int64_t lda, int p,
                                                   const double* __restrict__ B, int64_t ldb, int q,
                                                   double* __restrict__ partial, int nblk) {
    constexpr int RS = R + 4;
    constexpr int RW = R / (BLOCK / WAVE);   // rows per wavefront and slab
    static_assert(RW % 4 == 0, "whole MFMA steps per wavefront");
    constexpr int NSTAGE = (TP + TQ) * 16 * RS, NACC = TP * 16 * TQ * 16;
    __shared__ double smem[NSTAGE > NACC ? NSTAGE : NACC];
    double* As = smem;
    double* Bs = smem + TP * 16 * RS;
    double* acc_s = smem;   // reused once the last slab is done (every slab ends with a barrier)
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[TP][TQ];
#pragma unroll
    for (int a = 0; a < TP; ++a)
#pragma unroll
        for (int b = 0; b < TQ; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t nslab = (n + R - 1) / R;
    // the next slab's operands are loaded into registers while the current one is multiplied
    constexpr int NA = TP * 16 * R / BLOCK, NB = TQ * 16 * R / BLOCK;
    double pa[NA], pb[NB];
    auto fetch = [&](int64_t sl) {
        const int64_t r0 = sl * R;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int t = u * BLOCK + threadIdx.x, c = t / R, r = t % R;
            const int64_t row = r0 + r;
            pa[u] = (sl < nslab && c < p && row < n) ? A[(int64_t)c * lda + row] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int t = u * BLOCK + threadIdx.x, c = t / R, r = t % R;
            const int64_t row = r0 + r;
            pb[u] = (sl < nslab && c < q && row < n) ? B[(int64_t)c * ldb + row] : 0.0;
        }
    };
    fetch(blockIdx.x);
    for (int64_t sl = blockIdx.x; sl < nslab; sl += nblk) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int t = u * BLOCK + threadIdx.x;
            As[(t / R) * RS + t % R] = pa[u];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int t = u * BLOCK + threadIdx.x;
            Bs[(t / R) * RS + t % R] = pb[u];
        }
        __syncthreads();
        fetch(sl + nblk);
#pragma unroll
        for (int g = 0; g < RW / 4; ++g) {
            const int rr = wv * RW + g * 4 + lk;
            double av[TP], bv[TQ];
#pragma unroll
            for (int a = 0; a < TP; ++a) av[a] = As[(a * 16 + li) * RS + rr];
#pragma unroll
            for (int b = 0; b < TQ; ++b) bv[b] = Bs[(b * 16 + li) * RS + rr];
#pragma unroll
            for (int a = 0; a < TP; ++a)
#pragma unroll
                for (int b = 0; b < TQ; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // fixed-order combination of the wavefronts
    constexpr int LD = TP * 16;
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        if (wv == w) {
#pragma unroll
            for (int a = 0; a < TP; ++a)
#pragma unroll
                for (int b = 0; b < TQ; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = a * 16 + (lane >> 4) + 4 * r;
                        const int j = b * 16 + (lane & 15);
                        const double v = acc[a][b][r];
                        if (w == 0) acc_s[i + LD * j] = v;
                        else acc_s[i + LD * j] += v;
                    }
        }
        __syncthreads();
    }
    const int pq = p * q;
    for (int e = threadIdx.x; e < pq; e += BLOCK) {
        const int i = e % p, j = e / p;
        partial[(int64_t)e * nblk + blockIdx.x] = acc_s[i + LD * j];
    }
}

// dst[e] = sum over b of partial[e * nblk + b], each entry by a group of G lanes (power of two
// up to the wavefront) in a fixed order: lane-strided partial sums, then a butterfly.
__global__ __launch_bounds__(1024) void k_gram_reduce(const double* __restrict__ partial, int nblk, int pq, int G,
                                                      double* __restrict__ dst) {
    const int sub = threadIdx.x & (G - 1);
    const int per_pass = 1024 / G;
    for (int e0 = 0; e0 < pq; e0 += per_pass) {
        const int e = e0 + threadIdx.x / G;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (e < pq) {
            const double* src = partial + (int64_t)e * nblk;
            int b = sub;
            for (; b + 3 * G < nblk; b += 4 * G) {
                a0 += src[b];
                a1 += src[b + G];
                a2 += src[b + 2 * G];
                a3 += src[b + 3 * G];
            }
            for (; b < nblk; b += G) a0 += src[b];
        }
        double s = (a0 + a1) + (a2 + a3);
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
        if (e < pq && sub == 0) dst[e] = s;
    }
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of E (k x k <= 64), one wavefront, lane = row.
// cond1 = ||E||_1 ||E^{-1}||_1 with the inverse formed column by column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WAVE) void k_small_lu(const double* __restrict__ src, int k, Ctl* __restrict__ ctl) {
    constexpr int LDM = KMAX + 1;
    __shared__ double M[KMAX * LDM];
    __shared__ double X[KMAX * KMAX];
    __shared__ int perm[KMAX];
    const int lane = threadIdx.x;
    for (int t = lane; t < k * k; t += WAVE) {
        const int i = t % k, j = t / k;  // src column-major
        M[i * LDM + j] = src[t];
    }
    if (lane < k) perm[lane] = lane;
    __syncthreads();
    // ||E||_1: column sums
    double cs = 0.0;
    if (lane < k)
        for (int i = 0; i < k; ++i) cs += fabs(M[i * LDM + lane]);
    const double norm1 = wave_max(lane < k ? cs : 0.0);
    int fail = 0;
    for (int j = 0; j < k; ++j) {
        // pivot search among rows >= j (first index on ties)
        double v = (lane >= j && lane < k) ? fabs(M[lane * LDM + j]) : -1.0;
        int idx = lane;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(v, o, WAVE);
            const int oi = __shfl_xor(idx, o, WAVE);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        const int pr = idx;
        if (pr != j) {
            for (int c = lane; c < k; c += WAVE) {
                const double t = M[j * LDM + c];
                M[j * LDM + c] = M[pr * LDM + c];
                M[pr * LDM + c] = t;
            }
            if (lane == 0) {
                const int t = perm[j];
                perm[j] = perm[pr];
                perm[pr] = t;
            }
        }
        __syncthreads();
        const double d = M[j * LDM + j];
        if (d == 0.0 || !isfinite(d)) {
            fail = 1;
            break;
        }
        if (lane > j && lane < k) {
            const double l = M[lane * LDM + j] / d;
            M[lane * LDM + j] = l;
            for (int c = j + 1; c < k; ++c) M[lane * LDM + c] -= l * M[j * LDM + c];
        }
        __syncthreads();
    }
    double cond = INFINITY;
    if (!fail) {
        // column `lane` of E^{-1}: solve L U x = P e_lane
        if (lane < k) {
            for (int i = 0; i < k; ++i) {
                double s = (perm[i] == lane) ? 1.0 : 0.0;
                for (int j = 0; j < i; ++j) s -= M[i * LDM + j] * X[j * KMAX + lane];
                X[i * KMAX + lane] = s;
            }
            for (int i = k - 1; i >= 0; --i) {
                double s = X[i * KMAX + lane];
                for (int j = i + 1; j < k; ++j) s -= M[i * LDM + j] * X[j * KMAX + lane];
                X[i * KMAX + lane] = s / M[i * LDM + i];
            }
        }
        __syncthreads();
        double ics = 0.0;
        if (lane < k)
            for (int i = 0; i < k; ++i) ics += fabs(X[i * KMAX + lane]);
        const double inorm1 = wave_max(lane < k ? ics : 0.0);
        cond = norm1 * inorm1;
        if (!isfinite(cond)) cond = INFINITY;
    }
    for (int t = lane; t < k * k; t += WAVE) ctl->E[t] = M[(t / k) * LDM + (t % k)];
    if (lane < k) ctl->piv[lane] = perm[lane];
    if (lane == 0) {
        ctl->cond1 = cond;
        ctl->lu_fail = fail;
    }
}

// ---------------------------------------------------------------------------
// One TSQR level.  Block p factors rows [p*256, p*256+256) of M (zero beyond
// `rows`, columns padded with zeros up to C) by Householder reflections; thread
// t holds row t of the panel in registers.  The column being eliminated is
// always a[0]: after each reflection the finished column is written out (rows
// t <= cc of R) and the register array shifts down by one, so every register
// index is a compile-time constant.  Output: the c x c R factor of panel p in
// rows [p*c, p*c + c) of S.
// ---------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(TSQR_PANEL) void k_tsqr_level(int64_t rows, const double* __restrict__ M, int64_t ldm,
                                                           int c, double* __restrict__ S, int64_t lds) {
    __shared__ double red[TSQR_PANEL / WAVE][C];
    __shared__ double bc;
    const int t = threadIdx.x;
    const int wv = t / WAVE;
    const int64_t row = (int64_t)blockIdx.x * TSQR_PANEL + t;
    const int64_t orow = (int64_t)blockIdx.x * c + t;
    double a[C];
#pragma unroll
    for (int j = 0; j < C; ++j) a[j] = (row < rows && j < c) ? M[(int64_t)j * ldm + row] : 0.0;
    for (int cc = 0; cc < c; ++cc) {
        // squared norm of the current column on rows >= cc
        double s = (t >= cc) ? a[0] * a[0] : 0.0;
        s = wave_sum(s);
        __syncthreads();
        if ((t & (WAVE - 1)) == 0) red[wv][0] = s;
        if (t == cc) bc = a[0];
        __syncthreads();
        const double nrm2 = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        const double alpha = bc;
        if (nrm2 > 0.0) {  // uniform; a zero column needs no reflection
            const double nrm = sqrt(nrm2);
            const double beta = (alpha >= 0.0) ? -nrm : nrm;
            const double tau = (beta - alpha) / beta;
            const double v = (t > cc) ? a[0] / (alpha - beta) : ((t == cc) ? 1.0 : 0.0);
            double pr[C];
            pr[0] = 0.0;
#pragma unroll
            for (int j = 1; j < C; ++j) pr[j] = v * a[j];
            wave_tr_reduce<C>(pr);
            __syncthreads();
            if (wave_tr_owner<C>()) {
#pragma unroll
                for (int i = 0; i < wave_tr_left<C>(); ++i) red[wv][wave_tr_col<C>(i)] = pr[i];
            }
            __syncthreads();
#pragma unroll
            for (int j = 1; j < C; ++j) {
                const double d = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
                a[j] -= tau * v * d;
            }
            if (t == cc) a[0] = beta;
            else if (t > cc) a[0] = 0.0;
        }
        if (t < c) S[(int64_t)cc * lds + orow] = (t <= cc) ? a[0] : 0.0;
#pragma unroll
        for (int j = 0; j + 1 < C; ++j) a[j] = a[j + 1];
        a[C - 1] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// One TSQR level with one wavefront per panel of 64 RPL rows (lane l holds rows l, l + 64, ...),
// for c <= C <= 32.  No block barriers: for column CC the squared norm below the diagonal and the
// reflection's dot products all come from one transposed wavefront reduction of a[CC] a[j]
// (rows below CC, columns j >= CC), and the diagonal row is broadcast through LDS with the
// sums.  The column loop is unrolled at compile time, so iteration CC touches only columns
// CC..C-1.  Output as k_tsqr_level: the c x c R factor of panel p in rows [p c, p c + c) of S.
// ---------------------------------------------------------------------------
constexpr int pow2ceil(int x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

template <int C, int RPL, int CC>
__device__ __forceinline__ void tsqr_wave_column(double (&a)[RPL][C], int lane, int c, double* __restrict__ S,
                                                 int64_t lds, int64_t orow, double* rowb, double* sigb) {
    if constexpr (CC < C) {
        constexpr int NV = C - CC;          // columns CC..C-1
        constexpr int NT = pow2ceil(NV);    // values of the transposed reduction
        constexpr int OWN = WAVE / NT;      // column j's sum ends in lane j OWN
        if (CC < c) {
            double p[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) p[j] = 0.0;
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const double x = (lane + WAVE * q > CC) ? a[q][CC] : 0.0;
#pragma unroll
                for (int j = 0; j < NV; ++j) p[j] += x * a[q][CC + j];
            }
            wave_tr_reduce<NT>(p);
            if ((lane & (OWN - 1)) == 0 && lane / OWN < NV) sigb[lane / OWN] = p[0];
            if (lane == CC) {
#pragma unroll
                for (int j = 0; j < NV; ++j) rowb[j] = a[0][CC + j];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the LDS writes above have landed
            __builtin_amdgcn_wave_barrier();
            const double alpha = rowb[0];
            const double nrm2 = alpha * alpha + sigb[0];
            if (nrm2 > 0.0) {   // uniform; a zero column needs no reflection
                const double nrm = sqrt(nrm2);
                const double beta = (alpha >= 0.0) ? -nrm : nrm;
                const double tau = (beta - alpha) / beta;
                const double inv = 1.0 / (alpha - beta);
                // d_j = v^T a_j with v = (1, a_{CC+1..}[CC] / (alpha - beta))
                double d[NV];
#pragma unroll
                for (int j = 1; j < NV; ++j) d[j] = rowb[j] + sigb[j] * inv;
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const int t = lane + WAVE * q;
                    const double v = (t > CC) ? a[q][CC] * inv : ((t == CC) ? 1.0 : 0.0);
                    const double tv = tau * v;
#pragma unroll
                    for (int j = 1; j < NV; ++j) a[q][CC + j] -= tv * d[j];
                    if (t == CC) a[q][CC] = beta;
                    else if (t > CC) a[q][CC] = 0.0;
                }
            }
            __builtin_amdgcn_wave_barrier();   // the reads above precede the next column's writes
            if (lane < c) S[(int64_t)CC * lds + orow] = (lane <= CC) ? a[0][CC] : 0.0;
        }
        tsqr_wave_column<C, RPL, CC + 1>(a, lane, c, S, lds, orow, rowb, sigb);
    }
}

template <int C, int RPL>
__global__ __launch_bounds__(256) void k_tsqr_wave(int64_t rows, const double* __restrict__ M, int64_t ldm, int c,
                                                   double* __restrict__ S, int64_t lds) {
    __shared__ __attribute__((aligned(16))) double bufs[256 / WAVE][2][C];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int64_t panel = (int64_t)blockIdx.x * (256 / WAVE) + wv;
    const int64_t r0 = panel * WAVE * RPL;
    if (r0 >= rows) return;   // a wavefront past the last panel: nothing to factor or write
    double a[RPL][C];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int64_t row = r0 + lane + WAVE * q;
            a[q][j] = (row < rows && j < c) ? M[(int64_t)j * ldm + row] : 0.0;
        }
    tsqr_wave_column<C, RPL, 0>(a, lane, c, S, lds, panel * c + lane, bufs[wv][0], bufs[wv][1]);
}

// The same factorisation with a runtime column loop (the register arrays shift by one column per
// step, so every index stays a compile-time constant): a few kilobytes of code instead of tens,
// for the levels with few panels, where one wavefront's instruction fetches, not arithmetic, set
// the time.
template <int C, int RPL>
__global__ __launch_bounds__(256) void k_tsqr_wave_loop(int64_t rows, const double* __restrict__ M, int64_t ldm,
                                                        int c, double* __restrict__ S, int64_t lds) {
    __shared__ __attribute__((aligned(16))) double bufs[256 / WAVE][2][C];
    constexpr int OWN = WAVE / C;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int64_t panel = (int64_t)blockIdx.x * (256 / WAVE) + wv;
    const int64_t r0 = panel * WAVE * RPL;
    if (r0 >= rows) return;
    double* rowb = bufs[wv][0];
    double* sigb = bufs[wv][1];
    double a[RPL][C];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int j = 0; j < C; ++j) {
            const int64_t row = r0 + lane + WAVE * q;
            a[q][j] = (row < rows && j < c) ? M[(int64_t)j * ldm + row] : 0.0;
        }
    const int64_t orow = panel * c + lane;
    for (int cc = 0; cc < c; ++cc) {
        // a[q][0] is column cc; a[q][j] column cc + j
        double p[C];
#pragma unroll
        for (int j = 0; j < C; ++j) p[j] = 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const double x = (lane + WAVE * q > cc) ? a[q][0] : 0.0;
#pragma unroll
            for (int j = 0; j < C; ++j) p[j] += x * a[q][j];
        }
        wave_tr_reduce<C>(p);
        if ((lane & (OWN - 1)) == 0) sigb[lane / OWN] = p[0];
        if (lane == cc) {
#pragma unroll
            for (int j = 0; j < C; ++j) rowb[j] = a[0][j];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
        __builtin_amdgcn_wave_barrier();
        const double alpha = rowb[0];
        const double nrm2 = alpha * alpha + sigb[0];
        if (nrm2 > 0.0) {
            const double nrm = sqrt(nrm2);
            const double beta = (alpha >= 0.0) ? -nrm : nrm;
            const double tau = (beta - alpha) / beta;
            const double inv = 1.0 / (alpha - beta);
            double d[C];
#pragma unroll
            for (int j = 1; j < C; ++j) d[j] = rowb[j] + sigb[j] * inv;
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int t = lane + WAVE * q;
                const double v = (t > cc) ? a[q][0] * inv : ((t == cc) ? 1.0 : 0.0);
                const double tv = tau * v;
#pragma unroll
                for (int j = 1; j < C; ++j) a[q][j] -= tv * d[j];
                if (t == cc) a[q][0] = beta;
                else if (t > cc) a[q][0] = 0.0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < c) S[(int64_t)cc * lds + orow] = (lane <= cc) ? a[0][0] : 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
#pragma unroll
            for (int j = 0; j + 1 < C; ++j) a[q][j] = a[q][j + 1];
            a[q][C - 1] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of R (c x c <= 64) in one block: columns are rotated in
// pairs (round-robin ordering, 8 threads per pair) until all pairs are
// numerically orthogonal; the rotations accumulate in V, so R V = U Sigma.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_jacobi_svd(const double* __restrict__ R, int64_t ld, int c, int k,
                                                      int64_t n, Ctl* __restrict__ ctl, int smallest) {
    constexpr int LDC = SMAX + 1;
    __shared__ double Ac[(SMAX + 1) * LDC];   // column j at Ac[j * LDC + i]
    __shared__ double Vc[(SMAX + 1) * LDC];
    __shared__ double sig[SMAX + 1];
    __shared__ int order[SMAX + 1];
    __shared__ int rotated;
    const int tid = threadIdx.x;
    const int cp = (c + 1) & ~1;  // even number of players (a zero column pads odd c)
    for (int t = tid; t < cp * cp; t += BLOCK) {
        const int i = t % cp, j = t / cp;
        Ac[j * LDC + i] = (i < c && j < c) ? R[(int64_t)j * ld + i] : 0.0;
        Vc[j * LDC + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_svd_sweeps(Ac, Vc, cp, LDC, c, &rotated);
    const int rank = svd_order_rank(Ac, LDC, c, n, sig, order);
    const double s1 = (c > 0) ? sig[order[0]] : 0.0;
    const int keff = rank < k ? rank : k;
    for (int i = tid; i < c; i += BLOCK) ctl->sigma[i] = sig[order[i]];
    const int first = smallest ? rank - keff : 0;   // the modes kept: order[first .. first + keff)
    for (int t = tid; t < c * keff; t += BLOCK) {
        const int i = t / keff, j = t % keff;
        ctl->T[i * KMAX + j] = Vc[order[first + j] * LDC + i] / sig[order[first + j]];
    }
    if (tid == 0) {
        ctl->rank = rank;
        ctl->k_eff = keff;
        ctl->nonfinite = isfinite(s1) ? 0 : 1;
    }
}

// W = X T (T = V_k Sigma_k^{-1}, c x k row-major in ctl); rows in [n, npad) are zeroed.
template <int C>
__global__ __launch_bounds__(BLOCK) void k_form_w(int64_t n, int64_t npad, const double* __restrict__ X,
                                                  int64_t ldx, int c, int k, const Ctl* __restrict__ ctl,
                                                  double* __restrict__ W, int64_t ldw) {
    __shared__ double Ts[C * KMAX];
    for (int t = threadIdx.x; t < c * k; t += BLOCK) Ts[(t / k) * KMAX + (t % k)] = ctl->T[(t / k) * KMAX + (t % k)];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= npad) return;
    double x[C];
#pragma unroll
    for (int i = 0; i < C; ++i) x[i] = (r < n && i < c) ? X[(int64_t)i * ldx + r] : 0.0;
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (i < c) s += x[i] * Ts[i * KMAX + j];
        W[(int64_t)j * ldw + r] = s;
    }
}

// Cholesky of G = ctl->red (k x k, column-major) into ctl->L (row-major lower), one wavefront.
__global__ __launch_bounds__(WAVE) void k_cholesky(int k, Ctl* __restrict__ ctl) {
    constexpr int LDM = KMAX + 1;
    __shared__ double G[KMAX * LDM];
    const int lane = threadIdx.x;
    for (int t = lane; t < k * k; t += WAVE) G[(t % k) * LDM + (t / k)] = ctl->red[t];
    __syncthreads();
    int fail = 0;
    for (int j = 0; j < k; ++j) {
        // G[j][j] holds the updated pivot
        const double d = G[j * LDM + j];
        if (!(d > 0.0)) {
            fail = 1;
            break;
        }
        const double ljj = sqrt(d);
        __syncthreads();
        if (lane == j) G[j * LDM + j] = ljj;
        if (lane > j && lane < k) G[lane * LDM + j] /= ljj;
        __syncthreads();
        if (lane > j && lane < k) {
            const double lij = G[lane * LDM + j];
            for (int c2 = j + 1; c2 <= lane; ++c2) G[lane * LDM + c2] -= lij * G[c2 * LDM + j];
        }
        __syncthreads();
    }
    for (int t = lane; t < k * k; t += WAVE) {
        const int i = t / k, j = t % k;
        ctl->L[i * KMAX + j] = (j <= i) ? G[i * LDM + j] : 0.0;
    }
    if (lane == 0) ctl->lu_fail = fail;
}

// W[r, :] <- (L^{-1} W[r, :]^T)^T for every row: column-oriented forward
// substitution with L in LDS; the unknown being finished is always w[0] and the
// register array shifts down after each step.
template <int K>
__global__ __launch_bounds__(BLOCK) void k_trsm_rows(int64_t npad, double* __restrict__ W, int64_t ldw, int k,
                                                     const Ctl* __restrict__ ctl, double* __restrict__ Wr, int ldr,
                                                     float* __restrict__ W32) {
    __shared__ double Ls[K * K];
    for (int t = threadIdx.x; t < k * k; t += BLOCK) Ls[(t / k) * K + (t % k)] = ctl->L[(t / k) * KMAX + (t % k)];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= npad) return;
    // forward substitution with compile-time register indices (columns j >= k stay zero)
    double w[K];
#pragma unroll
    for (int j = 0; j < K; ++j) w[j] = (j < k) ? W[(int64_t)j * ldw + r] : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < k) {
            w[j] /= Ls[j * K + j];
#pragma unroll
            for (int i = j + 1; i < K; ++i)
                if (i < k) w[i] -= Ls[i * K + j] * w[j];
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < k) W[(int64_t)j * ldw + r] = w[j];
    if (W32) {
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) W32[(int64_t)j * ldw + r] = (float)w[j];
    }
    if (Wr) {
        // the row-major copy: this row's ldr-wide slot, written as 16-byte stores (zeros past k)
        double* dst = Wr + r * ldr;
#pragma unroll
        for (int j = 0; j < K; j += 2)
            if (j < ldr) {
                double pr[2] = {j < k ? w[j] : 0.0, j + 1 < k ? w[j + 1] : 0.0};
                __builtin_memcpy(__builtin_assume_aligned(dst + j, 16), pr, sizeof(pr));
            }
    }
}

}  // namespace

int launch_gram_tn(int64_t n, const double* A, int64_t lda, int p, const double* B, int64_t ldb, int q,
                   double* partial, int max_blocks, hipStream_t st) {
    const int tp = (p + 15) / 16, tq = (q + 15) / 16;
    const int R = (tp <= 1 && tq <= 1) ? 128 : ((tp <= 2 && tq <= 2) ? 128 : 64);
    const int64_t nslab = (n + R - 1) / R;
    const int nblk = (int)std::max<int64_t>(
        1, std::min<int64_t>({nslab, (int64_t)max_blocks, GRAM_PARTIAL / ((int64_t)p * q)}));
#define RS_G(TPv, TQv, Rv) k_gram_tn<TPv, TQv, Rv><<<nblk, BLOCK, 0, st>>>(n, A, lda, p, B, ldb, q, partial, nblk)
    if (tp <= 1 && tq <= 1) RS_G(1, 1, 128);
    else if (tp <= 2 && tq <= 2) RS_G(2, 2, 128);
    else RS_G(4, 4, 64);
#undef RS_G
    return nblk;
}

void launch_gram_reduce(const double* partial, int nblk, int pq, double* dst, hipStream_t st) {
    int G = 1;
    while (G < WAVE && G * 2 * pq <= 1024 && G * 2 <= nblk) G *= 2;
    k_gram_reduce<<<1, 1024, 0, st>>>(partial, nblk, pq, G, dst);
}

void launch_small_lu(const double* src, int k, Ctl* ctl, hipStream_t st) { k_small_lu<<<1, WAVE, 0, st>>>(src, k, ctl); }

int tsqr_panel_rows(int c) { return c <= 8 ? 512 : (c <= 16 ? 256 : (c <= 32 ? 128 : TSQR_PANEL)); }

void launch_tsqr_level(int64_t rows, const double* M, int64_t ldm, int c, double* S, int64_t lds, int npanels,
                       hipStream_t st) {
    const unsigned wb = (unsigned)((npanels + 3) / 4);   // four one-wavefront panels per block
    // many panels: the unrolled kernel (its code is shared by the waves of a compute unit); few:
    // the compact one
    const bool many = npanels >= 1024;
    if (c <= 8) {
        if (many) k_tsqr_wave<8, 8><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
        else k_tsqr_wave_loop<8, 8><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
    } else if (c <= 16) {
        if (many) k_tsqr_wave<16, 4><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
        else k_tsqr_wave_loop<16, 4><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
    } else if (c <= 32) {
        if (many) k_tsqr_wave<32, 2><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
        else k_tsqr_wave_loop<32, 2><<<wb, 256, 0, st>>>(rows, M, ldm, c, S, lds);
    } else {
        k_tsqr_level<64><<<npanels, TSQR_PANEL, 0, st>>>(rows, M, ldm, c, S, lds);
    }
}

void launch_jacobi_svd(const double* R, int64_t ld, int c, int k, int64_t n, Ctl* ctl, hipStream_t st,
                       bool smallest) {
    k_jacobi_svd<<<1, BLOCK, 0, st>>>(R, ld, c, k, n, ctl, smallest ? 1 : 0);
}

void launch_form_w(int64_t n, int64_t npad, const double* X, int64_t ldx, int c, int k, const Ctl* ctl, double* W,
                   int64_t ldw, hipStream_t st) {
    const unsigned g = (unsigned)((npad + BLOCK - 1) / BLOCK);
    if (c <= 8) k_form_w<8><<<g, BLOCK, 0, st>>>(n, npad, X, ldx, c, k, ctl, W, ldw);
    else if (c <= 16) k_form_w<16><<<g, BLOCK, 0, st>>>(n, npad, X, ldx, c, k, ctl, W, ldw);
    else if (c <= 32) k_form_w<32><<<g, BLOCK, 0, st>>>(n, npad, X, ldx, c, k, ctl, W, ldw);
    else k_form_w<64><<<g, BLOCK, 0, st>>>(n, npad, X, ldx, c, k, ctl, W, ldw);
}

void launch_cholesky(int k, Ctl* ctl, hipStream_t st) { k_cholesky<<<1, WAVE, 0, st>>>(k, ctl); }

void launch_trsm_rows(int64_t npad, double* W, int64_t ldw, int k, const Ctl* ctl, hipStream_t st, double* Wr,
                      int ldr, float* W32) {
    const unsigned g = (unsigned)((npad + BLOCK - 1) / BLOCK);
    if (k <= 8) k_trsm_rows<8><<<g, BLOCK, 0, st>>>(npad, W, ldw, k, ctl, Wr, ldr, W32);
    else if (k <= 16) k_trsm_rows<16><<<g, BLOCK, 0, st>>>(npad, W, ldw, k, ctl, Wr, ldr, W32);
    else if (k <= 32) k_trsm_rows<32><<<g, BLOCK, 0, st>>>(npad, W, ldw, k, ctl, Wr, ldr, W32);
    else k_trsm_rows<64><<<g, BLOCK, 0, st>>>(npad, W, ldw, k, ctl, Wr, ldr, W32);
}

}  // namespace rs
