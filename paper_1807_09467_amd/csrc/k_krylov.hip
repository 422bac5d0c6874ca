// Krylov-cycle kernels: fused multi-vector dot / update sweeps of classical
// Gram-Schmidt with reorthogonalisation (CGS2) and the oblique projector, the
// fixed-order reductions, the Givens update of the Hessenberg least-squares
// problem, and the end-of-cycle update.
//
// Streaming sweeps walk the rows with a grid-stride loop over `nblk` blocks and
// read every column of the tall operands with fully coalesced wavefront loads.
// Per-block partial sums go to partial[c * nblk + block]; the last block to
// finish (arrival counter) sums them in a fixed order, so results are bitwise
// reproducible for a given launch shape.
#include <algorithm>

#include "kernels.hpp"

namespace rs {

namespace {

// Up to three groups of columns, each dotted with its own vector: partial[c * nblk + block].
template <typename T>
struct DotGroups {
    const T* b0;
    const T* b1;
    const T* b2;
    const T* v0;
    const T* v1;
    const T* v2;
    int n0, n1, n2;
};

// Per-lane partial of sum_b p[b] over b = lane, lane + 64, ... < n with four independent
// accumulators (fixed order for a given n), so the loads of a lane are in flight together.
__device__ __forceinline__ double lane_strided_sum(const double* __restrict__ p, int n) {
    const int lane = threadIdx.x & (WAVE - 1);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = lane;
    for (; b + 3 * WAVE < n; b += 4 * WAVE) {
        a0 += p[b];
        a1 += p[b + WAVE];
        a2 += p[b + 2 * WAVE];
        a3 += p[b + 3 * WAVE];
    }
    for (; b < n; b += WAVE) a0 += p[b];
    return (a0 + a1) + (a2 + a3);
}

constexpr int RED_T = 1024;   // threads of the one-block reductions

// sums[c] = sum over b of partial[c * nblk + b] for c < ncol, by every thread of a RED_T block:
// each column gets a group of G threads (the largest power of two with G ncol <= RED_T, at most
// nblk rounded up), each thread sums a lane-strided share with sixteen accumulators, the group
// combines by butterfly within a wavefront and, for groups wider than one, over LDS in wave
// order.  All loads of a thread are independent, so the block keeps RED_T of them in flight.
// red: LDS scratch of RED_T / WAVE doubles.  Fixed order for given (nblk, ncol).  Ends with a
// barrier.
__device__ void reduce_columns(const double* __restrict__ partial, int nblk, int ncol, double* sums, double* red) {
    int G = 1;
    while (G * 2 * ncol <= RED_T && G < nblk) G *= 2;
    const int gw = G < WAVE ? G : WAVE;
    const int sub = threadIdx.x & (G - 1);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    for (int c0 = 0; c0 < ncol; c0 += RED_T / G) {
        const int c = c0 + threadIdx.x / G;
        // sixteen independent loads per round, so a thread waits for memory about nblk / (16 G)
        // times rather than once per four loads
        double a[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = 0.0;
        if (c < ncol) {
            const double* src = partial + (int64_t)c * nblk;
            int b = sub;
            for (; b + 15 * G < nblk; b += 16 * G) {
#pragma unroll
                for (int u = 0; u < 16; ++u) a[u] += src[b + u * G];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (b + u * G < nblk) a[u] += src[b + u * G];
        }
#pragma unroll
        for (int w = 8; w > 0; w >>= 1)
#pragma unroll
            for (int u = 0; u < w; ++u) a[u] += a[u + w];
        double v = a[0];
        for (int o = gw / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
        if (G > WAVE) {
            if (lane == 0) red[wv] = v;
            __syncthreads();
            if (sub == 0 && c < ncol) {
                double t = 0.0;
                for (int q = 0; q < G / WAVE; ++q) t += red[wv + q];
                sums[c] = t;
            }
            __syncthreads();
        } else if (sub == 0 && c < ncol) {
            sums[c] = v;
        }
    }
    __syncthreads();
}

// Solve E x = b (LU with row permutation in ctl) with one wavefront: lane i holds row i.
__device__ void wave_lu_solve(const Ctl* ctl, int k, const double* b, double* x, double* Es) {
    const int lane = threadIdx.x & (WAVE - 1);
    double v = (lane < k) ? b[ctl->piv[lane]] : 0.0;
    for (int j = 0; j < k; ++j) {  // unit lower
        const double yj = __shfl(v, j, WAVE);
        if (lane > j && lane < k) v -= Es[lane * k + j] * yj;
    }
    for (int j = k - 1; j >= 0; --j) {  // upper
        double xj = 0.0;
        if (lane == j) v = v / Es[j * k + j];
        xj = __shfl(v, j, WAVE);
        if (lane < j) v -= Es[lane * k + j] * xj;
    }
    if (lane < k) x[lane] = v;
}

__global__ __launch_bounds__(RED_T) void k_reduce(const double* __restrict__ partial, int nblk, int ncol,
                                                  double* __restrict__ dst, Ctl* __restrict__ ctl, int nv, int nw,
                                                  int lu_solve, int check_done) {
    if (check_done && ctl->done) return;
    __shared__ double sums[MMAX + KMAX];
    __shared__ double Es[KMAX * KMAX];
    __shared__ double red[RED_T / WAVE];
    const int wv = threadIdx.x / WAVE;
    if (lu_solve) {
        for (int t = threadIdx.x; t < nw * nw; t += RED_T) Es[t] = ctl->E[t];
    }
    reduce_columns(partial, nblk, ncol, sums, red);
    for (int c = threadIdx.x; c < ncol; c += RED_T) dst[c] = sums[c];
    if (lu_solve && wv == 0) wave_lu_solve(ctl, nw, sums + nv, ctl->cw, Es);
}

// Pass-1 coefficients of step j (nv = j + 1 basis vectors) with the oblique projector folded in:
// sums = [V^T w0 | W^T w0 | Z^T v_j]; F[j, :] = v_j^T Z; cw = E^{-1} W^T w0;
// h1 = V^T (w0 - Z cw) = V^T w0 - F cw.  Run by one block of any size (>= 1 wavefront).
// orth: the orthogonal projector I - W W^T (the third group then holds W^T v_j, and cw = W^T w0).
__device__ void pass1_coefficients(const double* __restrict__ partial, int nblk, int nv, int k, Ctl* __restrict__ ctl,
                                   double* sums, double* Es, double* cws, double* red, int orth = 0) {
    const int wv = threadIdx.x / WAVE;
    const int ncol = nv + 2 * k;
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) Es[t] = ctl->E[t];
    reduce_columns(partial, nblk, ncol, sums, red);
    if (k == 0) {
        for (int i = threadIdx.x; i < nv; i += blockDim.x) ctl->h1[i] = sums[i];
        return;
    }
    if (orth) {
        for (int c = threadIdx.x; c < k; c += blockDim.x) cws[c] = sums[nv + c];
    } else if (wv == 0) {
        wave_lu_solve(ctl, k, sums + nv, cws, Es);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        ctl->F[(nv - 1) * KMAX + c] = sums[nv + k + c];
        ctl->cw[c] = cws[c];
    }
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const double* Fi = (i == nv - 1) ? sums + nv + k : ctl->F + i * KMAX;
        double h0 = sums[i], h1 = 0.0, h2 = 0.0, h3 = 0.0;
        int c = 0;
        for (; c + 4 <= k; c += 4) {
            h0 -= Fi[c] * cws[c];
            h1 -= Fi[c + 1] * cws[c + 1];
            h2 -= Fi[c + 2] * cws[c + 2];
            h3 -= Fi[c + 3] * cws[c + 3];
        }
        for (; c < k; ++c) h0 -= Fi[c] * cws[c];
        ctl->h1[i] = (h0 + h1) + (h2 + h3);
    }
}

__global__ __launch_bounds__(RED_T) void k_reduce_pass1(const double* __restrict__ partial, int nblk, int nv, int k,
                                                        int orth, Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double sums[MMAX + 2 * KMAX];
    __shared__ double Es[KMAX * KMAX];
    __shared__ double cws[KMAX];
    __shared__ double red[RED_T / WAVE];
    pass1_coefficients(partial, nblk, nv, k, ctl, sums, Es, cws, red, orth);
}

// Sweep of dot products: wavefront w of the block owns columns [w CPW, w CPW + CPW) of the
// concatenated column list and walks the rows in 64-row tiles (one row per lane, grid-stride over
// tiles); the waves of a block share each tile's vector entries through L1.  Column pointers are
// wave-uniform and every slot loads unconditionally (an unused slot re-reads the wave's first
// column and is zeroed before the reduction), so the loads of a tile are issued together.
template <typename T, int CPW>
__global__ __launch_bounds__(1024) void k_dots(int64_t npad, int64_t ld, DotGroups<T> g,
                                               double* __restrict__ partial, int nblk,
                                               const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int n0 = g.n0, n1 = g.n1, ntot = n0 + n1 + g.n2;
    const int c0 = wv * CPW;
    const T* col[CPW];
    int sel[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
        const int c = (c0 + s < ntot) ? c0 + s : (c0 < ntot ? c0 : 0);
        sel[s] = (c < n0) ? 0 : ((c < n0 + n1) ? 1 : 2);
        col[s] = (sel[s] == 0) ? g.b0 + (int64_t)c * ld
                               : ((sel[s] == 1) ? g.b1 + (int64_t)(c - n0) * ld : g.b2 + (int64_t)(c - n0 - n1) * ld);
    }
    const T* x0p = g.v0;
    const T* x1p = n1 ? g.v1 : g.v0;
    const T* x2p = g.n2 ? g.v2 : g.v0;
    double acc[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) acc[s] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * WAVE + lane; i < npad; i += (int64_t)nblk * WAVE) {
        const double x0 = to_d(x0p[i]), x1 = to_d(x1p[i]), x2 = to_d(x2p[i]);
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
            const double xv = (sel[s] == 0) ? x0 : ((sel[s] == 1) ? x1 : x2);
            acc[s] += to_d(col[s][i]) * xv;
        }
    }
#pragma unroll
    for (int s = 0; s < CPW; ++s)
        if (c0 + s >= ntot) acc[s] = 0.0;
    wave_tr_reduce<CPW>(acc);
    if (wave_tr_owner<CPW>()) {
#pragma unroll
        for (int t = 0; t < wave_tr_left<CPW>(); ++t) {
            const int c = c0 + wave_tr_col<CPW>(t);
            if (c < ntot) partial[(int64_t)c * nblk + blockIdx.x] = acc[t];
        }
    }
}

// u - sum_{c < nc} col_c[i] coef[c] with the column loop unrolled by 8 into four partial sums
// (coefficients in LDS or registers), so eight independent loads are in flight per row.
template <typename T>
__device__ __forceinline__ double row_update(const T* __restrict__ B, int64_t ld, int nc, int64_t i,
                                             const double* __restrict__ cs, double u) {
    double u1 = 0.0, u2 = 0.0, u3 = 0.0;
    int c = 0;
    for (; c + 8 <= nc; c += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = to_d(B[(int64_t)(c + q) * ld + i]);
        u -= v[0] * cs[c] + v[4] * cs[c + 4];
        u1 -= v[1] * cs[c + 1] + v[5] * cs[c + 5];
        u2 -= v[2] * cs[c + 2] + v[6] * cs[c + 6];
        u3 -= v[3] * cs[c + 3] + v[7] * cs[c + 7];
    }
    for (; c < nc; ++c) u -= to_d(B[(int64_t)c * ld + i]) * cs[c];
    return (u + u1) + (u2 + u3);
}

// Column j of the Hessenberg matrix, Givens rotations, residual estimate, stop test.  Run by
// the first wavefront of one block; hcol is LDS scratch of MMAX + 1 doubles.
__device__ void givens_column(double s, int j, Ctl* __restrict__ ctl, double* hcol) {
    const int lane = threadIdx.x;
    if (lane >= WAVE) return;
    const double hn = sqrt(s);
    double cn = 0.0;
    for (int i = lane; i <= j; i += WAVE) {
        const double h = ctl->h1[i] + ctl->h2[i];
        cn += h * h;
    }
    cn = wave_sum(cn) + s;
    if (lane != 0) return;
    for (int i = 0; i <= j; ++i) hcol[i] = ctl->h1[i] + ctl->h2[i];
    hcol[j + 1] = hn;
    const double colnorm = sqrt(cn);
    for (int i = 0; i < j; ++i) {
        const double c = ctl->cs[i], sn = ctl->sn[i];
        const double t = c * hcol[i] + sn * hcol[i + 1];
        hcol[i + 1] = -sn * hcol[i] + c * hcol[i + 1];
        hcol[i] = t;
    }
    const double a = hcol[j], b = hn;
    const double rho = hypot(a, b);
    double c = 1.0, sn = 0.0;
    if (rho != 0.0) {
        c = a / rho;
        sn = b / rho;
    }
    ctl->cs[j] = c;
    ctl->sn[j] = sn;
    hcol[j] = rho;
    constexpr int LDR = MMAX + 1;
    for (int i = 0; i <= j; ++i) ctl->R[i + LDR * j] = hcol[i];
    const double gj = ctl->g[j];
    const double gn = -sn * gj;
    ctl->g[j + 1] = gn;
    ctl->g[j] = c * gj;
    const int steps = j + 1;
    ctl->steps = steps;
    ctl->gimp = fabs(gn);
    const bool lucky = !(hn > 1e-14 * colnorm);
    const bool bad = !isfinite(hn) || !isfinite(gn) || !isfinite(rho);
    if (bad) ctl->nonfinite = 1;
    if (lucky) ctl->lucky = 1;
    if (bad || lucky || fabs(gn) <= ctl->stop_abs || steps >= ctl->max_steps) ctl->done = 1;
    ctl->inv_h = (hn > 0.0) ? 1.0 / hn : 0.0;
}

__global__ __launch_bounds__(RED_T) void k_givens(const double* __restrict__ partial, int nblk, int j,
                                                  Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double hcol[MMAX + 1];
    __shared__ double sums[1];
    __shared__ double red[RED_T / WAVE];
    reduce_columns(partial, nblk, 1, sums, red);
    givens_column(sums[0], j, ctl, hcol);
}

// w -= V coefV + Z coefZ, then partial dots V^T w with the updated w.  Wavefront w owns V
// columns [w CPW, w CPW + CPW) and a share of the Z columns.  Rows go in pairs of 64-row tiles
// (lane l holds rows l and l + 64 of the pair): each wave forms its part of the row updates, the
// parts meet in LDS (double-buffered, one barrier per pair), every wave finishes the updated rows
// in the same fixed order, wave 0 stores them, and each wave accumulates the dots of its own
// columns (kept in registers) with the updated rows.
template <typename T, int CPW>
__global__ __launch_bounds__(1024) void k_update_dots(int64_t npad, const T* __restrict__ V, int64_t ld, int nv,
                                                      const T* __restrict__ Z, int nz, T* __restrict__ w,
                                                      const double* __restrict__ coefV,
                                                      const double* __restrict__ coefZ,
                                                      double* __restrict__ partial, int nblk,
                                                      const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double part[2][16][2 * WAVE];
    __shared__ double czs[KMAX];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int NW = blockDim.x / WAVE;
    const int c0 = wv * CPW;
    for (int t = threadIdx.x; t < nz; t += blockDim.x) czs[t] = coefZ[t];
    const T* col[CPW];
    double hc[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
        const bool ok = c0 + s < nv;
        col[s] = V + (int64_t)(ok ? c0 + s : 0) * ld;
        hc[s] = ok ? coefV[c0 + s] : 0.0;
    }
    const int zper = (nz + NW - 1) / NW;
    const int z0 = wv * zper < nz ? wv * zper : nz;
    const int z1 = (z0 + zper < nz) ? z0 + zper : nz;
    double acc[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) acc[s] = 0.0;
    __syncthreads();
    int buf = 0;
    for (int64_t t = blockIdx.x; t * 2 * WAVE < npad; t += nblk) {
        const int64_t i0 = t * 2 * WAVE + lane;
        const bool two = i0 + WAVE < npad;          // uniform: npad is a multiple of 64
        const int64_t i1 = two ? i0 + WAVE : i0;
        const double wi0 = to_d(w[i0]), wi1 = to_d(w[i1]);
        double va[CPW], vb[CPW];
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
            va[s] = to_d(col[s][i0]);
            vb[s] = to_d(col[s][i1]);
            p0 += va[s] * hc[s];
            p1 += vb[s] * hc[s];
        }
        {
            double q0 = 0.0, q1 = 0.0;
            int c = z0;
            for (; c + 2 <= z1; c += 2) {
                const T* za = Z + (int64_t)c * ld;
                const T* zb = za + ld;
                const double a0 = to_d(za[i0]), a1 = to_d(za[i1]), b0 = to_d(zb[i0]), b1 = to_d(zb[i1]);
                q0 += a0 * czs[c] + b0 * czs[c + 1];
                q1 += a1 * czs[c] + b1 * czs[c + 1];
            }
            if (c < z1) {
                const T* za = Z + (int64_t)c * ld;
                q0 += to_d(za[i0]) * czs[c];
                q1 += to_d(za[i1]) * czs[c];
            }
            p0 += q0;
            p1 += q1;
        }
        part[buf][wv][lane] = p0;
        part[buf][wv][WAVE + lane] = p1;
        __syncthreads();
        double u0 = wi0, u1 = wi1;
        for (int q = 0; q < NW; ++q) {
            u0 -= part[buf][q][lane];
            u1 -= part[buf][q][WAVE + lane];
        }
        const T us0 = (T)u0, us1 = (T)u1;
        if (wv == 0) {
            w[i0] = us0;
            if (two) w[i1] = us1;
        }
        const double ud0 = to_d(us0), ud1 = two ? to_d(us1) : 0.0;
#pragma unroll
        for (int s = 0; s < CPW; ++s) acc[s] += va[s] * ud0 + vb[s] * ud1;
        buf ^= 1;
    }
#pragma unroll
    for (int s = 0; s < CPW; ++s)
        if (c0 + s >= nv) acc[s] = 0.0;
    wave_tr_reduce<CPW>(acc);
    if (wave_tr_owner<CPW>()) {
#pragma unroll
        for (int t = 0; t < wave_tr_left<CPW>(); ++t) {
            const int c = c0 + wave_tr_col<CPW>(t);
            if (c < nv) partial[(int64_t)c * nblk + blockIdx.x] = acc[t];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_update_norm(int64_t npad, const T* __restrict__ V, int64_t ld, int nv,
                                                       T* __restrict__ w, const double* __restrict__ coef,
                                                       double* __restrict__ partial, int nblk,
                                                       const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double cv[MMAX];
    __shared__ double lds4[BLOCK / WAVE];
    for (int t = threadIdx.x; t < nv; t += BLOCK) cv[t] = coef[t];
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        const T us = (T)row_update(V, ld, nv, i, cv, to_d(w[i]));
        w[i] = us;
        const double ud = to_d(us);
        acc += ud * ud;
    }
    acc = block_sum(acc, lds4);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void k_cycle_init(Ctl* ctl, int max_steps, double stop_abs, int unit_scale) {
    if (threadIdx.x != 0) return;
    const double beta = ctl->rnorm;
    ctl->beta = beta;
    ctl->g[0] = beta;
    ctl->inv_h = unit_scale ? 1.0 : 1.0 / beta;
    ctl->steps = 0;
    ctl->done = 0;
    ctl->lucky = 0;
    ctl->max_steps = max_steps;
    ctl->stop_abs = stop_abs;
    ctl->gimp = beta;
}

// y = R^{-1} g, back substitution with one wavefront (two rows per lane when steps > 64).
__global__ __launch_bounds__(WAVE) void k_cycle_solve(Ctl* __restrict__ ctl) {
    const int lane = threadIdx.x;
    const int s = ctl->steps;
    constexpr int LDR = MMAX + 1;
    double v0 = (lane < s) ? ctl->g[lane] : 0.0;
    double v1 = (lane + WAVE < s) ? ctl->g[lane + WAVE] : 0.0;
    for (int j = s - 1; j >= 0; --j) {
        const double rjj = ctl->R[j + LDR * j];
        double yj;
        if (j < WAVE) {
            if (lane == j) v0 = v0 / rjj;
            yj = __shfl(v0, j, WAVE);
        } else {
            if (lane == j - WAVE) v1 = v1 / rjj;
            yj = __shfl(v1, j - WAVE, WAVE);
        }
        if (lane < j) v0 -= ctl->R[lane + LDR * j] * yj;
        if (lane + WAVE < j) v1 -= ctl->R[lane + WAVE + LDR * j] * yj;
    }
    if (lane < s) ctl->y[lane] = v0;
    if (lane + WAVE < s) ctl->y[lane + WAVE] = v1;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_x_update(int64_t n, const T* __restrict__ V, int64_t ld,
                                                    const double* __restrict__ dinv, double* __restrict__ x,
                                                    const Ctl* __restrict__ ctl) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int s = ctl->steps;
    const double acc = -row_update(V, ld, s, i, ctl->y, 0.0);
    x[i] += dinv ? acc * dinv[i] : acc;
}

__global__ __launch_bounds__(BLOCK) void k_correct(int64_t npad, const double* __restrict__ W,
                                                   const double* __restrict__ Z, int64_t ld, int k,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   const Ctl* __restrict__ ctl, double* __restrict__ partial,
                                                   int nblk) {
    __shared__ double lds4[BLOCK / WAVE];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        double ri = r[i];
        if (k > 0) {
            double xi = x[i];
            for (int c = 0; c < k; ++c) {
                const double cc = ctl->cw[c];
                xi += W[(int64_t)c * ld + i] * cc;
                ri -= Z[(int64_t)c * ld + i] * cc;
            }
            x[i] = xi;
            r[i] = ri;
        }
        acc += ri * ri;
    }
    acc = block_sum(acc, lds4);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(WAVE) void k_finish_norm(const double* __restrict__ partial, int nblk,
                                                      Ctl* __restrict__ ctl, int which) {
    const int lane = threadIdx.x;
    const double s = wave_sum(lane_strided_sum(partial, nblk));
    if (lane == 0) {
        const double nrm = sqrt(s);
        if (!isfinite(nrm)) ctl->nonfinite = 1;
        if (which == 0) ctl->rnorm = nrm;
        else ctl->bnorm = nrm;
    }
}

__global__ __launch_bounds__(BLOCK) void k_norm2(int64_t n, const double* __restrict__ v,
                                                 double* __restrict__ partial, int nblk) {
    __shared__ double lds4[BLOCK / WAVE];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)nblk * BLOCK) {
        const double t = v[i];
        acc += t * t;
    }
    acc = block_sum(acc, lds4);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(BLOCK) void k_copy_pad(int64_t n, int64_t npad, const double* __restrict__ in,
                                                    double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < npad) out[i] = (in && i < n) ? in[i] : 0.0;
}

// out = sum_{j<q} w_j x_j over the first n entries, zero up to npad: the extrapolated initial
// guess from the most recent solutions (section 4.1, eqs. (ext2)-(ext4)); one pass over the q
// inputs and the output.
__global__ __launch_bounds__(BLOCK) void k_extrapolate(int64_t n, int64_t npad, Extrap e, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= npad) return;
    double acc = 0.0;
    if (i < n) {
        for (int j = 0; j < e.q; ++j) acc += e.w[j] * e.x[j][i];
    }
    out[i] = acc;
}

// ---------------------------------------------------------------------------
// Arnoldi with delayed reorthogonalisation (two sweeps per step).  Step j holds the candidate
// u for basis vector j, orthogonalised once against V_j = [v_0 .. v_{j-1}] and not normalised,
// and z = A D^{-1} u.  One sweep forms V_j^T u, V_j^T z, W^T z, (A W)^T u, u.u and u.z; from them
// the reduction completes Hessenberg column j-1 (its second-pass part V_j^T u and subdiagonal
// ||u - V_j V_j^T u||), rotates it, and derives column j's first-pass coefficients for
// P A D^{-1} v_j through the Arnoldi relation; one update sweep then writes v_j and the next
// candidate.  In exact arithmetic this is the CGS2 Arnoldi process; the second pass of each
// vector is merged into the next step.
// ---------------------------------------------------------------------------

// Sweep of the columns [V_j, W, A W, u], each dotted with u and with z (CPW columns per
// wavefront, 64-row tiles): partial[(2c + e) nblk + b], e = 0 for u, 1 for z.  With zskip = kz
// the A W columns are left out of the sweep (the swept columns are [V_j, W, u], numbered
// 0 .. nq + k) and their slots of the partials stay unwritten: the update sweep of the previous
// step has already formed their dots with u, and the dots of A W with z are not used.
template <typename T, int CPW>
__global__ __launch_bounds__(1024) void k_dots2(int64_t npad, int64_t ld, const T* __restrict__ V, int nq,
                                                const T* __restrict__ W, const T* __restrict__ Z, int k, int kz,
                                                int zskip, const T* __restrict__ u, const T* __restrict__ z,
                                                int c_begin, int c_end, double* __restrict__ partial, int nblk,
                                                const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int c0 = c_begin + wv * CPW;
    const T* col[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
        int c = c0 + s < c_end ? c0 + s : (c0 < c_end ? c0 : c_begin);
        if (c >= nq + k) c += zskip;   // swept column -> slot of [V_j, W, A W, u]
        col[s] = c < nq ? V + (int64_t)c * ld
                        : (c < nq + k ? W + (int64_t)(c - nq) * ld : (c < nq + k + kz ? Z + (int64_t)(c - nq - k) * ld : u));
    }
    // 16-byte loads: VEC consecutive rows per lane (npad is a multiple of 64)
    constexpr int VEC = 16 / sizeof(T);
    double acc[2 * CPW];
#pragma unroll
    for (int s = 0; s < 2 * CPW; ++s) acc[s] = 0.0;
    const int64_t nvec = npad / VEC;
    for (int64_t q = (int64_t)blockIdx.x * WAVE + lane; q < nvec; q += (int64_t)nblk * WAVE) {
        const int64_t i = q * VEC;
        T xu[VEC], xz[VEC];
        __builtin_memcpy(xu, u + i, sizeof(xu));
        __builtin_memcpy(xz, z + i, sizeof(xz));
#pragma unroll
        for (int s = 0; s < CPW; ++s) {
            T v[VEC];
            __builtin_memcpy(v, col[s] + i, sizeof(v));
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                acc[2 * s] += to_d(v[e]) * to_d(xu[e]);
                acc[2 * s + 1] += to_d(v[e]) * to_d(xz[e]);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < CPW; ++s)
        if (c0 + s >= c_end) acc[2 * s] = acc[2 * s + 1] = 0.0;
    wave_tr_reduce<2 * CPW>(acc);
    if (wave_tr_owner<2 * CPW>()) {
#pragma unroll
        for (int t = 0; t < wave_tr_left<2 * CPW>(); ++t) {
            const int q = wave_tr_col<2 * CPW>(t);   // q = 2 s + e
            const int c = c0 + q / 2;
            const int slot = c >= nq + k ? c + zskip : c;
            if (c < c_end) partial[(int64_t)(2 * slot + (q & 1)) * nblk + blockIdx.x] = acc[t];
        }
    }
}

// sums[e] = sum over b of partial[e * nblk + b], e < nent: one wavefront per entry, eight loads
// in flight per lane, fixed order.  Spreads the cross-block reduction of a sweep over many
// compute units (one block reading every partial waits on remote caches for most of them).
// With zpart, the entries of the kz A W columns (slots zlo .. zlo + kz - 1) come from the update
// sweep's partials instead: their dots with u are the sum of zpart[c * nblk_z + b] minus
// (G cw)_c / nu with the previous step's cw and nu (still in the control block) and
// G = (A W)^T A W (gz, kz x kz row-major); their dots with z are not used and are set to zero.
__global__ __launch_bounds__(1024) void k_colsum(const double* __restrict__ partial, int nblk, int nent,
                                                 double* __restrict__ sums, const Ctl* __restrict__ ctl,
                                                 const double* __restrict__ zpart, int nblk_z, int zlo, int kz,
                                                 const double* __restrict__ gz) {
    if (ctl->done) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int e = blockIdx.x * (1024 / WAVE) + threadIdx.x / WAVE;
    if (e >= nent) return;
    const double* src = partial + (int64_t)e * nblk;
    double corr = 0.0;
    if (zpart && e >= 2 * zlo && e < 2 * (zlo + kz)) {
        if (e & 1) {
            if (lane == 0) sums[e] = 0.0;
            return;
        }
        const int c = (e - 2 * zlo) / 2;
        src = zpart + (int64_t)c * nblk_z;
        nblk = nblk_z;
        double g = lane < kz ? gz[c * kz + lane] * ctl->cw[lane] : 0.0;
        corr = wave_sum(g) * ctl->inv_nu;
    }
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int b = lane;
    for (; b + 7 * WAVE < nblk; b += 8 * WAVE) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += src[b + u * WAVE];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (b + u * WAVE < nblk) a[u] += src[b + u * WAVE];
    const double v = wave_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
    if (lane == 0) sums[e] = v - corr;
}

// One block: reduce the sweep, complete and rotate column j-1, prepare step j's update.
// has_z = 0 on the closing step of a cycle (no product was taken): only column j-1 completes.
// The loads of the control block are issued together at the start, and the sums over the
// Hessenberg matrix and F are split over the wavefronts, so the block waits for memory a few
// times rather than once per term.
__global__ __launch_bounds__(RED_T) void k_dcgs2_reduce(const double* __restrict__ dsum, int j, int k, int kz,
                                                        int orth, int has_z, Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    constexpr int LDH = MMAX + 1;
    constexpr int LDR = MMAX + 1;
    constexpr int NW = RED_T / WAVE;
    __shared__ double sums[2 * (MMAX + 2 * KMAX + 1)];
    __shared__ double Es[KMAX * KMAX];
    __shared__ double cws[KMAX];
    __shared__ double wz[KMAX];
    __shared__ double Qz[MMAX + 1];
    __shared__ double hcol[MMAX + 2];
    __shared__ double css[MMAX], sns[MMAX];
    constexpr int NH = 8, NF = NW - 1 - NH;   // wavefronts summing H h, and h^T F
    __shared__ double pH[NH][MMAX + 1];   // per-wavefront partial sums of H h
    __shared__ double pF[NF][KMAX];       // ... of h^T F (row j of F before scaling)
    static_assert(NW * MMAX <= KMAX * KMAX, "partial sums of F cws reuse the LU factors' space");
    double(*pQ)[MMAX] = reinterpret_cast<double(*)[MMAX]>(Es);   // ... of F cws, once the LU solve is done
    __shared__ double scal[4];
    __shared__ int stop;
    const int tid = threadIdx.x;
    const int wv = tid / WAVE, lane = tid & (WAVE - 1);
    const int ncol = j + k + kz + 1;
    // sweep columns: V (0..j-1), W (j..j+k-1), A W (kz = k columns, oblique projector only), u;
    // pz = first column of the projector's image (A W for the oblique projector; the W slot when
    // the sweep has no A W columns: W for the orthogonal projector, and for the least-squares one,
    // whose caller puts A W in the W slot), cu = the column of u
    const int pz = (kz == 0) ? j : j + k, cu = j + k + kz;
    const int jc = j - 1;   // the column completed here (none when j = 0)
    for (int t = tid; t < k * k; t += RED_T) Es[t] = ctl->E[t];
    for (int t = tid; t < jc; t += RED_T) {
        css[t] = ctl->cs[t];
        sns[t] = ctl->sn[t];
    }
    for (int t = tid; t < 2 * ncol; t += RED_T) sums[t] = dsum[t];
    __syncthreads();
    // sums[2 c] = col_c . u, sums[2 c + 1] = col_c . z; columns: V (0..j-1), W, A W, u
    const double* su = sums;
    if (wv == 0) {
        double hh = 0.0;
        for (int l = lane; l < j; l += WAVE) hh += su[2 * l] * su[2 * l];
        hh = wave_sum(hh);
        const double uu = su[2 * cu];
        const double nu = (j == 0) ? ctl->beta : sqrt(fmax(uu - hh, 0.0));
        if (lane == 0) {
            scal[0] = nu;
            stop = 0;
        }
        if (j >= 1) {
            // column j-1: first-pass part from the previous step plus the second-pass part
            double cn = 0.0;
            for (int l = lane; l < j; l += WAVE) {
                const double h = ctl->hp[l] + su[2 * l];
                hcol[l] = h;
                cn += h * h;
            }
            cn = wave_sum(cn) + nu * nu;
            if (lane == 0) hcol[j] = nu;
            __builtin_amdgcn_wave_barrier();
            for (int l = lane; l <= j; l += WAVE) ctl->Hs[l + LDH * jc] = hcol[l];
            if (lane == 0) {
                double a = hcol[0];
#pragma unroll 8
                for (int l = 0; l < jc; ++l) {
                    const double c = css[l], sn = sns[l], b = hcol[l + 1];
                    ctl->R[l + LDR * jc] = c * a + sn * b;
                    a = -sn * a + c * b;
                }
                const double rho = hypot(a, nu);
                double c = 1.0, sn = 0.0;
                if (rho != 0.0) {
                    c = a / rho;
                    sn = nu / rho;
                }
                ctl->cs[jc] = c;
                ctl->sn[jc] = sn;
                ctl->R[jc + LDR * jc] = rho;
                const double gj = ctl->g[jc];
                const double gn = -sn * gj;
                ctl->g[jc + 1] = gn;
                ctl->g[jc] = c * gj;
                ctl->steps = j;
                ctl->gimp = fabs(gn);
                const bool lucky = !(nu > 1e-14 * sqrt(cn));
                const bool bad = !isfinite(nu) || !isfinite(gn) || !isfinite(rho);
                if (bad) ctl->nonfinite = 1;
                if (lucky) ctl->lucky = 1;
                if (bad || lucky || fabs(gn) <= ctl->stop_abs || j >= ctl->max_steps || !has_z) {
                    ctl->done = 1;
                    stop = 1;
                }
            }
        }
    } else if (wv <= NH) {
        // waves 1..NH: partial sums of (H h)_i = sum_{l >= i-1} H[i, l] h_l over the columns
        // l < j - 1 kept in the control block (column j - 1 is hcol, added below)
        const int w = wv - 1;
        double ph0 = 0.0, ph1 = 0.0;
#pragma unroll 4
        for (int l = w; l < j - 1; l += NH) {
            const double h = su[2 * l];
            if (lane <= l + 1) ph0 += ctl->Hs[lane + LDH * l] * h;
            if (lane + WAVE <= l + 1) ph1 += ctl->Hs[lane + WAVE + LDH * l] * h;
        }
        pH[w][lane] = ph0;
        if (lane + WAVE <= MMAX) pH[w][lane + WAVE] = ph1;
        // rows from 2 WAVE on take no column kept in the control block (those columns end at row
        // j - 1 < 2 WAVE)
        for (int i = 2 * WAVE + lane; i <= MMAX; i += WAVE) pH[w][i] = 0.0;
    } else {
        // the other waves: partial sums of (h^T F)_c = sum_l h_l F[l, c]
        const int w = wv - 1 - NH;
        double pf = 0.0;
        if (lane < k) {
#pragma unroll 4
            for (int l = w; l < j; l += NF) pf += su[2 * l] * ctl->F[l * KMAX + lane];
        }
        pF[w][lane] = pf;
    }
    __syncthreads();
    if (stop || !has_z) return;
    const double nu = scal[0];
    const double inv = 1.0 / nu;
    // the projector's coefficients for z: c = E^{-1} W^T z (oblique) or W^T z (orthogonal)
    if (k > 0 && wv == 0) {
        if (lane < k) wz[lane] = su[2 * (j + lane) + 1];   // W^T z, contiguous for the solve
        __builtin_amdgcn_wave_barrier();
        if (orth) {
            if (lane < k) cws[lane] = wz[lane];
        } else {
            wave_lu_solve(ctl, k, wz, cws, Es);
        }
    }
    __syncthreads();
    // partial sums of (F cws)_l over groups of recycle columns: wavefront w takes c = w, w + NW, ...
    for (int l = lane; l < j; l += WAVE) {
        double q = 0.0;
#pragma unroll 4
        for (int c = wv; c < k; c += NW) q += ctl->F[l * KMAX + c] * cws[c];
        pQ[wv][l] = q;
    }
    // F row j and cw
    for (int c = tid; c < k; c += RED_T) {
        double f = 0.0;
        for (int w = 0; w < NF; ++w) f += pF[w][c];
        ctl->F[j * KMAX + c] = (su[2 * (pz + c)] - f) * inv;   // u . (A W or W)_c - h^T F[:, c]
        ctl->cw[c] = cws[c];
    }
    __syncthreads();
    // V_j^T (P z) and u^T (P z)
    for (int l = tid; l < j; l += RED_T) {
        double q = 0.0;
        for (int w = 0; w < NW; ++w) q += pQ[w][l];
        Qz[l] = su[2 * l + 1] - q;   // v_l . z - (F cws)_l
    }
    if (wv == NW - 1) {
        double uz = 0.0;
        for (int c = lane; c < k; c += WAVE) uz += su[2 * (pz + c)] * cws[c];
        uz = wave_sum(uz);
        if (lane == 0) scal[1] = su[2 * cu + 1] - uz;   // u . z - (u^T A W or u^T W) cws
    }
    __syncthreads();
    if (wv == 0) {
        double q = 0.0;
        for (int l = lane; l < j; l += WAVE) q += su[2 * l] * Qz[l];
        q = wave_sum(q);
        if (lane == 0) {
            Qz[j] = (scal[1] - q) * inv;   // v_j . (P z)
            ctl->inv_nu = inv;
        }
    }
    __syncthreads();
    // first-pass coefficients g of column j and the update coefficients d = H h / nu + g, with
    // h = V_j^T u the second-pass coefficients of v_j and H the unrotated Hessenberg (j+1 x j)
    for (int i = tid; i <= j; i += RED_T) {
        double hh = 0.0;
        for (int w = 0; w < NH; ++w) hh += pH[w][i];
        if (j >= 1) hh += hcol[i] * su[2 * (j - 1)];   // column j - 1 (zero below row j)
        const double g = (Qz[i] - hh) * inv;
        ctl->hp[i] = g;
        ctl->dq[i] = hh * inv + g;
    }
    for (int l = tid; l < j; l += RED_T) ctl->hr[l] = su[2 * l];
}

// v_j = (u - V hr) / nu; u <- (z - (A W) cw) / nu - V dq[0..j) - v_j dq[j]   (VEC rows per thread)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_dcgs2_update(int64_t npad, T* __restrict__ V, int64_t ld, int j,
                                                        const T* __restrict__ Z, int k, T* __restrict__ u,
                                                        const T* __restrict__ z, int nblk, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double hr[MMAX], dq[MMAX + 1], cw[KMAX];
    for (int t = threadIdx.x; t < j; t += BLOCK) hr[t] = ctl->hr[t];
    for (int t = threadIdx.x; t <= j; t += BLOCK) dq[t] = ctl->dq[t];
    for (int t = threadIdx.x; t < k; t += BLOCK) cw[t] = ctl->cw[t];
    const double inv = ctl->inv_nu;
    __syncthreads();
    T* vj = V + (int64_t)j * ld;
    // VEC consecutive rows per thread, 32 bytes of each column (two 16-byte loads; npad is a
    // multiple of 64): a wavefront reads 2 KB runs of every column, which streams measurably
    // faster than 1 KB runs on this memory system
    constexpr int VEC = 32 / sizeof(T);
    const int64_t nvec = npad / VEC;
    for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < nvec; q += (int64_t)nblk * BLOCK) {
        const int64_t i = q * VEC;
        T t[VEC];
        double a[VEC], b[VEC];
        __builtin_memcpy(t, u + i, sizeof(t));
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            a[e] = to_d(t[e]);
            b[e] = 0.0;
        }
#pragma unroll 4
        for (int l = 0; l < j; ++l) {
            T v[VEC];
            __builtin_memcpy(v, V + (int64_t)l * ld + i, sizeof(v));
            const double h = hr[l], d = dq[l];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                a[e] -= to_d(v[e]) * h;
                b[e] += to_d(v[e]) * d;
            }
        }
        T qs[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) qs[e] = (T)(a[e] * inv);
        __builtin_memcpy(vj + i, qs, sizeof(qs));
        __builtin_memcpy(t, z + i, sizeof(t));
        double zc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) zc[e] = to_d(t[e]);
#pragma unroll 4
        for (int c = 0; c < k; ++c) {
            T w[VEC];
            __builtin_memcpy(w, Z + (int64_t)c * ld + i, sizeof(w));
#pragma unroll
            for (int e = 0; e < VEC; ++e) zc[e] -= to_d(w[e]) * cw[c];
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) t[e] = (T)(zc[e] * inv - b[e] - to_d(qs[e]) * dq[j]);
        __builtin_memcpy(u + i, t, sizeof(t));
    }
}

// The update above for recycle dimensions k <= KZ, which also forms the per-block dots of the
// A W columns with the new candidate u: with y = V dq + v_j dq_j and s = z / nu - y (both known
// before the A W columns are read), u = s - (A W) cw / nu, so (A W)^T u = (A W)^T s -
// G cw / nu with G = (A W)^T A W.  The kernel accumulates (A W)^T s while it streams A W for
// the projector (zpart[c * nblk + b]); the column sums of the next step subtract G cw / nu.
// The next step's sweep then need not read A W at all.
template <typename T, int KZ>
__global__ __launch_bounds__(BLOCK) void k_dcgs2_update_zd(int64_t npad, T* __restrict__ V, int64_t ld, int j,
                                                           const T* __restrict__ Z, int k, T* __restrict__ u,
                                                           const T* __restrict__ z, int nblk,
                                                           const Ctl* __restrict__ ctl, double* __restrict__ zpart) {
    if (ctl->done) return;
    __shared__ double hr[MMAX], dq[MMAX + 1], cw[KMAX];
    __shared__ double zs[BLOCK / WAVE][KZ];
    for (int t = threadIdx.x; t < j; t += BLOCK) hr[t] = ctl->hr[t];
    for (int t = threadIdx.x; t <= j; t += BLOCK) dq[t] = ctl->dq[t];
    for (int t = threadIdx.x; t < k; t += BLOCK) cw[t] = ctl->cw[t];
    const double inv = ctl->inv_nu;
    __syncthreads();
    T* vj = V + (int64_t)j * ld;
    constexpr int VEC = 32 / sizeof(T);   // 32 bytes of each column per thread
    double acc[KZ];
#pragma unroll
    for (int c = 0; c < KZ; ++c) acc[c] = 0.0;
    const int64_t nvec = npad / VEC;
    for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < nvec; q += (int64_t)nblk * BLOCK) {
        const int64_t i = q * VEC;
        T t[VEC];
        double a[VEC], b[VEC];
        __builtin_memcpy(t, u + i, sizeof(t));
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            a[e] = to_d(t[e]);
            b[e] = 0.0;
        }
#pragma unroll 4
        for (int l = 0; l < j; ++l) {
            T v[VEC];
            __builtin_memcpy(v, V + (int64_t)l * ld + i, sizeof(v));
            const double h = hr[l], d = dq[l];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                a[e] -= to_d(v[e]) * h;
                b[e] += to_d(v[e]) * d;
            }
        }
        T qs[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) qs[e] = (T)(a[e] * inv);
        __builtin_memcpy(vj + i, qs, sizeof(qs));
        __builtin_memcpy(t, z + i, sizeof(t));
        double zc[VEC], sv[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            zc[e] = to_d(t[e]);
            sv[e] = zc[e] * inv - (b[e] + to_d(qs[e]) * dq[j]);
        }
#pragma unroll
        for (int c = 0; c < KZ; ++c) {
            if (c < k) {
                T w[VEC];
                __builtin_memcpy(w, Z + (int64_t)c * ld + i, sizeof(w));
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    zc[e] -= to_d(w[e]) * cw[c];
                    acc[c] += to_d(w[e]) * sv[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) t[e] = (T)(zc[e] * inv - b[e] - to_d(qs[e]) * dq[j]);
        __builtin_memcpy(u + i, t, sizeof(t));
    }
    wave_tr_reduce<KZ>(acc);
    const int wv = threadIdx.x / WAVE;
    if (wave_tr_owner<KZ>()) {
#pragma unroll
        for (int t = 0; t < wave_tr_left<KZ>(); ++t) zs[wv][wave_tr_col<KZ>(t)] = acc[t];
    }
    __syncthreads();
    if (threadIdx.x < k) {
        const int c = threadIdx.x;
        zpart[(int64_t)c * nblk + blockIdx.x] = (zs[0][c] + zs[1][c]) + (zs[2][c] + zs[3][c]);
    }
}

}  // namespace

template <typename T>
void launch_dots(int64_t npad, int64_t ld, const T* const* bases, const T* const* vecs, const int* counts,
                 int ngroups, double* partial, int nblk, Ctl* ctl, hipStream_t st, int pass1_nv, int pass1_k,
                 hipEvent_t ev0, hipEvent_t ev1, bool pass1_orth) {
    constexpr int CPW = 8;
    int ntot = 0;
    for (int q = 0; q < ngroups; ++q) ntot += counts[q];
    // at most 16 wavefronts (128 columns) per launch
    for (int a = 0; a < ntot; a += 16 * CPW) {
        const int b = (ntot - a) < 16 * CPW ? ntot : a + 16 * CPW;
        const T* gb[3] = {nullptr, nullptr, nullptr};
        const T* gv[3] = {nullptr, nullptr, nullptr};
        int gn[3] = {0, 0, 0};
        int gi = 0, off = 0;
        for (int q = 0; q < ngroups; ++q) {
            const int lo = off > a ? off : a;
            const int hi = (off + counts[q]) < b ? (off + counts[q]) : b;
            if (hi > lo) {
                gb[gi] = bases[q] + (int64_t)(lo - off) * ld;
                gv[gi] = vecs[q];
                gn[gi] = hi - lo;
                ++gi;
            }
            off += counts[q];
        }
        DotGroups<T> g{gb[0], gb[1], gb[2], gv[0], gv[1], gv[2], gn[0], gn[1], gn[2]};
        const int nw = (b - a + CPW - 1) / CPW;
        const bool first = a == 0, last = b == ntot;
        hipExtLaunchKernelGGL(k_dots<T, CPW>, dim3(nblk), dim3(nw * WAVE), 0, st, first ? ev0 : nullptr,
                              last ? ev1 : nullptr, 0, npad, ld, g, partial + (int64_t)a * nblk, nblk,
                              static_cast<const Ctl*>(ctl));
    }
    if (pass1_nv > 0) k_reduce_pass1<<<1, RED_T, 0, st>>>(partial, nblk, pass1_nv, pass1_k, pass1_orth ? 1 : 0, ctl);
}
template void launch_dots<double>(int64_t, int64_t, const double* const*, const double* const*, const int*, int,
                                  double*, int, Ctl*, hipStream_t, int, int, hipEvent_t, hipEvent_t, bool);
template void launch_dots<float>(int64_t, int64_t, const float* const*, const float* const*, const int*, int,
                                 double*, int, Ctl*, hipStream_t, int, int, hipEvent_t, hipEvent_t, bool);

void launch_reduce(const double* partial, int nblk, int ncol, double* dst, Ctl* ctl, int nv, int nw, bool lu_solve,
                   bool check_done, hipStream_t st) {
    k_reduce<<<1, RED_T, 0, st>>>(partial, nblk, ncol, dst, ctl, nv, nw, lu_solve ? 1 : 0, check_done ? 1 : 0);
}


template <typename T>
void launch_update_dots(int64_t npad, const T* V, int64_t ld, int nv, const T* Z, int nz, T* w, const double* coefV,
                        const double* coefZ, double* partial, int nblk, Ctl* ctl, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
    constexpr int CPW = 8;
    const int nw = (nv + CPW - 1) / CPW;   // nv <= 128 -> at most 16 wavefronts
    hipExtLaunchKernelGGL(k_update_dots<T, CPW>, dim3(nblk), dim3(nw * WAVE), 0, st, ev0, ev1, 0, npad, V, ld, nv, Z,
                          nz, w, coefV, coefZ, partial, nblk, static_cast<const Ctl*>(ctl));
    k_reduce<<<1, RED_T, 0, st>>>(partial, nblk, nv, ctl->h2, ctl, 0, 0, 0, 1);
}
template void launch_update_dots<double>(int64_t, const double*, int64_t, int, const double*, int, double*,
                                         const double*, const double*, double*, int, Ctl*, hipStream_t, hipEvent_t,
                                         hipEvent_t);
template void launch_update_dots<float>(int64_t, const float*, int64_t, int, const float*, int, float*,
                                        const double*, const double*, double*, int, Ctl*, hipStream_t, hipEvent_t,
                                        hipEvent_t);

template <typename T>
void launch_update_norm(int64_t npad, const T* V, int64_t ld, int nv, T* w, const double* coef, double* partial,
                        int nblk, Ctl* ctl, hipStream_t st, int givens_j, hipEvent_t ev0, hipEvent_t ev1) {
    hipExtLaunchKernelGGL(k_update_norm<T>, dim3(nblk), dim3(BLOCK), 0, st, ev0, ev1, 0, npad, V, ld, nv, w, coef,
                          partial, nblk, static_cast<const Ctl*>(ctl));
    if (givens_j >= 0) k_givens<<<1, RED_T, 0, st>>>(partial, nblk, givens_j, ctl);
}
template void launch_update_norm<double>(int64_t, const double*, int64_t, int, double*, const double*, double*, int,
                                         Ctl*, hipStream_t, int, hipEvent_t, hipEvent_t);
template void launch_update_norm<float>(int64_t, const float*, int64_t, int, float*, const double*, double*, int,
                                        Ctl*, hipStream_t, int, hipEvent_t, hipEvent_t);

void launch_givens(const double* partial, int nblk, int j, Ctl* ctl, hipStream_t st) {
    k_givens<<<1, RED_T, 0, st>>>(partial, nblk, j, ctl);
}

void launch_cycle_init(Ctl* ctl, int max_steps, double stop_abs, hipStream_t st, bool unit_scale) {
    k_cycle_init<<<1, 1, 0, st>>>(ctl, max_steps, stop_abs, unit_scale ? 1 : 0);
}

template <typename T>
void launch_dots2(int64_t npad, int64_t ld, const T* V, int nq, const T* W, const T* Z, int k, int kz, int zskip,
                  const T* u, const T* z, double* partial, int nblk, Ctl* ctl, hipStream_t st, hipEvent_t ev0,
                  hipEvent_t ev1) {
    const int ncol = nq + k + kz + 1 - zskip;   // swept columns
    // four columns per wavefront up to 64 columns, eight up to 128; at most 16 wavefronts per
    // launch, and u, z are read again by each further launch
    const int cpw = ncol > 64 ? 8 : 4;
    const int nl = (ncol + 16 * cpw - 1) / (16 * cpw);
    const int per = (ncol + nl - 1) / nl;   // columns per launch, balanced
    for (int a = 0; a < ncol; a += per) {
        const int b = (ncol - a) < per ? ncol : a + per;
        const int nw = (b - a + cpw - 1) / cpw;
        const bool first = a == 0, last = b == ncol;
        if (cpw == 8)
            hipExtLaunchKernelGGL(k_dots2<T, 8>, dim3(nblk), dim3(nw * WAVE), 0, st, first ? ev0 : nullptr,
                                  last ? ev1 : nullptr, 0, npad, ld, V, nq, W, Z, k, kz, zskip, u, z, a, b, partial,
                                  nblk, static_cast<const Ctl*>(ctl));
        else
            hipExtLaunchKernelGGL(k_dots2<T, 4>, dim3(nblk), dim3(nw * WAVE), 0, st, first ? ev0 : nullptr,
                                  last ? ev1 : nullptr, 0, npad, ld, V, nq, W, Z, k, kz, zskip, u, z, a, b, partial,
                                  nblk, static_cast<const Ctl*>(ctl));
    }
}
template void launch_dots2<double>(int64_t, int64_t, const double*, int, const double*, const double*, int, int, int,
                                   const double*, const double*, double*, int, Ctl*, hipStream_t, hipEvent_t,
                                   hipEvent_t);
template void launch_dots2<float>(int64_t, int64_t, const float*, int, const float*, const float*, int, int, int,
                                  const float*, const float*, double*, int, Ctl*, hipStream_t, hipEvent_t,
                                  hipEvent_t);

void launch_dcgs2_reduce(double* partial, int nblk, int j, int k, int kz, bool orth, bool has_z, Ctl* ctl,
                         hipStream_t st, const double* zpart, int nblk_z, const double* gz) {
    // the column sums go right after the partials
    const int nent = 2 * (j + k + kz + 1);
    double* dsum = partial + (int64_t)nent * nblk;
    k_colsum<<<(nent + 15) / 16, 1024, 0, st>>>(partial, nblk, nent, dsum, ctl, zpart, nblk_z, j + k, kz, gz);
    k_dcgs2_reduce<<<1, RED_T, 0, st>>>(dsum, j, k, kz, orth ? 1 : 0, has_z ? 1 : 0, ctl);
}

int dcgs2_update_blocks(int64_t npad, int elem_bytes, int max_blocks) {
    const int64_t want = (npad / (32 / elem_bytes) + BLOCK - 1) / BLOCK;   // one 32-byte slice per thread
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, max_blocks));
}

template <typename T>
void launch_dcgs2_update(int64_t npad, T* V, int64_t ld, int j, const T* Z, int k, T* u, const T* z, int nblk,
                         const Ctl* ctl, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, double* zpart) {
    if (zpart && k <= 8)
        hipExtLaunchKernelGGL(k_dcgs2_update_zd<T, 8>, dim3(nblk), dim3(BLOCK), 0, st, ev0, ev1, 0, npad, V, ld, j, Z,
                              k, u, z, nblk, ctl, zpart);
    else if (zpart && k <= DCGS2_ZD_KMAX)
        hipExtLaunchKernelGGL(k_dcgs2_update_zd<T, DCGS2_ZD_KMAX>, dim3(nblk), dim3(BLOCK), 0, st, ev0, ev1, 0, npad,
                              V, ld, j, Z, k, u, z, nblk, ctl, zpart);
    else
        hipExtLaunchKernelGGL(k_dcgs2_update<T>, dim3(nblk), dim3(BLOCK), 0, st, ev0, ev1, 0, npad, V, ld, j, Z, k, u,
                              z, nblk, ctl);
}
template void launch_dcgs2_update<double>(int64_t, double*, int64_t, int, const double*, int, double*,
                                          const double*, int, const Ctl*, hipStream_t, hipEvent_t, hipEvent_t,
                                          double*);
template void launch_dcgs2_update<float>(int64_t, float*, int64_t, int, const float*, int, float*, const float*, int,
                                         const Ctl*, hipStream_t, hipEvent_t, hipEvent_t, double*);

void launch_cycle_solve(Ctl* ctl, hipStream_t st) { k_cycle_solve<<<1, WAVE, 0, st>>>(ctl); }

template <typename T>
void launch_x_update(int64_t n, const T* V, int64_t ld, const double* dinv, double* x, const Ctl* ctl,
                     hipStream_t st) {
    k_x_update<T><<<(unsigned)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(n, V, ld, dinv, x, ctl);
}
template void launch_x_update<double>(int64_t, const double*, int64_t, const double*, double*, const Ctl*,
                                      hipStream_t);
template void launch_x_update<float>(int64_t, const float*, int64_t, const double*, double*, const Ctl*,
                                     hipStream_t);

void launch_correct(int64_t npad, const double* W, const double* Z, int64_t ld, int k, double* x, double* r,
                    const Ctl* ctl, double* partial, int nblk, hipStream_t st) {
    k_correct<<<nblk, BLOCK, 0, st>>>(npad, W, Z, ld, k, x, r, ctl, partial, nblk);
}

void launch_finish_norm(const double* partial, int nblk, Ctl* ctl, int which, hipStream_t st) {
    k_finish_norm<<<1, WAVE, 0, st>>>(partial, nblk, ctl, which);
}

void launch_norm2(int64_t n, const double* v, double* partial, int nblk, hipStream_t st) {
    k_norm2<<<nblk, BLOCK, 0, st>>>(n, v, partial, nblk);
}

void launch_copy_pad(int64_t n, int64_t npad, const double* in, double* out, hipStream_t st) {
    k_copy_pad<<<(unsigned)((npad + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(n, npad, in, out);
}

void launch_extrapolate(int64_t n, int64_t npad, const Extrap& e, double* out, hipStream_t st) {
    k_extrapolate<<<(unsigned)((npad + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(n, npad, e, out);
}

}  // namespace rs
