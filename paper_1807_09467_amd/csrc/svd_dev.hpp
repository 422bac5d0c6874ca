// One-sided (Hestenes) Jacobi SVD of a small square matrix held in LDS, shared by the
// multi-kernel recycle update and the one-block batched update (section 5.2, Algorithm 1:
// the SVD of the snapshot matrix, taken here of its triangular factor R).
#pragma once

#include "common.hpp"

namespace rs {

// Columns of Ac (cp x cp, cp even, column j at Ac[j * ldc + i]) are rotated in pairs, in
// round-robin order with 8 threads per pair, until every pair is orthogonal to working
// precision (|a_p . a_q| <= cp eps ||a_p|| ||a_q||); the rotations accumulate in Vc, so that
// on return Ac = R Vc = U Sigma.  Every thread of the block must call it; threads beyond
// 4 cp take part only in the barriers.  `rotated` is an LDS flag.
__device__ inline void jacobi_svd_sweeps(double* Ac, double* Vc, int cp, int ldc, int c, int* rotated) {
    const int tid = threadIdx.x;
    const double tol = (double)(c > 1 ? c : 1) * 2.220446049250313e-16;
    const int grp = tid >> 3, sub = tid & 7;
    for (int sweep = 0; sweep < 60 && cp >= 2; ++sweep) {
        if (tid == 0) *rotated = 0;
        __syncthreads();
        for (int rnd = 0; rnd < cp - 1; ++rnd) {
            if (grp < cp / 2) {
                const int ia = grp, ib = cp - 1 - grp;
                const int P = (ia == 0) ? 0 : 1 + ((ia - 1 + rnd) % (cp - 1));
                const int Q = 1 + ((ib - 1 + rnd) % (cp - 1));
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = sub; i < cp; i += 8) {
                    const double x = Ac[P * ldc + i], y = Ac[Q * ldc + i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
#pragma unroll
                for (int o = 4; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, WAVE);
                    be += __shfl_xor(be, o, WAVE);
                    ga += __shfl_xor(ga, o, WAVE);
                }
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tt * tt);
                    const double sn = cs * tt;
                    for (int i = sub; i < cp; i += 8) {
                        const double x = Ac[P * ldc + i], y = Ac[Q * ldc + i];
                        Ac[P * ldc + i] = cs * x - sn * y;
                        Ac[Q * ldc + i] = sn * x + cs * y;
                        const double vx = Vc[P * ldc + i], vy = Vc[Q * ldc + i];
                        Vc[P * ldc + i] = cs * vx - sn * vy;
                        Vc[Q * ldc + i] = sn * vx + cs * vy;
                    }
                    if (sub == 0) *rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!*rotated) break;
        __syncthreads();
    }
}

// Singular values sig[j] = ||Ac[:, j]|| and the descending order (stable on ties) in
// order[0..c).  Returns the numerical rank sigma_i > sigma_1 max(n, c) 2^-52 (0 when sigma_1
// is zero or not finite), the same value in every thread.
__device__ inline int svd_order_rank(const double* Ac, int ldc, int c, int64_t n, double* sig, int* order) {
    const int tid = threadIdx.x;
    if (tid < c) {
        double s = 0.0;
        for (int i = 0; i < c; ++i) s += Ac[tid * ldc + i] * Ac[tid * ldc + i];
        sig[tid] = sqrt(s);
    }
    __syncthreads();
    if (tid < c) {
        int pos = 0;
        for (int i = 0; i < c; ++i)
            if (sig[i] > sig[tid] || (sig[i] == sig[tid] && i < tid)) ++pos;
        order[pos] = tid;
    }
    __syncthreads();
    const double s1 = (c > 0) ? sig[order[0]] : 0.0;
    const double thr = s1 * (double)(n > c ? n : c) * 2.220446049250313e-16;
    int rank = 0;
    for (int i = 0; i < c; ++i)
        if (sig[order[i]] > thr) ++rank;
    if (!(s1 > 0.0) || !isfinite(s1)) rank = 0;
    return rank;
}

}  // namespace rs
