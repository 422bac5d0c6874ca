// Krylov-cycle kernels: fused multi-vector dot / update sweeps of classical
// Gram-Schmidt with reorthogonalisation (CGS2) and the oblique projector, the
// fixed-order reductions, the Givens update of the Hessenberg least-squares
// problem, and the end-of-cycle update.
//
// Streaming sweeps use one row per thread and a grid-stride loop over `nblk`
// blocks; every column of the tall operands is read with fully coalesced
// wavefront loads.  Per-block partial sums go to partial[c * nblk + block] and are
// summed in a fixed order by a separate kernel, so results are bitwise
// reproducible for a given launch shape.
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

template <typename T, int NT>
__global__ __launch_bounds__(BLOCK) void k_dots(int64_t npad, int64_t ld, DotGroups<T> g,
                                                double* __restrict__ partial, int nblk, const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    __shared__ double red[BLOCK / WAVE][NT];
    double acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = 0.0;
    const int n0 = g.n0, n1 = g.n1, ntot = n0 + n1 + g.n2;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        const double x0 = n0 ? to_d(g.v0[i]) : 0.0;
        const double x1 = n1 ? to_d(g.v1[i]) : 0.0;
        const double x2 = g.n2 ? to_d(g.v2[i]) : 0.0;
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            if (c < ntot) {
                const bool in0 = c < n0, in1 = c < n0 + n1;
                const T* col = in0 ? (g.b0 + (int64_t)c * ld)
                                   : (in1 ? (g.b1 + (int64_t)(c - n0) * ld) : (g.b2 + (int64_t)(c - n0 - n1) * ld));
                const double xv = in0 ? x0 : (in1 ? x1 : x2);
                acc[c] += to_d(col[i]) * xv;
            }
        }
    }
    wave_tr_reduce<NT>(acc);
    const int wv = threadIdx.x / WAVE;
    if (wave_tr_owner<NT>()) {
#pragma unroll
        for (int i = 0; i < wave_tr_left<NT>(); ++i) red[wv][wave_tr_col<NT>(i)] = acc[i];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ntot; c += BLOCK)
        partial[(int64_t)c * nblk + blockIdx.x] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
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

__global__ __launch_bounds__(BLOCK) void k_reduce(const double* __restrict__ partial, int nblk, int ncol,
                                                  double* __restrict__ dst, Ctl* __restrict__ ctl, int nv, int nw,
                                                  int lu_solve, int check_done) {
    if (check_done && ctl->done) return;
    __shared__ double sums[MMAX + KMAX];
    __shared__ double Es[KMAX * KMAX];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    for (int c = wv; c < ncol; c += BLOCK / WAVE) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += WAVE) s += partial[(int64_t)c * nblk + b];
        s = wave_sum(s);
        if (lane == 0) sums[c] = s;
    }
    if (lu_solve) {
        for (int t = threadIdx.x; t < nw * nw; t += BLOCK) Es[t] = ctl->E[t];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += BLOCK) dst[c] = sums[c];
    if (lu_solve && wv == 0) wave_lu_solve(ctl, nw, sums + nv, ctl->cw, Es);
}

// Pass-1 coefficients of step j (nv = j + 1 basis vectors) with the oblique projector folded in:
// sums = [V^T w0 | W^T w0 | Z^T v_j]; F[j, :] = v_j^T Z; cw = E^{-1} W^T w0;
// h1 = V^T (w0 - Z cw) = V^T w0 - F cw.
__global__ __launch_bounds__(BLOCK) void k_reduce_pass1(const double* __restrict__ partial, int nblk, int nv, int k,
                                                        Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double sums[MMAX + 2 * KMAX];
    __shared__ double Es[KMAX * KMAX];
    __shared__ double cws[KMAX];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int ncol = nv + 2 * k;
    for (int c = wv; c < ncol; c += BLOCK / WAVE) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += WAVE) s += partial[(int64_t)c * nblk + b];
        s = wave_sum(s);
        if (lane == 0) sums[c] = s;
    }
    for (int t = threadIdx.x; t < k * k; t += BLOCK) Es[t] = ctl->E[t];
    __syncthreads();
    if (k == 0) {
        for (int i = threadIdx.x; i < nv; i += BLOCK) ctl->h1[i] = sums[i];
        return;
    }
    if (wv == 0) wave_lu_solve(ctl, k, sums + nv, cws, Es);
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += BLOCK) {
        ctl->F[(nv - 1) * KMAX + c] = sums[nv + k + c];
        ctl->cw[c] = cws[c];
    }
    for (int i = threadIdx.x; i < nv; i += BLOCK) {
        double h = sums[i];
        for (int c = 0; c < k; ++c) {
            const double f = (i == nv - 1) ? sums[nv + k + c] : ctl->F[i * KMAX + c];
            h -= f * cws[c];
        }
        ctl->h1[i] = h;
    }
}

// w -= V coefV + Z coefZ, then partial dots V^T w with the updated w (nv <= NC <= 64).
template <typename T, int NC>
__global__ __launch_bounds__(BLOCK) void k_update_dots(int64_t npad, const T* __restrict__ V, int64_t ld, int nv,
                                                       const T* __restrict__ Z, int nz, T* __restrict__ w,
                                                       const double* __restrict__ coefV,
                                                       const double* __restrict__ coefZ,
                                                       double* __restrict__ partial, int nblk,
                                                       const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double red[BLOCK / WAVE][NC];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        double vv[NC];
        double u = to_d(w[i]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            vv[c] = 0.0;
            if (c < nv) {
                vv[c] = to_d(V[(int64_t)c * ld + i]);
                u -= vv[c] * coefV[c];
            }
        }
        for (int c = 0; c < nz; ++c) u -= to_d(Z[(int64_t)c * ld + i]) * coefZ[c];
        const T us = (T)u;
        w[i] = us;
        const double ud = to_d(us);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += vv[c] * ud;
    }
    wave_tr_reduce<NC>(acc);
    const int wv = threadIdx.x / WAVE;
    if (wave_tr_owner<NC>()) {
#pragma unroll
        for (int i = 0; i < wave_tr_left<NC>(); ++i) red[wv][wave_tr_col<NC>(i)] = acc[i];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nv; c += BLOCK)
        partial[(int64_t)c * nblk + blockIdx.x] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_update(int64_t npad, const T* __restrict__ V, int64_t ld, int nv,
                                                  const T* __restrict__ Z, int nz, T* __restrict__ w,
                                                  const double* __restrict__ coefV, const double* __restrict__ coefZ,
                                                  int nblk, const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        double u = to_d(w[i]);
        for (int c = 0; c < nv; ++c) u -= to_d(V[(int64_t)c * ld + i]) * coefV[c];
        for (int c = 0; c < nz; ++c) u -= to_d(Z[(int64_t)c * ld + i]) * coefZ[c];
        w[i] = (T)u;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_update_norm(int64_t npad, const T* __restrict__ V, int64_t ld, int nv,
                                                       T* __restrict__ w, const double* __restrict__ coef,
                                                       double* __restrict__ partial, int nblk,
                                                       const Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double lds4[BLOCK / WAVE];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < npad; i += (int64_t)nblk * BLOCK) {
        double u = to_d(w[i]);
        for (int c = 0; c < nv; ++c) u -= to_d(V[(int64_t)c * ld + i]) * coef[c];
        const T us = (T)u;
        w[i] = us;
        const double ud = to_d(us);
        acc += ud * ud;
    }
    acc = block_sum(acc, lds4);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Column j of the Hessenberg matrix, Givens rotations, residual estimate, stop test.
__global__ __launch_bounds__(WAVE) void k_givens(const double* __restrict__ partial, int nblk, int j,
                                                 Ctl* __restrict__ ctl) {
    if (ctl->done) return;
    __shared__ double hcol[MMAX + 1];
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += WAVE) s += partial[b];
    s = wave_sum(s);
    const double hn = sqrt(s);
    double cn = 0.0;
    for (int i = lane; i <= j; i += WAVE) {
        const double h = ctl->h1[i] + ctl->h2[i];
        hcol[i] = h;
        cn += h * h;
    }
    cn = wave_sum(cn) + s;
    __syncthreads();
    if (lane != 0) return;
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

__global__ void k_cycle_init(Ctl* ctl, int max_steps, double stop_abs) {
    if (threadIdx.x != 0) return;
    const double beta = ctl->rnorm;
    ctl->beta = beta;
    ctl->g[0] = beta;
    ctl->inv_h = 1.0 / beta;
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
    double acc = 0.0;
    for (int c = 0; c < s; ++c) acc += to_d(V[(int64_t)c * ld + i]) * ctl->y[c];
    if (dinv) acc *= dinv[i];
    x[i] += acc;
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
    double s = 0.0;
    for (int b = lane; b < nblk; b += WAVE) s += partial[b];
    s = wave_sum(s);
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

}  // namespace

template <typename T>
void launch_dots(int64_t npad, int64_t ld, const T* const* bases, const T* const* vecs, const int* counts,
                 int ngroups, double* partial, int nblk, const Ctl* ctl, hipStream_t st) {
    int ntot = 0;
    for (int q = 0; q < ngroups; ++q) ntot += counts[q];
    for (int a = 0; a < ntot; a += 64) {
        const int b = (ntot - a) < 64 ? ntot : a + 64;
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
        double* pp = partial + (int64_t)a * nblk;
        const int cnt = b - a;
        if (cnt <= 8)
            k_dots<T, 8><<<nblk, BLOCK, 0, st>>>(npad, ld, g, pp, nblk, ctl);
        else if (cnt <= 16)
            k_dots<T, 16><<<nblk, BLOCK, 0, st>>>(npad, ld, g, pp, nblk, ctl);
        else if (cnt <= 32)
            k_dots<T, 32><<<nblk, BLOCK, 0, st>>>(npad, ld, g, pp, nblk, ctl);
        else
            k_dots<T, 64><<<nblk, BLOCK, 0, st>>>(npad, ld, g, pp, nblk, ctl);
    }
}
template void launch_dots<double>(int64_t, int64_t, const double* const*, const double* const*, const int*, int,
                                  double*, int, const Ctl*, hipStream_t);
template void launch_dots<float>(int64_t, int64_t, const float* const*, const float* const*, const int*, int,
                                 double*, int, const Ctl*, hipStream_t);

void launch_reduce(const double* partial, int nblk, int ncol, double* dst, Ctl* ctl, int nv, int nw, bool lu_solve,
                   bool check_done, hipStream_t st) {
    k_reduce<<<1, BLOCK, 0, st>>>(partial, nblk, ncol, dst, ctl, nv, nw, lu_solve ? 1 : 0, check_done ? 1 : 0);
}

void launch_reduce_pass1(const double* partial, int nblk, int nv, int k, Ctl* ctl, hipStream_t st) {
    k_reduce_pass1<<<1, BLOCK, 0, st>>>(partial, nblk, nv, k, ctl);
}

template <typename T>
void launch_update_dots(int64_t npad, const T* V, int64_t ld, int nv, const T* Z, int nz, T* w, const double* coefV,
                        const double* coefZ, double* partial, int nblk, const Ctl* ctl, hipStream_t st) {
    if (nv <= 8)
        k_update_dots<T, 8><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, Z, nz, w, coefV, coefZ, partial, nblk, ctl);
    else if (nv <= 16)
        k_update_dots<T, 16><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, Z, nz, w, coefV, coefZ, partial, nblk, ctl);
    else if (nv <= 32)
        k_update_dots<T, 32><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, Z, nz, w, coefV, coefZ, partial, nblk, ctl);
    else
        k_update_dots<T, 64><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, Z, nz, w, coefV, coefZ, partial, nblk, ctl);
}
template void launch_update_dots<double>(int64_t, const double*, int64_t, int, const double*, int, double*,
                                         const double*, const double*, double*, int, const Ctl*, hipStream_t);
template void launch_update_dots<float>(int64_t, const float*, int64_t, int, const float*, int, float*,
                                        const double*, const double*, double*, int, const Ctl*, hipStream_t);

template <typename T>
void launch_update(int64_t npad, const T* V, int64_t ld, int nv, const T* Z, int nz, T* w, const double* coefV,
                   const double* coefZ, int nblk, const Ctl* ctl, hipStream_t st) {
    k_update<T><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, Z, nz, w, coefV, coefZ, nblk, ctl);
}
template void launch_update<double>(int64_t, const double*, int64_t, int, const double*, int, double*,
                                    const double*, const double*, int, const Ctl*, hipStream_t);
template void launch_update<float>(int64_t, const float*, int64_t, int, const float*, int, float*, const double*,
                                   const double*, int, const Ctl*, hipStream_t);

template <typename T>
void launch_update_norm(int64_t npad, const T* V, int64_t ld, int nv, T* w, const double* coef, double* partial,
                        int nblk, const Ctl* ctl, hipStream_t st) {
    k_update_norm<T><<<nblk, BLOCK, 0, st>>>(npad, V, ld, nv, w, coef, partial, nblk, ctl);
}
template void launch_update_norm<double>(int64_t, const double*, int64_t, int, double*, const double*, double*, int,
                                         const Ctl*, hipStream_t);
template void launch_update_norm<float>(int64_t, const float*, int64_t, int, float*, const double*, double*, int,
                                        const Ctl*, hipStream_t);

void launch_givens(const double* partial, int nblk, int j, Ctl* ctl, hipStream_t st) {
    k_givens<<<1, WAVE, 0, st>>>(partial, nblk, j, ctl);
}

void launch_cycle_init(Ctl* ctl, int max_steps, double stop_abs, hipStream_t st) {
    k_cycle_init<<<1, 1, 0, st>>>(ctl, max_steps, stop_abs);
}

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

}  // namespace rs
