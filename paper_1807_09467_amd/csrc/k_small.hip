// Persistent one-block path for small systems, batched: block b of a launch runs one whole
// recycled GMRES(m) solve, or one recycle update, of job b.  Every Arnoldi step, reduction,
// Givens rotation, restart decision and the SVD stay on the device, so a solve costs one launch
// instead of several per Arnoldi step, and independent sequences share that launch.
//
// The solve follows the same method and readings as the multi-kernel path: right Jacobi
// (operator P A D^{-1}); oblique projector P = I - A W E^{-1} W^T with E = W^T A W (section 3.2,
// Table 1 rows "augmented oblique" / "deflated oblique"), folded into CGS2 pass 1 as
// h1 = V^T w - F c with F = V^T A W and c = E^{-1} W^T w; projection guess and span(W) correction
// at every cycle end (section 4.2); explicit float64 residual stop ||b - A x|| <= tol ||b||;
// lucky breakdown at h_{j+1,j} <= 1e-14 ||h_j||; W dropped when cond_1(E) > 1e13.
// Everything is float64.
//
// The update follows Algorithm 1 (section 5.2): push the solution into the ring of the s most
// recent ones and, when due, take the SVD of the ring through a Householder QR X = Q R, the
// one-sided Jacobi SVD R = U_R Sigma V^T, and W = Q U_R[:, :k_eff] applied from the stored
// reflectors (orthonormal to working precision), k_eff = min(k, numerical rank).
//
// Job descriptors live in pinned host memory: each block copies its descriptor to LDS at the
// start and writes its results back at the end.
#include <rsolve.h>

#include "kernels.hpp"
#include "svd_dev.hpp"

namespace rs {

namespace {

constexpr int TB = 1024;          // threads per block
constexpr int NWV = TB / WAVE;    // wavefronts per block
constexpr int SM_M = SMALL_MMAX;
constexpr int SM_K = SMALL_KMAX;
constexpr int LDR = SM_M + 1;     // leading dimension of the rotated Hessenberg R
constexpr int LDE = SM_K + 1;     // leading dimension of the LU factors of E
constexpr int LPR_S = 4;          // lanes per row of the sparse products

static_assert(sizeof(SmallJob) % 8 == 0 && sizeof(SmallUpd) % 8 == 0, "descriptors are copied as 8-byte words");
static_assert(SM_M <= WAVE && SM_K <= WAVE, "one lane per row of the small dense solves");

struct SolveLds {
    double R[LDR * SM_M];          // rotated Hessenberg, column-major
    double g[SM_M + 1];
    double cs[SM_M], sn[SM_M];
    double hc[SM_M + 1];           // raw column j of H (h1 + h2)
    double h1[SM_M], h2[SM_M];
    double y[SM_M];
    double cw[SM_K];
    double E[SM_K * LDE];          // LU factors of E = W^T A W, row-major
    double d[SM_K * SM_K];         // dot results of a sweep; columns of E^{-1} while estimating cond_1
    double red[NWV];
    double scal[4];
    int piv[SM_K];
    int flag[4];
};

template <typename T>
__device__ __forceinline__ void copy_words(T* dst, const T* src) {
    constexpr int nw = (int)(sizeof(T) / sizeof(int64_t));
    const int64_t* s = reinterpret_cast<const int64_t*>(src);
    int64_t* d = reinterpret_cast<int64_t*>(dst);
    for (int t = threadIdx.x; t < nw; t += TB) d[t] = s[t];
}

// Block-wide sum; the result is the same in every thread.  Begins with a barrier, so the
// caller may reuse `red` right after.
__device__ __forceinline__ double blk_sum(double v, double* red) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) s += red[q];
    return s;
}

// y = scale * (A x), and vout = scale * x when vout is given (rows < n).  LPR_S lanes per row,
// four consecutive entries per lane per round; the lanes of a row always share the loop trip.
__device__ void blk_spmv(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const double* __restrict__ val, const double* __restrict__ x, double scale,
                         double* __restrict__ y, double* __restrict__ vout) {
    const int sub = threadIdx.x % LPR_S;
    for (int64_t row = threadIdx.x / LPR_S; row < n; row += TB / LPR_S) {
        const int a = rp[row], e = rp[row + 1];
        double acc = 0.0;
        for (int k0 = a + 4 * sub; k0 < e; k0 += 4 * LPR_S) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (k0 + t < e) acc += val[k0 + t] * x[ci[k0 + t]];
        }
#pragma unroll
        for (int o = LPR_S / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        if (sub == 0) {
            y[row] = scale * acc;
            if (vout) vout[row] = scale * x[row];
        }
    }
}

// out[c] = a_c . v_c over n rows for c < ncol, one wavefront per column (fixed order), then a
// barrier.
template <typename ColF, typename VecF>
__device__ void blk_dots(int64_t n, int ncol, ColF colp, VecF vecp, double* out) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    for (int c = wv; c < ncol; c += NWV) {
        const double* a = colp(c);
        const double* v = vecp(c);
        double s0 = 0.0, s1 = 0.0;
        int64_t i = lane;
        for (; i + WAVE < n; i += 2 * WAVE) {
            s0 += a[i] * v[i];
            s1 += a[i + WAVE] * v[i + WAVE];
        }
        if (i < n) s0 += a[i] * v[i];
        const double s = wave_sum(s0 + s1);
        if (lane == 0) out[c] = s;
    }
    __syncthreads();
}

// x = E^{-1} b with the LU factors in L (wavefront 0 only, lane = row).
__device__ void wave_lu_solve(const SolveLds& L, int k, const double* b, double* x) {
    const int lane = threadIdx.x & (WAVE - 1);
    double v = (lane < k) ? b[L.piv[lane]] : 0.0;
    for (int j = 0; j < k; ++j) {
        const double yj = __shfl(v, j, WAVE);
        if (lane > j && lane < k) v -= L.E[lane * LDE + j] * yj;
    }
    for (int j = k - 1; j >= 0; --j) {
        if (lane == j) v = v / L.E[j * LDE + j];
        const double xj = __shfl(v, j, WAVE);
        if (lane < j) v -= L.E[lane * LDE + j] * xj;
    }
    if (lane < k) x[lane] = v;
}

// LU with partial pivoting of E (k x k in L.E) and cond_1(E) into L.scal[3] (infinite on a zero
// or non-finite pivot).  Wavefront 0 only, lane = row.
__device__ void wave_lu_factor(SolveLds& L, int k) {
    const int lane = threadIdx.x & (WAVE - 1);
    double colsum = 0.0;
    if (lane < k)
        for (int i = 0; i < k; ++i) colsum += fabs(L.E[i * LDE + lane]);
    const double norm1 = wave_max(lane < k ? colsum : 0.0);
    if (lane < k) L.piv[lane] = lane;
    bool fail = false;
    for (int j = 0; j < k && !fail; ++j) {
        double v = (lane >= j && lane < k) ? fabs(L.E[lane * LDE + j]) : -1.0;
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
        if (idx != j) {
            for (int c = lane; c < k; c += WAVE) {
                const double t = L.E[j * LDE + c];
                L.E[j * LDE + c] = L.E[idx * LDE + c];
                L.E[idx * LDE + c] = t;
            }
            if (lane == 0) {
                const int t = L.piv[j];
                L.piv[j] = L.piv[idx];
                L.piv[idx] = t;
            }
        }
        __builtin_amdgcn_wave_barrier();
        const double dg = L.E[j * LDE + j];
        if (dg == 0.0 || !isfinite(dg)) {
            fail = true;
        } else if (lane > j && lane < k) {
            const double l = L.E[lane * LDE + j] / dg;
            L.E[lane * LDE + j] = l;
            for (int c = j + 1; c < k; ++c) L.E[lane * LDE + c] -= l * L.E[j * LDE + c];
        }
        __builtin_amdgcn_wave_barrier();
    }
    double cond = INFINITY;
    if (!fail) {
        // column `lane` of E^{-1}: solve L U x = P e_lane, stored in d (row i at d[i * SM_K + lane])
        double* X = L.d;
        if (lane < k) {
            for (int i = 0; i < k; ++i) {
                double s = (L.piv[i] == lane) ? 1.0 : 0.0;
                for (int j = 0; j < i; ++j) s -= L.E[i * LDE + j] * X[j * SM_K + lane];
                X[i * SM_K + lane] = s;
            }
            for (int i = k - 1; i >= 0; --i) {
                double s = X[i * SM_K + lane];
                for (int j = i + 1; j < k; ++j) s -= L.E[i * LDE + j] * X[j * SM_K + lane];
                X[i * SM_K + lane] = s / L.E[i * LDE + i];
            }
        }
        double icol = 0.0;
        if (lane < k)
            for (int i = 0; i < k; ++i) icol += fabs(X[i * SM_K + lane]);
        const double inorm1 = wave_max(lane < k ? icol : 0.0);
        cond = norm1 * inorm1;
        if (!isfinite(cond)) cond = INFINITY;
    }
    if (lane == 0) L.scal[3] = cond;
}

// r = b - A x (unscaled values), then, with k > 0, x += W c and r -= Z c with c = E^{-1} W^T r.
// Returns ||r|| in every thread.
__device__ double blk_residual_correct(const SmallJob& J, SolveLds& L, int k) {
    blk_spmv(J.n, J.rp, J.ci, J.val, J.xw, 1.0, J.w, nullptr);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < J.n; i += TB) J.r[i] = J.b[i] - J.w[i];
    __syncthreads();
    if (k > 0) {
        blk_dots(
            J.n, k, [&](int c) { return J.W + (int64_t)c * J.ld; }, [&](int) { return (const double*)J.r; }, L.d);
        if (threadIdx.x < WAVE) wave_lu_solve(L, k, L.d, L.cw);
        __syncthreads();
        for (int64_t i = threadIdx.x; i < J.n; i += TB) {
            double xi = J.xw[i], ri = J.r[i];
            for (int c = 0; c < k; ++c) {
                xi += J.W[(int64_t)c * J.ld + i] * L.cw[c];
                ri -= J.Z[(int64_t)c * J.ld + i] * L.cw[c];
            }
            J.xw[i] = xi;
            J.r[i] = ri;
        }
        __syncthreads();
    }
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < J.n; i += TB) acc += J.r[i] * J.r[i];
    return sqrt(blk_sum(acc, L.red));
}

__device__ void finish_job(SmallJob* hj, int status, int its, int cycles, int converged, uint32_t flags, int k,
                           double rnorm, double bnorm, double gimp) {
    if (threadIdx.x != 0) return;
    hj->status = status;
    hj->iterations = its;
    hj->cycles = cycles;
    hj->converged = converged;
    hj->flags = flags;
    hj->k_used = k;
    hj->rnorm = rnorm;
    hj->bnorm = bnorm;
    hj->gimp = gimp;
}

__global__ __launch_bounds__(TB) void k_small_solve(SmallBatch batch) {
    __shared__ SolveLds L;
    __shared__ SmallJob J;
    SmallJob* hj = batch.job[blockIdx.x];
    copy_words(&J, hj);
    __syncthreads();
    const int64_t n = J.n, ld = J.ld;
    const int m = J.m;

    // a1: pattern check (row pointers monotone and in range, columns sorted, in range, with a
    // diagonal entry)
    if (J.validate) {
        int bad = 0;
        for (int64_t i = threadIdx.x; i < n; i += TB) {
            const int64_t a = J.rp[i], e = J.rp[i + 1];
            if (a < 0 || e < a || e > J.nnz) {
                bad = 1;
                continue;
            }
            int64_t prev = -1;
            bool diag = false;
            for (int64_t q = a; q < e; ++q) {
                const int64_t c = J.ci[q];
                if (c < 0 || c >= n || c <= prev) bad = 1;
                if (c == i) diag = true;
                prev = c;
            }
            if (!diag) bad = 1;
        }
        if (threadIdx.x == 0 && (J.rp[0] != 0 || J.rp[n] != J.nnz)) bad = 1;
        if (blk_sum(bad ? 1.0 : 0.0, L.red) > 0.0) {
            finish_job(hj, RSOLVE_E_INVALID, 0, 0, 0, 0u, 0, 0.0, 0.0, 0.0);
            return;
        }
    }
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += TB) acc += J.b[i] * J.b[i];
    const double bnorm = sqrt(blk_sum(acc, L.red));
    if (!isfinite(bnorm)) {
        finish_job(hj, RSOLVE_E_NONFINITE, 0, 0, 0, RSOLVE_FLAG_NONFINITE, 0, 0.0, bnorm, 0.0);
        return;
    }
    if (bnorm == 0.0) {
        for (int64_t i = threadIdx.x; i < ld; i += TB) {
            J.xw[i] = 0.0;
            if (i < n) J.x[i] = 0.0;
        }
        finish_job(hj, RSOLVE_OK, 0, 0, 1, 0u, 0, 0.0, 0.0, 0.0);
        return;
    }
    // a1: right Jacobi, values of A D^{-1}
    const double* kval = J.val;
    if (J.jacobi) {
        for (int64_t i = threadIdx.x; i < n; i += TB) {
            const int a = J.rp[i], e = J.rp[i + 1];
            double dg = 0.0;
            for (int q = a; q < e; ++q)
                if (J.ci[q] == i) dg = J.val[q];
            J.dinv[i] = 1.0 / dg;
        }
        __syncthreads();
        for (int64_t q = threadIdx.x; q < J.nnz; q += TB) J.vals[q] = J.val[q] * J.dinv[J.ci[q]];
        kval = J.vals;
        __syncthreads();
    }
    // a2: Z = A W, E = W^T Z and its LU
    int k = J.k;
    uint32_t flags = 0;
    if (k > 0) {
        const int sub = threadIdx.x % LPR_S;
        for (int64_t row = threadIdx.x / LPR_S; row < n; row += TB / LPR_S) {
            const int a = J.rp[row], e = J.rp[row + 1];
            for (int c = 0; c < k; ++c) {
                const double* wc = J.W + (int64_t)c * ld;
                double s = 0.0;
                for (int q = a + sub; q < e; q += LPR_S) s += J.val[q] * wc[J.ci[q]];
#pragma unroll
                for (int o = LPR_S / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
                if (sub == 0) J.Z[(int64_t)c * ld + row] = s;
            }
        }
        __syncthreads();
        blk_dots(
            n, k * k, [&](int p) { return J.W + (int64_t)(p / k) * ld; },
            [&](int p) { return (const double*)(J.Z + (int64_t)(p % k) * ld); }, L.d);
        for (int p = threadIdx.x; p < k * k; p += TB) L.E[(p / k) * LDE + (p % k)] = L.d[p];
        __syncthreads();
        if (threadIdx.x < WAVE) wave_lu_factor(L, k);
        __syncthreads();
        if (!(L.scal[3] <= 1e13)) {
            k = 0;
            flags |= RSOLVE_FLAG_RECYCLE_DROPPED;
        }
    }
    // a3: x0, then the projection guess x0 + W E^{-1} W^T (b - A x0)
    for (int64_t i = threadIdx.x; i < ld; i += TB) J.xw[i] = (J.x0 && i < n) ? J.x0[i] : 0.0;
    __syncthreads();
    double rnorm = blk_residual_correct(J, L, k);
    const double stop_abs = J.tol * bnorm;
    int its = 0, cycles = 0, status = RSOLVE_OK, converged = 0;
    double gimp = rnorm;
    for (;;) {
        if (!isfinite(rnorm)) {
            status = RSOLVE_E_NONFINITE;
            flags |= RSOLVE_FLAG_NONFINITE;
            break;
        }
        if (rnorm <= stop_abs) {
            converged = 1;
            break;
        }
        if (its >= J.max_iters) {
            status = RSOLVE_NOT_CONVERGED;
            break;
        }
        const int max_steps = (m < J.max_iters - its) ? m : J.max_iters - its;
        if (threadIdx.x == 0) L.g[0] = rnorm;
        double scale = 1.0 / rnorm;
        int steps = 0;
        for (int j = 0; j < max_steps; ++j) {
            // the unnormalised vector of step j lives in one work buffer, its product in the other
            const double* vin = (j & 1) ? J.w : J.r;
            double* wv = (j & 1) ? J.r : J.w;
            double* vj = J.V + (int64_t)j * ld;
            // a4: w = A D^{-1} v_j, with v_j = scale * vin stored on the way
            blk_spmv(n, J.rp, J.ci, kval, vin, scale, wv, vj);
            __syncthreads();
            const int nv = j + 1;
            // a5 + a6 pass 1: V^T w, W^T w and v_j^T Z in one sweep
            blk_dots(
                n, nv + 2 * k,
                [&](int c) {
                    return c < nv ? J.V + (int64_t)c * ld
                                  : (c < nv + k ? J.W + (int64_t)(c - nv) * ld : J.Z + (int64_t)(c - nv - k) * ld);
                },
                [&](int c) { return (const double*)(c < nv + k ? wv : vj); }, L.d);
            if (k > 0) {
                if (threadIdx.x < WAVE) wave_lu_solve(L, k, L.d + nv, L.cw);
                for (int c = threadIdx.x; c < k; c += TB) J.F[j * SM_K + c] = L.d[nv + k + c];
                __syncthreads();
            }
            for (int i = threadIdx.x; i < nv; i += TB) {
                double h = L.d[i];
                for (int c = 0; c < k; ++c) h -= J.F[i * SM_K + c] * L.cw[c];
                L.h1[i] = h;
            }
            __syncthreads();
            for (int64_t i = threadIdx.x; i < n; i += TB) {
                double u = wv[i];
                for (int c = 0; c < nv; ++c) u -= J.V[(int64_t)c * ld + i] * L.h1[c];
                for (int c = 0; c < k; ++c) u -= J.Z[(int64_t)c * ld + i] * L.cw[c];
                wv[i] = u;
            }
            __syncthreads();
            // pass 2
            blk_dots(
                n, nv, [&](int c) { return J.V + (int64_t)c * ld; }, [&](int) { return (const double*)wv; }, L.h2);
            double nacc = 0.0;
            for (int64_t i = threadIdx.x; i < n; i += TB) {
                double u = wv[i];
                for (int c = 0; c < nv; ++c) u -= J.V[(int64_t)c * ld + i] * L.h2[c];
                wv[i] = u;
                nacc += u * u;
            }
            const double hn2 = blk_sum(nacc, L.red);
            // a7: Givens update and stop test (thread 0)
            if (threadIdx.x == 0) {
                const double hn = sqrt(hn2);
                double cn = hn2;
                for (int i = 0; i <= j; ++i) {
                    const double h = L.h1[i] + L.h2[i];
                    L.hc[i] = h;
                    cn += h * h;
                }
                double a = L.hc[0];
                for (int i = 0; i < j; ++i) {
                    const double c = L.cs[i], sn = L.sn[i], b = L.hc[i + 1];
                    L.R[i + LDR * j] = c * a + sn * b;
                    a = -sn * a + c * b;
                }
                const double rho = hypot(a, hn);
                double c = 1.0, sn = 0.0;
                if (rho != 0.0) {
                    c = a / rho;
                    sn = hn / rho;
                }
                L.cs[j] = c;
                L.sn[j] = sn;
                L.R[j + LDR * j] = rho;
                const double gj = L.g[j];
                const double gn = -sn * gj;
                L.g[j + 1] = gn;
                L.g[j] = c * gj;
                const bool lucky = !(hn > 1e-14 * sqrt(cn));
                const bool bad = !isfinite(hn) || !isfinite(gn) || !isfinite(rho);
                L.flag[0] = (bad || lucky || fabs(gn) <= stop_abs || j + 1 >= max_steps) ? 1 : 0;
                L.flag[1] = lucky ? 1 : 0;
                L.flag[2] = bad ? 1 : 0;
                L.scal[0] = (hn > 0.0) ? 1.0 / hn : 0.0;
                L.scal[1] = fabs(gn);
            }
            __syncthreads();
            steps = j + 1;
            if (L.flag[1]) flags |= RSOLVE_FLAG_BREAKDOWN_LUCKY;
            if (L.flag[2]) flags |= RSOLVE_FLAG_NONFINITE;
            gimp = L.scal[1];
            scale = L.scal[0];
            if (L.flag[0]) break;
        }
        its += steps;
        cycles += 1;
        // a8: y = R^{-1} g (wavefront 0, lane = row), x += D^{-1} V y
        if (threadIdx.x < WAVE) {
            const int lane = threadIdx.x;
            double t = (lane < steps) ? L.g[lane] : 0.0;
            for (int jj = steps - 1; jj >= 0; --jj) {
                double yj = (lane == jj) ? t / L.R[jj + LDR * jj] : 0.0;
                yj = __shfl(yj, jj, WAVE);
                if (lane < jj) t -= L.R[lane + LDR * jj] * yj;
                if (lane == jj) L.y[jj] = yj;
            }
        }
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += TB) {
            double s = 0.0;
            for (int c = 0; c < steps; ++c) s += J.V[(int64_t)c * ld + i] * L.y[c];
            J.xw[i] += J.jacobi ? s * J.dinv[i] : s;
        }
        __syncthreads();
        // explicit residual and span(W) correction
        rnorm = blk_residual_correct(J, L, k);
        if (flags & RSOLVE_FLAG_NONFINITE) {
            status = RSOLVE_E_NONFINITE;
            break;
        }
    }
    for (int64_t i = threadIdx.x; i < n; i += TB) J.x[i] = J.xw[i];
    finish_job(hj, status, its, cycles, converged, flags, k, rnorm, bnorm, gimp);
}

// ---------------------------------------------------------------------------
// Recycle update (Algorithm 1) for one sequence per block.
// ---------------------------------------------------------------------------
constexpr int LDC = SMALL_SMAX + 1;

struct UpdLds {
    double Ac[LDC * LDC];   // R, then R V = U_R Sigma (column j at Ac[j * LDC + i])
    double Vc[LDC * LDC];
    double sig[LDC];
    double tau[SMALL_SMAX];
    double dq[SMALL_SMAX];  // tau times the dots of a reflector
    double red[NWV];
    int order[LDC];
    int rotated;
};

__global__ __launch_bounds__(TB) void k_small_update(SmallUpdBatch batch) {
    __shared__ UpdLds L;
    __shared__ SmallUpd J;
    SmallUpd* hj = batch.job[blockIdx.x];
    copy_words(&J, hj);
    __syncthreads();
    const int64_t n = J.n, ld = J.ld;
    const int c = J.c;
    // push into the ring
    for (int64_t i = threadIdx.x; i < n; i += TB) J.X[(int64_t)J.slot * ld + i] = J.src[i];
    if (!J.svd) {
        if (threadIdx.x == 0) {
            hj->status = RSOLVE_OK;
            hj->rank = -1;
            hj->k_eff = -1;
        }
        return;
    }
    __syncthreads();
    double* Q = J.Q;
    for (int q = 0; q < c; ++q)
        for (int64_t i = threadIdx.x; i < n; i += TB) Q[(int64_t)q * ld + i] = J.X[(int64_t)q * ld + i];
    __syncthreads();
    // Householder QR: column j keeps R[0..j][j] on and above the diagonal and the reflector v_j
    // below it (v_j[j] = 1 implicit); tau[j] = 0 marks an identity reflector.
    for (int j = 0; j < c; ++j) {
        double* qj = Q + (int64_t)j * ld;
        // a0 is read before the barriers of blk_sum: thread 0 overwrites it with beta below
        const double a0 = (j < n) ? qj[j] : 0.0;
        double acc = 0.0;
        for (int64_t i = j + 1 + threadIdx.x; i < n; i += TB) acc += qj[i] * qj[i];
        const double ss = blk_sum(acc, L.red);
        const double alpha = sqrt(a0 * a0 + ss);
        double tau = 0.0;
        if (alpha > 0.0) {
            const double beta = -copysign(alpha, a0);
            const double v0 = a0 - beta;
            tau = (beta - a0) / beta;
            const double inv = 1.0 / v0;
            for (int64_t i = j + 1 + threadIdx.x; i < n; i += TB) qj[i] *= inv;
            if (threadIdx.x == 0 && j < n) qj[j] = beta;
        }
        if (threadIdx.x == 0) L.tau[j] = tau;
        __syncthreads();
        if (tau == 0.0 || j + 1 >= c) continue;
        // d_q = tau (v_j . Q[:, q]) for the trailing columns, then Q[:, q] -= d_q v_j
        const int nt = c - j - 1;
        {
            const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
            for (int t = wv; t < nt; t += NWV) {
                const double* qq = Q + (int64_t)(j + 1 + t) * ld;
                double s = (lane == 0 && j < n) ? qq[j] : 0.0;
                for (int64_t i = j + 1 + lane; i < n; i += WAVE) s += qj[i] * qq[i];
                s = wave_sum(s);
                if (lane == 0) L.dq[t] = tau * s;
            }
        }
        __syncthreads();
        for (int64_t i = j + threadIdx.x; i < n; i += TB) {
            const double vi = (i == j) ? 1.0 : qj[i];
            for (int t = 0; t < nt; ++t) Q[(int64_t)(j + 1 + t) * ld + i] -= L.dq[t] * vi;
        }
        __syncthreads();
    }
    // SVD of R (c x c, padded to an even size with a zero column)
    const int cp = (c + 1) & ~1;
    for (int t = threadIdx.x; t < cp * cp; t += TB) {
        const int i = t % cp, j = t / cp;
        L.Ac[j * LDC + i] = (i < c && j < c && i <= j && i < n) ? Q[(int64_t)j * ld + i] : 0.0;
        L.Vc[j * LDC + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_svd_sweeps(L.Ac, L.Vc, cp, LDC, c, &L.rotated);
    const int rank = svd_order_rank(L.Ac, LDC, c, n, L.sig, L.order);
    const double s1 = (c > 0) ? L.sig[L.order[0]] : 0.0;
    const int keff = isfinite(s1) ? (rank < J.k ? rank : J.k) : 0;
    // W = Q [U_R[:, :keff]; 0]: U_R in the top c rows, then the reflectors in reverse order
    double* W = J.W;
    const int first = J.smallest ? rank - keff : 0;   // the modes kept: order[first .. first + keff)
    for (int q = 0; q < keff; ++q) {
        const int col = L.order[first + q];
        const double inv = 1.0 / L.sig[col];
        for (int64_t i = threadIdx.x; i < ld; i += TB)
            W[(int64_t)q * ld + i] = (i < c && i < n) ? L.Ac[col * LDC + i] * inv : 0.0;
    }
    __syncthreads();
    for (int j = c - 1; j >= 0 && keff > 0; --j) {
        const double tau = L.tau[j];
        if (tau == 0.0) continue;
        const double* qj = Q + (int64_t)j * ld;
        {
            const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
            for (int q = wv; q < keff; q += NWV) {
                const double* wq = W + (int64_t)q * ld;
                double s = (lane == 0 && j < n) ? wq[j] : 0.0;
                for (int64_t i = j + 1 + lane; i < n; i += WAVE) s += qj[i] * wq[i];
                s = wave_sum(s);
                if (lane == 0) L.dq[q] = tau * s;
            }
        }
        __syncthreads();
        for (int64_t i = j + threadIdx.x; i < n; i += TB) {
            const double vi = (i == j) ? 1.0 : qj[i];
            for (int q = 0; q < keff; ++q) W[(int64_t)q * ld + i] -= L.dq[q] * vi;
        }
        __syncthreads();
    }
    if (threadIdx.x < c) hj->sigma[threadIdx.x] = L.sig[L.order[threadIdx.x]];
    if (threadIdx.x == 0) {
        hj->status = isfinite(s1) ? RSOLVE_OK : RSOLVE_E_NONFINITE;
        hj->rank = rank;
        hj->k_eff = keff;
    }
}

}  // namespace

void launch_small_solve(const SmallBatch& batch, int count, hipStream_t st) {
    if (count > 0) k_small_solve<<<count, TB, 0, st>>>(batch);
}

void launch_small_update(const SmallUpdBatch& batch, int count, hipStream_t st) {
    if (count > 0) k_small_update<<<count, TB, 0, st>>>(batch);
}

}  // namespace rs
