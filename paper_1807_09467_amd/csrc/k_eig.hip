// Ritz and harmonic Ritz pairs of a small projected problem (section 5.1, eqs.
// (eigenvalues_hessenberg) and (eigenvalues_harmonic)), one wavefront on the device.
//
// Input: Ga = Q^T A Q (Ritz) or Ga = (A Q)^T (A Q) and Gb = (A Q)^T Q (harmonic), r x r column-major,
// Q with orthonormal columns.  The harmonic problem Ga z = theta Gb z becomes Gb^{-1} Ga z = theta z
// (LU with partial pivoting).  The real r x r matrix is reduced to Hessenberg form by Householder
// reflections, then to complex Schur form T = Z^H M Z by single-shift QR steps (Wilkinson shift,
// Givens rotations, deflation from the bottom); the eigenvectors of T come from back substitution
// and are mapped back with Z.  The k eigenvalues of smallest modulus are kept (a complex
// conjugate pair only whole, as the real and imaginary parts of its vector) and the kept vectors
// are written as the r x kk coefficient matrix ctl->T (row-major, ld KMAX) of W = Q T, with
// kk in ctl->k_eff and the kept moduli |theta| in ctl->sigma.  ctl->lu_fail = 1 when Gb is
// singular or the QR steps do not converge (then kk = 0).
//
// Lane l owns row or column l of every r-vector operation; the matrices live in a scratch buffer
// (L2-resident at r <= 64), and the block is one wavefront, so __syncthreads orders the phases.
#include "kernels.hpp"

namespace rs {

namespace {

struct cplx {
    double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    // Smith's division
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    const double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ cplx csqrt_(cplx a) {
    const double m = cabs(a);
    if (m == 0.0) return {0.0, 0.0};
    double re = sqrt(0.5 * (m + fabs(a.re)));
    double im = 0.5 * a.im / re;
    if (a.re < 0.0) {
        const double t = re;
        re = fabs(im);
        im = (a.im >= 0.0) ? t : -t;
    }
    return {re, im};
}

constexpr int LD = SMAX;   // leading dimension of the r x r scratch matrices (r <= SMAX = WAVE)

}  // namespace

// scratch: 9 SMAX^2 doubles (M, then H and Z as complex, eigenvectors X and V as complex)
__global__ __launch_bounds__(WAVE) void k_small_eig(const double* __restrict__ Ga, const double* __restrict__ Gb,
                                                    int r, int k, int harmonic, double* __restrict__ scratch,
                                                    Ctl* __restrict__ ctl) {
    const int l = threadIdx.x;
    double* M = scratch;                                          // r x r real, column-major
    cplx* H = reinterpret_cast<cplx*>(scratch + SMAX * SMAX);     // complex Schur form
    cplx* Z = H + SMAX * SMAX;                                    // Schur vectors
    cplx* X = Z + SMAX * SMAX;                                    // eigenvectors of T
    cplx* V = X + SMAX * SMAX;                                    // eigenvectors of M
    __shared__ int fail;
    __shared__ double lam_abs[SMAX];
    if (l == 0) fail = 0;
    // ---- M = Ga, or the solution of Gb M = Ga (LU with partial pivoting of Gb in place) ----
    if (l < r)
        for (int j = 0; j < r; ++j) M[j * LD + l] = Ga[j * r + l];
    if (harmonic) {
        double* B = reinterpret_cast<double*>(X);   // r x r working copy of Gb
        if (l < r)
            for (int j = 0; j < r; ++j) B[j * LD + l] = Gb[j * r + l];
        __syncthreads();
        double bmax = 0.0;
        for (int t = l; t < r * r; t += WAVE) bmax = fmax(bmax, fabs(B[(t / r) * LD + t % r]));
        bmax = wave_max(bmax);
        for (int c = 0; c < r; ++c) {
            // pivot: the largest |B[i][c]|, i >= c (ties to the smaller row)
            const double v = (l >= c && l < r) ? fabs(B[c * LD + l]) : -1.0;
            double best = v;
            int bi = l;
            for (int o = WAVE / 2; o > 0; o >>= 1) {
                const double ov = __shfl_xor(best, o, WAVE);
                const int oi = __shfl_xor(bi, o, WAVE);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            if (!(best > 1e-14 * bmax)) {
                if (l == 0) fail = 1;
                break;
            }
            // swap rows c and bi of B and M (lanes over the columns)
            if (bi != c && l < r) {
                double t = B[l * LD + c];
                B[l * LD + c] = B[l * LD + bi];
                B[l * LD + bi] = t;
                t = M[l * LD + c];
                M[l * LD + c] = M[l * LD + bi];
                M[l * LD + bi] = t;
            }
            __syncthreads();
            // eliminate below the pivot (lanes over the rows)
            if (l > c && l < r) {
                const double f = B[c * LD + l] / B[c * LD + c];
                for (int j = c + 1; j < r; ++j) B[j * LD + l] -= f * B[j * LD + c];
                for (int j = 0; j < r; ++j) M[j * LD + l] -= f * M[j * LD + c];
                B[c * LD + l] = 0.0;
            }
            __syncthreads();
        }
        __syncthreads();
        if (!fail && l < r) {
            // back substitution, lane l for column l of M
            for (int i = r - 1; i >= 0; --i) {
                double sacc = M[l * LD + i];
                for (int j = i + 1; j < r; ++j) sacc -= B[j * LD + i] * M[l * LD + j];
                M[l * LD + i] = sacc / B[i * LD + i];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (fail) {
        if (l == 0) {
            ctl->lu_fail = 1;
            ctl->k_eff = 0;
            ctl->rank = 0;
        }
        return;
    }
    // ---- Hessenberg reduction of M (real Householder), Z accumulates the reflections ----
    double* Zr = reinterpret_cast<double*>(V);   // real Z during the reduction
    if (l < r)
        for (int j = 0; j < r; ++j) Zr[j * LD + l] = (j == l) ? 1.0 : 0.0;
    __syncthreads();
    double* vh = reinterpret_cast<double*>(X);   // Householder vector
    for (int c = 0; c + 2 < r; ++c) {
        const double xi = (l > c && l < r) ? M[c * LD + l] : 0.0;
        const double nrm2 = wave_sum(xi * xi);
        const double alpha = M[c * LD + c + 1];
        const double tail = nrm2 - alpha * alpha;
        if (tail <= 0.0) continue;   // already zero below the subdiagonal
        const double nrm = sqrt(nrm2);
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        // v = x - beta e_{c+1}, tau = 2 / v^T v
        const double v = (l == c + 1) ? alpha - beta : xi;
        const double vtv = wave_sum((l > c && l < r) ? v * v : 0.0);
        const double tau = 2.0 / vtv;
        vh[l] = (l > c && l < r) ? v : 0.0;
        __syncthreads();
        // M <- (I - tau v v^T) M: lanes over the columns
        if (l < r) {
            double w = 0.0;
            for (int i = c + 1; i < r; ++i) w += vh[i] * M[l * LD + i];
            for (int i = c + 1; i < r; ++i) M[l * LD + i] -= tau * vh[i] * w;
        }
        __syncthreads();
        // M <- M (I - tau v v^T) and Z <- Z (I - tau v v^T): lanes over the rows
        if (l < r) {
            double w = 0.0, wz = 0.0;
            for (int j = c + 1; j < r; ++j) {
                w += M[j * LD + l] * vh[j];
                wz += Zr[j * LD + l] * vh[j];
            }
            for (int j = c + 1; j < r; ++j) {
                M[j * LD + l] -= tau * w * vh[j];
                Zr[j * LD + l] -= tau * wz * vh[j];
            }
        }
        __syncthreads();
        if (l > c + 1 && l < r) M[c * LD + l] = 0.0;
        __syncthreads();
    }
    // complex copies
    double hnorm = 0.0;
    if (l < r)
        for (int j = 0; j < r; ++j) {
            H[j * LD + l] = {M[j * LD + l], 0.0};
            hnorm = fmax(hnorm, fabs(M[j * LD + l]));
        }
    hnorm = wave_max(hnorm);
    __syncthreads();
    if (l < r)
        for (int j = 0; j < r; ++j) Z[j * LD + l] = {Zr[j * LD + l], 0.0};
    __syncthreads();
    // ---- complex Schur form by single-shift QR steps ----
    const double eps = 2.220446049250313e-16;
    int hi = r - 1, iter = 0;
    const int max_iter = 30 * (r + 1);
    int total = 0;
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double sub = cabs(H[(lo - 1) * LD + lo]);
            const double dia = cabs(H[lo * LD + lo]) + cabs(H[(lo - 1) * LD + lo - 1]);
            if (sub <= eps * (dia > 0.0 ? dia : hnorm)) break;
            --lo;
        }
        if (lo > 0) {
            if (l == 0) H[(lo - 1) * LD + lo] = {0.0, 0.0};
            __syncthreads();
        }
        if (lo == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > max_iter) {
            if (l == 0) fail = 1;
            break;
        }
        ++iter;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer its last entry
        cplx mu;
        {
            const cplx a = H[(hi - 1) * LD + hi - 1], b = H[hi * LD + hi - 1], c = H[(hi - 1) * LD + hi],
                       d = H[hi * LD + hi];
            if (iter % 11 == 10) {
                // exceptional shift
                mu = cadd(d, {cabs(H[(hi - 1) * LD + hi]) + (hi >= 2 ? cabs(H[(hi - 2) * LD + hi - 1]) : 0.0), 0.0});
            } else {
                const cplx tr2 = {0.5 * (a.re - d.re), 0.5 * (a.im - d.im)};
                const cplx disc = csqrt_(cadd(cmul(tr2, tr2), cmul(b, c)));
                const cplx m1 = cadd(d, csub(tr2, disc)), m2 = cadd(d, cadd(tr2, disc));
                // eigenvalues d + tr2 -+ disc... take the one closer to d
                mu = (cabs2(csub(m1, d)) <= cabs2(csub(m2, d))) ? m1 : m2;
            }
        }
        // implicit single-shift QR sweep over rows lo..hi
        cplx x = csub(H[lo * LD + lo], mu), y = H[lo * LD + lo + 1];
        for (int i = lo; i < hi; ++i) {
            if (i > lo) {
                x = H[(i - 1) * LD + i];
                y = H[(i - 1) * LD + i + 1];
            }
            // G = [c s; -conj(s) c] with c real: G [x; y] = [rho; 0]
            const double nx = cabs(x), ny = cabs(y);
            double cs = 1.0;
            cplx sn = {0.0, 0.0};
            if (ny != 0.0) {
                const double rho = hypot(nx, ny);
                if (nx == 0.0) {
                    cs = 0.0;
                    sn = cdiv(cconj(y), {ny, 0.0});
                } else {
                    cs = nx / rho;
                    const cplx ph = {x.re / nx, x.im / nx};   // x / |x|
                    sn = cmul(ph, {cconj(y).re / rho, cconj(y).im / rho});
                }
            }
            __syncthreads();
            // rows i, i+1 of H, columns (i > lo ? i - 1 : lo) .. r - 1 (lanes over the columns)
            const int c0 = (i > lo) ? i - 1 : lo;
            if (l >= c0 && l < r) {
                const cplx hi0 = H[l * LD + i], hi1 = H[l * LD + i + 1];
                H[l * LD + i] = cadd(cmul({cs, 0.0}, hi0), cmul(sn, hi1));
                H[l * LD + i + 1] = csub(cmul({cs, 0.0}, hi1), cmul(cconj(sn), hi0));
            }
            __syncthreads();
            // columns i, i+1 of H times G^H, rows 0 .. min(i + 2, hi); and of Z, every row
            const int r1 = (i + 2 < hi) ? i + 2 : hi;
            if (l <= r1) {
                const cplx h0 = H[i * LD + l], h1 = H[(i + 1) * LD + l];
                H[i * LD + l] = cadd(cmul({cs, 0.0}, h0), cmul(cconj(sn), h1));
                H[(i + 1) * LD + l] = csub(cmul({cs, 0.0}, h1), cmul(sn, h0));
            }
            if (l < r) {
                const cplx z0 = Z[i * LD + l], z1 = Z[(i + 1) * LD + l];
                Z[i * LD + l] = cadd(cmul({cs, 0.0}, z0), cmul(cconj(sn), z1));
                Z[(i + 1) * LD + l] = csub(cmul({cs, 0.0}, z1), cmul(sn, z0));
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (fail) {
        if (l == 0) {
            ctl->lu_fail = 1;
            ctl->k_eff = 0;
            ctl->rank = 0;
        }
        return;
    }
    // ---- eigenvectors of the upper triangular T (lane l: eigenvalue T_ll), then V = Z X ----
    double tnorm = 0.0;
    if (l < r)
        for (int j = l; j < r; ++j) tnorm = fmax(tnorm, cabs(H[j * LD + l]));
    tnorm = wave_max(tnorm);
    const double small = eps * (tnorm > 0.0 ? tnorm : 1.0);
    {
        const cplx lam = (l < r) ? H[l * LD + l] : cplx{0.0, 0.0};
        for (int i = r - 1; i >= 0; --i) {
            if (l < r) {
                cplx xi = {0.0, 0.0};
                if (i == l) {
                    xi = {1.0, 0.0};
                } else if (i < l) {
                    cplx acc = {0.0, 0.0};
                    for (int j = i + 1; j <= l; ++j) acc = cadd(acc, cmul(H[j * LD + i], X[l * LD + j]));
                    cplx den = csub(H[i * LD + i], lam);
                    if (cabs(den) < small) den = {small, 0.0};
                    xi = cdiv({-acc.re, -acc.im}, den);
                }
                X[l * LD + i] = xi;
            }
        }
    }
    __syncthreads();
    if (l < r) {
        double nrm2 = 0.0;
        int big = 0;
        double bigv = -1.0;
        for (int i = 0; i < r; ++i) {
            cplx acc = {0.0, 0.0};
            for (int j = 0; j <= l; ++j) acc = cadd(acc, cmul(Z[j * LD + i], X[l * LD + j]));
            V[l * LD + i] = acc;
            const double a2 = cabs2(acc);
            nrm2 += a2;
            if (a2 > bigv) {
                bigv = a2;
                big = i;
            }
        }
        // unit norm, largest entry real and positive (a real eigenvalue's vector is then real)
        const cplx ph = V[l * LD + big];
        const double pa = cabs(ph);
        const cplx scale = cdiv({pa / sqrt(nrm2), 0.0}, ph);
        for (int i = 0; i < r; ++i) V[l * LD + i] = cmul(V[l * LD + i], scale);
        lam_abs[l] = cabs(H[l * LD + l]);
    }
    __syncthreads();
    // ---- the k of smallest modulus, a complex pair only whole ----
    if (l == 0) {
        double lmax = 0.0;
        for (int i = 0; i < r; ++i) lmax = fmax(lmax, lam_abs[i]);
        const double imtol = 64.0 * eps * (lmax > 0.0 ? lmax : 1.0);
        unsigned long long used = 0ull;
        int kk = 0;
        for (int step = 0; step < r; ++step) {
            // next unused index of smallest modulus (ties to the smaller index)
            int idx = -1;
            for (int i = 0; i < r; ++i)
                if (!((used >> i) & 1ull) && isfinite(lam_abs[i]) && (idx < 0 || lam_abs[i] < lam_abs[idx])) idx = i;
            if (idx < 0) break;
            const cplx lam = H[idx * LD + idx];
            if (fabs(lam.im) > imtol) {
                if (kk + 2 > k) break;
                int partner = -1;
                double pd = 0.0;
                for (int j = 0; j < r; ++j) {
                    if (j == idx || ((used >> j) & 1ull)) continue;
                    const double d = cabs(csub(H[j * LD + j], cconj(lam)));
                    if (partner < 0 || d < pd) {
                        partner = j;
                        pd = d;
                    }
                }
                for (int i = 0; i < r; ++i) {
                    ctl->T[i * KMAX + kk] = V[idx * LD + i].re;
                    ctl->T[i * KMAX + kk + 1] = V[idx * LD + i].im;
                }
                ctl->sigma[kk] = lam_abs[idx];
                ctl->sigma[kk + 1] = lam_abs[idx];
                kk += 2;
                used |= 1ull << idx;
                if (partner >= 0) used |= 1ull << partner;
            } else {
                if (kk + 1 > k) break;
                for (int i = 0; i < r; ++i) ctl->T[i * KMAX + kk] = V[idx * LD + i].re;
                ctl->sigma[kk] = lam_abs[idx];
                kk += 1;
                used |= 1ull << idx;
            }
        }
        ctl->k_eff = kk;
        ctl->rank = kk;
        ctl->lu_fail = 0;
    }
}

void launch_small_eig(const double* Ga, const double* Gb, int r, int k, int harmonic, double* scratch, Ctl* ctl,
                      hipStream_t st) {
    k_small_eig<<<1, WAVE, 0, st>>>(Ga, Gb, r, k, harmonic, scratch, ctl);
}

}  // namespace rs

namespace rs {

namespace {
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_scale_cols(int64_t n, int64_t ld, const T* __restrict__ V, int cols,
                                                      const double* __restrict__ dinv, double* __restrict__ out,
                                                      int64_t ldo) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const double d = dinv ? dinv[i] : 1.0;
    for (int c = 0; c < cols; ++c) out[(int64_t)c * ldo + i] = d * static_cast<double>(V[(int64_t)c * ld + i]);
}
}  // namespace

template <typename T>
void launch_scale_cols(int64_t n, int64_t ld, const T* V, int cols, const double* dinv, double* out, int64_t ldo,
                       hipStream_t st) {
    if (cols <= 0) return;
    k_scale_cols<T><<<(unsigned)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(n, ld, V, cols, dinv, out, ldo);
}
template void launch_scale_cols<double>(int64_t, int64_t, const double*, int, const double*, double*, int64_t,
                                        hipStream_t);
template void launch_scale_cols<float>(int64_t, int64_t, const float*, int, const double*, double*, int64_t,
                                       hipStream_t);

}  // namespace rs
