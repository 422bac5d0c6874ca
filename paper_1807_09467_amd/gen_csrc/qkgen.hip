// qkgen: GPU assembly for the synthetic input generator (workload.py).
//
// Builds A(u_prev) and b(u_prev) of the backward-Euler / Picard Q_p finite-element
// systems on a uniform N x N mesh directly in device memory, so that long
// sequences of large systems can be produced without host round trips.  This
// library belongs to the input generator: it holds finite-element assembly only
// and shares nothing with the solver library.
//
//   qkgen_element_values: element matrices M/dt + eps K + C(u_prev) (one block
//       handles one or more elements; the lagged coefficient u_prev beta is
//       evaluated at the Gauss points once per element in LDS);
//   qkgen_gather: CSR values as a fixed-order sum of element entries (the
//       contribution list is sorted by element index, so the result is
//       deterministic);
//   qkgen_set_value: writes a constant at listed CSR positions (identity rows);
//   qkgen_spmv_scaled: b = s * M u for the stored mass matrix.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int BLK = 256;
constexpr int MAXQ = 32;
constexpr int MAXEPB = 16;

__global__ __launch_bounds__(BLK) void k_elem(int64_t E, int nl, int nq, int epb, const int32_t* __restrict__ en,
                                              const double* __restrict__ u, const double* __restrict__ phi,
                                              const double* __restrict__ wq, const double* __restrict__ Bx,
                                              const double* __restrict__ By, const double* __restrict__ st,
                                              int rotating, double bx0, double by0, const double* __restrict__ qxi,
                                              const double* __restrict__ qeta, int N, double h,
                                              double* __restrict__ ev) {
    __shared__ double axs[MAXEPB][MAXQ];
    __shared__ double ays[MAXEPB][MAXQ];
    const int nl2 = nl * nl;
    for (int t = threadIdx.x; t < epb * nq; t += BLK) {
        const int le = t / nq, q = t % nq;
        const int64_t e = (int64_t)blockIdx.x * epb + le;
        double ax = 0.0, ay = 0.0;
        if (e < E) {
            double uq = 0.0;
            for (int l = 0; l < nl; ++l) uq += u[en[e * nl + l]] * phi[q * nl + l];
            double bx = bx0, by = by0;
            if (rotating) {
                const int64_t ex = e % N, ey = e / N;
                const double x = ((double)ex + qxi[q]) * h;
                const double y = ((double)ey + qeta[q]) * h;
                bx = -2.0 * M_PI * (y - 0.5);
                by = 2.0 * M_PI * (x - 0.5);
            }
            const double s = h * wq[q] * uq;
            ax = s * bx;
            ay = s * by;
        }
        axs[le][q] = ax;
        ays[le][q] = ay;
    }
    __syncthreads();
    const int le = threadIdx.x / nl2, ij = threadIdx.x % nl2;
    const int64_t e = (int64_t)blockIdx.x * epb + le;
    if (le < epb && e < E) {
        double v = 0.0;
        for (int q = 0; q < nq; ++q) v += axs[le][q] * Bx[q * nl2 + ij] + ays[le][q] * By[q * nl2 + ij];
        ev[e * nl2 + ij] = v + st[ij];
    }
}

__global__ __launch_bounds__(BLK) void k_gather(int64_t nnz, const int32_t* __restrict__ cptr,
                                                const int32_t* __restrict__ cidx, const double* __restrict__ ev,
                                                double* __restrict__ vals) {
    const int64_t k = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (k >= nnz) return;
    double s = 0.0;
    for (int32_t t = cptr[k]; t < cptr[k + 1]; ++t) s += ev[cidx[t]];
    vals[k] = s;
}

__global__ __launch_bounds__(BLK) void k_set(int64_t cnt, const int32_t* __restrict__ pos, double value,
                                             double* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i < cnt) vals[pos[i]] = value;
}

__global__ __launch_bounds__(BLK) void k_spmv_scaled(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ mv,
                                                     const double* __restrict__ u, double scale,
                                                     double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += mv[k] * u[ci[k]];
    b[i] = s * scale;
}

inline unsigned grid(int64_t n) { return (unsigned)((n + BLK - 1) / BLK); }

}  // namespace

extern "C" {

// Element matrices of A(u): ev[e * nl^2 + i * nl + j], e < E.  Returns 0, or -1 on bad sizes.
int qkgen_element_values(int64_t E, int32_t nl, int32_t nq, const int32_t* elem_nodes, const double* u,
                         const double* phi, const double* wq, const double* Bx, const double* By,
                         const double* static_e, int32_t rotating, double bx0, double by0, const double* qxi,
                         const double* qeta, int32_t N, double h, double* ev, void* stream) {
    const int nl2 = nl * nl;
    if (E < 1 || nl < 1 || nl2 > BLK || nq < 1 || nq > MAXQ) return -1;
    int epb = BLK / nl2;
    if (epb > MAXEPB) epb = MAXEPB;
    const unsigned g = (unsigned)((E + epb - 1) / epb);
    k_elem<<<g, BLK, 0, (hipStream_t)stream>>>(E, nl, nq, epb, elem_nodes, u, phi, wq, Bx, By, static_e, rotating,
                                               bx0, by0, qxi, qeta, N, h, ev);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// vals[k] = sum_{t in [cptr[k], cptr[k+1])} ev[cidx[t]]
int qkgen_gather(int64_t nnz, const int32_t* cptr, const int32_t* cidx, const double* ev, double* vals,
                 void* stream) {
    if (nnz < 1) return -1;
    k_gather<<<grid(nnz), BLK, 0, (hipStream_t)stream>>>(nnz, cptr, cidx, ev, vals);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int qkgen_set_value(int64_t cnt, const int32_t* pos, double value, double* vals, void* stream) {
    if (cnt < 1) return 0;
    k_set<<<grid(cnt), BLK, 0, (hipStream_t)stream>>>(cnt, pos, value, vals);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int qkgen_spmv_scaled(int64_t n, const int32_t* rp, const int32_t* ci, const double* mv, const double* u,
                      double scale, double* b, void* stream) {
    if (n < 1) return -1;
    k_spmv_scaled<<<grid(n), BLK, 0, (hipStream_t)stream>>>(n, rp, ci, mv, u, scale, b);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
