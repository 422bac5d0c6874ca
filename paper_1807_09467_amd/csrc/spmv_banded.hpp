// The Arnoldi product on the banded padded copy of the matrix (device code and its launcher).
// Kept apart from the other sparse kernels: the rocprofv3 counter figures of this product are
// tied to this file's contents.
#pragma once

#include "kernels.hpp"

namespace rs {

// Banded padded CSR.
// Row r owns the chunks [p[r], p[r+1]) of E entries each: its entries, then zeros up to a whole
// chunk.  Columns are kept as 16-bit offsets col - r, so a finite-element row of E entries costs
// E (w + 2) bytes instead of E (w + 4).  The LPR lanes of a row take the chunks p[r] + sub,
// p[r] + sub + LPR, ...; inside each round of LPR chunks the row's entries are dealt round-robin
// over the lanes that hold a chunk of it, so at every step the lanes of a row read neighbouring
// entries and gather neighbouring columns of x.  Padding entries have offset 0 and value 0.

// Position of entry kk (0 <= kk < E LP) of a row whose chunks start at c0 (LP chunks).
__device__ __forceinline__ int64_t bp_pos(int64_t c0, int LP, int kk, int E, int LPR) {
    const int R = E * LPR;
    const int it = kk / R, w = kk - it * R;
    const int g = min(LPR, LP - LPR * it);
    return (c0 + (int64_t)LPR * it + w % g) * E + w / g;
}

template <int LPR>
__device__ __forceinline__ double bp_group_sum(double v) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// y = s A win, vout = s win (vout may be null), s = ctl->inv_h; float64 accumulation.
template <typename T, int E, int LPR>
__global__ __launch_bounds__(BLOCK) void k_spmv_bp(int64_t n, const int32_t* __restrict__ p,
                                                   const int16_t* __restrict__ off, const T* __restrict__ val,
                                                   const T* __restrict__ win, T* __restrict__ vout,
                                                   T* __restrict__ y, const Ctl* __restrict__ ctl, int remap) {
    if (ctl->done) return;
    const double s = ctl->inv_h;
    const unsigned lb = remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int64_t gt = (int64_t)lb * BLOCK + threadIdx.x;
    const int64_t row = gt / LPR;
    const int sub = (int)(gt % LPR);
    double acc = 0.0;
    const bool active = row < n;
    if (active) {
        const int a = p[row], e = p[row + 1];
        const T* xr = win + row;
        for (int q = a + sub; q < e; q += LPR) {
            int16_t c[E];
            T v[E];
            __builtin_memcpy(c, __builtin_assume_aligned(off + (int64_t)q * E, 2 * E), sizeof(c));
            __builtin_memcpy(v, __builtin_assume_aligned(val + (int64_t)q * E, 16), sizeof(v));
            double pr[E];
#pragma unroll
            for (int t = 0; t < E; ++t) pr[t] = to_d(v[t]) * to_d(xr[c[t]]);
#pragma unroll
            for (int t = 0; t < E; ++t) acc += pr[t];
        }
    }
    acc = bp_group_sum<LPR>(acc);
    if (active && sub == 0) {
        y[row] = (T)(s * acc);
        if (vout) vout[row] = (T)(s * to_d(win[row]));
    }
}

template <typename T>
void launch_spmv_bp(int E, int LPR, int remap, int64_t n, const int32_t* p, const int16_t* off, const T* val,
                    const T* win, T* vout, T* y, const Ctl* ctl, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const auto grid = [n](int L) { return dim3((unsigned)((n * L + BLOCK - 1) / BLOCK)); };
#define RS_BP(EE, L)                                                                                          \
    hipExtLaunchKernelGGL(k_spmv_bp<T, EE, L>, grid(L), dim3(BLOCK), 0, st, ev0, ev1, 0, n, p, off, val, win, vout, \
                          y, ctl, remap)
    if (E == 8) {
        if (LPR == 2) RS_BP(8, 2);
        else if (LPR == 4) RS_BP(8, 4);
        else RS_BP(8, 8);
    } else {
        if (LPR == 2) RS_BP(4, 2);
        else if (LPR == 4) RS_BP(4, 4);
        else RS_BP(4, 8);
    }
#undef RS_BP
}

}  // namespace rs
