// Banded padded SpMV with shared offset lists.
//
// The rows of a finite-element matrix on a structured mesh fall into a few classes whose column
// offsets col - row are the same (for tensor-product Q_p elements: the position of the node
// inside its element and its distance to the boundary).  The banded copy keeps every row's
// offsets in its own chunks; here each class keeps one copy of them (dict, in the chunk order of
// the banded layout) and each row keeps the 16-bit chunk index where its class's list starts in
// dict, so the product streams the values, the chunk offsets p and two bytes per row instead of
// two bytes per entry.  The values are the banded copy's (same chunks, same padding), so the
// result equals that of k_spmv_bp bit for bit.
//
// Latency: every wavefront makes one pass, so the kernel's time is the number of passes per
// compute unit times the length of one pass's chain of dependent loads.  The row's list start is
// read directly (not through a class table) and together with the row's chunk offsets, so the
// chain is {p, list start} -> {values, offset list} -> x.
#pragma once

#include <cstdint>

#include "spmv_banded.hpp"

namespace rs {

// y = s A win, vout = s win (vout may be null), s = ctl->inv_h; float64 accumulation.  Row r reads
// its offsets from dict + first[r] E, chunk by chunk as k_spmv_bp reads off + p[r] E.
template <typename T, int E, int LPR>
__global__ __launch_bounds__(BLOCK) void k_spmv_bc(int64_t n, const int32_t* __restrict__ p,
                                                   const uint16_t* __restrict__ first,
                                                   const int16_t* __restrict__ dict, const T* __restrict__ val,
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
        int f = first[row];
        // taking the value here keeps its load beside p's instead of under the loop test below
        __asm__ volatile("" : "+v"(f));
        const int16_t* offr = dict + (int64_t)f * E;
        const T* xr = win + row;
        for (int q = a + sub; q < e; q += LPR) {
            int16_t c[E];
            T v[E];
            __builtin_memcpy(c, __builtin_assume_aligned(offr + (int64_t)(q - a) * E, 2 * E), sizeof(c));
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
void launch_spmv_bc(int E, int LPR, int remap, int64_t n, const int32_t* p, const uint16_t* first,
                    const int16_t* dict, const T* val, const T* win, T* vout, T* y,
                    const Ctl* ctl, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const auto grid = [n](int L) { return dim3((unsigned)((n * L + BLOCK - 1) / BLOCK)); };
#define RS_BC(EE, L)                                                                                              \
    hipExtLaunchKernelGGL(k_spmv_bc<T, EE, L>, grid(L), dim3(BLOCK), 0, st, ev0, ev1, 0, n, p, first, dict, val, win, \
                          vout, y, ctl, remap)
    if (E == 8) {
        if (LPR == 2) RS_BC(8, 2);
        else if (LPR == 4) RS_BC(8, 4);
        else RS_BC(8, 8);
    } else {
        if (LPR == 2) RS_BC(4, 2);
        else if (LPR == 4) RS_BC(4, 4);
        else RS_BC(4, 8);
    }
#undef RS_BC
}

}  // namespace rs
