// Sparse kernels: CSR validation, Jacobi scaling, SpMV variants and the A W product.
//
// CSR SpMV uses LPR consecutive lanes of a 64-wide wavefront per row (LPR = 2..32):
// a Q_p finite-element row holds 9..49 entries stored contiguously, so each lane
// takes 4 consecutive entries per round with 16-byte index / value loads, gathers
// x, and the LPR lanes combine their partial sums with shuffles.  Accumulation is
// float64.
#include <cstdlib>

#include <algorithm>

#include "kernels.hpp"
#include "spmv_banded.hpp"
#include "spmv_classes.hpp"

namespace rs {

namespace {

__global__ __launch_bounds__(BLOCK) void k_validate(int64_t n, int64_t nnz, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, int32_t* __restrict__ diag_pos,
                                                    int32_t* __restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    if (i == 0 && rp[0] != 0) err[0] = 1;
    if (i == n - 1 && (int64_t)rp[n] != nnz) err[0] = 1;
    const int64_t a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || b > nnz) {
        err[0] = 1;
        diag_pos[i] = -1;
        return;
    }
    int32_t d = -1;
    int64_t prev = -1;
    bool bad_col = false, bad_order = false, wide = false;
    for (int64_t k = a; k < b; ++k) {
        const int64_t c = ci[k];
        if (c < 0 || c >= n) bad_col = true;
        if (c <= prev) bad_order = true;
        if (c == i) d = (int32_t)k;
        if (c - i > BP_MAX_OFFSET || i - c > BP_MAX_OFFSET) wide = true;
        prev = c;
    }
    if (bad_col) err[1] = 1;
    if (bad_order) err[2] = 1;
    if (d < 0) err[3] = 1;
    if (wide) err[4] = 1;   // not an error: the banded format cannot hold this pattern
    diag_pos[i] = d;
}

__global__ __launch_bounds__(BLOCK) void k_diag_inv(int64_t n, const int32_t* __restrict__ dp,
                                                    const double* __restrict__ val, double* __restrict__ dinv) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    dinv[i] = 1.0 / val[dp[i]];
}

__global__ __launch_bounds__(BLOCK) void k_scale_values(int64_t nnz, const int32_t* __restrict__ ci,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ dinv, double* __restrict__ o64,
                                                        float* __restrict__ o32) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= nnz) return;
    double v = val[k];
    if (dinv) v *= dinv[ci[k]];
    if (o64) o64[k] = v;
    if (o32) o32[k] = (float)v;
}

// Partial dot product of one CSR row with x over the entries k = a + sub + LPR t: four entries
// per lane per round, indices and values loaded together before the four gathers of x.  Rounds
// past the row end clamp to the row's first entry and contribute zero.
template <typename T, int LPR>
__device__ __forceinline__ double csr_row_part(const int32_t* __restrict__ ci, const T* __restrict__ val,
                                               const T* __restrict__ x, int a, int e, int sub) {
    double acc = 0.0;
    for (int k0 = a + sub; k0 < e; k0 += 4 * LPR) {
        int c[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * LPR;
            const bool ok = k < e;
            const int kk = ok ? k : a;
            c[u] = ci[kk];
            v[u] = ok ? to_d(val[kk]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u] * to_d(x[c[u]]);
    }
    return acc;
}

// Variant with each lane owning E (4 or 8) consecutive entries per round: 16-byte index and value
// loads (rows start at arbitrary offsets, so the loads are only dword-aligned, which the memory
// system accepts).  The last partial chunk of a row falls back to guarded scalar loads.
template <typename T, int LPR, int E>
__device__ __forceinline__ double csr_row_part_vec(const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                   const T* __restrict__ x, int a, int e, int sub) {
    double acc = 0.0;
    for (int k0 = a + E * sub; k0 < e; k0 += E * LPR) {
        if (k0 + E <= e) {
            int c[E];
            T v[E];
            __builtin_memcpy(c, ci + k0, sizeof(c));
            __builtin_memcpy(v, val + k0, sizeof(v));
            double p[E];
#pragma unroll
            for (int t = 0; t < E; ++t) p[t] = to_d(v[t]) * to_d(x[c[t]]);
#pragma unroll
            for (int t = 0; t < E; ++t) acc += p[t];
        } else {
            for (int k = k0; k < e; ++k) acc += to_d(val[k]) * to_d(x[ci[k]]);
        }
    }
    return acc;
}

template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// y = s * A win ; vout = s * win  (row-wise, s = ctl->inv_h)
template <typename T, int LPR>
__global__ __launch_bounds__(BLOCK) void k_spmv_arnoldi(int64_t n, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                        const T* __restrict__ win, T* __restrict__ vout,
                                                        T* __restrict__ y, const Ctl* __restrict__ ctl, int remap,
                                                        int vec) {
    if (ctl->done) return;
    const double s = ctl->inv_h;
    const unsigned lb = remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int64_t gt = (int64_t)lb * BLOCK + threadIdx.x;
    const int64_t row = gt / LPR;
    const int sub = (int)(gt % LPR);
    double acc = 0.0;
    const bool active = row < n;
    if (active)
        acc = (vec == 8)   ? csr_row_part_vec<T, LPR, 8>(ci, val, win, rp[row], rp[row + 1], sub)
              : (vec == 4) ? csr_row_part_vec<T, LPR, 4>(ci, val, win, rp[row], rp[row + 1], sub)
                           : csr_row_part<T, LPR>(ci, val, win, rp[row], rp[row + 1], sub);
    acc = group_sum<LPR>(acc);
    if (active && sub == 0) {
        y[row] = (T)(s * acc);
        if (vout) vout[row] = (T)(s * to_d(win[row]));
    }
}

// p[i] = sum_{r < i} ceil(len_r / E), i = 0..n, in three launches: tile-local exclusive sums
// and tile totals (tiles of BP_TILE rows, 4 per thread), an exclusive scan of the totals by one
// block, and the tile offsets added back.
constexpr int BP_TILE = 4 * 1024;

// Exclusive scan of v over a 1024-thread block; *total gets the block's sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wtot, int* total) {
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    int inc = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        const int t = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += t;
    }
    if (lane == WAVE - 1) wtot[wv] = inc;
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < 1024 / WAVE; ++w) {
        const int t = wtot[w];
        if (w < wv) before += t;
        all += t;
    }
    __syncthreads();   // wtot may be reused by the caller
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(1024) void k_bp_tiles(int64_t n, const int32_t* __restrict__ rp, int E,
                                                   int32_t* __restrict__ p, int32_t* __restrict__ tsum) {
    __shared__ int wtot[1024 / WAVE];
    const int64_t i0 = (int64_t)blockIdx.x * BP_TILE + 4 * (int64_t)threadIdx.x;
    int c[4], loc = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u;
        c[u] = i < n ? (rp[i + 1] - rp[i] + E - 1) / E : 0;
        loc += c[u];
    }
    int total = 0;
    int ex = block_exclusive_scan(loc, wtot, &total);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (i0 + u < n) p[i0 + u] = ex;
        ex += c[u];
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

// In place: tsum[t] <- sum_{t' < t} tsum[t'] for t < nt, and p[n] = the grand total.
__global__ __launch_bounds__(1024) void k_bp_tile_offsets(int64_t n, int nt, int32_t* __restrict__ tsum,
                                                          int32_t* __restrict__ p) {
    __shared__ int wtot[1024 / WAVE];
    int carry = 0;
    for (int t0 = 0; t0 < nt; t0 += 1024) {
        const int t = t0 + (int)threadIdx.x;
        const int v = t < nt ? tsum[t] : 0;
        int total = 0;
        const int ex = block_exclusive_scan(v, wtot, &total);
        if (t < nt) tsum[t] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) p[n] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_bp_add(int64_t n, const int32_t* __restrict__ tsum, int32_t* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] += tsum[i / BP_TILE];
}

// Offsets of every entry and zero values at the padding (once per pattern): 8 lanes per row.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_bp_pack(int64_t n, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, const int32_t* __restrict__ p,
                                                   int E, int LPR, int16_t* __restrict__ off, T* __restrict__ val) {
    const int64_t gt = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t i = gt / 8;
    const int sub = (int)(gt % 8);
    if (i >= n) return;
    const int a = rp[i], L = rp[i + 1] - a;
    const int c0 = p[i], LP = p[i + 1] - c0;
    for (int kk = sub; kk < LP * E; kk += 8) {
        const int64_t q = bp_pos(c0, LP, kk, E, LPR);
        if (kk < L) {
            off[q] = (int16_t)(ci[a + kk] - i);
        } else {
            off[q] = 0;
            val[q] = (T)0;
        }
    }
}

// The values of one matrix (times D^{-1} by column when dinv is given) into their positions:
// 8 lanes per row, each lane writing VEC consecutive positions of the row's chunks with one
// 16-byte store (padding positions get 0), so the row's region is written whole and in order.
// The entry at row-local position t (chunk t / E, slot t % E) is the inverse of bp_pos: with
// it = chunk / LPR, l = chunk % LPR and g the lanes of that round, entry it E LPR + slot g + l.
constexpr int BPV_ROWS = BLOCK / 8;     // rows per block of the value refill
constexpr int BPV_STAGE = 2048;         // CSR entries staged (32 rows of up to 64 entries)

template <typename T, int E, int LPR>
__global__ __launch_bounds__(BLOCK) void k_bp_values(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                     const double* __restrict__ dinv, const int32_t* __restrict__ p,
                                                     T* __restrict__ out) {
    // the block's rows are one contiguous CSR slice: scaled and rounded once, by coalesced loads,
    // into LDS when it fits, then written in the banded copy's order
    __shared__ T lv[BPV_STAGE];
    const int64_t row0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * BPV_ROWS;
    const int64_t rowe = row0 + BPV_ROWS < n ? row0 + BPV_ROWS : n;
    const int e0 = rp[row0], e1 = rp[rowe];
    const bool staged = e1 - e0 <= BPV_STAGE;   // the same for the whole block
    if (staged) {
        for (int e = e0 + (int)threadIdx.x; e < e1; e += BLOCK) {
            double v = val[e];
            if (dinv) v *= dinv[ci[e]];
            lv[e - e0] = (T)v;
        }
    }
    __syncthreads();
    const int64_t i = row0 + threadIdx.x / 8;
    const int sub = (int)(threadIdx.x % 8);
    if (i >= n) return;
    const int a = rp[i], L = rp[i + 1] - a;
    const int c0 = p[i], LP = p[i + 1] - c0;
    constexpr int VEC = 16 / sizeof(T);   // divides E (4 or 8), so a store never leaves its chunk
    T* dst = out + (int64_t)c0 * E;
    const int tot = LP * E, R = E * LPR;
    for (int t0 = sub * VEC; t0 < tot; t0 += 8 * VEC) {
        T o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int t = t0 + e;
            const int chunk = t / E, slot = t - chunk * E;
            const int it = chunk / LPR, l = chunk - it * LPR;
            const int g = min(LPR, LP - LPR * it);
            const int kk = it * R + slot * g + l;
            T v = (T)0;
            if (kk < L) {
                if (staged) {
                    v = lv[a - e0 + kk];
                } else {
                    double d = val[a + kk];
                    if (dinv) d *= dinv[ci[a + kk]];
                    v = (T)d;
                }
            }
            o[e] = v;
        }
        __builtin_memcpy(dst + t0, o, sizeof(o));
    }
}

template <int LPR>
__global__ __launch_bounds__(BLOCK) void k_residual(int64_t n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                    const double* __restrict__ x, const double* __restrict__ b,
                                                    double* __restrict__ r) {
    const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    const int64_t row = gt / LPR;
    const int sub = (int)(gt % LPR);
    double acc = 0.0;
    const bool active = row < n;
    if (active) acc = csr_row_part_vec<double, LPR, 4>(ci, val, x, rp[row], rp[row + 1], sub);
    acc = group_sum<LPR>(acc);
    if (active && sub == 0) r[row] = (b ? b[row] : 0.0) - acc;
}

template <int LPR>
__global__ __launch_bounds__(BLOCK) void k_spmv(int64_t n, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                const double* __restrict__ x, double* __restrict__ y) {
    const int64_t gt = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t row = gt / LPR;
    const int sub = (int)(gt % LPR);
    double acc = 0.0;
    const bool active = row < n;
    if (active) acc = csr_row_part_vec<double, LPR, 4>(ci, val, x, rp[row], rp[row + 1], sub);
    acc = group_sum<LPR>(acc);
    if (active && sub == 0) y[row] = acc;
}

// Z[:, c0 + c] = A W[:, c0 + c], c < kc <= 16, with W given row-major (Wr[row * ldr + col],
// ldr a multiple of 16): four lanes per row, lane s owning columns c0 + 4 s .. c0 + 4 s + 3;
// every lane walks all entries of its row, so each entry costs the four lanes one 128-byte line of
// W between them and no reduction across lanes is needed.  (Measured on Q3 with k = 16: 0.88 ms,
// against 1.1 ms for lanes that split the row's entries and take all 16 columns.)  The column
// indices and values of the block's rows, one contiguous CSR slice, are first staged in LDS by
// coalesced loads when the slice fits, so the four lanes of a row read them from LDS rather than
// each loading them again.
constexpr int SPMM_ROWS = BLOCK / 4;      // rows per block
constexpr int SPMM_STAGE = 3200;          // CSR entries staged (64 rows of up to 50 entries)

template <typename I, typename V>
__device__ __forceinline__ void spmm_row(const I* __restrict__ cs, const V* __restrict__ vs, int a, int e,
                                         const double* __restrict__ wb, int ldr, double acc[4]) {
    int j = a;
    // eight entries at a time: their column indices and values first, then the eight W gathers
    // together, so each round trip to memory carries eight entries rather than two
    for (; j + 7 < e; j += 8) {
        int c[8];
        double v[8], w[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = cs[j + u];
            v[u] = vs[j + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            __builtin_memcpy(w[u], __builtin_assume_aligned(wb + (int64_t)c[u] * ldr, 32), sizeof(w[u]));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) acc[cc] += v[u] * w[u][cc];
        }
    }
    for (; j < e; ++j) {
        const double v0 = vs[j];
        double w0[4];
        __builtin_memcpy(w0, __builtin_assume_aligned(wb + (int64_t)cs[j] * ldr, 32), sizeof(w0));
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += v0 * w0[c];
    }
}

__global__ __launch_bounds__(BLOCK) void k_spmm_rows(int64_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                     const double* __restrict__ Wr, int ldr, int c0, int kc,
                                                     double* __restrict__ Z, float* __restrict__ Z32, int64_t ld) {
    __shared__ int32_t lci[SPMM_STAGE];
    __shared__ double lval[SPMM_STAGE];
    // XCD-aware rows: each XCD takes a contiguous share, so the W rows a block gathers (the columns
    // near its rows) are fetched into that XCD's L2 once rather than once per XCD
    const int64_t row0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SPMM_ROWS;
    const int64_t rowe = row0 + SPMM_ROWS < n ? row0 + SPMM_ROWS : n;
    const int e0 = rp[row0], e1 = rp[rowe];
    const bool staged = e1 - e0 <= SPMM_STAGE;   // the same for the whole block
    if (staged) {
        for (int e = e0 + (int)threadIdx.x; e < e1; e += BLOCK) {
            lci[e - e0] = ci[e];
            lval[e - e0] = val[e];
        }
    }
    __syncthreads();
    const int64_t row = row0 + threadIdx.x / 4;
    const int sub = (int)(threadIdx.x % 4);
    if (row >= n) return;
    const int a = rp[row], e = rp[row + 1];
    const double* wb = Wr + c0 + 4 * sub;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (staged) spmm_row(lci, lval, a - e0, e - e0, wb, ldr, acc);
    else spmm_row(ci, val, a, e, wb, ldr, acc);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (4 * sub + c < kc) {
            Z[(int64_t)(c0 + 4 * sub + c) * ld + row] = acc[c];
            if (Z32) Z32[(int64_t)(c0 + 4 * sub + c) * ld + row] = (float)acc[c];
        }
}

// Wr[r * ldr + c] = W[c * ld + r] for r < n, c < k.
__global__ __launch_bounds__(BLOCK) void k_to_rows(int64_t n, const double* __restrict__ W, int64_t ld, int k,
                                                   double* __restrict__ Wr, int ldr) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= n) return;
    for (int c = 0; c < k; ++c) Wr[r * ldr + c] = W[(int64_t)c * ld + r];
}

__global__ __launch_bounds__(BLOCK) void k_to_f32(int64_t count, const double* __restrict__ in,
                                                  float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < count) out[i] = (float)in[i];
}

// a = b + s c over n doubles, two per thread (16-byte loads and stores; grid-stride if the grid is
// capped): the streaming rate the hot kernels are measured against.
__global__ __launch_bounds__(BLOCK) void k_triad(int64_t n, double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ c, double s) {
    const int64_t npair = n / 2;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x; q < npair; q += stride) {
        double bb[2], cc[2], aa[2];
        __builtin_memcpy(bb, __builtin_assume_aligned(b + 2 * q, 16), sizeof(bb));
        __builtin_memcpy(cc, __builtin_assume_aligned(c + 2 * q, 16), sizeof(cc));
        aa[0] = bb[0] + s * cc[0];
        aa[1] = bb[1] + s * cc[1];
        __builtin_memcpy(__builtin_assume_aligned(a + 2 * q, 16), aa, sizeof(aa));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) a[n - 1] = b[n - 1] + s * c[n - 1];
}

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + BLOCK - 1) / BLOCK); }

}  // namespace

void launch_triad(int64_t n, double* a, const double* b, const double* c, double s, int cus, hipStream_t st) {
    // one pair per thread: on this device a full grid streams about a third faster than 8 to 32
    // grid-striding blocks per compute unit (6.0 against 4.4-4.9 TB/s measured at n = 2^27)
    (void)cus;
    const int64_t want = (n / 2 + BLOCK - 1) / BLOCK;
    k_triad<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(want, INT32_MAX)), BLOCK, 0, st>>>(n, a, b, c, s);
}

void launch_validate(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, int32_t* diag_pos, int32_t* err,
                     hipStream_t st) {
    k_validate<<<grid_for(n), BLOCK, 0, st>>>(n, nnz, rp, ci, diag_pos, err);
}

void launch_diag_inv(int64_t n, const int32_t* dp, const double* val, double* dinv, hipStream_t st) {
    k_diag_inv<<<grid_for(n), BLOCK, 0, st>>>(n, dp, val, dinv);
}

void launch_scale_values(int64_t nnz, const int32_t* ci, const double* val, const double* dinv, double* o64,
                         float* o32, hipStream_t st) {
    k_scale_values<<<grid_for(nnz), BLOCK, 0, st>>>(nnz, ci, val, dinv, o64, o32);
}

#define RS_LPR_DISPATCH(lpr, CALL) \
    switch (lpr) {                 \
        case 2: CALL(2); break;    \
        case 4: CALL(4); break;    \
        case 8: CALL(8); break;    \
        case 16: CALL(16); break;  \
        default: CALL(32); break;  \
    }

template <typename T>
void launch_spmv_arnoldi(int lpr, int vec, int remap, int64_t n, const int32_t* rp, const int32_t* ci, const T* val,
                         const T* win, T* vout, T* y, const Ctl* ctl, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
#define RS_CALL(L)                                                                                       \
    hipExtLaunchKernelGGL(k_spmv_arnoldi<T, L>, dim3(grid_for(n * L)), dim3(BLOCK), 0, st, ev0, ev1, 0, n, rp, ci, \
                          val, win, vout, y, ctl, remap, vec)
    RS_LPR_DISPATCH(lpr, RS_CALL)
#undef RS_CALL
}
template void launch_spmv_arnoldi<double>(int, int, int, int64_t, const int32_t*, const int32_t*, const double*,
                                          const double*, double*, double*, const Ctl*, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template void launch_spmv_arnoldi<float>(int, int, int, int64_t, const int32_t*, const int32_t*, const float*,
                                         const float*, float*, float*, const Ctl*, hipStream_t, hipEvent_t,
                                         hipEvent_t);

int64_t bp_scratch_ints(int64_t n) { return (n + BP_TILE - 1) / BP_TILE; }

int bp_setup(int64_t n, const int32_t* rp, const int32_t* ci, int E, int LPR, int32_t* p, int16_t* off, void* val,
             bool f32, int32_t* scratch, int64_t scratch_ints, hipStream_t st) {
    if ((E != 4 && E != 8) || (LPR != 2 && LPR != 4 && LPR != 8) || n < 1) return -1;
    const int64_t nt = bp_scratch_ints(n);
    if (nt > scratch_ints || nt > INT32_MAX) return -1;
    k_bp_tiles<<<(unsigned)nt, 1024, 0, st>>>(n, rp, E, p, scratch);
    k_bp_tile_offsets<<<1, 1024, 0, st>>>(n, (int)nt, scratch, p);
    k_bp_add<<<grid_for(n), BLOCK, 0, st>>>(n, scratch, p);
    if (f32) k_bp_pack<float><<<grid_for(n * 8), BLOCK, 0, st>>>(n, rp, ci, p, E, LPR, off, static_cast<float*>(val));
    else k_bp_pack<double><<<grid_for(n * 8), BLOCK, 0, st>>>(n, rp, ci, p, E, LPR, off, static_cast<double*>(val));
    return 0;
}

template <typename T>
void launch_bp_values(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* dinv,
                      const int32_t* p, int E, int LPR, T* out, hipStream_t st) {
    const unsigned g = (unsigned)((n + BPV_ROWS - 1) / BPV_ROWS);
#define RS_BPV(EE, L) k_bp_values<T, EE, L><<<g, BLOCK, 0, st>>>(n, rp, ci, val, dinv, p, out)
    if (E == 4) {
        if (LPR == 2) RS_BPV(4, 2);
        else if (LPR == 4) RS_BPV(4, 4);
        else RS_BPV(4, 8);
    } else {
        if (LPR == 2) RS_BPV(8, 2);
        else if (LPR == 4) RS_BPV(8, 4);
        else RS_BPV(8, 8);
    }
#undef RS_BPV
}
template void launch_bp_values<double>(int64_t, const int32_t*, const int32_t*, const double*, const double*,
                                       const int32_t*, int, int, double*, hipStream_t);
template void launch_bp_values<float>(int64_t, const int32_t*, const int32_t*, const double*, const double*,
                                      const int32_t*, int, int, float*, hipStream_t);

template void launch_spmv_bp<double>(int, int, int, int64_t, const int32_t*, const int16_t*, const double*,
                                     const double*, double*, double*, const Ctl*, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_spmv_bp<float>(int, int, int, int64_t, const int32_t*, const int16_t*, const float*,
                                    const float*, float*, float*, const Ctl*, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_spmv_bc<double>(int, int, int, int64_t, const int32_t*, const uint16_t*, const int16_t*,
                                     const double*, const double*, double*, double*, const Ctl*, hipStream_t,
                                     hipEvent_t, hipEvent_t);
template void launch_spmv_bc<float>(int, int, int, int64_t, const int32_t*, const uint16_t*, const int16_t*,
                                    const float*, const float*, float*, float*, const Ctl*, hipStream_t, hipEvent_t,
                                    hipEvent_t);

void launch_residual(int lpr, int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* x,
                     const double* b, double* r, hipStream_t st) {
#define RS_CALL(L) k_residual<L><<<grid_for(n * L), BLOCK, 0, st>>>(n, rp, ci, val, x, b, r)
    RS_LPR_DISPATCH(lpr, RS_CALL)
#undef RS_CALL
}

void launch_spmv(int lpr, int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* x,
                 double* y, hipStream_t st) {
#define RS_CALL(L) k_spmv<L><<<grid_for(n * L), BLOCK, 0, st>>>(n, rp, ci, val, x, y)
    RS_LPR_DISPATCH(lpr, RS_CALL)
#undef RS_CALL
}

void launch_spmm_rows(int64_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* Wr, int ldr,
                      int k, double* Z, int64_t ld, hipStream_t st, float* Z32) {
    for (int c0 = 0; c0 < k; c0 += 16) {
        const int kc = (k - c0) < 16 ? (k - c0) : 16;
        k_spmm_rows<<<(unsigned)((n + SPMM_ROWS - 1) / SPMM_ROWS), BLOCK, 0, st>>>(n, rp, ci, val, Wr, ldr, c0, kc,
                                                                                Z, Z32, ld);
    }
}

void launch_to_rows(int64_t n, const double* W, int64_t ld, int k, double* Wr, int ldr, hipStream_t st) {
    k_to_rows<<<grid_for(n), BLOCK, 0, st>>>(n, W, ld, k, Wr, ldr);
}

void launch_to_f32(int64_t count, const double* in, float* out, hipStream_t st) {
    k_to_f32<<<grid_for(count), BLOCK, 0, st>>>(count, in, out);
}

}  // namespace rs
