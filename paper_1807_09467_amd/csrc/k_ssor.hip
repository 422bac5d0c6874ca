// Multicolour SSOR (the symmetric SOR preconditioner of section 6.1) on the device.
//
// The rows carry a colour such that rows of one colour never couple (a_ij = a_ji = 0 for i != j
// of equal colour).  With D the diagonal and L, U the couplings of each row to rows of lower and
// of higher colour, M = (D + w L) D^{-1} (D + w U) / (w (2 - w)), and t = M^{-1} r takes two
// sweeps over the colours, each colour a set of independent rows:
//
//   forward, colours ascending:   t_i = (w (2 - w) r_i - w sum_{colour j < colour i} a_ij t_j) / a_ii
//   backward, colours descending: t_i -= w sum_{colour j > colour i} a_ij t_j / a_ii
//
// (the second line is (D + w U) z = D y solved in place over y).  A row is read by LPR lanes, each
// taking every LPR-th entry, float64 throughout.  Small systems take the whole application in
// one workgroup that walks the colours with a barrier between them; larger ones take one launch
// per colour and sweep.
//
// The colouring itself is first fit in natural row order over the symmetrised pattern, on the
// host, once per pattern.
#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace rs {

namespace {

constexpr int SSOR_BLOCK_THREADS = 1024;
constexpr int64_t SSOR_LDS_ROWS = 3640;   // 18 bytes a row within 64 KB of LDS

template <int LPR>
__device__ __forceinline__ double lane_group_sum(double v) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// The part of row i's sum that a sweep takes: couplings to lower colours (forward) or higher
// colours (backward); lane `sub` of LPR takes entries rp[i] + sub, rp[i] + sub + LPR, ..., four at a
// time.
template <bool FWD, int LPR>
__device__ __forceinline__ double colour_part(int i, int c, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ val,
                                              const int32_t* __restrict__ colour, const double* t, int sub) {
    double acc = 0.0;
    const int e1 = rp[i + 1];
    int e = rp[i] + sub;
    for (; e + 3 * LPR < e1; e += 4 * LPR) {   // four entries' indices and values before any use
        int jj[4];
        double vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            jj[u] = ci[e + u * LPR];
            vv[u] = val[e + u * LPR];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int cj = colour[jj[u]];
            if (FWD ? (cj < c) : (cj > c)) acc += vv[u] * t[jj[u]];
        }
    }
    for (; e < e1; e += LPR) {
        const int j = ci[e];
        const int cj = colour[j];
        if (FWD ? (cj < c) : (cj > c)) acc += val[e] * t[j];
    }
    return acc;
}

// One colour step of one sweep over rows[0..cnt), all of colour c.  Forward also writes
// vout_i = inv_h r_i when vout is given (the normalised Arnoldi vector).
template <bool FWD, int LPR>
__global__ __launch_bounds__(BLOCK) void k_ssor_colour(int32_t cnt, const int32_t* __restrict__ rows, int c,
                                                       const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                       const double* __restrict__ val, const int32_t* __restrict__ dpos,
                                                       const int32_t* __restrict__ colour,
                                                       const double* __restrict__ r, double* t,
                                                       double* __restrict__ vout, double omega,
                                                       const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    const int64_t gt = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t q = gt / LPR;
    const int sub = (int)(gt % LPR);
    const bool active = q < cnt;
    const int i = active ? rows[q] : 0;
    double acc = active ? colour_part<FWD, LPR>(i, c, rp, ci, val, colour, t, sub) : 0.0;
    acc = lane_group_sum<LPR>(acc);
    if (active && sub == 0) {
        const double d = val[dpos[i]];
        if (FWD) {
            t[i] = (omega * (2.0 - omega) * r[i] - omega * acc) / d;
            if (vout) vout[i] = ctl->inv_h * r[i];
        } else {
            t[i] -= omega * acc / d;
        }
    }
}

// The whole application in one workgroup: colours coff[c] .. coff[c + 1] of `rows`, forward then
// backward, a barrier after every colour (it orders the writes of t for the next colour).
template <int LPR>
__global__ __launch_bounds__(SSOR_BLOCK_THREADS) void k_ssor_block(int ncol, const int32_t* __restrict__ coff,
                                                                  const int32_t* __restrict__ rows,
                                                                  const int32_t* __restrict__ rp,
                                                                  const int32_t* __restrict__ ci,
                                                                  const double* __restrict__ val,
                                                                  const int32_t* __restrict__ dpos,
                                                                  const int32_t* __restrict__ colour,
                                                                  const double* __restrict__ r, double* t,
                                                                  double* __restrict__ vout, double omega,
                                                                  const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    constexpr int GROUPS = SSOR_BLOCK_THREADS / LPR;
    const int group = threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    const double alpha = omega * (2.0 - omega);
    for (int c = 0; c < ncol; ++c) {
        const int q1 = coff[c + 1];
        for (int q = coff[c] + group; q < q1; q += GROUPS) {
            const int i = rows[q];
            const double acc = lane_group_sum<LPR>(colour_part<true, LPR>(i, c, rp, ci, val, colour, t, sub));
            if (sub == 0) {
                t[i] = (alpha * r[i] - omega * acc) / val[dpos[i]];
                if (vout) vout[i] = ctl->inv_h * r[i];
            }
        }
        __syncthreads();
    }
    for (int c = ncol - 2; c >= 0; --c) {   // the highest colour has no higher neighbours
        const int q1 = coff[c + 1];
        for (int q = coff[c] + group; q < q1; q += GROUPS) {
            const int i = rows[q];
            const double acc = lane_group_sum<LPR>(colour_part<false, LPR>(i, c, rp, ci, val, colour, t, sub));
            if (sub == 0) t[i] -= omega * acc / val[dpos[i]];
        }
        __syncthreads();
    }
}

// Row i's couplings to lower (FWD) or higher colours than c, with the colours and t in LDS; the
// lane's entries are taken eight at a time, their indices and values loaded before any is used.
template <bool FWD, int LPR>
__device__ __forceinline__ double colour_part_lds(int a, int e1, int c, const int32_t* __restrict__ ci,
                                                  const double* __restrict__ val, const uint16_t* cls,
                                                  const double* ts, int sub) {
    double acc = 0.0;
    int e = a + sub;
    for (; e + 7 * LPR < e1; e += 8 * LPR) {
        int jj[8];
        double vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            jj[u] = ci[e + u * LPR];
            vv[u] = val[e + u * LPR];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int cj = cls[jj[u]];
            if (FWD ? (cj < c) : (cj > c)) acc += vv[u] * ts[jj[u]];
        }
    }
    for (; e < e1; e += LPR) {
        const int j = ci[e];
        const int cj = cls[j];
        if (FWD ? (cj < c) : (cj > c)) acc += val[e] * ts[j];
    }
    return acc;
}

// The one-workgroup application for systems of at most SSOR_LDS_ROWS rows, with t, the colours,
// the rows grouped by colour and the row pointers held in LDS (18 bytes a row): each colour
// step then waits on one global load, the row's entries, instead of four.  t is written back
// to global memory at the end.
template <int LPR>
__global__ __launch_bounds__(SSOR_BLOCK_THREADS) void k_ssor_block_lds(int ncol, int n, const int32_t* __restrict__ coff,
                                                                      const int32_t* __restrict__ rows,
                                                                      const int32_t* __restrict__ rp,
                                                                      const int32_t* __restrict__ ci,
                                                                      const double* __restrict__ val,
                                                                      const int32_t* __restrict__ dpos,
                                                                      const int32_t* __restrict__ colour,
                                                                      const double* __restrict__ r, double* __restrict__ t,
                                                                      double* __restrict__ vout, double omega,
                                                                      const Ctl* __restrict__ ctl) {
    if (ctl && ctl->done) return;
    extern __shared__ double lds_ssor[];
    double* ts = lds_ssor;                                                  // n
    int32_t* rps = reinterpret_cast<int32_t*>(ts + n);                      // n + 1
    int32_t* rws = rps + (n + 1);                                           // n
    uint16_t* cls = reinterpret_cast<uint16_t*>(rws + n);                   // n
    for (int i = threadIdx.x; i <= n; i += SSOR_BLOCK_THREADS) rps[i] = rp[i];
    for (int i = threadIdx.x; i < n; i += SSOR_BLOCK_THREADS) {
        rws[i] = rows[i];
        cls[i] = (uint16_t)colour[i];
    }
    __syncthreads();
    constexpr int GROUPS = SSOR_BLOCK_THREADS / LPR;
    const int group = threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    const double alpha = omega * (2.0 - omega);
    for (int c = 0; c < ncol; ++c) {
        const int q1 = coff[c + 1];
        for (int q = coff[c] + group; q < q1; q += GROUPS) {
            const int i = rws[q];
            const double acc =
                lane_group_sum<LPR>(colour_part_lds<true, LPR>(rps[i], rps[i + 1], c, ci, val, cls, ts, sub));
            if (sub == 0) {
                ts[i] = (alpha * r[i] - omega * acc) / val[dpos[i]];
                if (vout) vout[i] = ctl->inv_h * r[i];
            }
        }
        __syncthreads();
    }
    for (int c = ncol - 2; c >= 0; --c) {
        const int q1 = coff[c + 1];
        for (int q = coff[c] + group; q < q1; q += GROUPS) {
            const int i = rws[q];
            const double acc =
                lane_group_sum<LPR>(colour_part_lds<false, LPR>(rps[i], rps[i + 1], c, ci, val, cls, ts, sub));
            if (sub == 0) ts[i] -= omega * acc / val[dpos[i]];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += SSOR_BLOCK_THREADS) t[i] = ts[i];
}

__global__ __launch_bounds__(BLOCK) void k_fill(int64_t n, double* __restrict__ x, double v) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(BLOCK) void k_axpy(int64_t n, const double* __restrict__ t, double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) x[i] += t[i];
}

inline unsigned grid_of(int64_t threads) { return (unsigned)((threads + BLOCK - 1) / BLOCK); }

}  // namespace

int ssor_lanes(int64_t n, int64_t nnz) {
    const double avg = n > 0 ? (double)nnz / (double)n : 1.0;
    return avg <= 12.0 ? 4 : (avg <= 96.0 ? 16 : 64);
}

void launch_ssor_apply(const SsorPlan& p, const int32_t* rp, const int32_t* ci, const double* val,
                       const int32_t* dpos, const double* r, double* t, double* vout, const Ctl* ctl,
                       hipStream_t st) {
    if (p.single && p.n <= SSOR_LDS_ROWS && p.ncol <= 65535) {
        const size_t bytes = (size_t)p.n * 18 + 4;
#define RS_SSOR_L(L)                                                                                          \
    k_ssor_block_lds<L><<<1, SSOR_BLOCK_THREADS, bytes, st>>>(p.ncol, (int)p.n, p.coff_dev, p.rows, rp, ci, val, dpos, \
                                                              p.colour, r, t, vout, p.omega, ctl)
        if (p.lpr == 4) RS_SSOR_L(4);
        else if (p.lpr == 16) RS_SSOR_L(16);
        else RS_SSOR_L(64);
#undef RS_SSOR_L
        return;
    }
    if (p.single) {
#define RS_SSOR_B(L)                                                                                           \
    k_ssor_block<L><<<1, SSOR_BLOCK_THREADS, 0, st>>>(p.ncol, p.coff_dev, p.rows, rp, ci, val, dpos, p.colour, r, \
                                                      t, vout, p.omega, ctl)
        if (p.lpr == 4) RS_SSOR_B(4);
        else if (p.lpr == 16) RS_SSOR_B(16);
        else RS_SSOR_B(64);
#undef RS_SSOR_B
        return;
    }
    for (int dir = 0; dir < 2; ++dir) {
        const bool fwd = dir == 0;
        for (int s = 0; s < p.ncol; ++s) {
            const int c = fwd ? s : p.ncol - 1 - s;
            if (!fwd && c == p.ncol - 1) continue;   // no higher colour
            const int32_t q0 = p.coff_host[c], cnt = p.coff_host[c + 1] - q0;
            if (cnt == 0) continue;
            const unsigned g = grid_of((int64_t)cnt * p.lpr);
#define RS_SSOR_C(F, L)                                                                                          \
    k_ssor_colour<F, L><<<g, BLOCK, 0, st>>>(cnt, p.rows + q0, c, rp, ci, val, dpos, p.colour, r, t, F ? vout : nullptr, \
                                             p.omega, ctl)
            if (fwd) {
                if (p.lpr == 4) RS_SSOR_C(true, 4);
                else if (p.lpr == 16) RS_SSOR_C(true, 16);
                else RS_SSOR_C(true, 64);
            } else {
                if (p.lpr == 4) RS_SSOR_C(false, 4);
                else if (p.lpr == 16) RS_SSOR_C(false, 16);
                else RS_SSOR_C(false, 64);
            }
#undef RS_SSOR_C
        }
    }
}

void launch_fill(int64_t n, double* x, double v, hipStream_t st) {
    k_fill<<<grid_of(n), BLOCK, 0, st>>>(n, x, v);
}

void launch_axpy(int64_t n, const double* t, double* x, hipStream_t st) {
    k_axpy<<<grid_of(n), BLOCK, 0, st>>>(n, t, x);
}

int colour_first_fit(int64_t n, const int32_t* rp, const int32_t* ci, int32_t* colour, std::vector<int32_t>& rows,
                     std::vector<int32_t>& coff) {
    // rows j < i that hold column i: the earlier neighbours row i does not list itself
    std::vector<int64_t> tp((size_t)n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t e = rp[j]; e < rp[j + 1]; ++e)
            if (ci[e] > j) tp[(size_t)ci[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) tp[(size_t)i + 1] += tp[(size_t)i];
    std::vector<int32_t> tj((size_t)tp[(size_t)n]);
    {
        std::vector<int64_t> pos(tp.begin(), tp.end() - 1);
        for (int64_t j = 0; j < n; ++j)
            for (int64_t e = rp[j]; e < rp[j + 1]; ++e)
                if (ci[e] > j) tj[(size_t)pos[(size_t)ci[e]]++] = (int32_t)j;
    }
    // first fit: mark[c] == i when an earlier neighbour of row i holds colour c
    std::vector<int64_t> mark(16, -1);
    int ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] < i) mark[(size_t)colour[ci[e]]] = i;
        for (int64_t q = tp[(size_t)i]; q < tp[(size_t)i + 1]; ++q) mark[(size_t)colour[tj[(size_t)q]]] = i;
        int c = 0;
        while (mark[(size_t)c] == i) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
        if ((size_t)ncol + 1 >= mark.size()) mark.resize(mark.size() * 2, -1);
    }
    // rows grouped by colour, natural order inside a colour
    coff.assign((size_t)ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) coff[(size_t)colour[i] + 1]++;
    for (int c = 0; c < ncol; ++c) coff[(size_t)c + 1] += coff[(size_t)c];
    rows.assign((size_t)n, 0);
    std::vector<int32_t> pos(coff.begin(), coff.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[(size_t)pos[(size_t)colour[i]]++] = (int32_t)i;
    return ncol;
}

}  // namespace rs
