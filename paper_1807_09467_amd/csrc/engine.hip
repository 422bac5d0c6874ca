// Host engine and C-ABI of the rsolve library: one sequence = one time-stepping
// sequence of systems, solved by restarted GMRES(m) with the oblique projector
// of the recycle basis W (section 3.2, eq. (left_deflation); Table 1 rows
// "augmented / deflated oblique"), the projection initial guess (section 4.2),
// and the SVD snapshot-ring update (section 5.2, Algorithm 1).
//
// All device work of a sequence goes to its stream.  Within a GMRES cycle the
// host enqueues every Arnoldi step without waiting: the Givens kernel sets a
// device flag when the cycle must stop and later kernels of the cycle return
// at once.  The host synchronises once per cycle (explicit FP64 residual).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <type_traits>
#include <mutex>
#include <unordered_map>
#include <tuple>
#include <vector>

#include "../../include/rsolve.h"
#include "../../include/rsolve_kernels.h"
#include "engine_internal.hpp"
#include "kernels.hpp"

using namespace rs;

namespace {

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

// Sequential carving of the caller's workspace (base == nullptr: size only).
struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = align_up(off, ALIGN);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_err("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            return RSOLVE_E_DEVICE;                                                    \
        }                                                                              \
    } while (0)

constexpr size_t CTL_HEAD = offsetof(Ctl, g);   // fields the host reads after a sync

// Order of the extrapolated initial guess (eqs. (ext2)-(ext4)), 0 for the other methods.
int extrap_order(int method) {
    return (method >= RSOLVE_GUESS_EXTRAP2 && method <= RSOLVE_GUESS_EXTRAP4) ? method - RSOLVE_GUESS_EXTRAP2 + 2 : 0;
}

bool ritz_mode(const rsolve_config& c) {
    return c.select == RSOLVE_SELECT_RITZ || c.select == RSOLVE_SELECT_HARMONIC;
}

int cfg_check(const rsolve_config* c) {
    if (!c) return RSOLVE_E_INVALID;
    if (c->restart_m < 1 || c->restart_m > RSOLVE_MAX_RESTART) return RSOLVE_E_INVALID;
    if (c->recycle_k < 0 || c->recycle_k > RSOLVE_MAX_RECYCLE) return RSOLVE_E_INVALID;
    if (c->snapshots_s < 0 || c->snapshots_s > RSOLVE_MAX_SNAPSHOTS) return RSOLVE_E_INVALID;
    const bool ritz = c->select == RSOLVE_SELECT_RITZ || c->select == RSOLVE_SELECT_HARMONIC;
    // the Ritz spaces come from the search space [W, D^{-1} V_m] (no ring needed), at most SMAX wide
    if (ritz && (c->recycle_k < 1 || c->recycle_k + c->restart_m > SMAX)) return RSOLVE_E_INVALID;
    if (c->recycle_k > 0 && !ritz && c->snapshots_s < c->recycle_k) return RSOLVE_E_INVALID;
    if (c->svd_interval < 1) return RSOLVE_E_INVALID;
    if (c->method < RSOLVE_PLAIN || c->method > RSOLVE_DEFL_LS) return RSOLVE_E_INVALID;
    // the extrapolation methods keep a ring of at least `order` solutions and no recycle space
    if (extrap_order(c->method) && (c->recycle_k != 0 || c->snapshots_s < extrap_order(c->method)))
        return RSOLVE_E_INVALID;
    if (c->precond != RSOLVE_PRECOND_NONE && c->precond != RSOLVE_PRECOND_JACOBI && c->precond != RSOLVE_PRECOND_SSOR)
        return RSOLVE_E_INVALID;
    // multicolour SSOR: FP64 sweeps, and the Ritz search space would need M^{-1} of every basis vector
    if (c->precond == RSOLVE_PRECOND_SSOR &&
        (c->precision != RSOLVE_FP64 || ritz || !(c->ssor_omega == 0.0 || (c->ssor_omega > 0.0 && c->ssor_omega < 2.0))))
        return RSOLVE_E_INVALID;
    if (c->precision != RSOLVE_FP64 && c->precision != RSOLVE_FP32_IR) return RSOLVE_E_INVALID;
    if (c->max_iters < 1) return RSOLVE_E_INVALID;
    if (c->select < RSOLVE_SELECT_LARGEST || c->select > RSOLVE_SELECT_HARMONIC) return RSOLVE_E_INVALID;
    if (c->ortho != RSOLVE_ORTHO_CGS2 && c->ortho != RSOLVE_ORTHO_DCGS2) return RSOLVE_E_INVALID;
    if (c->precision == RSOLVE_FP32_IR && !(c->inner_tol > 0.0 && c->inner_tol < 1.0)) return RSOLVE_E_INVALID;
    return RSOLVE_OK;
}

int pick_lpr(int64_t n, int64_t nnz) {
    // lanes per row for the 4-entries-per-lane product: about one round of loads per row
    const double avg = n > 0 ? (double)nnz / (double)n : 1.0;
    if (avg <= 8.0) return 2;
    if (avg <= 32.0) return 4;
    return 8;
}

// Grid of the row-per-thread streaming kernels (256-thread blocks): enough blocks for
// 8 per compute unit, never more blocks than 256-row slabs.
int pick_nblk(int64_t npad, int cus) {
    const int64_t slabs = (npad + BLOCK - 1) / BLOCK;
    return (int)std::max<int64_t>(1, std::min<int64_t>({slabs, (int64_t)cus * 8, (int64_t)NBLK_MAX}));
}

// Grid of the column-per-wavefront sweeps with `nw` wavefronts per block: as many blocks as fit
// on the device at once (32 wavefronts per compute unit), never more than 64-row tiles.
// The per-block partials (ncol per block) are summed by one block afterwards, so the grid
// also keeps nblk * ncol near 48k values.
int cols_grid(int64_t npad, int cus, int nw, int waves_per_cu, int ncol) {
    const int64_t tiles = npad / WAVE;
    int per_cu = std::max(1, waves_per_cu / std::max(1, nw));
    per_cu = std::max(1, std::min(per_cu, (int)(49152 / ((int64_t)std::max(ncol, 1) * cus))));
    return (int)std::max<int64_t>(1, std::min<int64_t>({tiles, (int64_t)cus * per_cu, (int64_t)NBLK_MAX}));
}

// Most blocks of the Gram kernel (two per compute unit of the device); the launcher also
// keeps one slab per block at least and the partials within their buffer.
int pick_gblk(int64_t n) {
    (void)n;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 2 * std::max(cus, 1);
}

}  // namespace

struct rsolve_seq {
    rsolve_config cfg;
    int64_t n = 0, ld = 0, nnz_max = 0, nnz_cur = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Ctl* ctl = nullptr;
    Ctl* hctl = nullptr;     // pinned host mirror of the control header
    double* hsig = nullptr;  // pinned host copy of the singular values
    int32_t* err = nullptr;
    int32_t* herr = nullptr;
    int32_t* diag_pos = nullptr;
    double *V = nullptr, *W = nullptr, *Z = nullptr, *X = nullptr, *xw = nullptr, *dinv = nullptr;
    double* Wr = nullptr;          // W row-major (row r at Wr + r ldr), for Z = A W
    int ldr = 0;                   // recycle_k rounded up to 16
    bool wr_ok = false;            // Wr holds the current W
    double* wb[2] = {nullptr, nullptr};
    double *vals = nullptr, *partial = nullptr, *gpart = nullptr;
    double* zpart = nullptr;   // per-block A W dots of the delayed scheme's update (k <= DCGS2_ZD_KMAX)
    double* gz = nullptr;      // (A W)^T A W for them
    double* tsq[2] = {nullptr, nullptr};
    int64_t tsq_ld = 0;
    float *V32 = nullptr, *W32 = nullptr, *Z32 = nullptr, *vals32 = nullptr;
    float* w32[2] = {nullptr, nullptr};
    int nblk = 1, gblk = 1, lpr = 8, cus = 256;
    int svec = 4, sremap = 0;      // Arnoldi SpMV shape (entries per lane, XCD-aware block order)
    int sfmt = RSOLVE_SPMV_CSR;    // Arnoldi SpMV storage (CSR or banded padded)
    bool shape_set = false;        // lpr / svec / sremap / sfmt chosen by the caller (rsolve_set_spmv_shape)
    // banded padded copy of the matrix for the Arnoldi product (RSOLVE_SPMV_BANDED)
    int32_t* bp_p = nullptr;       // chunk offsets, n + 1
    int16_t* bp_off = nullptr;     // column offsets col - row, bp_cap
    void* bp_val = nullptr;        // values (float in FP32_IR mode, else double), bp_cap
    int64_t bp_cap = 0;            // 0: the format is not available for this size
    bool band_ok = false;          // the current pattern fits the 16-bit offsets
    int bp_e = 0, bp_l = 0;        // chunk size and lanes the copy is laid out for (0: not built)
    // shared offset lists of the banded copy: rows of equal offsets form a class, each class keeps
    // one list in cls_dict, and cls_first[r] is the chunk where row r's list starts
    uint16_t* cls_first = nullptr;
    int16_t* cls_dict = nullptr;
    bool cls_ok = false;           // the classes describe the banded copy as laid out now
    bool cls_allowed = true;       // build them at all (the serving loop turns this off)
    int ncls = 0;
    const int32_t* pat_rp = nullptr;
    const int32_t* pat_ci = nullptr;
    int64_t pat_nnz = -1;
    bool pat_ok = false;
    // Ritz and harmonic Ritz recycle spaces: the search space U = [W, D^{-1} V_j] of the last
    // solve, its orthonormal basis Q and A Q, the pairs' basis before orthonormalisation, and the
    // new W prepared at the end of the solve (A is not available to the update)
    double *rz_u = nullptr, *rz_q = nullptr, *rz_aq = nullptr, *rz_tmp = nullptr, *rz_w = nullptr;
    double *rz_g = nullptr, *rz_eig = nullptr;
    int rz_k = 0;                  // columns of rz_w
    bool rz_pending = false;       // rz_w holds the next W
    double rz_theta[SMAX];         // |theta| of the kept pairs
    int last_steps = 0;            // Arnoldi steps of the last cycle of the last solve
    int cycle_hint = 0;            // Arnoldi steps of the last cycle that took any (kept across solves)
    // multicolour SSOR: the colouring of the current pattern (device arrays in the workspace, the
    // colour offsets also on the host) and two work vectors
    bool ssor = false;
    SsorPlan sp;
    int32_t *ss_colour = nullptr, *ss_rows = nullptr, *ss_coff = nullptr;
    std::vector<int32_t> ss_coff_host;
    double *ss_t = nullptr, *ss_u = nullptr;
    int k_w = 0, rank = 0, nsig = 0;
    int64_t count = 0;
    double sigma[SMAX];
    bool have_x = false;
    // pipelined polling of the cycle's done flag
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    int32_t* poll_done = nullptr;  // pinned, 2 slots
    // per-kernel timing
    static constexpr int NPK = 4, NVAR = 4;
    bool prof_on = false;
    int prof_mask = 0;                   // bit RSOLVE_PROF_* set: that kernel kind is timed
    int prof_stride = 1;                 // time steps j with j % prof_stride == prof_stride / 2
    hipEvent_t* pev = nullptr;           // [NPK][MMAX][2]
    int pvar[NPK][MMAX];                 // variant recorded for step j
    double pbytes[NPK][MMAX];            // algorithmic bytes of step j's launch
    bool pset[NPK][MMAX] = {};           // events of step j recorded since the last collection
    double pms[NPK][NVAR];
    double pb[NPK][NVAR];
    int64_t pcnt[NPK][NVAR];
    // captured Arnoldi chunks: one graph per chunk, keyed by everything its kernels bake in
    struct GraphKey {
        int j0, j1, k, ir, lpr, vec, remap, fmt, dg, allowed;
        const void* rp;
        const void* ci;
        const void* off;
        const void* vals;
        bool operator<(const GraphKey& o) const {
            return std::tie(j0, j1, k, ir, lpr, vec, remap, fmt, dg, allowed, rp, ci, off, vals) <
                   std::tie(o.j0, o.j1, o.k, o.ir, o.lpr, o.vec, o.remap, o.fmt, o.dg, o.allowed, o.rp, o.ci, o.off,
                            o.vals);
        }
    };
    bool graphs_on = false;
    hipStream_t cap_stream = nullptr;   // capture happens here: the caller's stream may be the null stream
    std::map<GraphKey, hipGraphExec_t> graphs;
    int64_t graph_captures = 0, graph_launches = 0;
    // one-block batched path: pinned job descriptors and its own pattern cache
    SmallJob* hjob = nullptr;
    SmallUpd* hupd = nullptr;
    const int32_t* spat_rp = nullptr;
    const int32_t* spat_ci = nullptr;
    int64_t spat_nnz = -1;
};

namespace {

// The split-n reductions' partial sums (also the scratch of the banded layout's prefix sums).
constexpr int64_t PARTIAL_DOUBLES = (int64_t)NBLK_MAX * (MMAX + 2 * KMAX + 1);
constexpr int64_t PARTIAL_INTS = 2 * PARTIAL_DOUBLES;

// Lays the sequence's buffers out in the workspace; returns the bytes used.
size_t layout(rsolve_seq* s, const rsolve_config& c, int64_t n, int64_t nnz_max, char* base) {
    Carver cv{base};
    const int64_t ld = pad64(n);
    const bool ir = c.precision == RSOLVE_FP32_IR;
    const bool jac = c.precond == RSOLVE_PRECOND_JACOBI;
    const int m = c.restart_m, k = c.recycle_k, sn = c.snapshots_s;
    Ctl* ctl = cv.take<Ctl>(1);
    int32_t* err = cv.take<int32_t>(8);
    int32_t* dp = cv.take<int32_t>((size_t)n);
    double* V = ir ? nullptr : cv.take<double>((size_t)(m + 1) * ld);
    float* V32 = ir ? cv.take<float>((size_t)(m + 1) * ld) : nullptr;
    double* W = k ? cv.take<double>((size_t)k * ld) : nullptr;
    double* Z = k ? cv.take<double>((size_t)k * ld) : nullptr;
    const int ldr = (k + 15) / 16 * 16;
    double* Wr = k ? cv.take<double>((size_t)ldr * ld) : nullptr;
    float* W32 = (k && ir) ? cv.take<float>((size_t)k * ld) : nullptr;
    float* Z32 = (k && ir) ? cv.take<float>((size_t)k * ld) : nullptr;
    double* X = ((k || extrap_order(c.method)) && sn) ? cv.take<double>((size_t)sn * ld) : nullptr;
    double* wb0 = cv.take<double>((size_t)ld);
    double* wb1 = cv.take<double>((size_t)ld);
    float* w320 = ir ? cv.take<float>((size_t)ld) : nullptr;
    float* w321 = ir ? cv.take<float>((size_t)ld) : nullptr;
    double* xw = cv.take<double>((size_t)ld);
    double* dinv = jac ? cv.take<double>((size_t)ld) : nullptr;
    double* vals = (jac && !ir) ? cv.take<double>((size_t)nnz_max) : nullptr;
    float* vals32 = ir ? cv.take<float>((size_t)nnz_max) : nullptr;
    // the banded copy holds every row padded to whole chunks of at most 8 entries
    const int64_t bp_cap = (nnz_max + 7 * n < (int64_t)INT32_MAX) ? align_up(nnz_max + 7 * n, 64) : 0;
    int32_t* bp_p = bp_cap ? cv.take<int32_t>((size_t)n + 1) : nullptr;
    int16_t* bp_off = bp_cap ? cv.take<int16_t>((size_t)bp_cap) : nullptr;
    void* bp_val = bp_cap ? (ir ? static_cast<void*>(cv.take<float>((size_t)bp_cap))
                                : static_cast<void*>(cv.take<double>((size_t)bp_cap)))
                          : nullptr;
    uint16_t* cls_first = bp_cap ? cv.take<uint16_t>((size_t)n) : nullptr;
    int16_t* cls_dict = bp_cap ? cv.take<int16_t>((size_t)CLS_DICT_CHUNKS * 8) : nullptr;
    double* partial = cv.take<double>((size_t)PARTIAL_DOUBLES);
    double* gpart = cv.take<double>((size_t)GRAM_PARTIAL);
    double* zpart = (k > 0 && k <= DCGS2_ZD_KMAX) ? cv.take<double>((size_t)k * NBLK_MAX) : nullptr;
    double* gz = zpart ? cv.take<double>((size_t)k * k) : nullptr;
    const bool rz = ritz_mode(c) && k > 0;
    const int rzc = rz ? k + m : 0;   // widest search space
    double *rz_u = nullptr, *rz_q = nullptr, *rz_aq = nullptr, *rz_tmp = nullptr, *rz_w = nullptr;
    double *rz_g = nullptr, *rz_eig = nullptr;
    if (rz) {
        rz_u = cv.take<double>((size_t)rzc * ld);
        rz_q = cv.take<double>((size_t)rzc * ld);
        rz_aq = cv.take<double>((size_t)rzc * ld);
        rz_tmp = cv.take<double>((size_t)k * ld);
        rz_w = cv.take<double>((size_t)k * ld);
        rz_g = cv.take<double>((size_t)2 * SMAX * SMAX);
        rz_eig = cv.take<double>((size_t)9 * SMAX * SMAX);
    }
    const bool ssor = c.precond == RSOLVE_PRECOND_SSOR;
    int32_t* ss_colour = ssor ? cv.take<int32_t>((size_t)n) : nullptr;
    int32_t* ss_rows = ssor ? cv.take<int32_t>((size_t)n) : nullptr;
    int32_t* ss_coff = ssor ? cv.take<int32_t>((size_t)n + 1) : nullptr;
    double* ss_t = ssor ? cv.take<double>((size_t)ld) : nullptr;
    double* ss_u = ssor ? cv.take<double>((size_t)ld) : nullptr;
    const int tcols = std::max(rz ? rzc : 0, (k || extrap_order(c.method)) ? sn : 0);   // TSQR width
    int64_t tsq_rows = 0, tsq_ld = 0;
    double *t0 = nullptr, *t1 = nullptr;
    if (k && tcols) {
        tsq_rows = ((n + TSQR_MIN_PANEL - 1) / TSQR_MIN_PANEL) * tcols;
        tsq_ld = pad64(tsq_rows);
        t0 = cv.take<double>((size_t)tsq_ld * tcols);
        t1 = cv.take<double>((size_t)tsq_ld * tcols);
    }
    if (s) {
        s->ld = ld;
        s->ctl = ctl;
        s->err = err;
        s->diag_pos = dp;
        s->V = V;
        s->V32 = V32;
        s->W = W;
        s->Wr = Wr;
        s->ldr = ldr;
        s->Z = Z;
        s->W32 = W32;
        s->Z32 = Z32;
        s->X = X;
        s->wb[0] = wb0;
        s->wb[1] = wb1;
        s->w32[0] = w320;
        s->w32[1] = w321;
        s->xw = xw;
        s->dinv = dinv;
        s->vals = vals;
        s->vals32 = vals32;
        s->partial = partial;
        s->gpart = gpart;
        s->zpart = zpart;
        s->gz = gz;
        s->bp_p = bp_p;
        s->bp_off = bp_off;
        s->bp_val = bp_val;
        s->bp_cap = bp_cap;
        s->cls_first = cls_first;
        s->cls_dict = cls_dict;
        s->tsq[0] = t0;
        s->tsq[1] = t1;
        s->tsq_ld = tsq_ld;
        s->rz_u = rz_u;
        s->rz_q = rz_q;
        s->rz_aq = rz_aq;
        s->rz_tmp = rz_tmp;
        s->rz_w = rz_w;
        s->rz_g = rz_g;
        s->rz_eig = rz_eig;
        s->ssor = ssor;
        s->ss_colour = ss_colour;
        s->ss_rows = ss_rows;
        s->ss_coff = ss_coff;
        s->ss_t = ss_t;
        s->ss_u = ss_u;
    }
    return align_up(cv.off, ALIGN);
}

// Multicolour SSOR: colour the (validated) pattern on the host and upload the colour of every row,
// the rows grouped by colour and the colour offsets; the plan then serves every solve until the
// pattern changes.
int ssor_colour(rsolve_seq* s, const rsolve_csr* A) {
    hipStream_t stm = s->stream;
    const int64_t n = s->n;
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)A->nnz), colour((size_t)n), rows;
    HIP_TRY(hipMemcpyAsync(rp.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, stm));
    HIP_TRY(hipMemcpyAsync(ci.data(), A->col_idx, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost, stm));
    HIP_TRY(hipStreamSynchronize(stm));
    const int ncol = colour_first_fit(n, rp.data(), ci.data(), colour.data(), rows, s->ss_coff_host);
    HIP_TRY(hipMemcpyAsync(s->ss_colour, colour.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stm));
    HIP_TRY(hipMemcpyAsync(s->ss_rows, rows.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stm));
    HIP_TRY(hipMemcpyAsync(s->ss_coff, s->ss_coff_host.data(), sizeof(int32_t) * (ncol + 1), hipMemcpyHostToDevice,
                           stm));
    HIP_TRY(hipStreamSynchronize(stm));   // the host vectors go out of scope
    SsorPlan& p = s->sp;
    p.n = n;
    p.ncol = ncol;
    p.lpr = ssor_lanes(n, A->nnz);
    // one workgroup when the colours hold few rows on average (its barrier is cheaper than a
    // launch), one launch per colour otherwise
    p.single = n <= 16384 || (int64_t)ncol * 512 >= n;
    p.omega = s->cfg.ssor_omega == 0.0 ? 1.0 : s->cfg.ssor_omega;
    p.colour = s->ss_colour;
    p.rows = s->ss_rows;
    p.coff_dev = s->ss_coff;
    p.coff_host = s->ss_coff_host.data();
    return RSOLVE_OK;
}

// Pattern check on the device (row pointers, column range and order, diagonal present); on
// success the pattern is cached for RSOLVE_SAME_PATTERN calls and the SpMV lanes per row are
// chosen for it (unless the caller fixed the shape).
int validate_pattern(rsolve_seq* s, const rsolve_csr* A) {
    hipStream_t stm = s->stream;
    const int64_t n = s->n;
    s->pat_ok = false;
    HIP_TRY(hipMemsetAsync(s->err, 0, sizeof(int32_t) * 8, stm));
    launch_validate(n, A->nnz, A->row_ptr, A->col_idx, s->diag_pos, s->err, stm);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(s->herr, s->err, sizeof(int32_t) * 5, hipMemcpyDeviceToHost, stm));
    HIP_TRY(hipStreamSynchronize(stm));
    if (s->herr[0] || s->herr[1] || s->herr[2] || s->herr[3]) {
        set_err("corrupt CSR: row_ptr=%d col_range=%d col_order=%d no_diagonal=%d", s->herr[0], s->herr[1],
                s->herr[2], s->herr[3]);
        return RSOLVE_E_INVALID;
    }
    if (s->ssor) {
        const int crc = ssor_colour(s, A);
        if (crc) return crc;
    }
    s->pat_rp = A->row_ptr;
    s->pat_ci = A->col_idx;
    s->pat_nnz = A->nnz;
    s->pat_ok = true;
    s->band_ok = s->bp_cap > 0 && s->herr[4] == 0;
    s->bp_e = s->bp_l = 0;   // the banded copy (if used) is laid out again for this pattern
    s->cls_ok = false;
    if (!s->shape_set) {
        // banded padded format with 8-entry chunks and 4 lanes per row for finite-element rows of
        // about a dozen entries or more; CSR otherwise (always with SSOR, whose product takes the
        // caller's values as they are)
        if (s->band_ok && (double)A->nnz >= 12.0 * (double)n && !s->ssor) {
            s->sfmt = RSOLVE_SPMV_BANDED;
            s->svec = 8;
            s->lpr = 4;
        } else {
            s->sfmt = RSOLVE_SPMV_CSR;
            s->svec = 4;
            s->lpr = pick_lpr(n, A->nnz);
        }
        s->sremap = 0;
    }
    return RSOLVE_OK;
}

// The matrix operand of the Arnoldi product: CSR (the caller's pattern and a value array) or the
// sequence's banded padded copy.
struct SpOp {
    int fmt;
    const int32_t* rp;    // CSR row pointers, or the banded chunk offsets
    const int32_t* ci;    // CSR column indices (null for the banded copy)
    const int16_t* off;   // banded column offsets (null for CSR)
    const void* vals;
};

// Lays the banded copy out for the current pattern and shape if needed, then writes this
// matrix's values (times D^{-1} by column when dinv is given) into it.
// The offset classes of the banded copy just laid out (chunk size E): the copy's chunk offsets
// and column offsets are read back once, rows are grouped by their offset lists (hash, then an
// exact comparison), and each row's list start and the lists are written to the workspace.
// Leaves cls_ok false (no error) when the pattern has more than CLS_MAX classes or their lists
// exceed CLS_DICT_CHUNKS chunks: the product then reads the copy's own offsets.
int cls_build(rsolve_seq* s, int E) {
    s->cls_ok = false;
    if (!CLS_ON || !s->cls_allowed) return RSOLVE_OK;
    hipStream_t stm = s->stream;
    const int64_t n = s->n;
    std::vector<int32_t> hp((size_t)n + 1);
    HIP_TRY(hipMemcpyAsync(hp.data(), s->bp_p, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, stm));
    HIP_TRY(hipStreamSynchronize(stm));
    const int64_t total = (int64_t)hp[n] * E;
    std::vector<int16_t> hoff((size_t)total);
    HIP_TRY(hipMemcpyAsync(hoff.data(), s->bp_off, sizeof(int16_t) * total, hipMemcpyDeviceToHost, stm));
    HIP_TRY(hipStreamSynchronize(stm));
    std::vector<uint16_t> rowc((size_t)n);
    std::vector<int32_t> cstart, clen;
    std::vector<int16_t> dict;
    std::unordered_multimap<uint64_t, int> by_hash;
    for (int64_t r = 0; r < n; ++r) {
        const int LP = hp[r + 1] - hp[r];
        const int16_t* sp = hoff.data() + (int64_t)hp[r] * E;
        const int len = LP * E;
        uint64_t h = 1469598103934665603ull ^ (uint64_t)LP;
        for (int t = 0; t < len; ++t) h = (h ^ (uint16_t)sp[t]) * 1099511628211ull;
        int id = -1;
        auto range = by_hash.equal_range(h);
        for (auto it = range.first; it != range.second; ++it) {
            const int c = it->second;
            if (clen[c] == LP && std::memcmp(dict.data() + (int64_t)cstart[c] * E, sp, sizeof(int16_t) * len) == 0) {
                id = c;
                break;
            }
        }
        if (id < 0) {
            const int64_t chunks = (int64_t)dict.size() / E;
            // every list start stays below CLS_DICT_CHUNKS, so it fits the 16-bit row entry
            if ((int)cstart.size() >= CLS_MAX || chunks + std::max(LP, 1) > CLS_DICT_CHUNKS) return RSOLVE_OK;
            id = (int)cstart.size();
            cstart.push_back((int32_t)chunks);
            clen.push_back(LP);
            dict.insert(dict.end(), sp, sp + len);
            by_hash.emplace(h, id);
        }
        rowc[r] = (uint16_t)cstart[id];
    }
    HIP_TRY(hipMemcpyAsync(s->cls_first, rowc.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice, stm));
    if (!dict.empty())
        HIP_TRY(hipMemcpyAsync(s->cls_dict, dict.data(), sizeof(int16_t) * dict.size(), hipMemcpyHostToDevice, stm));
    HIP_TRY(hipStreamSynchronize(stm));   // the host vectors go out of scope
    s->ncls = (int)cstart.size();
    s->cls_ok = true;
    return RSOLVE_OK;
}

int bp_prepare(rsolve_seq* s, const rsolve_csr* A, const double* dinv, bool f32) {
    if (!s->band_ok) {
        set_err("the banded SpMV format needs |col - row| <= %d for every entry and room for the padding",
                BP_MAX_OFFSET);
        return RSOLVE_E_INVALID;
    }
    hipStream_t stm = s->stream;
    if (s->bp_e != s->svec || s->bp_l != s->lpr) {
        if (bp_setup(s->n, A->row_ptr, A->col_idx, s->svec, s->lpr, s->bp_p, s->bp_off, s->bp_val, f32,
                     reinterpret_cast<int32_t*>(s->partial), PARTIAL_INTS, stm) != 0) {
            set_err("invalid banded SpMV shape (entries %d, lanes %d)", s->svec, s->lpr);
            return RSOLVE_E_INVALID;
        }
        s->bp_e = s->svec;
        s->bp_l = s->lpr;
        const int crc = cls_build(s, s->svec);
        if (crc) return crc;
    }
    if (f32) launch_bp_values<float>(s->n, A->row_ptr, A->col_idx, A->val, dinv, s->bp_p, s->svec, s->lpr,
                                     static_cast<float*>(s->bp_val), stm);
    else launch_bp_values<double>(s->n, A->row_ptr, A->col_idx, A->val, dinv, s->bp_p, s->svec, s->lpr,
                                  static_cast<double*>(s->bp_val), stm);
    return RSOLVE_OK;
}

// Algorithmic bytes of one Arnoldi product (entries counted without padding), w = value width.
double spmv_bytes(const rsolve_seq* s, double w, bool vout) {
    const double nn = (double)s->n, nz = (double)s->nnz_cur;
    if (s->sfmt == RSOLVE_SPMV_BANDED && s->cls_ok)   // values, chunk offsets, 16-bit list starts
        return w * nz + 4.0 * (nn + 1.0) + 2.0 * nn + (vout ? 3.0 : 2.0) * w * nn;
    const double idx = s->sfmt == RSOLVE_SPMV_BANDED ? 2.0 : 4.0;
    return (w + idx) * nz + 4.0 * (nn + 1.0) + (vout ? 3.0 : 2.0) * w * nn;
}

template <typename T>
void arnoldi_product(rsolve_seq* s, const SpOp& op, const T* win, T* vout, T* y, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (std::is_same<T, double>::value) {
        if (s->ssor) {
            // y = s A M^{-1} win: the sweeps give M^{-1} win (and vout = s win), the product scales
            launch_ssor_apply(s->sp, op.rp, op.ci, static_cast<const double*>(op.vals), s->diag_pos, win, s->ss_t,
                              vout, s->ctl, s->stream);
            launch_spmv_arnoldi<double>(s->lpr, s->svec, s->sremap, s->n, op.rp, op.ci,
                                        static_cast<const double*>(op.vals), s->ss_t, nullptr, y, s->ctl, s->stream,
                                        e0, e1);
            return;
        }
    }
    if (op.fmt == RSOLVE_SPMV_BANDED && s->cls_ok)
        launch_spmv_bc<T>(s->svec, s->lpr, s->sremap, s->n, op.rp, s->cls_first, s->cls_dict,
                          static_cast<const T*>(op.vals), win, vout, y, s->ctl, s->stream, e0, e1);
    else if (op.fmt == RSOLVE_SPMV_BANDED)
        launch_spmv_bp<T>(s->svec, s->lpr, s->sremap, s->n, op.rp, op.off, static_cast<const T*>(op.vals), win, vout,
                          y, s->ctl, s->stream, e0, e1);
    else
        launch_spmv_arnoldi<T>(s->lpr, s->svec, s->sremap, s->n, op.rp, op.ci, static_cast<const T*>(op.vals), win,
                               vout, y, s->ctl, s->stream, e0, e1);
}

// The executable graph of one Arnoldi chunk (kernel launches only, captured on the sequence's
// stream in thread-local mode), captured on first use and kept while its key holds.
template <class F>
int chunk_graph(rsolve_seq* s, const rsolve_seq::GraphKey& key, F&& enqueue, hipGraphExec_t* out) {
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) {
        *out = it->second;
        return RSOLVE_OK;
    }
    if (s->graphs.size() >= 512) {   // keys of earlier matrices: start over
        for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
        s->graphs.clear();
    }
    if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    // the chunk's kernels are recorded on the capture stream (nothing runs there), then the graph
    // is launched on the sequence's own stream
    hipStream_t own = s->stream;
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    s->stream = s->cap_stream;
    enqueue();
    s->stream = own;
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_err("graph capture failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return RSOLVE_E_DEVICE;
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        set_err("graph instantiation failed: %s", hipGetErrorString(e3));
        return RSOLVE_E_DEVICE;
    }
    s->graphs[key] = ge;
    s->graph_captures++;
    *out = ge;
    return RSOLVE_OK;
}

inline double* ctl_h1(Ctl* c) { return reinterpret_cast<double*>(reinterpret_cast<char*>(c) + offsetof(Ctl, h1)); }
inline double* ctl_h2(Ctl* c) { return reinterpret_cast<double*>(reinterpret_cast<char*>(c) + offsetof(Ctl, h2)); }
inline double* ctl_cw(Ctl* c) { return reinterpret_cast<double*>(reinterpret_cast<char*>(c) + offsetof(Ctl, cw)); }
inline double* ctl_red(Ctl* c) { return reinterpret_cast<double*>(reinterpret_cast<char*>(c) + offsetof(Ctl, red)); }
inline double* ctl_sigma(Ctl* c) {
    return reinterpret_cast<double*>(reinterpret_cast<char*>(c) + offsetof(Ctl, sigma));
}

int read_head(rsolve_seq* s) {
    HIP_TRY(hipMemcpyAsync(s->hctl, s->ctl, CTL_HEAD, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return RSOLVE_OK;
}

inline int var_of(int cols) { return cols <= 8 ? 0 : (cols <= 16 ? 1 : (cols <= 32 ? 2 : 3)); }

// Per-kernel timing: the events of (kernel kind, step j) are handed to the launch itself, which
// stamps them with the start and end of the kernel's dispatch.
struct ProfEv {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfEv(rsolve_seq* s, int kind, int j, int var, double bytes) {
        if (!(s->prof_mask & (1 << kind)) || j >= MMAX || j % s->prof_stride != s->prof_stride / 2) return;
        s->pvar[kind][j] = var;
        s->pbytes[kind][j] = bytes;
        s->pset[kind][j] = true;
        e0 = s->pev[(kind * MMAX + j) * 2 + 0];
        e1 = s->pev[(kind * MMAX + j) * 2 + 1];
    }
};

// After a cycle's synchronisation: accumulate the event times of the steps that ran.
void prof_collect(rsolve_seq* s, int steps) {
    if (!s->prof_on) return;
    for (int kd = 0; kd < rsolve_seq::NPK; ++kd)
        for (int j = 0; j < steps && (s->prof_mask & (1 << kd)); ++j) {
            // only kernels that ran in this cycle (the two schemes use different kinds); an event
            // never recorded would leave an error behind in the runtime
            if (!s->pset[kd][j]) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->pev[(kd * MMAX + j) * 2], s->pev[(kd * MMAX + j) * 2 + 1]) != hipSuccess)
                continue;
            const int v = s->pvar[kd][j];
            s->pms[kd][v] += ms;
            s->pb[kd][v] += s->pbytes[kd][j];
            s->pcnt[kd][v] += 1;
        }
    memset(s->pset, 0, sizeof(s->pset));
}

// One Arnoldi step j of the current cycle on storage type T.
template <typename T>
void arnoldi_step(rsolve_seq* s, int j, const SpOp& op, T* V, T* const* wbuf, const T* Wt, const T* Zt, int k,
                  bool orth) {
    // the orthogonal projector I - W W^T takes W where the oblique one takes A W
    const T* Pt = orth ? Wt : Zt;
    hipStream_t st = s->stream;
    const int64_t ld = s->ld;
    T* win = wbuf[j & 1];
    T* wout = wbuf[(j + 1) & 1];
    T* vj = V + (int64_t)j * ld;
    const double w = sizeof(T), nn = (double)s->n;
    {
        ProfEv pe(s, RSOLVE_PROF_SPMV, j, 0, spmv_bytes(s, w, true));
        arnoldi_product<T>(s, op, win, vj, wout, pe.e0,
                               pe.e1);
    }
    const int nv = j + 1;
    const int ntot = k > 0 ? nv + 2 * k : nv;
    const int nb1 = cols_grid(ld, s->cus, std::min(16, (ntot + 7) / 8), 32, ntot);
    if (k > 0) {
        const T* bases[3] = {V, Wt, Pt};
        const T* vecs[3] = {wout, wout, vj};
        const int counts[3] = {nv, k, k};
        ProfEv pe(s, RSOLVE_PROF_DOTS, j, var_of(ntot), (nv + 2.0 * k + 1.0) * w * nn);
        launch_dots<T>(ld, ld, bases, vecs, counts, 3, s->partial, nb1, s->ctl, st, nv, k, pe.e0, pe.e1, orth);
    } else {
        const T* bases[1] = {V};
        const T* vecs[1] = {wout};
        const int counts[1] = {nv};
        ProfEv pe(s, RSOLVE_PROF_DOTS, j, var_of(ntot), (nv + 1.0) * w * nn);
        launch_dots<T>(ld, ld, bases, vecs, counts, 1, s->partial, nb1, s->ctl, st, nv, 0, pe.e0, pe.e1);
    }
    const int nb2 = cols_grid(ld, s->cus, (nv + 7) / 8, 16, nv);
    {
        ProfEv pe(s, RSOLVE_PROF_UPDATE_DOTS, j, var_of(nv), (nv + k + 2.0) * w * nn);
        launch_update_dots<T>(ld, V, ld, nv, Pt, k, wout, ctl_h1(s->ctl), ctl_cw(s->ctl), s->partial, nb2, s->ctl, st,
                              pe.e0, pe.e1);
    }
    {
        ProfEv pe(s, RSOLVE_PROF_UPDATE_NORM, j, 0, (nv + 2.0) * w * nn);
        launch_update_norm<T>(ld, V, ld, nv, wout, ctl_h2(s->ctl), s->partial, s->nblk, s->ctl, st, j, pe.e0, pe.e1);
    }
}

// One step j of a cycle with delayed reorthogonalisation (RSOLVE_ORTHO_DCGS2): z = A D^{-1} u
// (skipped on the closing step j = allowed), the sweep over [V_j, W, A W, u] with u and z, the
// reduction that completes column j-1, and the update sweep writing v_j and the next candidate.
// ls: the least-squares projector, called with Wt = Zt = A W; the sweep then reads A W once (its
// dots with z give the projector's right-hand side, those with u the row of F).
template <typename T>
void dcgs2_step(rsolve_seq* s, int j, int allowed, const SpOp& op, T* V, T* const* wbuf, const T* Wt, const T* Zt,
                int k, bool orth, bool ls) {
    // the orthogonal projector I - W W^T needs no A W columns in the sweep and takes W in the update
    const int kz = (orth || ls) ? 0 : k;
    hipStream_t st = s->stream;
    const int64_t ld = s->ld;
    T* u = wbuf[0];
    T* z = wbuf[1];
    const bool has_z = j < allowed;
    const double w = sizeof(T), nn = (double)s->n;
    if (has_z) {
        ProfEv pe(s, RSOLVE_PROF_SPMV, j, 0, spmv_bytes(s, w, false));
        arnoldi_product<T>(s, op, u, nullptr, z, pe.e0, pe.e1);
    }
    const int ncol = j + k + kz + 1;
    // oblique projector, k <= DCGS2_ZD_KMAX: every update writes the dots of A W with the candidate
    // it forms, so from step 1 on the sweep reads [V_j, W, u] and not A W (k columns fewer)
    double* zpart = (kz > 0 && s->zpart) ? s->zpart : nullptr;
    const int zskip = (zpart && j >= 1) ? kz : 0;
    const int nsw = ncol - zskip;   // swept columns
    // two blocks per compute unit once a block has 8 or more wavefronts (measured on Q3 for 34..83
    // columns: one block per unit leaves the wide sweeps a third slower, three or four are slower
    // too), about 32 wavefronts per unit for narrower sweeps; the partials within their buffer
    const int nw = std::min(16, (nsw + (nsw > 64 ? 7 : 3)) / (nsw > 64 ? 8 : 4));   // as the launcher
    const int64_t per_cu = nw >= 8 ? 2 : 32 / nw;
    const int64_t tiles = std::max<int64_t>(1, ld / (WAVE * (16 / (int64_t)sizeof(T))));
    const int nb1 = (int)std::min<int64_t>({per_cu * s->cus, tiles, PARTIAL_DOUBLES / (2 * ncol) - 1, (int64_t)NBLK_MAX});
    {
        ProfEv pe(s, RSOLVE_PROF_DOTS, has_z ? j : MMAX, var_of(nsw), (nsw + 1.0) * w * nn);
        launch_dots2<T>(ld, ld, V, j, Wt, Zt, k, kz, zskip, u, has_z ? z : u, s->partial, nb1, s->ctl, st, pe.e0,
                        pe.e1);
    }
    // the update's grid: one 32-byte slice of every column per thread; its A W partials number the same
    const int nbu = dcgs2_update_blocks(ld, (int)sizeof(T), s->nblk);
    launch_dcgs2_reduce(s->partial, nb1, j, k, kz, orth, has_z, s->ctl, st, zskip ? zpart : nullptr, nbu, s->gz);
    if (has_z) {
        ProfEv pe(s, RSOLVE_PROF_UPDATE_DOTS, j, var_of(j + 1), (j + k + 4.0) * w * nn);
        launch_dcgs2_update<T>(ld, V, ld, j, orth ? Wt : Zt, k, u, z, nbu, s->ctl, st, pe.e0, pe.e1, zpart);
    }
}

// The span(W) correction of r (wb[0]) and x: c = M^{-1} Q^T r, x += W c, r -= A W c, then
// ctl->rnorm = ||r||.  Q = W with M = E = W^T A W (the projection guess and the Galerkin
// correction, section 4.2, eq. (projection_t_s)); Q = A W with M = (A W)^T A W (the least-squares
// correction); M's LU factors are those in the control block.
void correct(rsolve_seq* s, const double* Q, int k) {
    hipStream_t st = s->stream;
    if (k > 0) {
        const double* bases[1] = {Q};
        const double* vecs[1] = {s->wb[0]};
        const int counts[1] = {k};
        const int nb = cols_grid(s->ld, s->cus, (k + 7) / 8, 32, k);
        launch_dots<double>(s->ld, s->ld, bases, vecs, counts, 1, s->partial, nb, nullptr, st);
        launch_reduce(s->partial, nb, k, ctl_red(s->ctl), s->ctl, 0, k, true, false, st);
    }
    launch_correct(s->ld, s->W, s->Z, s->ld, k, s->xw, s->wb[0], s->ctl, s->partial, s->nblk, st);
    launch_finish_norm(s->partial, s->nblk, s->ctl, 0, st);
}

// r (wb[0]) = b - A xw, then the span(W) correction with dot basis Q (see correct).
void residual_and_correct(rsolve_seq* s, const rsolve_csr* A, const double* b, int k, const double* Q) {
    launch_residual(s->lpr, s->n, A->row_ptr, A->col_idx, A->val, s->xw, b, s->wb[0], s->stream);
    correct(s, Q, k);
}

// SVD step of Algorithm 1 on an n x c matrix X (section 5.2): TSQR of X to one c x c R factor,
// one-sided Jacobi SVD of R, then W_out = X V_k Sigma_k^{-1} re-orthonormalised by the Cholesky
// factor of its Gram matrix, k_eff = min(kmax, rank) with the rank cut sigma_i > sigma_1 max(n, c)
// eps (the k_eff smallest above the cut when `smallest`).  The singular values land in s->hsig;
// Wr (nullable) receives W row-major with leading dimension ldr.  Synchronous (two read-backs).
int svd_basis_dev(rsolve_seq* s, const double* X, int64_t ldx, int c, int kmax, bool smallest, double* W_out,
                  int64_t ldw, double* Wr, int ldr, int* keff_out, int* rank_out, int* nonfinite, int* lu_fail,
                  float* W32_out = nullptr) {
    hipStream_t stm = s->stream;
    const int64_t n = s->n, ld = s->ld;
    const double* M = X;
    int64_t ldm = ldx, rows = n;
    int lvl = 0;
    const double* R = nullptr;
    for (;;) {
        const int pr = tsqr_panel_rows(c);
        const int P = (int)((rows + pr - 1) / pr);
        double* out = s->tsq[lvl & 1];
        launch_tsqr_level(rows, M, ldm, c, out, s->tsq_ld, P, stm);
        R = out;
        if (P == 1) break;
        M = out;
        ldm = s->tsq_ld;
        rows = (int64_t)P * c;
        ++lvl;
    }
    HIP_TRY(hipMemsetAsync(s->ctl, 0, CTL_HEAD, stm));
    launch_jacobi_svd(R, s->tsq_ld, c, kmax, n, s->ctl, stm, smallest);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(s->hsig, ctl_sigma(s->ctl), sizeof(double) * c, hipMemcpyDeviceToHost, stm));
    int rc = read_head(s);
    if (rc) return rc;
    *rank_out = s->hctl->rank;
    *nonfinite = s->hctl->nonfinite;
    *lu_fail = 0;
    const int keff = s->hctl->nonfinite ? 0 : s->hctl->k_eff;
    *keff_out = keff;
    if (keff > 0) {
        launch_form_w(n, ld, X, ldx, c, keff, s->ctl, W_out, ldw, stm);
        const int gb = launch_gram_tn(ld, W_out, ldw, keff, W_out, ldw, keff, s->gpart, s->gblk, stm);
        launch_gram_reduce(s->gpart, gb, keff * keff, ctl_red(s->ctl), stm);
        launch_cholesky(keff, s->ctl, stm);
        launch_trsm_rows(ld, W_out, ldw, keff, s->ctl, stm, Wr, ldr, W32_out);
        HIP_TRY(hipGetLastError());
        rc = read_head(s);
        if (rc) return rc;
        *lu_fail = s->hctl->lu_fail;
    }
    return RSOLVE_OK;
}

// Ritz or harmonic Ritz recycle basis for the next solve (section 5.1), prepared at the end of a
// solve while A is valid: U = [W, D^{-1} V_j] (the solve's W and the x-space directions of its
// last cycle), Q = an orthonormal basis of span(U) (its SVD, rank cut), A Q by sparse products,
// the small (generalised) eigenproblem on the device, the kept pairs' real basis Q T, and its
// orthonormal basis (SVD again) into rz_w.  W itself changes in rsolve_update_recycle.
int ritz_prepare(rsolve_seq* s, const rsolve_csr* A, int kw) {
    const rsolve_config& c = s->cfg;
    hipStream_t stm = s->stream;
    const int64_t n = s->n, ld = s->ld;
    const int j = s->last_steps;
    s->rz_pending = false;
    if (j < 1) return RSOLVE_OK;   // no Krylov step: keep W
    const int cu = kw + j;
    if (kw > 0) HIP_TRY(hipMemcpyAsync(s->rz_u, s->W, sizeof(double) * ld * kw, hipMemcpyDeviceToDevice, stm));
    const double* dv = c.precond == RSOLVE_PRECOND_JACOBI ? s->dinv : nullptr;
    if (c.precision == RSOLVE_FP32_IR) launch_scale_cols<float>(n, ld, s->V32, j, dv, s->rz_u + (int64_t)kw * ld, ld, stm);
    else launch_scale_cols<double>(n, ld, s->V, j, dv, s->rz_u + (int64_t)kw * ld, ld, stm);
    int r = 0, rank = 0, bad = 0, luf = 0;
    int rc = svd_basis_dev(s, s->rz_u, ld, cu, cu, false, s->rz_q, ld, nullptr, 0, &r, &rank, &bad, &luf);
    if (rc) return rc;
    if (bad) {
        set_err("non-finite search space");
        return RSOLVE_E_NONFINITE;
    }
    int keep = 0;
    if (r > 0 && !luf) {
        for (int i = 0; i < r; ++i)
            launch_spmv(s->lpr, n, A->row_ptr, A->col_idx, A->val, s->rz_q + (int64_t)i * ld, s->rz_aq + (int64_t)i * ld,
                        stm);
        const bool harm = c.select == RSOLVE_SELECT_HARMONIC;
        double* Ga = s->rz_g;
        double* Gb = s->rz_g + SMAX * SMAX;
        const double* left = harm ? s->rz_aq : s->rz_q;
        int gb = launch_gram_tn(ld, left, ld, r, s->rz_aq, ld, r, s->gpart, s->gblk, stm);
        launch_gram_reduce(s->gpart, gb, r * r, Ga, stm);
        if (harm) {
            gb = launch_gram_tn(ld, s->rz_aq, ld, r, s->rz_q, ld, r, s->gpart, s->gblk, stm);
            launch_gram_reduce(s->gpart, gb, r * r, Gb, stm);
        }
        HIP_TRY(hipMemsetAsync(s->ctl, 0, CTL_HEAD, stm));
        launch_small_eig(Ga, Gb, r, c.recycle_k, harm ? 1 : 0, s->rz_eig, s->ctl, stm);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(s->hsig, ctl_sigma(s->ctl), sizeof(double) * SMAX, hipMemcpyDeviceToHost, stm));
        rc = read_head(s);
        if (rc) return rc;
        const int kk = s->hctl->lu_fail ? 0 : s->hctl->k_eff;
        for (int i = 0; i < kk; ++i) s->rz_theta[i] = s->hsig[i];
        if (kk > 0) {
            launch_form_w(n, ld, s->rz_q, ld, r, kk, s->ctl, s->rz_tmp, ld, stm);
            rc = svd_basis_dev(s, s->rz_tmp, ld, kk, kk, false, s->rz_w, ld, nullptr, 0, &keep, &rank, &bad, &luf);
            if (rc) return rc;
            if (bad || luf) keep = 0;
        }
    }
    s->rz_k = keep;
    s->rz_pending = true;
    return RSOLVE_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static_assert(SMALL_MMAX == RSOLVE_SMALL_MAX_RESTART && SMALL_KMAX == RSOLVE_SMALL_MAX_RECYCLE &&
                  SMALL_SMAX == RSOLVE_SMALL_MAX_SNAPSHOTS,
              "one-block limits of the header and the kernels agree");

bool small_solve_ok(const rsolve_seq* s) {
    const rsolve_config& c = s->cfg;
    // the one-block solve implements the oblique projector (or none) only
    return c.precision == RSOLVE_FP64 && c.restart_m <= SMALL_MMAX && c.recycle_k <= SMALL_KMAX &&
           s->n <= RSOLVE_SMALL_MAX_N && c.method <= RSOLVE_DEFL_OBLIQUE && !ritz_mode(c) &&
           c.precond != RSOLVE_PRECOND_SSOR;
}

bool small_update_ok(const rsolve_seq* s) {
    const rsolve_config& c = s->cfg;
    return c.precision == RSOLVE_FP64 && c.snapshots_s <= SMALL_SMAX && c.snapshots_s <= c.restart_m + 1 &&
           s->n >= c.snapshots_s && s->n <= RSOLVE_SMALL_MAX_N && extrap_order(c.method) == 0 && !ritz_mode(c);
}

// Argument checks shared with rsolve_solve; returns RSOLVE_OK or E_INVALID (message set).
int check_solve_args(const rsolve_seq* s, const rsolve_csr* A, const double* b, const double* x, double tol) {
    if (!s || !A || !b || !x) {
        set_err("null argument");
        return RSOLVE_E_INVALID;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_err("tol must be positive and finite");
        return RSOLVE_E_INVALID;
    }
    if (A->n != s->n || A->nnz < A->n || A->nnz > s->nnz_max || !A->row_ptr || !A->col_idx || !A->val ||
        A->reserved != 0) {
        set_err("matrix header does not match the sequence (n=%lld nnz=%lld)", (long long)A->n, (long long)A->nnz);
        return RSOLVE_E_INVALID;
    }
    return RSOLVE_OK;
}

}  // namespace

void rs::seq_set_stream(rsolve_seq* s, hipStream_t st) { s->stream = st; }

void rs::seq_set_offset_classes(rsolve_seq* s, bool on) {
    s->cls_allowed = on;
    if (!on) s->cls_ok = false;
}

extern "C" {

size_t rsolve_workspace_bytes(const rsolve_config* cfg, int64_t n, int64_t nnz_max) {
    if (cfg_check(cfg) != RSOLVE_OK || n < 1 || nnz_max < n || nnz_max > INT32_MAX) return 0;
    return layout(nullptr, *cfg, n, nnz_max, nullptr);
}

int rsolve_create_sequence(const rsolve_config* cfg, int64_t n, int64_t nnz_max, void* hip_stream, void* workspace,
                           size_t ws_bytes, rsolve_seq** out) {
    g_err[0] = 0;
    if (!out) return RSOLVE_E_INVALID;
    *out = nullptr;
    if (cfg_check(cfg) != RSOLVE_OK) {
        set_err("invalid configuration");
        return RSOLVE_E_INVALID;
    }
    if (n < 1 || nnz_max < n || nnz_max > INT32_MAX) {
        set_err("invalid n=%lld / nnz_max=%lld", (long long)n, (long long)nnz_max);
        return RSOLVE_E_INVALID;
    }
    const size_t need = layout(nullptr, *cfg, n, nnz_max, nullptr);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0) {
        set_err("workspace needs %zu bytes (got %zu) aligned to %zu", need, ws_bytes, ALIGN);
        return RSOLVE_E_WORKSPACE;
    }
    rsolve_seq* s = new rsolve_seq();
    s->cfg = *cfg;
    s->n = n;
    s->nnz_max = nnz_max;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->ws = static_cast<char*>(workspace);
    s->ws_bytes = ws_bytes;
    layout(s, *cfg, n, nnz_max, s->ws);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
    s->nblk = pick_nblk(s->ld, s->cus);
    s->gblk = pick_gblk(s->ld);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->hctl), CTL_HEAD + 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->hsig), sizeof(double) * SMAX, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->herr), sizeof(int32_t) * 8, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->poll_done), sizeof(int32_t) * 2, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->hjob), sizeof(SmallJob), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->hupd), sizeof(SmallUpd), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->poll_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->poll_ev[1], hipEventDisableTiming);
    // zero the whole workspace once: padding rows of every tall buffer stay zero forever
    if (e == hipSuccess) e = hipMemsetAsync(s->ws, 0, need, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        set_err("create: %s", hipGetErrorString(e));
        if (s->hctl) (void)hipHostFree(s->hctl);
        if (s->hsig) (void)hipHostFree(s->hsig);
        if (s->herr) (void)hipHostFree(s->herr);
        if (s->poll_done) (void)hipHostFree(s->poll_done);
        if (s->hjob) (void)hipHostFree(s->hjob);
        if (s->hupd) (void)hipHostFree(s->hupd);
        for (auto& ev : s->poll_ev)
            if (ev) (void)hipEventDestroy(ev);
        delete s;
        return RSOLVE_E_DEVICE;
    }
    *out = s;
    return RSOLVE_OK;
}

int rsolve_profile_enable(rsolve_seq* s, int32_t kinds) {
    if (!s || kinds < 0 || (kinds & ~(RSOLVE_PROF_ALL | 0xFF00))) return RSOLVE_E_INVALID;
    s->prof_stride = ((kinds >> 8) & 0xFF) + 1;
    kinds &= RSOLVE_PROF_ALL;
    if (kinds && !s->pev) {
        HIP_TRY(hipSetDevice(s->device));
        const int cnt = rsolve_seq::NPK * MMAX * 2;
        s->pev = new hipEvent_t[cnt]();
        // timing-only events: no system-scope fence, so recording them does not flush caches
        for (int i = 0; i < cnt; ++i) HIP_TRY(hipEventCreateWithFlags(&s->pev[i], hipEventDisableSystemFence));
    }
    s->prof_mask = kinds;
    s->prof_on = kinds != 0;
    return RSOLVE_OK;
}

int rsolve_profile_read(rsolve_seq* s, rsolve_prof_entry* out, int32_t cap, int32_t* count, int32_t reset) {
    if (!s || (cap > 0 && !out)) return RSOLVE_E_INVALID;
    int c = 0;
    for (int kd = 0; kd < rsolve_seq::NPK; ++kd)
        for (int v = 0; v < rsolve_seq::NVAR; ++v) {
            if (s->pcnt[kd][v] == 0) continue;
            if (c < cap) out[c] = rsolve_prof_entry{kd, v, s->pcnt[kd][v], s->pms[kd][v], s->pb[kd][v]};
            ++c;
        }
    if (count) *count = c;
    if (reset) {
        memset(s->pms, 0, sizeof(s->pms));
        memset(s->pb, 0, sizeof(s->pb));
        memset(s->pcnt, 0, sizeof(s->pcnt));
    }
    return RSOLVE_OK;
}

int rsolve_set_spmv_shape(rsolve_seq* s, const rsolve_spmv_shape* shape) {
    if (!s || !shape) return RSOLVE_E_INVALID;
    const int l = shape->lanes_per_row, v = shape->vec, f = shape->format;
    const bool csr_ok = f == RSOLVE_SPMV_CSR && (l == 2 || l == 4 || l == 8 || l == 16 || l == 32) &&
                        (v == 1 || v == 4 || v == 8);
    const bool bp_ok = f == RSOLVE_SPMV_BANDED && (l == 2 || l == 4 || l == 8) && (v == 4 || v == 8);
    if (!(csr_ok || bp_ok) || (shape->xcd_remap != 0 && shape->xcd_remap != 1) || shape->reserved != 0) {
        set_err("invalid SpMV shape (format %d, lanes %d, vec %d, remap %d)", f, l, v, shape->xcd_remap);
        return RSOLVE_E_INVALID;
    }
    s->sfmt = f;
    s->lpr = l;
    s->svec = v;
    s->sremap = shape->xcd_remap;
    s->shape_set = true;
    return RSOLVE_OK;
}

int rsolve_get_spmv_shape(rsolve_seq* s, rsolve_spmv_shape* shape) {
    if (!s || !shape) return RSOLVE_E_INVALID;
    *shape = rsolve_spmv_shape{s->lpr, s->svec, s->sremap, s->shape_set ? 1 : 0, s->sfmt, 0, 0.0};
    return RSOLVE_OK;
}

int rsolve_tune_spmv(rsolve_seq* s, const rsolve_csr* A, int32_t reps, rsolve_spmv_shape* out, int32_t cap,
                     int32_t* count) {
    g_err[0] = 0;
    if (!s || !A || !count || reps < 1 || reps > 1000 || cap < 0 || (cap > 0 && !out)) return RSOLVE_E_INVALID;
    if (A->n != s->n || A->nnz < A->n || A->nnz > s->nnz_max || !A->row_ptr || !A->col_idx || !A->val ||
        A->reserved != 0) {
        set_err("matrix header does not match the sequence");
        return RSOLVE_E_INVALID;
    }
    HIP_TRY(hipSetDevice(s->device));
    hipStream_t stm = s->stream;
    // the candidates read A's indices: check the pattern first, as a solve would (this also
    // picks the default shape, unless the caller set one)
    const int vrc = validate_pattern(s, A);
    if (vrc != RSOLVE_OK) return vrc;
    s->pat_ok = false;     // the next solve checks again (the caller did not promise the pattern)
    const bool ir = s->cfg.precision == RSOLVE_FP32_IR;
    const int64_t n = s->n;
    HIP_TRY(hipMemsetAsync(s->ctl, 0, CTL_HEAD, stm));
    if (ir) launch_scale_values(A->nnz, A->col_idx, A->val, nullptr, nullptr, s->vals32, stm);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_err("event creation failed");
        return RSOLVE_E_DEVICE;
    }
    std::vector<rsolve_spmv_shape> res;
    hipError_t err = hipSuccess;
    auto time_it = [&](auto&& run, rsolve_spmv_shape sh) {
        if (err != hipSuccess) return;
        run();   // warm-up
        err = hipEventRecord(e0, stm);
        for (int r = 0; r < reps && err == hipSuccess; ++r) run();
        if (err == hipSuccess) err = hipEventRecord(e1, stm);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess) err = hipGetLastError();
        sh.us = 1e3 * (double)ms / reps;
        res.push_back(sh);
    };
    for (int l : {2, 4, 8, 16, 32})
        for (int v : {1, 4, 8})
            for (int rm = 0; rm < 2; ++rm)
                time_it(
                    [&] {
                        if (ir)
                            launch_spmv_arnoldi<float>(l, v, rm, n, A->row_ptr, A->col_idx, s->vals32, s->w32[0],
                                                       s->V32, s->w32[1], s->ctl, stm);
                        else
                            launch_spmv_arnoldi<double>(l, v, rm, n, A->row_ptr, A->col_idx, A->val, s->wb[0], s->V,
                                                        s->wb[1], s->ctl, stm);
                    },
                    rsolve_spmv_shape{l, v, rm, 0, RSOLVE_SPMV_CSR, 0, 0.0});
    if (s->band_ok)
        for (int l : {2, 4, 8})
            for (int v : {4, 8}) {
                // lay the copy out for this shape and fill it with A's values
                s->cls_ok = false;
                if (err == hipSuccess && bp_setup(n, A->row_ptr, A->col_idx, v, l, s->bp_p, s->bp_off, s->bp_val, ir,
                                                  reinterpret_cast<int32_t*>(s->partial), PARTIAL_INTS, stm) == 0) {
                    s->bp_e = v;
                    s->bp_l = l;
                    if (cls_build(s, v) != RSOLVE_OK) err = hipErrorUnknown;
                    if (ir) launch_bp_values<float>(n, A->row_ptr, A->col_idx, A->val, nullptr, s->bp_p, v, l,
                                                    static_cast<float*>(s->bp_val), stm);
                    else launch_bp_values<double>(n, A->row_ptr, A->col_idx, A->val, nullptr, s->bp_p, v, l,
                                                  static_cast<double*>(s->bp_val), stm);
                }
                for (int rm = 0; rm < 2; ++rm)
                    time_it(
                        [&] {
                            if (ir && s->cls_ok)
                                launch_spmv_bc<float>(v, l, rm, n, s->bp_p, s->cls_first, s->cls_dict,
                                                      static_cast<const float*>(s->bp_val), s->w32[0], s->V32,
                                                      s->w32[1], s->ctl, stm);
                            else if (ir)
                                launch_spmv_bp<float>(v, l, rm, n, s->bp_p, s->bp_off,
                                                      static_cast<const float*>(s->bp_val), s->w32[0], s->V32,
                                                      s->w32[1], s->ctl, stm);
                            else if (s->cls_ok)
                                launch_spmv_bc<double>(v, l, rm, n, s->bp_p, s->cls_first, s->cls_dict,
                                                       static_cast<const double*>(s->bp_val), s->wb[0], s->V,
                                                       s->wb[1], s->ctl, stm);
                            else
                                launch_spmv_bp<double>(v, l, rm, n, s->bp_p, s->bp_off,
                                                       static_cast<const double*>(s->bp_val), s->wb[0], s->V,
                                                       s->wb[1], s->ctl, stm);
                        },
                        rsolve_spmv_shape{l, v, rm, 0, RSOLVE_SPMV_BANDED, 0, 0.0});
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) {
        set_err("tuning run failed: %s", hipGetErrorString(err));
        return RSOLVE_E_DEVICE;
    }
    std::stable_sort(res.begin(), res.end(),
                     [](const rsolve_spmv_shape& a, const rsolve_spmv_shape& b) { return a.us < b.us; });
    for (int i = 0; i < std::min<int>(cap, (int)res.size()); ++i) out[i] = res[i];
    *count = (int32_t)res.size();
    return RSOLVE_OK;
}

int rsolve_enable_graphs(rsolve_seq* s, int32_t on) {
    if (!s || (on != 0 && on != 1)) return RSOLVE_E_INVALID;
    s->graphs_on = on != 0;
    return RSOLVE_OK;
}

int rsolve_graph_counts(rsolve_seq* s, int64_t* captures, int64_t* launches) {
    if (!s) return RSOLVE_E_INVALID;
    if (captures) *captures = s->graph_captures;
    if (launches) *launches = s->graph_launches;
    return RSOLVE_OK;
}

int rsolve_destroy_sequence(rsolve_seq* s) {
    if (!s) return RSOLVE_E_INVALID;
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->pev) {
        for (int i = 0; i < rsolve_seq::NPK * MMAX * 2; ++i)
            if (s->pev[i]) (void)hipEventDestroy(s->pev[i]);
        delete[] s->pev;
    }
    if (s->hctl) (void)hipHostFree(s->hctl);
    if (s->hsig) (void)hipHostFree(s->hsig);
    if (s->herr) (void)hipHostFree(s->herr);
    if (s->poll_done) (void)hipHostFree(s->poll_done);
    if (s->hjob) (void)hipHostFree(s->hjob);
    if (s->hupd) (void)hipHostFree(s->hupd);
    for (auto& ev : s->poll_ev)
        if (ev) (void)hipEventDestroy(ev);
    delete s;
    return RSOLVE_OK;
}

int rsolve_solve(rsolve_seq* s, const rsolve_csr* A, const double* b, const double* x0, double* x, double tol,
                 rsolve_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    g_err[0] = 0;
    if (!s || !A || !b || !x) {
        set_err("null argument");
        return RSOLVE_E_INVALID;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_err("tol must be positive and finite");
        return RSOLVE_E_INVALID;
    }
    if (A->n != s->n || A->nnz < A->n || A->nnz > s->nnz_max || !A->row_ptr || !A->col_idx || !A->val ||
        A->reserved != 0) {
        set_err("matrix header does not match the sequence (n=%lld nnz=%lld)", (long long)A->n, (long long)A->nnz);
        return RSOLVE_E_INVALID;
    }
    HIP_TRY(hipSetDevice(s->device));
    hipStream_t stm = s->stream;
    const int64_t n = s->n, ld = s->ld;
    const rsolve_config& c = s->cfg;
    const bool ir = c.precision == RSOLVE_FP32_IR;
    const bool jac = c.precond == RSOLVE_PRECOND_JACOBI;
    s->have_x = false;

    // a1: pattern validation (device) unless the caller vouches for an unchanged pattern
    const bool same = (A->flags & RSOLVE_SAME_PATTERN) && s->pat_ok && s->pat_rp == A->row_ptr &&
                      s->pat_ci == A->col_idx && s->pat_nnz == A->nnz;
    if (!same) {
        const int vrc = validate_pattern(s, A);
        if (vrc != RSOLVE_OK) return vrc;
    }
    HIP_TRY(hipMemsetAsync(s->ctl, 0, CTL_HEAD, stm));
    s->nnz_cur = A->nnz;
    s->last_steps = 0;
    s->rz_pending = false;

    // ||b||
    launch_norm2(n, b, s->partial, s->nblk, stm);
    launch_finish_norm(s->partial, s->nblk, s->ctl, 1, stm);

    // a1: Jacobi scaling A D^{-1} (and the FP32 copy in mixed mode)
    // into the Arnoldi product's operand: the banded copy, or CSR values (the caller's FP64
    // values when neither scaling nor conversion is needed)
    if (jac) launch_diag_inv(n, s->diag_pos, A->val, s->dinv, stm);
    const double* dv = jac ? s->dinv : nullptr;
    SpOp op{RSOLVE_SPMV_CSR, A->row_ptr, A->col_idx, nullptr, A->val};
    if (s->sfmt == RSOLVE_SPMV_BANDED && !s->ssor) {
        const int brc = bp_prepare(s, A, dv, ir);
        if (brc) return brc;
        op = SpOp{RSOLVE_SPMV_BANDED, s->bp_p, nullptr, s->bp_off, s->bp_val};
    } else if (ir) {
        launch_scale_values(A->nnz, A->col_idx, A->val, dv, nullptr, s->vals32, stm);
        op.vals = s->vals32;
    } else if (jac) {
        launch_scale_values(A->nnz, A->col_idx, A->val, dv, s->vals, nullptr, stm);
        op.vals = s->vals;
    }

    // a2: recycle setup A W, E = W^T A W, LU(E)
    int k = (c.method != RSOLVE_PLAIN) ? s->k_w : 0;   // always 0 for the extrapolation methods
    uint32_t flags = 0;
    if (k > 0) {
        if (!s->wr_ok) {   // W came from the one-block update, which keeps no row-major copy
            launch_to_rows(n, s->W, ld, k, s->Wr, s->ldr, stm);
            s->wr_ok = true;
        }
        // A W, and in mixed precision its float copy for the inner cycles, in one pass
        launch_spmm_rows(n, A->row_ptr, A->col_idx, A->val, s->Wr, s->ldr, k, s->Z, ld, stm, ir ? s->Z32 : nullptr);
        const int gb = launch_gram_tn(ld, s->W, ld, k, s->Z, ld, k, s->gpart, s->gblk, stm);
        launch_gram_reduce(s->gpart, gb, k * k, ctl_red(s->ctl), stm);
        launch_small_lu(ctl_red(s->ctl), k, s->ctl, stm);
    }
    // a3: r = b - A x0, x0 the caller's or (extrapolation methods, once solutions are stored) the
    // extrapolation of the most recent ones: order min(q, stored), weights (-1)^{j+1} C(order, j)
    const int q_ext = extrap_order(c.method);
    const int stored = (int)std::min<int64_t>(s->count, c.snapshots_s);
    if (q_ext && stored > 0) {
        Extrap e{};
        e.q = std::min(q_ext, stored);
        int64_t binom = 1;
        for (int j = 0; j < e.q; ++j) {
            binom = binom * (e.q - j) / (j + 1);   // C(q, j + 1)
            const int64_t slot = (s->count - 1 - j) % c.snapshots_s;
            e.x[j] = s->X + slot * ld;
            e.w[j] = (j % 2 == 0) ? (double)binom : -(double)binom;
        }
        launch_extrapolate(n, ld, e, s->xw, stm);
    } else {
        launch_copy_pad(n, ld, x0, s->xw, stm);
    }
    HIP_TRY(hipGetLastError());
    int rc = read_head(s);
    if (rc) return rc;
    const double bnorm = s->hctl->bnorm;
    if (!std::isfinite(bnorm)) {
        set_err("non-finite right-hand side");
        return RSOLVE_E_NONFINITE;
    }
    if (bnorm == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, stm));
        HIP_TRY(hipMemsetAsync(s->xw, 0, sizeof(double) * ld, stm));
        HIP_TRY(hipStreamSynchronize(stm));
        s->have_x = true;
        if (st) {
            memset(st, 0, sizeof(*st));
            st->converged = 1;
            st->t_total_ms = ms_since(t0);
        }
        return RSOLVE_OK;
    }
    if (k > 0 && (s->hctl->lu_fail || !(s->hctl->cond1 <= 1e13))) {
        k = 0;
        flags |= RSOLVE_FLAG_RECYCLE_DROPPED;
    }
    residual_and_correct(s, A, b, k, s->W);
    HIP_TRY(hipGetLastError());
    // the projection-guess method uses W for the guess only: plain Krylov cycles (kry = 0)
    int kry = (c.method == RSOLVE_GUESS_PROJECT) ? 0 : k;
    // least-squares projector: once the guess has used E, the control block's factors become
    // those of (A W)^T A W (symmetric positive definite for A W of full rank), which the Arnoldi
    // reductions and the cycle-end correction then apply, with A W in the place of W in the dots
    const bool ls = c.method == RSOLVE_AUG_LS || c.method == RSOLVE_DEFL_LS;
    if (ls && kry > 0) {
        const int gb = launch_gram_tn(ld, s->Z, ld, kry, s->Z, ld, kry, s->gpart, s->gblk, stm);
        launch_gram_reduce(s->gpart, gb, kry * kry, ctl_red(s->ctl), stm);
        launch_small_lu(ctl_red(s->ctl), kry, s->ctl, stm);
        HIP_TRY(hipGetLastError());
    }
    // delayed scheme with the oblique projector: G = (A W)^T A W, with which the column sums turn
    // the update's dots of A W into (A W)^T u for the next step
    if (!ls && kry > 0 && s->zpart && c.ortho == RSOLVE_ORTHO_DCGS2 && c.method != RSOLVE_AUG_ORTHO &&
        c.method != RSOLVE_DEFL_ORTHO) {
        const int gb = launch_gram_tn(ld, s->Z, ld, kry, s->Z, ld, kry, s->gpart, s->gblk, stm);
        launch_gram_reduce(s->gpart, gb, kry * kry, s->gz, stm);
        HIP_TRY(hipGetLastError());
    }
    const double* Qd = ls ? s->Z : s->W;   // dot basis of the cycle-end correction
    const double stop_abs = tol * bnorm;
    const double t_setup = ms_since(t0);

    int its = 0, cycles = 0;
    int its_est = -1;   // steps when a cycle first ended with its estimate within tol ||b||
    bool converged = false;
    int status = RSOLVE_OK;
    double gimp = 0.0;
    const int m = c.restart_m;
    const float* W32 = s->W32;
    const float* Z32 = s->Z32;
    bool head_fresh = false;   // the control block's head was read after the last enqueued work
    for (;;) {
        if (!head_fresh) {
            rc = read_head(s);
            if (rc) return rc;
        }
        head_fresh = false;
        const double rnorm = s->hctl->rnorm;
        if (s->hctl->nonfinite || !std::isfinite(rnorm)) {
            flags |= RSOLVE_FLAG_NONFINITE;
            status = RSOLVE_E_NONFINITE;
            set_err("non-finite value in the iteration");
            break;
        }
        if (rnorm <= stop_abs) {
            converged = true;
            if (its_est < 0 && cycles == 0) its_est = 0;
            break;
        }
        if (its >= c.max_iters) {
            status = RSOLVE_NOT_CONVERGED;
            break;
        }
        if (cycles == 0 && ls && kry > 0) {
            if (s->hctl->lu_fail) {   // (A W)^T A W numerically singular: plain cycles from here
                kry = 0;
                flags |= RSOLVE_FLAG_RECYCLE_DROPPED;
            } else if (c.method == RSOLVE_DEFL_LS) {
                // deflated LS: the Krylov initial vector P_LS r, taken as the least-squares
                // correction of x and r (the final residual, hence x, is the same as projecting
                // only the initial vector, since P_LS is idempotent)
                correct(s, s->Z, kry);
                HIP_TRY(hipGetLastError());
            }
        }
        const int max_steps = std::min(m, c.max_iters - its);
        const double cyc_stop = ir ? std::max(c.inner_tol * rnorm, stop_abs) : stop_abs;
        const bool dg = c.ortho == RSOLVE_ORTHO_DCGS2;
        const bool orth = c.method == RSOLVE_AUG_ORTHO || c.method == RSOLVE_DEFL_ORTHO;
        // the least-squares projector takes A W where the oblique one takes W (dots) as well
        const double* Wd = ls ? s->Z : s->W;
        const float* Wf = ls ? Z32 : W32;
        launch_cycle_init(s->ctl, max_steps, cyc_stop, stm, dg);
        if (ir) launch_to_f32(ld, s->wb[0], s->w32[0], stm);
        // Enqueue the cycle in chunks; after chunk c the done flag is copied to pinned memory, and
        // before chunk c + 2 is enqueued the host waits for chunk c (chunk c + 1 keeps the GPU busy),
        // so at most two chunks of early-exiting kernels follow the step that converges.  Chunks of
        // four steps, or of two when the sequence's last cycle took at most 12: there the steps after
        // the stop are a large share of the launches (Q1 32x32, about 7 steps a solve: 6 and 19
        // percent more solves/s recycled and plain), while on longer cycles the extra waits of short
        // chunks cost more than they save (Q1 64x64 with Jacobi, 29-53 steps: 6 percent slower).
        // with delayed reorthogonalisation step max_steps closes the last column (no product)
        const int nsteps = dg ? max_steps + 1 : max_steps;
        const int CHUNK = (s->cycle_hint > 0 && s->cycle_hint <= 12) ? 2 : 4;
        int chunk = 0;
        for (int j0 = 0; j0 < nsteps; j0 += CHUNK, ++chunk) {
            if (chunk >= 2) {
                HIP_TRY(hipEventSynchronize(s->poll_ev[chunk & 1]));
                if (s->poll_done[chunk & 1]) break;
            }
            const int j1 = std::min(nsteps, j0 + CHUNK);
            auto enqueue = [&] {
                for (int j = j0; j < j1; ++j) {
                    if (dg) {
                        if (ir) dcgs2_step<float>(s, j, max_steps, op, s->V32, s->w32, Wf, Z32, kry, orth, ls);
                        else dcgs2_step<double>(s, j, max_steps, op, s->V, s->wb, Wd, s->Z, kry, orth, ls);
                    } else {
                        if (ir) arnoldi_step<float>(s, j, op, s->V32, s->w32, Wf, Z32, kry, orth);
                        else arnoldi_step<double>(s, j, op, s->V, s->wb, Wd, s->Z, kry, orth);
                    }
                }
            };
            if (s->graphs_on && !s->prof_on && !s->ssor) {
                const rsolve_seq::GraphKey key{j0,      j1,         kry,       ir ? 1 : 0, s->lpr, s->svec, s->sremap,
                                               op.fmt,  (dg ? 1 : 0) | (orth ? 2 : 0) | (ls ? 4 : 0) | (s->cls_ok ? 8 : 0),
                                               dg ? max_steps : 0, op.rp, op.ci,
                                               op.off,  op.vals};
                hipGraphExec_t ge = nullptr;
                rc = chunk_graph(s, key, enqueue, &ge);
                if (rc) return rc;
                HIP_TRY(hipGraphLaunch(ge, stm));
                s->graph_launches++;
            } else {
                enqueue();
            }
            if (j1 < nsteps) {
                HIP_TRY(hipMemcpyAsync(s->poll_done + (chunk & 1), reinterpret_cast<char*>(s->ctl) + offsetof(Ctl, done),
                                       sizeof(int32_t), hipMemcpyDeviceToHost, stm));
                HIP_TRY(hipEventRecord(s->poll_ev[chunk & 1], stm));
            }
        }
        launch_cycle_solve(s->ctl, stm);
        if (ir) {
            launch_x_update<float>(n, s->V32, ld, jac ? s->dinv : nullptr, s->xw, s->ctl, stm);
        } else if (s->ssor) {
            // x += M^{-1} (V y): V y into ss_u, the sweeps (not stopped by the cycle's done flag)
            launch_fill(n, s->ss_u, 0.0, stm);
            launch_x_update<double>(n, s->V, ld, nullptr, s->ss_u, s->ctl, stm);
            launch_ssor_apply(s->sp, A->row_ptr, A->col_idx, A->val, s->diag_pos, s->ss_u, s->ss_t, nullptr,
                              nullptr, stm);
            launch_axpy(n, s->ss_t, s->xw, stm);
        } else {
            launch_x_update<double>(n, s->V, ld, jac ? s->dinv : nullptr, s->xw, s->ctl, stm);
        }
        residual_and_correct(s, A, b, kry, Qd);
        HIP_TRY(hipGetLastError());
        rc = read_head(s);
        if (rc) return rc;
        head_fresh = true;
        prof_collect(s, s->hctl->steps);
        its += s->hctl->steps;
        s->last_steps = s->hctl->steps;
        if (s->hctl->steps > 0) s->cycle_hint = s->hctl->steps;
        cycles += 1;
        gimp = s->hctl->gimp;
        if (its_est < 0 && s->hctl->steps > 0 && gimp <= stop_abs) its_est = its;
        if (s->hctl->lucky) flags |= RSOLVE_FLAG_BREAKDOWN_LUCKY;
        if (s->hctl->steps == 0) {
            // a cycle that cannot take a step cannot make progress
            status = RSOLVE_NOT_CONVERGED;
            break;
        }
    }
    HIP_TRY(hipMemcpyAsync(x, s->xw, sizeof(double) * n, hipMemcpyDeviceToDevice, stm));
    HIP_TRY(hipStreamSynchronize(stm));
    s->have_x = true;
    const double rnorm_final = s->hctl->rnorm;
    if (ritz_mode(c) && c.recycle_k > 0 && status != RSOLVE_E_NONFINITE) {
        rc = ritz_prepare(s, A, s->k_w);
        if (rc) return rc;
    }
    if (st) {
        st->iterations = its;
        st->cycles = cycles;
        st->k_eff = k;
        st->converged = converged ? 1 : 0;
        st->flags = flags;
        st->its_estimate_met = its_est;
        st->rel_res_true = rnorm_final / bnorm;
        st->rel_res_implicit = gimp / bnorm;
        st->t_setup_ms = t_setup;
        st->t_total_ms = ms_since(t0);
        st->t_cycles_ms = st->t_total_ms - t_setup;
    }
    return status;
}

int rsolve_update_recycle(rsolve_seq* s, const double* x) {
    g_err[0] = 0;
    if (!s) return RSOLVE_E_INVALID;
    const double* src = x;
    if (!src) {
        if (!s->have_x) {
            set_err("no solution to store yet");
            return RSOLVE_E_STATE;
        }
        src = s->xw;
    }
    const rsolve_config& c = s->cfg;
    const bool extrap = extrap_order(c.method) != 0;
    if (ritz_mode(c)) {
        // the basis the last solve prepared from its search space (x itself is not stored)
        s->count++;
        if (!s->rz_pending) return RSOLVE_OK;
        HIP_TRY(hipSetDevice(s->device));
        const int kk = s->rz_k;
        if (kk > 0) {
            HIP_TRY(hipMemcpyAsync(s->W, s->rz_w, sizeof(double) * s->ld * kk, hipMemcpyDeviceToDevice, s->stream));
            if (s->W32) launch_to_f32(kk * s->ld, s->W, s->W32, s->stream);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipStreamSynchronize(s->stream));
        s->wr_ok = false;
        for (int i = 0; i < kk; ++i) s->sigma[i] = s->rz_theta[i];
        s->nsig = kk;
        s->rank = kk;
        s->k_w = kk;
        s->rz_pending = false;
        return RSOLVE_OK;
    }
    if ((c.recycle_k == 0 && !extrap) || c.snapshots_s == 0) {
        s->count++;
        return RSOLVE_OK;
    }
    HIP_TRY(hipSetDevice(s->device));
    hipStream_t stm = s->stream;
    const int64_t n = s->n, ld = s->ld;
    const int slot = (int)(s->count % c.snapshots_s);
    HIP_TRY(hipMemcpyAsync(s->X + (int64_t)slot * ld, src, sizeof(double) * n, hipMemcpyDeviceToDevice, stm));
    s->count++;
    if (extrap || s->count % c.svd_interval != 0) {   // the extrapolation methods keep the ring only
        HIP_TRY(hipStreamSynchronize(stm));
        return RSOLVE_OK;
    }
    const int cc = (int)std::min<int64_t>(s->count, c.snapshots_s);
    int keff = 0, rank = 0, bad = 0, lu_fail = 0;
    // the re-orthonormalised W is also written rounded to float (the inner cycles' copy in mixed precision)
    int rc = svd_basis_dev(s, s->X, ld, cc, c.recycle_k, c.select == RSOLVE_SELECT_SMALLEST, s->W, ld, s->Wr,
                           s->ldr, &keff, &rank, &bad, &lu_fail, s->W32);
    if (rc) return rc;
    for (int i = 0; i < cc; ++i) s->sigma[i] = s->hsig[i];
    s->nsig = cc;
    s->rank = rank;
    if (bad) {
        s->k_w = 0;
        set_err("non-finite snapshot");
        return RSOLVE_E_NONFINITE;
    }
    if (keff > 0) {
        s->wr_ok = true;
        HIP_TRY(hipGetLastError());
        if (lu_fail) {
            s->k_w = 0;
            return RSOLVE_OK;
        }
    }
    s->k_w = keff;
    return RSOLVE_OK;
}

int rsolve_solve_batch(rsolve_batch_solve_item* items, int32_t count, void* hip_stream) {
    const auto t0 = std::chrono::steady_clock::now();
    g_err[0] = 0;
    if (count < 0 || (count > 0 && !items)) {
        set_err("invalid batch");
        return RSOLVE_E_INVALID;
    }
    if (count == 0) return RSOLVE_OK;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    // 0 = invalid, 1 = one-block launch, 2 = multi-kernel path
    std::vector<int> route(count, 0);
    std::vector<int> small;
    for (int i = 0; i < count; ++i) {
        rsolve_batch_solve_item& it = items[i];
        it.status = RSOLVE_E_INVALID;
        memset(&it.stats, 0, sizeof(it.stats));
        if (check_solve_args(it.seq, &it.A, it.b, it.x, it.tol) != RSOLVE_OK) continue;
        if (it.seq->device != dev) continue;
        bool dup = false;
        for (int q = 0; q < i && !dup; ++q) dup = route[q] != 0 && items[q].seq == it.seq;
        if (dup) continue;
        route[i] = small_solve_ok(it.seq) ? 1 : 2;
        if (route[i] == 1) small.push_back(i);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (!st && !small.empty()) st = items[small[0]].seq->stream;
    for (size_t b0 = 0; b0 < small.size(); b0 += SMALL_BATCH) {
        SmallBatch batch{};
        const int cnt = (int)std::min<size_t>(SMALL_BATCH, small.size() - b0);
        for (int q = 0; q < cnt; ++q) {
            rsolve_batch_solve_item& it = items[small[b0 + q]];
            rsolve_seq* s = it.seq;
            const rsolve_config& c = s->cfg;
            const bool same = (it.A.flags & RSOLVE_SAME_PATTERN) && s->spat_rp == it.A.row_ptr &&
                              s->spat_ci == it.A.col_idx && s->spat_nnz == it.A.nnz;
            SmallJob& J = *s->hjob;
            memset(&J, 0, sizeof(J));
            J.n = s->n;
            J.nnz = it.A.nnz;
            J.ld = s->ld;
            J.rp = it.A.row_ptr;
            J.ci = it.A.col_idx;
            J.val = it.A.val;
            J.b = it.b;
            J.x0 = it.x0;
            J.x = it.x;
            J.tol = it.tol;
            J.m = c.restart_m;
            J.k = (c.method != RSOLVE_PLAIN) ? s->k_w : 0;
            J.max_iters = c.max_iters;
            J.jacobi = c.precond == RSOLVE_PRECOND_JACOBI ? 1 : 0;
            J.validate = same ? 0 : 1;
            J.W = s->W;
            J.Z = s->Z;
            J.V = s->V;
            J.w = s->wb[0];
            J.r = s->wb[1];
            J.xw = s->xw;
            J.dinv = s->dinv;
            J.vals = s->vals;
            J.F = s->partial;
            J.status = RSOLVE_E_DEVICE;
            batch.job[q] = s->hjob;
            // the multi-kernel path keeps its own pattern cache (with the diagonal positions)
            s->pat_ok = false;
            s->have_x = false;
        }
        launch_small_solve(batch, cnt, st);
        HIP_TRY(hipGetLastError());
    }
    // items outside the one-block limits: the multi-kernel path, while the launch runs
    for (int i = 0; i < count; ++i) {
        if (route[i] != 2) continue;
        rsolve_batch_solve_item& it = items[i];
        it.status = rsolve_solve(it.seq, &it.A, it.b, it.x0, it.x, it.tol, &it.stats);
    }
    if (!small.empty()) HIP_TRY(hipStreamSynchronize(st));
    const double total = ms_since(t0);
    for (int i : small) {
        rsolve_batch_solve_item& it = items[i];
        rsolve_seq* s = it.seq;
        const SmallJob& J = *s->hjob;
        it.status = J.status;
        if (J.status == RSOLVE_OK || J.status == RSOLVE_NOT_CONVERGED) {
            s->spat_rp = it.A.row_ptr;
            s->spat_ci = it.A.col_idx;
            s->spat_nnz = it.A.nnz;
            s->have_x = true;
            s->nnz_cur = it.A.nnz;
        } else if (J.status == RSOLVE_E_INVALID) {
            s->spat_nnz = -1;
        }
        rsolve_stats& o = it.stats;
        o.iterations = J.iterations;
        o.cycles = J.cycles;
        o.k_eff = J.k_used;
        o.converged = J.converged;
        o.its_estimate_met = J.converged ? J.iterations : -1;
        o.flags = J.flags;
        o.rel_res_true = J.bnorm > 0.0 ? J.rnorm / J.bnorm : 0.0;
        o.rel_res_implicit = J.bnorm > 0.0 ? J.gimp / J.bnorm : 0.0;
        o.t_setup_ms = 0.0;
        o.t_cycles_ms = total;
        o.t_total_ms = total;
    }
    return RSOLVE_OK;
}

int rsolve_update_recycle_batch(rsolve_batch_update_item* items, int32_t count, void* hip_stream) {
    g_err[0] = 0;
    if (count < 0 || (count > 0 && !items)) {
        set_err("invalid batch");
        return RSOLVE_E_INVALID;
    }
    if (count == 0) return RSOLVE_OK;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<int> route(count, 0);
    std::vector<int> small;
    for (int i = 0; i < count; ++i) {
        rsolve_batch_update_item& it = items[i];
        it.status = RSOLVE_E_INVALID;
        rsolve_seq* s = it.seq;
        if (!s || s->device != dev) continue;
        bool dup = false;
        for (int q = 0; q < i && !dup; ++q) dup = route[q] != 0 && items[q].seq == s;
        if (dup) continue;
        if (!it.x && !s->have_x) {
            it.status = RSOLVE_E_STATE;
            continue;
        }
        const rsolve_config& c = s->cfg;
        if ((c.recycle_k == 0 && extrap_order(c.method) == 0) || c.snapshots_s == 0) {
            s->count++;
            it.status = RSOLVE_OK;
            continue;
        }
        route[i] = small_update_ok(s) ? 1 : 2;
        if (route[i] == 1) small.push_back(i);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (!st && !small.empty()) st = items[small[0]].seq->stream;
    for (size_t b0 = 0; b0 < small.size(); b0 += SMALL_BATCH) {
        SmallUpdBatch batch{};
        const int cnt = (int)std::min<size_t>(SMALL_BATCH, small.size() - b0);
        for (int q = 0; q < cnt; ++q) {
            rsolve_batch_update_item& it = items[small[b0 + q]];
            rsolve_seq* s = it.seq;
            const rsolve_config& c = s->cfg;
            SmallUpd& U = *s->hupd;
            memset(&U, 0, sizeof(U));
            s->wr_ok = false;   // this update writes W only
            U.n = s->n;
            U.ld = s->ld;
            U.src = it.x ? it.x : s->xw;
            U.X = s->X;
            U.Q = s->V;
            U.W = s->W;
            U.slot = (int32_t)(s->count % c.snapshots_s);
            U.c = (int32_t)std::min<int64_t>(s->count + 1, c.snapshots_s);
            U.k = c.recycle_k;
            U.svd = ((s->count + 1) % c.svd_interval == 0) ? 1 : 0;
            U.smallest = c.select == RSOLVE_SELECT_SMALLEST ? 1 : 0;
            U.status = RSOLVE_E_DEVICE;
            batch.job[q] = s->hupd;
        }
        launch_small_update(batch, cnt, st);
        HIP_TRY(hipGetLastError());
    }
    for (int i = 0; i < count; ++i) {
        if (route[i] != 2) continue;
        items[i].status = rsolve_update_recycle(items[i].seq, items[i].x);
    }
    if (!small.empty()) HIP_TRY(hipStreamSynchronize(st));
    for (int i : small) {
        rsolve_batch_update_item& it = items[i];
        rsolve_seq* s = it.seq;
        const SmallUpd& U = *s->hupd;
        s->count++;
        it.status = U.status;
        if (!U.svd) continue;
        if (U.status == RSOLVE_OK) {
            s->k_w = U.k_eff;
            s->rank = U.rank;
            s->nsig = U.c;
            for (int q = 0; q < U.c; ++q) s->sigma[q] = U.sigma[q];
        } else {
            s->k_w = 0;
        }
    }
    return RSOLVE_OK;
}

int rsolve_get_recycle(rsolve_seq* s, int32_t* k_eff, int32_t* rank, double* sigma_host, int32_t cap, double* W_out,
                       int64_t ld_out) {
    if (!s) return RSOLVE_E_INVALID;
    if (k_eff) *k_eff = s->k_w;
    if (rank) *rank = s->rank;
    if (sigma_host)
        for (int i = 0; i < std::min<int>(cap, s->nsig); ++i) sigma_host[i] = s->sigma[i];
    if (W_out && s->k_w > 0) {
        if (ld_out < s->n) return RSOLVE_E_INVALID;
        HIP_TRY(hipSetDevice(s->device));
        HIP_TRY(hipMemcpy2DAsync(W_out, sizeof(double) * ld_out, s->W, sizeof(double) * s->ld, sizeof(double) * s->n,
                                 s->k_w, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return RSOLVE_OK;
}

// ---- checkpoint / resume of a sequence's recycling state ----

namespace {

// The state blob: this header, then float64 columns of n values each: W (k_w columns), the
// snapshot ring by slot (ring_cols columns), the last solution (if have_x) and a pending Ritz
// basis (rz_k columns, if rz_pending).  Native byte order; the checksum is FNV-1a over the header
// (its checksum field zero) followed by the columns.
struct StateHeader {
    uint64_t magic;
    uint32_t version, header_bytes;
    int32_t recycle_k, snapshots_s, svd_interval, method, select, precision;
    int64_t n, count;
    int32_t k_w, rank, nsig, have_x;
    int32_t ring_cols, rz_pending, rz_k, shape_set;
    int32_t lpr, svec, sremap, sfmt;
    double sigma[SMAX];
    double rz_theta[SMAX];
    uint64_t payload_bytes, checksum;
};
constexpr uint64_t STATE_MAGIC = 0x31545345564c4f53ull;   // "SOLVEST1"
constexpr uint32_t STATE_VERSION = 1;

// stored solutions of the snapshot ring (the Ritz spaces keep none)
int state_ring_cols(const rsolve_seq* s, int64_t count) {
    return (s->X && !ritz_mode(s->cfg)) ? (int)std::min<int64_t>(count, s->cfg.snapshots_s) : 0;
}

uint64_t state_columns(int ring, int have_x, int rz_pending, int rz_k, int k_w) {
    return (uint64_t)k_w + (uint64_t)ring + (uint64_t)have_x + (rz_pending ? (uint64_t)rz_k : 0);
}

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    return h;
}

uint64_t state_checksum(StateHeader h, const unsigned char* payload) {
    h.checksum = 0;
    return fnv1a(payload, (size_t)h.payload_bytes, fnv1a(reinterpret_cast<const unsigned char*>(&h), sizeof(h)));
}

}  // namespace

size_t rsolve_state_bytes(rsolve_seq* s) {
    if (!s) return 0;
    const uint64_t cols = state_columns(state_ring_cols(s, s->count), s->have_x ? 1 : 0, s->rz_pending ? 1 : 0, s->rz_k,
                                        s->k_w);
    return sizeof(StateHeader) + sizeof(double) * (size_t)s->n * (size_t)cols;
}

int rsolve_export_state(rsolve_seq* s, void* buf, size_t bytes, size_t* written) {
    g_err[0] = 0;
    if (written) *written = 0;
    if (!s || !buf) return RSOLVE_E_INVALID;
    const size_t need = rsolve_state_bytes(s);
    if (bytes < need) {
        set_err("state buffer of %zu bytes, %zu needed", bytes, need);
        return RSOLVE_E_INVALID;
    }
    HIP_TRY(hipSetDevice(s->device));
    StateHeader h{};
    h.magic = STATE_MAGIC;
    h.version = STATE_VERSION;
    h.header_bytes = (uint32_t)sizeof(StateHeader);
    const rsolve_config& c = s->cfg;
    h.recycle_k = c.recycle_k;
    h.snapshots_s = c.snapshots_s;
    h.svd_interval = c.svd_interval;
    h.method = c.method;
    h.select = c.select;
    h.precision = c.precision;
    h.n = s->n;
    h.count = s->count;
    h.k_w = s->k_w;
    h.rank = s->rank;
    h.nsig = s->nsig;
    h.have_x = s->have_x ? 1 : 0;
    h.ring_cols = state_ring_cols(s, s->count);
    h.rz_pending = s->rz_pending ? 1 : 0;
    h.rz_k = s->rz_pending ? s->rz_k : 0;
    h.shape_set = s->shape_set ? 1 : 0;
    h.lpr = s->lpr;
    h.svec = s->svec;
    h.sremap = s->sremap;
    h.sfmt = s->sfmt;
    for (int i = 0; i < SMAX; ++i) {
        h.sigma[i] = i < s->nsig ? s->sigma[i] : 0.0;
        h.rz_theta[i] = i < h.rz_k ? s->rz_theta[i] : 0.0;
    }
    const size_t col = sizeof(double) * (size_t)s->n;
    h.payload_bytes = need - sizeof(StateHeader);
    unsigned char* out = static_cast<unsigned char*>(buf) + sizeof(StateHeader);
    const size_t pitch = sizeof(double) * (size_t)s->ld;
    auto take = [&](const double* src, int cols) -> int {
        if (cols > 0) {
            HIP_TRY(hipMemcpy2DAsync(out, col, src, pitch, col, cols, hipMemcpyDeviceToHost, s->stream));
            out += col * (size_t)cols;
        }
        return RSOLVE_OK;
    };
    int rc = take(s->W, h.k_w);
    if (rc == RSOLVE_OK) rc = take(s->X, h.ring_cols);
    if (rc == RSOLVE_OK) rc = take(s->xw, h.have_x);
    if (rc == RSOLVE_OK && h.rz_pending) rc = take(s->rz_w, h.rz_k);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    h.checksum = state_checksum(h, static_cast<const unsigned char*>(buf) + sizeof(StateHeader));
    std::memcpy(buf, &h, sizeof(h));
    if (written) *written = need;
    return RSOLVE_OK;
}

int rsolve_import_state(rsolve_seq* s, const void* buf, size_t bytes) {
    g_err[0] = 0;
    if (!s || !buf) return RSOLVE_E_INVALID;
    StateHeader h;
    if (bytes < sizeof(h)) {
        set_err("state of %zu bytes is shorter than its header", bytes);
        return RSOLVE_E_INVALID;
    }
    std::memcpy(&h, buf, sizeof(h));
    const rsolve_config& c = s->cfg;
    if (h.magic != STATE_MAGIC || h.version != STATE_VERSION || h.header_bytes != sizeof(StateHeader)) {
        set_err("not a sequence state of this library version");
        return RSOLVE_E_INVALID;
    }
    if (h.n != s->n || h.recycle_k != c.recycle_k || h.snapshots_s != c.snapshots_s ||
        h.svd_interval != c.svd_interval || h.method != c.method || h.select != c.select ||
        h.precision != c.precision) {
        set_err("state of another configuration or size (n %lld, k %d, s %d, method %d)", (long long)h.n,
                h.recycle_k, h.snapshots_s, h.method);
        return RSOLVE_E_INVALID;
    }
    const int ring = state_ring_cols(s, std::max<int64_t>(h.count, 0));
    const bool ranges_ok = h.count >= 0 && h.k_w >= 0 && h.k_w <= c.recycle_k && h.rank >= 0 &&
                           h.nsig >= 0 && h.nsig <= SMAX && (h.have_x == 0 || h.have_x == 1) &&
                           h.ring_cols == ring && (h.rz_pending == 0 || h.rz_pending == 1) && h.rz_k >= 0 &&
                           h.rz_k <= c.recycle_k && (h.rz_pending || h.rz_k == 0) &&
                           (h.shape_set == 0 || h.shape_set == 1);
    const uint64_t cols = ranges_ok ? state_columns(ring, h.have_x, h.rz_pending, h.rz_k, h.k_w) : 0;
    const uint64_t payload = sizeof(double) * (uint64_t)s->n * cols;
    if (!ranges_ok || h.payload_bytes != payload || bytes < sizeof(h) + payload) {
        set_err("inconsistent or truncated sequence state");
        return RSOLVE_E_INVALID;
    }
    const unsigned char* in = static_cast<const unsigned char*>(buf) + sizeof(h);
    if (state_checksum(h, in) != h.checksum) {
        set_err("sequence state checksum mismatch");
        return RSOLVE_E_INVALID;
    }
    if (h.shape_set) {
        const rsolve_spmv_shape shape{h.lpr, h.svec, h.sremap, 1, h.sfmt, 0, 0.0};
        const int rc = rsolve_set_spmv_shape(s, &shape);
        if (rc) return rc;
    }
    HIP_TRY(hipSetDevice(s->device));
    const size_t col = sizeof(double) * (size_t)s->n;
    const size_t pitch = sizeof(double) * (size_t)s->ld;
    auto put = [&](double* dst, int ncols) -> int {
        if (ncols > 0) {
            HIP_TRY(hipMemcpy2DAsync(dst, pitch, in, col, col, ncols, hipMemcpyHostToDevice, s->stream));
            in += col * (size_t)ncols;
        }
        return RSOLVE_OK;
    };
    int rc = put(s->W, h.k_w);
    if (rc == RSOLVE_OK) rc = put(s->X, ring);
    if (rc == RSOLVE_OK) rc = put(s->xw, h.have_x);
    if (rc == RSOLVE_OK && h.rz_pending) rc = put(s->rz_w, h.rz_k);
    if (rc) return rc;
    if (s->W32 && h.k_w > 0) launch_to_f32((int64_t)h.k_w * s->ld, s->W, s->W32, s->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->count = h.count;
    s->k_w = h.k_w;
    s->rank = h.rank;
    s->nsig = h.nsig;
    for (int i = 0; i < SMAX; ++i) s->sigma[i] = h.sigma[i];
    s->have_x = h.have_x != 0;
    s->rz_pending = h.rz_pending != 0;
    s->rz_k = h.rz_k;
    for (int i = 0; i < SMAX; ++i) s->rz_theta[i] = h.rz_theta[i];
    s->wr_ok = false;   // the row-major copy of W is rebuilt by the next solve
    return RSOLVE_OK;
}

const char* rsolve_status_string(int status) {
    switch (status) {
        case RSOLVE_OK: return "ok";
        case RSOLVE_NOT_CONVERGED: return "not converged";
        case RSOLVE_E_INVALID: return "invalid argument";
        case RSOLVE_E_NONFINITE: return "non-finite value";
        case RSOLVE_E_WORKSPACE: return "workspace too small or misaligned";
        case RSOLVE_E_DEVICE: return "HIP runtime error";
        case RSOLVE_E_STATE: return "call out of order";
        case RSOLVE_E_BUDGET: return "no room in the server's pool or slots";
        default: return "unknown status";
    }
}

const char* rsolve_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// kernel-level entry points
// ---------------------------------------------------------------------------

int rsolve_triad(int64_t n, double* a, const double* b, const double* c, double s, void* hip_stream) {
    g_err[0] = 0;
    const auto mis = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; };
    if (n < 1 || !a || !b || !c || mis(a) || mis(b) || mis(c)) return RSOLVE_E_INVALID;
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    launch_triad(n, a, b, c, s, cus, reinterpret_cast<hipStream_t>(hip_stream));
    HIP_TRY(hipGetLastError());
    return RSOLVE_OK;
}

int rsolve_colour_first_fit(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* colour,
                            int32_t* ncolours) {
    g_err[0] = 0;
    if (n < 1 || !row_ptr || !col_idx || !colour || !ncolours || row_ptr[0] != 0) return RSOLVE_E_INVALID;
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return RSOLVE_E_INVALID;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col_idx[e] < 0 || col_idx[e] >= n) return RSOLVE_E_INVALID;
    }
    std::vector<int32_t> rows, coff;
    *ncolours = colour_first_fit(n, row_ptr, col_idx, colour, rows, coff);
    return RSOLVE_OK;
}

int rsolve_spmv(const rsolve_csr* A, const double* x, double* y, void* hip_stream) {
    if (!A || !x || !y || !A->row_ptr || !A->col_idx || !A->val || A->n < 1) return RSOLVE_E_INVALID;
    launch_spmv(pick_lpr(A->n, A->nnz), A->n, A->row_ptr, A->col_idx, A->val, x, y,
                reinterpret_cast<hipStream_t>(hip_stream));
    HIP_TRY(hipGetLastError());
    return RSOLVE_OK;
}

namespace {
struct KWs {
    Ctl* ctl;
    double* gpart;
    double* t0;
    double* t1;
    int64_t tld;
};
size_t kws_layout(int64_t n, int cols, char* base, KWs* o) {
    Carver cv{base};
    Ctl* ctl = cv.take<Ctl>(1);
    double* gp = cv.take<double>((size_t)GRAM_PARTIAL);
    const int64_t rows = ((n + TSQR_MIN_PANEL - 1) / TSQR_MIN_PANEL) * std::max(cols, 1);
    const int64_t tld = pad64(rows);
    double* t0 = cv.take<double>((size_t)tld * std::max(cols, 1));
    double* t1 = cv.take<double>((size_t)tld * std::max(cols, 1));
    if (o) *o = KWs{ctl, gp, t0, t1, tld};
    return align_up(cv.off, ALIGN);
}
}  // namespace

size_t rsolve_kernel_workspace_bytes(int64_t n, int32_t cols) {
    if (n < 1 || cols < 0 || cols > 64) return 0;
    return kws_layout(n, cols, nullptr, nullptr);
}

int rsolve_gram_tn(int64_t n, const double* A, int64_t lda, int32_t p, const double* B, int64_t ldb, int32_t q,
                   double* C_host, void* workspace, size_t ws_bytes, void* hip_stream) {
    if (n < 1 || !A || !B || !C_host || p < 1 || q < 1 || p > 64 || q > 64 || lda < n || ldb < n)
        return RSOLVE_E_INVALID;
    const int cols = std::max(p, q);
    if (!workspace || ws_bytes < kws_layout(n, cols, nullptr, nullptr) ||
        (reinterpret_cast<uintptr_t>(workspace) % ALIGN))
        return RSOLVE_E_WORKSPACE;
    KWs w;
    kws_layout(n, cols, static_cast<char*>(workspace), &w);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int gblk = launch_gram_tn(n, A, lda, p, B, ldb, q, w.gpart, pick_gblk(n), st);
    launch_gram_reduce(w.gpart, gblk, p * q, ctl_red(w.ctl), st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C_host, ctl_red(w.ctl), sizeof(double) * p * q, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RSOLVE_OK;
}

}  // extern "C"

// ---- the Gram product without a workspace argument ----
namespace {
// split-n partial sums (as many as the Gram kernel may write for any p, q <= 64), then the
// reduced p x q result
constexpr size_t NOALLOC_PARTIAL = (size_t)GRAM_PARTIAL;
constexpr size_t NOALLOC_RESULT = (size_t)RSOLVE_GRAM_NOALLOC_MAX_COLS * RSOLVE_GRAM_NOALLOC_MAX_COLS;
static_assert((NOALLOC_PARTIAL + NOALLOC_RESULT) * sizeof(double) == RSOLVE_GRAM_NOALLOC_SCRATCH_BYTES,
              "scratch size stated in the header");
static_assert(RSOLVE_GRAM_NOALLOC_MAX_COLS <= KMAX, "the Gram kernel's column limit");

// One copy per GPU, placed by the loader.  In host code this name stands for the symbol only:
// kernels and copies get the device address taken below.
static __device__ __align__(256) double scratch[NOALLOC_PARTIAL + NOALLOC_RESULT];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per device (with that
// device current) and kept.
int scratch_address(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_err("device %d beyond the %d devices the static scratch table covers", dev, NOALLOC_MAX_DEVICES);
        return RSOLVE_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_err("hipGetSymbolAddress returned no address for the static scratch");
            return RSOLVE_E_DEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return RSOLVE_OK;
}
}  // namespace

extern "C" {

int rsolve_gram_tn_noalloc(int64_t n, const double* A, int64_t lda, int32_t p, const double* B, int64_t ldb,
                           int32_t q, double* C_host, void* hip_stream) {
    g_err[0] = 0;
    if (n < 1 || !A || !B || !C_host || lda < n || ldb < n) {
        set_err("null pointer, n < 1 or leading dimension below n");
        return RSOLVE_E_INVALID;
    }
    if (p < 1 || q < 1 || p > RSOLVE_GRAM_NOALLOC_MAX_COLS || q > RSOLVE_GRAM_NOALLOC_MAX_COLS) {
        set_err("p = %d, q = %d: the static scratch holds products of at most %d x %d", p, q,
                RSOLVE_GRAM_NOALLOC_MAX_COLS, RSOLVE_GRAM_NOALLOC_MAX_COLS);
        return RSOLVE_E_INVALID;
    }
    double* base = nullptr;
    const int rc = scratch_address(&base);
    if (rc) return rc;
    double* partial = base;
    double* result = base + NOALLOC_PARTIAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int gblk = launch_gram_tn(n, A, lda, p, B, ldb, q, partial, pick_gblk(n), st);
    launch_gram_reduce(partial, gblk, p * q, result, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(C_host, result, sizeof(double) * p * q, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RSOLVE_OK;
}

int rsolve_snapshot_svd(int64_t n, const double* X, int64_t ldx, int32_t c, int32_t k, double* W_out, int64_t ldw,
                        double* sigma_host, int32_t* k_eff, int32_t* rank, void* workspace, size_t ws_bytes,
                        void* hip_stream) {
    if (n < 1 || !X || c < 1 || c > 64 || k < 0 || k > 64 || ldx < n || (k > 0 && (!W_out || ldw < n)))
        return RSOLVE_E_INVALID;
    if (!workspace || ws_bytes < kws_layout(n, c, nullptr, nullptr) ||
        (reinterpret_cast<uintptr_t>(workspace) % ALIGN))
        return RSOLVE_E_WORKSPACE;
    KWs w;
    kws_layout(n, c, static_cast<char*>(workspace), &w);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), st));
    const double* M = X;
    int64_t ldm = ldx, rows = n;
    const double* R = nullptr;
    int lvl = 0;
    for (;;) {
        const int pr = tsqr_panel_rows(c);
        const int P = (int)((rows + pr - 1) / pr);
        double* out = (lvl & 1) ? w.t1 : w.t0;
        launch_tsqr_level(rows, M, ldm, c, out, w.tld, P, st);
        R = out;
        if (P == 1) break;
        M = out;
        ldm = w.tld;
        rows = (int64_t)P * c;
        ++lvl;
    }
    launch_jacobi_svd(R, w.tld, c, k, n, w.ctl, st);
    HIP_TRY(hipGetLastError());
    Ctl head;
    HIP_TRY(hipMemcpyAsync(&head, w.ctl, CTL_HEAD, hipMemcpyDeviceToHost, st));
    if (sigma_host) HIP_TRY(hipMemcpyAsync(sigma_host, ctl_sigma(w.ctl), sizeof(double) * c, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (rank) *rank = head.rank;
    if (k_eff) *k_eff = head.k_eff;
    const int keff = head.k_eff;
    if (keff > 0) {
        launch_form_w(n, n, X, ldx, c, keff, w.ctl, W_out, ldw, st);
        const int gblk = launch_gram_tn(n, W_out, ldw, keff, W_out, ldw, keff, w.gpart, pick_gblk(n), st);
        launch_gram_reduce(w.gpart, gblk, keff * keff, ctl_red(w.ctl), st);
        launch_cholesky(keff, w.ctl, st);
        launch_trsm_rows(n, W_out, ldw, keff, w.ctl, st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
    }
    return RSOLVE_OK;
}

}  // extern "C"
