// Host-side memory and undefined-behaviour check of the rsolve C ABI.
//
// build_host_check.py compiles every library source with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host half only (the device code is the library's own), links
// this driver against the objects and runs it as
//   host_check cpu   the entry points that never touch the GPU: the first-fit colouring on random
//                    patterns (checked for properness), argument checks, workspace sizing over a
//                    grid of configurations, status strings;
//   host_check gpu   every entry point on a small convection-diffusion time-stepping sequence: each
//                    valid solver configuration (method x preconditioner x precision x recycle
//                    selection x orthogonalisation), the recycle read-back, a checkpoint moved to a
//                    fresh sequence, profiling, graph replay, the SpMV tuner, batched solves, the
//                    serving loop, the kernel-level calls and the documented error returns.
// Every residual a solve reports is recomputed on the host in float64.  Exit status 0 when all
// checks hold; a sanitizer report ends the run with a non-zero status.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "rsolve.h"
#include "rsolve_kernels.h"
#include "rsolve_server.h"

namespace {

int g_fail = 0;

void fail(const char* what, const std::string& detail) {
    ++g_fail;
    std::printf("FAIL %s: %s (last error: %s)\n", what, detail.c_str(), rsolve_last_error());
    std::fflush(stdout);
}

#define EXPECT(cond, detail)                   \
    do {                                       \
        if (!(cond)) fail(#cond, (detail));    \
    } while (0)

#define HIP_OK(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            std::printf("HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            std::exit(3);                                                            \
        }                                                                            \
    } while (0)

// ---------------------------------------------------------------- host-only phase

bool proper_colouring(int n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                      const std::vector<int32_t>& colour, int nc) {
    for (int i = 0; i < n; ++i) {
        if (colour[i] < 0 || colour[i] >= nc) return false;
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i && colour[ci[e]] == colour[i]) return false;
    }
    return true;
}

void cpu_phase() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 300; ++trial) {
        const int n = 1 + (int)(rng() % 400);
        const double dens = 0.002 + (double)(rng() % 1000) * 1e-4;
        std::vector<int32_t> rp(n + 1, 0), ci;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j)
                if (j == i || (double)(rng() % 100000) * 1e-5 < dens) ci.push_back(j);
            rp[i + 1] = (int32_t)ci.size();
        }
        std::vector<int32_t> colour(n);
        int32_t nc = 0;
        const int rc = rsolve_colour_first_fit(n, rp.data(), ci.data(), colour.data(), &nc);
        EXPECT(rc == RSOLVE_OK, "colouring of trial " + std::to_string(trial));
        if (rc == RSOLVE_OK)
            EXPECT(proper_colouring(n, rp, ci, colour, nc), "colouring of trial " + std::to_string(trial));
    }
    // rejected patterns: a column out of range, a decreasing row pointer, n < 1, null arrays
    std::vector<int32_t> rp = {0, 1, 2}, ci = {0, 5}, colour(2);
    int32_t nc = 0;
    EXPECT(rsolve_colour_first_fit(2, rp.data(), ci.data(), colour.data(), &nc) == RSOLVE_E_INVALID, "column 5 of 2");
    const std::vector<int32_t> rp_dec = {0, 2, 1}, ci_ok = {0, 1};
    EXPECT(rsolve_colour_first_fit(2, rp_dec.data(), ci_ok.data(), colour.data(), &nc) == RSOLVE_E_INVALID,
           "decreasing row pointer");
    EXPECT(rsolve_colour_first_fit(0, rp.data(), ci.data(), colour.data(), &nc) == RSOLVE_E_INVALID, "n = 0");
    EXPECT(rsolve_colour_first_fit(2, nullptr, ci.data(), colour.data(), &nc) == RSOLVE_E_INVALID, "null row_ptr");

    // workspace sizing over valid and invalid configurations and sizes
    int valid = 0, total = 0;
    for (int m : {0, 1, 5, 30, 64, 128, 129})
        for (int k : {0, 1, 8, 64, 65})
            for (int s : {0, 1, 8, 64, 65})
                for (int meth = -1; meth <= 11; ++meth)
                    for (int pc = 0; pc <= 3; ++pc)
                        for (int prec = 0; prec <= 2; ++prec)
                            for (int sel = 0; sel <= 4; ++sel) {
                                rsolve_config c{};
                                c.restart_m = m;
                                c.recycle_k = k;
                                c.snapshots_s = s;
                                c.svd_interval = 1;
                                c.method = meth;
                                c.precond = pc;
                                c.precision = prec;
                                c.max_iters = 100;
                                c.select = sel;
                                c.ortho = m % 2;
                                c.inner_tol = 1e-5;
                                c.ssor_omega = pc == RSOLVE_PRECOND_SSOR ? 1.3 : 0.0;
                                for (int64_t n : {(int64_t)1, (int64_t)63, (int64_t)100000}) {
                                    ++total;
                                    const size_t b = rsolve_workspace_bytes(&c, n, n * 9);
                                    if (b) {
                                        ++valid;
                                        EXPECT(b % 256 == 0, "workspace size not a multiple of 256");
                                    }
                                }
                            }
    EXPECT(rsolve_workspace_bytes(nullptr, 10, 10) == 0, "null configuration");
    EXPECT(valid > 0 && valid < total, "workspace sizing accepted all or nothing");

    // handle checks that return before any device call
    rsolve_stats st{};
    double dummy = 0.0;
    const rsolve_csr A{};
    EXPECT(rsolve_solve(nullptr, &A, &dummy, nullptr, &dummy, 1e-8, &st) == RSOLVE_E_INVALID, "solve(null)");
    EXPECT(rsolve_update_recycle(nullptr, nullptr) == RSOLVE_E_INVALID, "update(null)");
    EXPECT(rsolve_destroy_sequence(nullptr) == RSOLVE_E_INVALID, "destroy(null)");
    EXPECT(rsolve_get_recycle(nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0) == RSOLVE_E_INVALID, "get(null)");
    rsolve_config bad{};
    rsolve_seq* seq = nullptr;
    EXPECT(rsolve_create_sequence(&bad, 10, 10, nullptr, nullptr, 0, &seq) == RSOLVE_E_INVALID && !seq,
           "create with a zero configuration");
    unsigned char blob[64] = {};
    EXPECT(rsolve_state_bytes(nullptr) == 0, "state_bytes(null)");
    EXPECT(rsolve_export_state(nullptr, blob, sizeof blob, nullptr) == RSOLVE_E_INVALID, "export(null)");
    EXPECT(rsolve_import_state(nullptr, blob, sizeof blob) == RSOLVE_E_INVALID, "import(null)");
    rsolve_server* srv = nullptr;
    rsolve_server_config sc{};
    EXPECT(rsolve_server_create(&sc, &srv) == RSOLVE_E_INVALID && !srv, "server without a pool");
    for (int code = -8; code <= 2; ++code) EXPECT(rsolve_status_string(code) != nullptr, "status string");
    EXPECT(rsolve_last_error() != nullptr, "last error string");
    std::printf("cpu phase: %d of %d configurations sized, %d failures\n", valid, total, g_fail);
}

// ---------------------------------------------------------------- device phase

// A 9-point convection-diffusion operator on an nx x nx interior grid of the unit square (Q1-like
// diffusion stencil, central convection by a rotating field whose strength changes with the step),
// plus a mass term 1/dt: non-symmetric, positive definite symmetric part.
struct Problem {
    int nx = 0, n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> val, b;

    explicit Problem(int nx_) : nx(nx_), n(nx_ * nx_) {
        rp.assign(n + 1, 0);
        for (int iy = 0; iy < nx; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int jx = ix + dx, jy = iy + dy;
                        if (jx >= 0 && jx < nx && jy >= 0 && jy < nx) ci.push_back(jy * nx + jx);
                    }
                rp[iy * nx + ix + 1] = (int32_t)ci.size();
            }
        val.resize(ci.size());
        b.resize(n);
    }

    void set_step(int step) {
        const double h = 1.0 / (nx + 1), nu = 0.01, inv_dt = 20.0;
        const double amp = 2.0 * (1.0 + 0.3 * std::sin(0.7 * step));
        for (int iy = 0; iy < nx; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const int i = iy * nx + ix;
                const double x = (ix + 1) * h, y = (iy + 1) * h;
                const double bx = -amp * (y - 0.5), by = amp * (x - 0.5);
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    const int j = ci[e], dx = j % nx - ix, dy = j / nx - iy;
                    double a = (dx == 0 && dy == 0) ? inv_dt + nu * (8.0 / 3.0) / (h * h) : -nu / (3.0 * h * h);
                    if (dy == 0) a += dx * bx / (2.0 * h);
                    if (dx == 0) a += dy * by / (2.0 * h);
                    val[e] = a;
                }
                b[i] = std::sin(M_PI * x) * std::sin(M_PI * y) * (1.0 + 0.1 * step) +
                       0.2 * y * std::cos(2.0 * M_PI * x + 0.3 * step);
            }
    }

    // ||b - A x||_2 / ||b||_2 in float64 on the host
    double rel_residual(const std::vector<double>& x) const {
        double rr = 0.0, bb = 0.0;
        for (int i = 0; i < n; ++i) {
            double r = b[i];
            for (int e = rp[i]; e < rp[i + 1]; ++e) r -= val[e] * x[ci[e]];
            rr += r * r;
            bb += b[i] * b[i];
        }
        return std::sqrt(rr / bb);
    }
};

// The problem's arrays on the device
struct DeviceProblem {
    int32_t *rp = nullptr, *ci = nullptr;
    double *val = nullptr, *b = nullptr;
    int64_t n = 0, nnz = 0;

    explicit DeviceProblem(const Problem& p) : n(p.n), nnz((int64_t)p.ci.size()) {
        HIP_OK(hipMalloc(&rp, (n + 1) * sizeof(int32_t)));
        HIP_OK(hipMalloc(&ci, nnz * sizeof(int32_t)));
        HIP_OK(hipMalloc(&val, nnz * sizeof(double)));
        HIP_OK(hipMalloc(&b, n * sizeof(double)));
        HIP_OK(hipMemcpy(rp, p.rp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(ci, p.ci.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    ~DeviceProblem() {
        (void)hipFree(rp);
        (void)hipFree(ci);
        (void)hipFree(val);
        (void)hipFree(b);
    }
    void upload(const Problem& p) {
        HIP_OK(hipMemcpy(val, p.val.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(b, p.b.data(), n * sizeof(double), hipMemcpyHostToDevice));
    }
    rsolve_csr csr(bool same_pattern) const {
        return rsolve_csr{n, nnz, rp, ci, val, same_pattern ? RSOLVE_SAME_PATTERN : 0u, 0u};
    }
};

std::vector<double> download(const double* d, int64_t n) {
    std::vector<double> h(n);
    HIP_OK(hipMemcpy(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost));
    return h;
}

// A solve's status and reported residual against the host's own residual of the returned x
void check_solve(const char* what, int rc, const rsolve_stats& st, const Problem& p, const double* dx, double tol,
                 int* not_converged) {
    if (rc == RSOLVE_NOT_CONVERGED) {
        ++*not_converged;
    } else if (rc != RSOLVE_OK) {
        fail(what, "status " + std::to_string(rc));
        return;
    }
    const double rel = p.rel_residual(download(dx, p.n));
    char buf[160];
    std::snprintf(buf, sizeof buf, "host residual %.3e, reported %.3e, converged %d", rel, st.rel_res_true,
                  st.converged);
    if (!(std::fabs(rel - st.rel_res_true) <= 1e-3 * std::max(rel, tol))) fail(what, buf);
    if (rc == RSOLVE_OK && !(st.converged == 1 && rel <= 1.05 * tol)) fail(what, buf);
}

rsolve_config base_config(int method, int precond, int precision, int select, int ortho) {
    const bool extrap = method >= RSOLVE_GUESS_EXTRAP2 && method <= RSOLVE_GUESS_EXTRAP4;
    rsolve_config c{};
    c.restart_m = 30;
    c.recycle_k = (method == RSOLVE_PLAIN || extrap) ? 0 : 8;
    c.snapshots_s = extrap ? 4 : (c.recycle_k ? 10 : 0);
    c.svd_interval = 1 + method % 2;
    c.method = method;
    c.precond = precond;
    c.precision = precision;
    c.max_iters = 3000;
    c.select = select;
    c.ortho = ortho;
    c.inner_tol = 1e-5;
    c.ssor_omega = precond == RSOLVE_PRECOND_SSOR ? 1.2 : 0.0;
    return c;
}

void solver_configurations(Problem& p, DeviceProblem& dp, hipStream_t stream) {
    const double tol = 1e-8;
    const int steps = 4;
    double *x = nullptr, *Wout = nullptr;
    HIP_OK(hipMalloc(&x, p.n * sizeof(double)));
    HIP_OK(hipMalloc(&Wout, (size_t)p.n * 64 * sizeof(double)));
    int configs = 0, solves = 0, not_converged = 0, profiled = 0, graphed = 0, tuned = 0;
    for (int method = RSOLVE_PLAIN; method <= RSOLVE_DEFL_LS; ++method) {
        std::printf("  method %d: %d configurations so far\n", method, configs);
        std::fflush(stdout);
        for (int precond = RSOLVE_PRECOND_NONE; precond <= RSOLVE_PRECOND_SSOR; ++precond)
            for (int precision = RSOLVE_FP64; precision <= RSOLVE_FP32_IR; ++precision)
                for (int select = RSOLVE_SELECT_LARGEST; select <= RSOLVE_SELECT_HARMONIC; ++select)
                    for (int ortho = RSOLVE_ORTHO_CGS2; ortho <= RSOLVE_ORTHO_DCGS2; ++ortho) {
                        const rsolve_config c = base_config(method, precond, precision, select, ortho);
                        if (c.recycle_k == 0 && select != RSOLVE_SELECT_LARGEST) continue;
                        const size_t ws = rsolve_workspace_bytes(&c, p.n, dp.nnz);
                        if (!ws) continue;
                        ++configs;
                        char name[96];
                        std::snprintf(name, sizeof name, "method %d precond %d precision %d select %d ortho %d",
                                      method, precond, precision, select, ortho);
                        void* w = nullptr;
                        HIP_OK(hipMalloc(&w, ws));
                        rsolve_seq* s = nullptr;
                        if (rsolve_create_sequence(&c, p.n, dp.nnz, stream, w, ws, &s) != RSOLVE_OK) {
                            fail("create", name);
                            HIP_OK(hipFree(w));
                            continue;
                        }
                        EXPECT(rsolve_update_recycle(s, nullptr) == RSOLVE_E_STATE, name);
                        const bool probe = precond == RSOLVE_PRECOND_JACOBI && select == RSOLVE_SELECT_LARGEST &&
                                           ortho == RSOLVE_ORTHO_CGS2;
                        if (probe && precision == RSOLVE_FP64) {
                            EXPECT(rsolve_profile_enable(s, RSOLVE_PROF_ALL | RSOLVE_PROF_STRIDE(2)) == RSOLVE_OK,
                                   name);
                            ++profiled;
                        }
                        if (probe && precision == RSOLVE_FP32_IR) {
                            EXPECT(rsolve_enable_graphs(s, 1) == RSOLVE_OK, name);
                            ++graphed;
                        }
                        for (int step = 0; step < steps; ++step) {
                            p.set_step(step);
                            dp.upload(p);
                            const rsolve_csr A = dp.csr(step > 0);
                            if (probe && method == RSOLVE_AUG_OBLIQUE && step == 1) {
                                rsolve_spmv_shape shapes[64];
                                int32_t count = 0;
                                EXPECT(rsolve_tune_spmv(s, &A, 2, shapes, 64, &count) == RSOLVE_OK && count > 0, name);
                                if (count > 0) {
                                    EXPECT(rsolve_set_spmv_shape(s, &shapes[0]) == RSOLVE_OK, name);
                                    rsolve_spmv_shape got{};
                                    EXPECT(rsolve_get_spmv_shape(s, &got) == RSOLVE_OK && got.user_set == 1 &&
                                               got.format == shapes[0].format &&
                                               got.lanes_per_row == shapes[0].lanes_per_row,
                                           name);
                                }
                                ++tuned;
                            }
                            rsolve_stats st{};
                            const int rc = rsolve_solve(s, &A, dp.b, step ? x : nullptr, x, tol, &st);
                            check_solve(name, rc, st, p, x, tol, &not_converged);
                            ++solves;
                            const int uc = rsolve_update_recycle(s, nullptr);
                            EXPECT(uc == RSOLVE_OK, name);
                        }
                        int32_t k_eff = -1, rank = -1;
                        double sigma[64];
                        EXPECT(rsolve_get_recycle(s, &k_eff, &rank, sigma, 64, Wout, p.n) == RSOLVE_OK, name);
                        EXPECT(k_eff >= 0 && k_eff <= c.recycle_k, name);
                        if (probe && precision == RSOLVE_FP64) {
                            rsolve_prof_entry prof[64];
                            int32_t count = 0;
                            EXPECT(rsolve_profile_read(s, prof, 64, &count, 1) == RSOLVE_OK && count > 0, name);
                            for (int i = 0; i < std::min(count, 64); ++i)
                                EXPECT(prof[i].launches >= 0 && prof[i].ms >= 0.0 && prof[i].bytes >= 0.0, name);
                        }
                        if (probe && precision == RSOLVE_FP32_IR) {
                            int64_t captures = -1, launches = -1;
                            EXPECT(rsolve_graph_counts(s, &captures, &launches) == RSOLVE_OK && captures >= 0 &&
                                       launches >= 0,
                                   name);
                        }
                        // checkpoint: the state moves to a fresh sequence of the same configuration
                        std::vector<unsigned char> blob(rsolve_state_bytes(s));
                        size_t written = 0;
                        EXPECT(rsolve_export_state(s, blob.data(), blob.size(), &written) == RSOLVE_OK &&
                                   written == blob.size(),
                               name);
                        void* w2 = nullptr;
                        HIP_OK(hipMalloc(&w2, ws));
                        rsolve_seq* s2 = nullptr;
                        EXPECT(rsolve_create_sequence(&c, p.n, dp.nnz, stream, w2, ws, &s2) == RSOLVE_OK, name);
                        if (s2) {
                            EXPECT(rsolve_import_state(s2, blob.data(), blob.size() / 2) == RSOLVE_E_INVALID, name);
                            EXPECT(rsolve_import_state(s2, blob.data(), blob.size()) == RSOLVE_OK, name);
                            int32_t k2 = -1, rank2 = -1;
                            double sigma2[64];
                            EXPECT(rsolve_get_recycle(s2, &k2, &rank2, sigma2, 64, nullptr, 0) == RSOLVE_OK &&
                                       k2 == k_eff && rank2 == rank &&
                                       std::memcmp(sigma, sigma2, sizeof(double) * std::min(64, std::max(rank, 0))) == 0,
                                   name);
                            EXPECT(rsolve_destroy_sequence(s2) == RSOLVE_OK, name);
                        }
                        HIP_OK(hipFree(w2));
                        EXPECT(rsolve_destroy_sequence(s) == RSOLVE_OK, name);
                        HIP_OK(hipFree(w));
                    }
    }
    HIP_OK(hipFree(x));
    HIP_OK(hipFree(Wout));
    std::printf("solver configurations: %d, solves %d (not converged %d), profiled %d, graphs %d, tuned %d\n",
                configs, solves, not_converged, profiled, graphed, tuned);
    EXPECT(configs >= 200 && profiled > 0 && graphed > 0 && tuned > 0, "coverage of the configuration loop");
    EXPECT(not_converged == 0, std::to_string(not_converged) + " solves did not converge");
}

void error_returns(Problem& p, DeviceProblem& dp, hipStream_t stream) {
    const rsolve_config c = base_config(RSOLVE_AUG_OBLIQUE, RSOLVE_PRECOND_JACOBI, RSOLVE_FP64, 0, 0);
    const size_t ws = rsolve_workspace_bytes(&c, p.n, dp.nnz);
    void* w = nullptr;
    HIP_OK(hipMalloc(&w, ws));
    rsolve_seq* s = nullptr;
    EXPECT(rsolve_create_sequence(&c, p.n, dp.nnz, stream, w, ws - 256, &s) == RSOLVE_E_WORKSPACE && !s,
           "workspace one block short");
    EXPECT(rsolve_create_sequence(&c, p.n, dp.nnz, stream, (char*)w + 64, ws - 256, &s) == RSOLVE_E_WORKSPACE,
           "misaligned workspace");
    EXPECT(rsolve_create_sequence(&c, p.n, dp.nnz, stream, w, ws, &s) == RSOLVE_OK, "create");
    double* x = nullptr;
    HIP_OK(hipMalloc(&x, p.n * sizeof(double)));
    p.set_step(0);
    dp.upload(p);
    rsolve_csr A = dp.csr(false);
    rsolve_stats st{};
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 0.0, &st) == RSOLVE_E_INVALID, "tol = 0");
    A.n = p.n - 1;
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st) == RSOLVE_E_INVALID, "n mismatch");
    A = dp.csr(false);
    A.nnz = dp.nnz + 1;
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st) == RSOLVE_E_INVALID, "nnz above nnz_max");
    // a column index out of range in device memory
    A = dp.csr(false);
    const int32_t bad_col = (int32_t)p.n + 7;
    int32_t saved = 0;
    HIP_OK(hipMemcpy(&saved, dp.ci + 5, sizeof saved, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(dp.ci + 5, &bad_col, sizeof bad_col, hipMemcpyHostToDevice));
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st) == RSOLVE_E_INVALID, "corrupt column index");
    HIP_OK(hipMemcpy(dp.ci + 5, &saved, sizeof saved, hipMemcpyHostToDevice));
    // a NaN in b
    const double nan = std::nan("");
    HIP_OK(hipMemcpy(dp.b + 3, &nan, sizeof nan, hipMemcpyHostToDevice));
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st) == RSOLVE_E_NONFINITE, "NaN in b");
    dp.upload(p);
    int nc = 0;
    EXPECT(rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st) == RSOLVE_OK, "solve after the errors");
    check_solve("solve after the errors", RSOLVE_OK, st, p, x, 1e-8, &nc);
    EXPECT(rsolve_destroy_sequence(s) == RSOLVE_OK, "destroy");
    // the iteration cap
    rsolve_config one = c;
    one.max_iters = 1;
    EXPECT(rsolve_create_sequence(&one, p.n, dp.nnz, stream, w, ws, &s) == RSOLVE_OK, "create max_iters 1");
    const int rc = rsolve_solve(s, &A, dp.b, nullptr, x, 1e-8, &st);
    EXPECT(rc == RSOLVE_NOT_CONVERGED && st.iterations == 1 && st.converged == 0, "max_iters = 1");
    check_solve("max_iters = 1", rc, st, p, x, 1e-8, &nc);
    EXPECT(rsolve_destroy_sequence(s) == RSOLVE_OK, "destroy");
    HIP_OK(hipFree(x));
    HIP_OK(hipFree(w));
    std::printf("error returns checked\n");
}

void batched(Problem& p, DeviceProblem& dp, hipStream_t stream) {
    // four one-block sequences and one FP32_IR sequence that takes the multi-kernel path
    const int count = 5, steps = 4;
    std::vector<rsolve_seq*> seqs(count, nullptr);
    std::vector<void*> ws(count, nullptr);
    std::vector<double*> x(count, nullptr);
    for (int i = 0; i < count; ++i) {
        const int method = i % 2 ? RSOLVE_DEFL_OBLIQUE : RSOLVE_AUG_OBLIQUE;
        const rsolve_config c = base_config(method, RSOLVE_PRECOND_JACOBI, i == 4 ? RSOLVE_FP32_IR : RSOLVE_FP64, 0, 0);
        const size_t b = rsolve_workspace_bytes(&c, p.n, dp.nnz);
        HIP_OK(hipMalloc(&ws[i], b));
        HIP_OK(hipMalloc(&x[i], p.n * sizeof(double)));
        EXPECT(rsolve_create_sequence(&c, p.n, dp.nnz, stream, ws[i], b, &seqs[i]) == RSOLVE_OK, "batch create");
    }
    int nc = 0;
    for (int step = 0; step < steps; ++step) {
        p.set_step(step);
        dp.upload(p);
        std::vector<rsolve_batch_solve_item> items(count);
        for (int i = 0; i < count; ++i) {
            items[i] = rsolve_batch_solve_item{};
            items[i].seq = seqs[i];
            items[i].A = dp.csr(step > 0);
            items[i].b = dp.b;
            items[i].x0 = step ? x[i] : nullptr;
            items[i].x = x[i];
            items[i].tol = 1e-8;
        }
        EXPECT(rsolve_solve_batch(items.data(), count, stream) == RSOLVE_OK, "solve_batch");
        for (int i = 0; i < count; ++i) check_solve("batched solve", items[i].status, items[i].stats, p, x[i], 1e-8, &nc);
        std::vector<rsolve_batch_update_item> ups(count);
        for (int i = 0; i < count; ++i) ups[i] = rsolve_batch_update_item{seqs[i], nullptr, -99, 0};
        EXPECT(rsolve_update_recycle_batch(ups.data(), count, stream) == RSOLVE_OK, "update_recycle_batch");
        for (int i = 0; i < count; ++i) EXPECT(ups[i].status == RSOLVE_OK, "batched update");
    }
    for (int i = 0; i < count; ++i) {
        EXPECT(rsolve_destroy_sequence(seqs[i]) == RSOLVE_OK, "batch destroy");
        HIP_OK(hipFree(ws[i]));
        HIP_OK(hipFree(x[i]));
    }
    EXPECT(nc == 0, "batched solves did not converge");
    std::printf("batched solves checked\n");
}

void serving(Problem& p, DeviceProblem& dp) {
    // three one-block FP64 sequences, one FP32_IR and one SSOR sequence on the large workers
    const int count = 5, steps = 4;
    std::vector<rsolve_config> cfgs;
    for (int i = 0; i < 3; ++i) cfgs.push_back(base_config(RSOLVE_AUG_OBLIQUE, RSOLVE_PRECOND_JACOBI, RSOLVE_FP64, 0, 0));
    cfgs.push_back(base_config(RSOLVE_AUG_OBLIQUE, RSOLVE_PRECOND_JACOBI, RSOLVE_FP32_IR, 0, 1));
    cfgs.push_back(base_config(RSOLVE_AUG_ORTHO, RSOLVE_PRECOND_SSOR, RSOLVE_FP64, 0, 0));
    size_t need = 0;
    for (const auto& c : cfgs) need += rsolve_workspace_bytes(&c, p.n, dp.nnz);
    const size_t pool_bytes = (need * 3 / 2 + 255) / 256 * 256;
    void* pool = nullptr;
    HIP_OK(hipMalloc(&pool, pool_bytes));
    rsolve_server_config sc{pool, pool_bytes, 2, 8, 8, 0};
    rsolve_server* srv = nullptr;
    EXPECT(rsolve_server_create(&sc, &srv) == RSOLVE_OK, "server create");
    std::vector<uint64_t> ids(count, 0);
    for (int i = 0; i < count; ++i)
        EXPECT(rsolve_server_open(srv, &cfgs[i], p.n, dp.nnz, &ids[i]) == RSOLVE_OK, "server open");
    // admission: a sequence as large as the pool does not fit next to the others
    uint64_t extra = 0;
    const rsolve_config big = base_config(RSOLVE_AUG_OBLIQUE, RSOLVE_PRECOND_JACOBI, RSOLVE_FP64, 0, 0);
    EXPECT(rsolve_server_open(srv, &big, (int64_t)p.n * 40, dp.nnz * 40, &extra) == RSOLVE_E_BUDGET,
           "admission beyond the pool");
    std::vector<double*> x(count, nullptr);
    for (int i = 0; i < count; ++i) HIP_OK(hipMalloc(&x[i], p.n * sizeof(double)));
    int nc = 0;
    for (int step = 0; step < steps; ++step) {
        p.set_step(step);
        dp.upload(p);
        const rsolve_csr A = dp.csr(step > 0);
        for (int i = 0; i < count; ++i)
            EXPECT(rsolve_server_submit(srv, ids[i], &A, dp.b, step ? x[i] : nullptr, x[i], 1e-8, nullptr,
                                        (uint64_t)(step * 100 + i)) == RSOLVE_OK,
                   "submit");
        int got = 0;
        const auto t0 = std::chrono::steady_clock::now();
        while (got < count && std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60)) {
            rsolve_completion out[8];
            int32_t k = 0;
            EXPECT(rsolve_server_poll(srv, out, 8, &k, 1000) == RSOLVE_OK, "poll");
            for (int j = 0; j < k; ++j) {
                const int i = (int)(out[j].tag % 100);
                EXPECT(out[j].tag / 100 == (uint64_t)step && i < count && out[j].seq_id == ids[i], "completion tag");
                if (i < count) check_solve("served solve", out[j].status, out[j].stats, p, x[i], 1e-8, &nc);
            }
            got += k;
        }
        EXPECT(got == count, "completions of step " + std::to_string(step));
    }
    rsolve_server_info info{};
    EXPECT(rsolve_server_info_get(srv, &info) == RSOLVE_OK && info.sequences == count && info.pending == 0 &&
               info.completed == (int64_t)count * steps && info.batched_solves > 0,
           "server info");
    for (int i = 0; i < count; ++i) EXPECT(rsolve_server_close(srv, ids[i]) == RSOLVE_OK, "close");
    EXPECT(rsolve_server_info_get(srv, &info) == RSOLVE_OK && info.sequences == 0 && info.pool_used == 0,
           "pool empty after closing");
    EXPECT(rsolve_server_destroy(srv) == RSOLVE_OK, "server destroy");
    for (int i = 0; i < count; ++i) HIP_OK(hipFree(x[i]));
    HIP_OK(hipFree(pool));
    EXPECT(nc == 0, "served solves did not converge");
    std::printf("serving loop checked\n");
}

void kernel_calls(Problem& p, DeviceProblem& dp, hipStream_t stream) {
    const int64_t n = p.n;
    std::mt19937_64 rng(11);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    p.set_step(1);
    dp.upload(p);
    // SpMV
    std::vector<double> hx(n);
    for (auto& v : hx) v = U(rng);
    double *dx = nullptr, *dy = nullptr;
    HIP_OK(hipMalloc(&dx, n * sizeof(double)));
    HIP_OK(hipMalloc(&dy, n * sizeof(double)));
    HIP_OK(hipMemcpy(dx, hx.data(), n * sizeof(double), hipMemcpyHostToDevice));
    const rsolve_csr A = dp.csr(false);
    EXPECT(rsolve_spmv(&A, dx, dy, stream) == RSOLVE_OK, "spmv");
    HIP_OK(hipStreamSynchronize(stream));
    const std::vector<double> y = download(dy, n);
    double err = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0, a = 0.0;
        for (int e = p.rp[i]; e < p.rp[i + 1]; ++e) {
            s += p.val[e] * hx[p.ci[e]];
            a += std::fabs(p.val[e] * hx[p.ci[e]]);
        }
        err = std::max(err, std::fabs(y[i] - s) / a);
    }
    EXPECT(err <= 1e-15 * 9, "spmv against the host product");
    // Gram products on the matrix cores, with and without a workspace
    const int c = 12;
    std::vector<double> hX((size_t)n * c);
    for (auto& v : hX) v = U(rng);
    double* dX = nullptr;
    HIP_OK(hipMalloc(&dX, hX.size() * sizeof(double)));
    HIP_OK(hipMemcpy(dX, hX.data(), hX.size() * sizeof(double), hipMemcpyHostToDevice));
    const size_t kws = rsolve_kernel_workspace_bytes(n, c);
    void* kw = nullptr;
    HIP_OK(hipMalloc(&kw, kws));
    std::vector<double> G(c * c), G2(c * c);
    EXPECT(rsolve_gram_tn(n, dX, n, c, dX, n, c, G.data(), kw, kws, stream) == RSOLVE_OK, "gram_tn");
    EXPECT(rsolve_gram_tn_noalloc(n, dX, n, c, dX, n, c, G2.data(), stream) == RSOLVE_OK, "gram_tn_noalloc");
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int64_t r = 0; r < n; ++r) s += hX[r + n * i] * hX[r + n * j];
            EXPECT(std::fabs(G[i + c * j] - s) <= 1e-12 * n, "gram_tn entry");
            EXPECT(std::fabs(G2[i + c * j] - s) <= 1e-12 * n, "gram_tn_noalloc entry");
        }
    EXPECT(rsolve_gram_tn(n, dX, n - 1, c, dX, n, c, G.data(), kw, kws, stream) == RSOLVE_E_INVALID, "lda < n");
    EXPECT(rsolve_gram_tn_noalloc(n, dX, n, 65, dX, n, c, G2.data(), stream) == RSOLVE_E_INVALID, "p = 65");
    // the SVD step of Algorithm 1 on the same columns
    const int k = 6;
    double* dW = nullptr;
    HIP_OK(hipMalloc(&dW, (size_t)n * k * sizeof(double)));
    double sigma[64];
    int32_t k_eff = -1, rank = -1;
    EXPECT(rsolve_snapshot_svd(n, dX, n, c, k, dW, n, sigma, &k_eff, &rank, kw, kws, stream) == RSOLVE_OK,
           "snapshot_svd");
    EXPECT(k_eff == k && rank == c, "snapshot_svd rank");
    for (int i = 1; i < c; ++i) EXPECT(sigma[i] <= sigma[i - 1] && sigma[i] > 0.0, "singular values descending");
    std::vector<double> WtW(k * k);
    EXPECT(rsolve_gram_tn(n, dW, n, k, dW, n, k, WtW.data(), kw, kws, stream) == RSOLVE_OK, "gram of W");
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) EXPECT(std::fabs(WtW[i + k * j] - (i == j)) <= 1e-12, "W orthonormal");
    // the streaming reference kernel
    double* da = nullptr;
    HIP_OK(hipMalloc(&da, n * sizeof(double)));
    EXPECT(rsolve_triad(n, da, dx, dy, 0.75, stream) == RSOLVE_OK, "triad");
    HIP_OK(hipStreamSynchronize(stream));
    const std::vector<double> a = download(da, n);
    for (int64_t i = 0; i < n; ++i)
        EXPECT(std::fabs(a[i] - (hx[i] + 0.75 * y[i])) <= 2.3e-16 * (std::fabs(hx[i]) + 0.75 * std::fabs(y[i])),
               "triad entry");
    EXPECT(rsolve_triad(n, da + 1, dx, dy, 0.75, stream) == RSOLVE_E_INVALID, "misaligned triad");
    for (void* ptr : {(void*)dx, (void*)dy, (void*)dX, kw, (void*)dW, (void*)da}) HIP_OK(hipFree(ptr));
    std::printf("kernel-level calls checked\n");
}

void gpu_phase() {
    hipStream_t stream = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    Problem p(64);
    DeviceProblem dp(p);
    // the first-fit colouring of the 9-point pattern needs four colours
    std::vector<int32_t> colour(p.n);
    int32_t nc = 0;
    EXPECT(rsolve_colour_first_fit(p.n, p.rp.data(), p.ci.data(), colour.data(), &nc) == RSOLVE_OK && nc == 4 &&
               proper_colouring(p.n, p.rp, p.ci, colour, nc),
           "colouring of the 9-point grid");
    const auto t0 = std::chrono::steady_clock::now();
    auto stamp = [&](const char* what) {
        std::printf("[%6.1f s] %s\n", std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(),
                    what);
        std::fflush(stdout);
    };
    stamp("start: error returns");
    error_returns(p, dp, stream);
    stamp("kernel-level calls");
    kernel_calls(p, dp, stream);
    stamp("batched solves");
    batched(p, dp, stream);
    stamp("serving loop");
    serving(p, dp);
    stamp("solver configurations");
    solver_configurations(p, dp, stream);
    stamp("done");
    HIP_OK(hipStreamDestroy(stream));
}

}  // namespace

int main(int argc, char** argv) {
    const std::string phase = argc > 1 ? argv[1] : "cpu";
    if (phase == "cpu") {
        cpu_phase();
    } else if (phase == "gpu") {
        cpu_phase();
        gpu_phase();
    } else {
        std::printf("usage: host_check cpu|gpu\n");
        return 2;
    }
    std::printf("%s\n", g_fail ? "host check FAILED" : "host check passed");
    std::fflush(stdout);
    // End without the static destructors: the HIP runtime's own teardown at exit frees memory
    // through the sanitizer allocator's device hooks after they have been unloaded, which the
    // AddressSanitizer runtime reports as an internal CHECK failure unrelated to this library.
    std::_Exit(g_fail ? 1 : 0);
}
