"""GPU parity of the delayed-reorthogonalisation Arnoldi (ortho="dcgs2") against the FP64 oracle.

The delayed scheme computes the same Arnoldi relation as classical Gram-Schmidt applied twice
(the second pass of each basis vector is merged into the next step's sweep and the Hessenberg
column completes one step later), so it answers to the same bars as the CGS2 path: float64
solutions within 1e-9 relative of the oracle at tol 1e-10, Arnoldi-step counts within +-2 per
solve and the same effective recycle dimension; float32-inner refinement within the refinement
bar.  It also agrees with the CGS2 GPU path to the same bar."""
import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL

from test_gpu_parity import _check_parity, _t, run_pair

pytestmark = pytest.mark.gpu


def test_dcgs2_plain_c1(gpu_ctx):
    out = run_pair(gpu_ctx, WL.C1, 5, 1e-10, restart_m=30, method="plain", ortho="dcgs2")
    _check_parity(out)


def test_dcgs2_recycled_c1_full_sequence(gpu_ctx):
    out = run_pair(gpu_ctx, WL.C1, 20, 1e-10, restart_m=30, recycle_k=5, snapshots_s=10, ortho="dcgs2")
    _check_parity(out)


@pytest.mark.parametrize("prob,m,k,s", [(WL.C2_SMALL, 30, 10, 20), (WL.C3_SMALL, 50, 16, 32)])
def test_dcgs2_recycled_jacobi(gpu_ctx, prob, m, k, s):
    out = run_pair(gpu_ctx, prob, 12, 1e-10, restart_m=m, recycle_k=k, snapshots_s=s, precond="jacobi",
                   ortho="dcgs2")
    _check_parity(out)


def test_dcgs2_short_restart_many_cycles(gpu_ctx):
    """Restart 5: every cycle runs to its closing step, where only the last column completes."""
    out = run_pair(gpu_ctx, WL.C3_SMALL, 4, 1e-10, restart_m=5, recycle_k=4, snapshots_s=6, precond="jacobi",
                   ortho="dcgs2")
    _check_parity(out, its_bar=3)
    assert max(r["st"]["cycles"] for r in out) > 2


def test_dcgs2_long_restart_over_64(gpu_ctx):
    """Restart 100: sweeps of more than 64 columns are split over several launches."""
    hard = WL.Problem(p=3, N=16, eps=1e-3, dt=0.05, beta="rotating")
    out = run_pair(gpu_ctx, hard, 2, 1e-12, restart_m=100, method="plain", ortho="dcgs2")
    _check_parity(out)
    assert out[0]["st"]["iterations"] > 64
    # and with a recycle space of 24 columns (sweeps of j + 49 columns)
    out = run_pair(gpu_ctx, hard, 3, 1e-12, restart_m=100, recycle_k=24, snapshots_s=28, ortho="dcgs2")
    _check_parity(out)


def test_dcgs2_mixed_precision_c3_small(gpu_ctx):
    out = run_pair(gpu_ctx, WL.C3_SMALL, 10, 1e-8, precision="fp32_ir", oracle_tol=1e-12, restart_m=50,
                   recycle_k=16, snapshots_s=32, precond="jacobi", inner_tol=1e-5, ortho="dcgs2")
    for r in out:
        assert r["status"] == 0 and r["st"]["converged"] == 1
        assert r["res"] <= 1e-8 * (1 + 1e-6)
        kappa = np.linalg.cond(r["A"].toarray(), 1)
        assert r["rel"] <= max(1e-8, kappa * 1e-8 * 2), (r["step"], r["rel"], kappa)


def test_dcgs2_agrees_with_cgs2(gpu_ctx):
    kw = dict(restart_m=30, recycle_k=10, snapshots_s=20, precond="jacobi")
    a = run_pair(gpu_ctx, WL.C2_SMALL, 8, 1e-10, **kw)
    d = run_pair(gpu_ctx, WL.C2_SMALL, 8, 1e-10, ortho="dcgs2", **kw)
    for ra, rd in zip(a, d):
        assert np.linalg.norm(ra["xg"] - rd["xg"]) <= 1e-9 * np.linalg.norm(ra["xg"]), ra["step"]
        assert abs(ra["st"]["iterations"] - rd["st"]["iterations"]) <= 2, ra["step"]


def test_dcgs2_tiny_systems_lucky_breakdown(gpu_ctx):
    """n = 1 and n = 2: the Krylov space is exhausted after n steps (lucky breakdown detected
    when column n-1 completes)."""
    import scipy.sparse as sp
    from paper_1807_09467_amd import rsolve
    for dense in (np.array([[4.0]]), np.array([[3.0, 1.0], [-2.0, 5.0]])):
        A = sp.csr_matrix(dense)
        n = dense.shape[0]
        b = np.arange(1.0, n + 1.0)
        seq = rsolve.Sequence(n, A.nnz, device=gpu_ctx, restart_m=4, ortho="dcgs2")
        x, st, status = seq.solve(_t(A.indptr.astype(np.int32), gpu_ctx), _t(A.indices.astype(np.int32), gpu_ctx),
                                  _t(A.data, gpu_ctx), _t(b, gpu_ctx), tol=1e-14)
        assert status == 0 and st["iterations"] <= n
        assert np.allclose(x.cpu().numpy(), np.linalg.solve(dense, b), rtol=1e-13)
        seq.close()


def test_dcgs2_profiling(gpu_ctx):
    """Per-kernel event timing with the delayed scheme reports its own kernels (and only kernels
    that ran), and leaves no error behind for the next solve."""
    import torch
    from paper_1807_09467_amd import rsolve
    asm, systems, _ = WL.march(WL.C1, 3, 0)
    rp, ci = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx)
    seq = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, recycle_k=5, snapshots_s=10,
                          ortho="dcgs2")
    seq.profile(True)
    x_prev = torch.zeros(asm.pat.n, dtype=torch.float64, device=gpu_ctx)
    for i, (v, b) in enumerate(systems):
        x, st, status = seq.solve(rp, ci, _t(v, gpu_ctx), _t(b, gpu_ctx), x0=x_prev, tol=1e-10, same_pattern=i > 0)
        assert status == 0 and st["converged"] == 1
        seq.update()
        x_prev = x
    prof = seq.profile_read()
    names = {e["kernel"] for e in prof}
    assert names == {"spmv_arnoldi", "dots2", "dcgs2_update"}, names
    assert all(e["launches"] > 0 and e["ms"] > 0 for e in prof)
    seq.close()


def _check_slow_tail(out, tol):
    """Bars for a solve whose last cycle converges slowly (a few percent per step near the
    tolerance), where rounding moves the stopping step: the true residual meets tol, the step
    count is within 3 of the oracle's, and the solutions differ by at most what two solutions
    that both meet tol can differ by (2 kappa_1 tol)."""
    for r in out:
        assert r["status"] == 0 and r["st"]["converged"] == 1, r["step"]
        assert r["res"] <= tol * (1 + 1e-6), (r["step"], r["res"])
        assert abs(r["st"]["iterations"] - r["ores"].iterations) <= 3, (
            r["step"], r["st"]["iterations"], r["ores"].iterations)
        assert r["st"]["k_eff"] == r["ores"].k_eff
        kappa = np.linalg.cond(r["A"].toarray(), 1)
        assert r["rel"] <= max(1e-9, 2 * kappa * tol), (r["step"], r["rel"], kappa)


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_restart_at_the_maximum(gpu_ctx, ortho):
    """GMRES(128), the largest restart: full 128-step cycles (about 270 steps per plain solve), so
    the Hessenberg matrix and the sweeps reach their largest sizes; plain and recycled."""
    hard = WL.Problem(p=3, N=16, eps=1e-4, dt=0.1, beta="rotating")
    out = run_pair(gpu_ctx, hard, 2, 1e-10, restart_m=128, method="plain", ortho=ortho)
    _check_slow_tail(out, 1e-10)
    assert out[0]["st"]["iterations"] > 256 and out[0]["st"]["cycles"] >= 3
    out = run_pair(gpu_ctx, hard, 3, 1e-10, restart_m=128, recycle_k=16, snapshots_s=20, ortho=ortho)
    _check_slow_tail(out, 1e-10)


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_maximum_recycle_dimensions(gpu_ctx, ortho):
    """k = s = 64 (the largest recycle dimension and ring): the ring fills after 64 solves and
    the recycle space keeps all 64 directions (the smallest singular value of the ring stays an
    order of magnitude above the rank cut), so the sweeps carry 2 k + j columns and the small LU
    is 64 x 64."""
    out = run_pair(gpu_ctx, WL.C1, 68, 1e-10, restart_m=30, recycle_k=64, snapshots_s=64, ortho=ortho)
    _check_parity(out)
    assert [r["st"]["k_eff"] for r in out][-4:] == [64] * 4
