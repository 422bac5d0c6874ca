"""GPU parity of the initial-guess strategies of section 4: the projection guess onto span(W)
followed by plain GMRES (section 4.2, eq. (iteration_projection)) and Lagrange extrapolation of
order 2-4 (section 4.1, eqs. (ext2)-(ext4)).  Against the FP64 oracle on the same sequences (bars
as for the recycled path: solutions within 1e-9 relative at tol 1e-10, Arnoldi steps within +-2
per solve), and against closed forms: a solution polynomial in the step index of degree below the
order, or lying in the span of the stored solutions, is reached by the guess alone."""
import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL

from test_gpu_parity import _check_parity, _t, run_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
@pytest.mark.parametrize("method,k,s", [("guess_project", 5, 10), ("guess_project", 10, 10),
                                        ("guess_extrap2", 0, 2), ("guess_extrap3", 0, 3),
                                        ("guess_extrap4", 0, 6)])
def test_guess_methods_c1_sequence(gpu_ctx, method, k, s, ortho):
    out = run_pair(gpu_ctx, WL.C1, 14, 1e-10, restart_m=30, recycle_k=k, snapshots_s=s, method=method, ortho=ortho)
    _check_parity(out)
    assert all(r["st"]["k_eff"] == (min(k, r["step"]) if k else 0) for r in out)


@pytest.mark.parametrize("method,k,s", [("guess_project", 10, 20), ("guess_extrap3", 0, 3)])
def test_guess_methods_jacobi_c2(gpu_ctx, method, k, s):
    out = run_pair(gpu_ctx, WL.C2_SMALL, 10, 1e-10, restart_m=30, recycle_k=k, snapshots_s=s, method=method,
                   precond="jacobi", ortho="dcgs2")
    _check_parity(out)


def test_guess_project_mixed_precision(gpu_ctx):
    """FP32 Arnoldi inside FP64 refinement with the projection guess: the final iterate meets the
    FP64 stopping rule and agrees with a tight oracle solve."""
    out = run_pair(gpu_ctx, WL.C1, 8, 1e-10, precision="fp32_ir", oracle_tol=1e-13, restart_m=30, recycle_k=5,
                   snapshots_s=10, method="guess_project", precond="jacobi")
    for r in out:
        assert r["status"] == 0 and r["res"] <= 1e-10 and r["rel"] <= 1e-8, (r["step"], r["res"], r["rel"])


def _fixed_system(dev):
    asm, systems, _ = WL.march(WL.C1, 2, 5)
    vals, _ = systems[-1]
    A = asm.csr(vals)
    return asm, A, _t(asm.pat.row_ptr, dev), _t(asm.pat.col_idx, dev), _t(vals, dev)


@pytest.mark.parametrize("order,s", [(2, 2), (3, 4), (4, 4), (4, 7)])
def test_extrapolation_reaches_polynomial_solutions(gpu_ctx, order, s):
    """The ring holds exact values of x(t) = sum_{d<order} c_d t^d (stored through the update
    call); the next solve's extrapolated guess is x(t) itself, so no Arnoldi step is taken.  Ring
    sizes above the order wrap the slot index."""
    import torch
    from paper_1807_09467_amd import rsolve
    asm, A, rp, ci, v = _fixed_system(gpu_ctx)
    n = asm.pat.n
    rng = np.random.default_rng(order * 10 + s)
    C = rng.standard_normal((order, n))
    xt = lambda t: sum(C[d] * float(t) ** d for d in range(order))
    seq = rsolve.Sequence(n, asm.pat.nnz, device=gpu_ctx, restart_m=30, snapshots_s=s,
                          method="guess_extrap%d" % order)
    for t in range(order):
        seq.update(_t(xt(t), gpu_ctx))
    for t in range(order, order + 9):
        want = xt(t)
        x, st, status = seq.solve(rp, ci, v, _t(A @ want, gpu_ctx), tol=1e-10, same_pattern=t > order)
        assert status == 0 and st["iterations"] == 0 and st["k_eff"] == 0, (t, st["iterations"])
        assert np.linalg.norm(x.cpu().numpy() - want) <= 1e-11 * np.linalg.norm(want)
        seq.update(_t(want, gpu_ctx))
    seq.close()


def test_extrapolation_lowers_order_while_ring_fills(gpu_ctx):
    """Order 4 with one or two stored solutions: a constant sequence is reached from one stored
    solution and a linear one from two (the highest order the stored solutions allow); the
    caller's x0 is ignored once a solution is stored."""
    import torch
    from paper_1807_09467_amd import rsolve
    asm, A, rp, ci, v = _fixed_system(gpu_ctx)
    n = asm.pat.n
    rng = np.random.default_rng(7)
    c0, c1 = rng.standard_normal(n), rng.standard_normal(n)
    junk = _t(rng.standard_normal(n) * 1e3, gpu_ctx)
    seq = rsolve.Sequence(n, asm.pat.nnz, device=gpu_ctx, restart_m=30, snapshots_s=4, method="guess_extrap4")
    seq.update(_t(c0, gpu_ctx))
    x, st, status = seq.solve(rp, ci, v, _t(A @ c0, gpu_ctx), x0=junk, tol=1e-10)
    assert status == 0 and st["iterations"] == 0
    seq.close()
    seq = rsolve.Sequence(n, asm.pat.nnz, device=gpu_ctx, restart_m=30, snapshots_s=4, method="guess_extrap4")
    seq.update(_t(c0, gpu_ctx))
    seq.update(_t(c0 + c1, gpu_ctx))
    want = c0 + 2 * c1
    x, st, status = seq.solve(rp, ci, v, _t(A @ want, gpu_ctx), x0=junk, tol=1e-10)
    assert status == 0 and st["iterations"] == 0
    assert np.linalg.norm(x.cpu().numpy() - want) <= 1e-11 * np.linalg.norm(want)
    seq.close()
    # an empty ring starts from x0 (here the solution itself)
    seq = rsolve.Sequence(n, asm.pat.nnz, device=gpu_ctx, restart_m=30, snapshots_s=4, method="guess_extrap2")
    x, st, status = seq.solve(rp, ci, v, _t(A @ c1, gpu_ctx), x0=_t(c1, gpu_ctx), tol=1e-10)
    assert status == 0 and st["iterations"] == 0
    seq.close()


def test_projection_guess_reaches_solutions_in_the_span(gpu_ctx):
    """Stored solutions spanning a two-dimensional space: any solution in that space is the
    projection guess (eq. (projection_t_s)), no Arnoldi step follows; outside it the Krylov
    iteration is the plain one and converges."""
    from paper_1807_09467_amd import rsolve
    asm, A, rp, ci, v = _fixed_system(gpu_ctx)
    n = asm.pat.n
    rng = np.random.default_rng(11)
    U = rng.standard_normal((n, 2))
    seq = rsolve.Sequence(n, asm.pat.nnz, device=gpu_ctx, restart_m=30, recycle_k=2, snapshots_s=2,
                          method="guess_project")
    seq.update(_t(U[:, 0], gpu_ctx))
    seq.update(_t(U[:, 1], gpu_ctx))
    for i, cf in enumerate(([0.3, -1.2], [2.0, 0.5], [-1.0, 1.0])):
        want = U @ np.array(cf)
        x, st, status = seq.solve(rp, ci, v, _t(A @ want, gpu_ctx), tol=1e-10, same_pattern=i > 0)
        assert status == 0 and st["iterations"] == 0 and st["k_eff"] == 2
        assert np.linalg.norm(x.cpu().numpy() - want) <= 1e-11 * np.linalg.norm(want)
    b = rng.standard_normal(n)
    x, st, status = seq.solve(rp, ci, v, _t(b, gpu_ctx), tol=1e-10, same_pattern=True)
    xn = x.cpu().numpy()
    assert status == 0 and st["iterations"] > 0
    assert np.linalg.norm(b - A @ xn) <= 1e-10 * np.linalg.norm(b)
    seq.close()


def test_guess_methods_on_the_batched_calls(gpu_ctx):
    """The batched solve call routes the guess methods to the multi-kernel path, alongside a
    one-block item: with extrapolation (whose update only stores the solution) the iterates equal
    those of rsolve_solve / rsolve_update_recycle bit for bit; with the projection guess the
    batched update computes W with the one-block SVD, so the iterates agree to the parity bar."""
    import torch
    from paper_1807_09467_amd import rsolve
    asm, systems, _ = WL.march(WL.C1, 6, 9)
    n, nnz = asm.pat.n, asm.pat.nnz
    rp, ci = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx)
    kws = [dict(restart_m=30, snapshots_s=3, method="guess_extrap3"),
           dict(restart_m=30, recycle_k=4, snapshots_s=6, method="guess_project"),
           dict(restart_m=30, recycle_k=4, snapshots_s=6, method="aug_oblique")]
    single = [rsolve.Sequence(n, nnz, device=gpu_ctx, **kw) for kw in kws]
    batched = [rsolve.Sequence(n, nnz, device=gpu_ctx, **kw) for kw in kws]
    xp = [torch.zeros(n, dtype=torch.float64, device=gpu_ctx) for _ in kws]
    for i, (vals, b) in enumerate(systems):
        vd, bd = _t(vals, gpu_ctx), _t(b, gpu_ctx)
        xs_single = []
        for q, sq in enumerate(single):
            x, st, status = sq.solve(rp, ci, vd, bd, x0=xp[q], tol=1e-10, same_pattern=i > 0)
            assert status == 0
            sq.update(x)
            xs_single.append(x)
        res = rsolve.solve_batch([dict(seq=sq, row_ptr=rp, col_idx=ci, val=vd, b=bd, x0=xp[q], tol=1e-10,
                                       same_pattern=i > 0) for q, sq in enumerate(batched)])
        rsolve.update_batch(batched, [r[0] for r in res])
        assert torch.equal(res[0][0], xs_single[0]), i
        for q in (1, 2):
            assert res[q][2] == 0
            assert np.linalg.norm(res[q][0].cpu().numpy() - xs_single[q].cpu().numpy()) <= \
                1e-9 * np.linalg.norm(xs_single[q].cpu().numpy()), (i, q)
        xp = [r[0] for r in res]
    for sq in single + batched:
        sq.close()
