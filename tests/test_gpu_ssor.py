"""GPU parity of the multicolour SSOR preconditioner (the paper's SSOR of section 6.1 on a colour
ordering, applied on the right) against the oracle's, which computes the same first-fit
colouring on its own and applies M^{-1} by two sparse triangular solves of the permuted matrix.

Cases: the one-workgroup application (Q1 64 x 64 with 4 colours, the Q3 reduced mesh with 16,
the order-8 spectral elements with 64) and the one-launch-per-colour application (a Q2 mesh of
37,249 rows, 9 colours); plain, oblique and orthogonal rows; both Arnoldi schemes; omega other
than 1; a change of pattern inside a sequence (colouring again); the batched call routing SSOR
sequences to the multi-kernel path; configurations SSOR does not support.  Bars as for Jacobi:
solutions within 1e-9 (2-norm and entry by entry) at tol 1e-10, Arnoldi steps within 2 (the
orthogonal rows one more per cycle), the same k_eff."""
import numpy as np
import pytest

from oracle import rgmres as O
from paper_1807_09467_amd import workload as WL

from test_gpu_parity import _check_parity, _t, run_pair
from test_gpu_variants import _check_ortho

pytestmark = pytest.mark.gpu

Q2_MID = WL.Problem(p=2, N=96, eps=1e-3, dt=5e-3, beta="const")   # n = 37,249: one launch per colour


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_ssor_plain_and_oblique_q1_paper(gpu_ctx, ortho):
    for method, k in (("plain", 0), ("aug_oblique", 10)):
        print(f"[ssor] Q1 64 paper nu=1e-2 {method} {ortho}", flush=True)
        out = run_pair(gpu_ctx, WL.PAPER_Q1[1e-2], 8, 1e-10, restart_m=30, recycle_k=k, snapshots_s=max(k, 0),
                       precond="ssor", method=method, ortho=ortho)
        _check_parity(out)


def test_ssor_table3_protocol_q1(gpu_ctx):
    """Table 3's augmented orthogonal 'aug 20' with SSOR, the paper's preconditioner: no recycle
    space for 20 solves, then 20 directions."""
    print("[ssor] Q1 64 aug_ortho k=20 s=20 ell=20", flush=True)
    out = run_pair(gpu_ctx, WL.PAPER_Q1[1e-2], 23, 1e-10, restart_m=30, recycle_k=20, snapshots_s=20,
                   svd_interval=20, precond="ssor", method="aug_ortho")
    _check_ortho(out)
    assert [r["st"]["k_eff"] for r in out] == [0] * 20 + [20] * 3


@pytest.mark.parametrize("prob,name", [(WL.C3_SMALL, "c3_small"), (WL.PAPER_SEM8, "sem8")])
def test_ssor_many_colours(gpu_ctx, prob, name):
    print(f"[ssor] {name} aug_oblique", flush=True)
    out = run_pair(gpu_ctx, prob, 6, 1e-10, restart_m=40, recycle_k=6, snapshots_s=8, precond="ssor",
                   method="aug_oblique", ortho="dcgs2")
    _check_parity(out)


def test_ssor_one_launch_per_colour(gpu_ctx):
    print("[ssor] Q2 96x96 plain and aug_oblique", flush=True)
    out = run_pair(gpu_ctx, Q2_MID, 3, 1e-10, restart_m=40, recycle_k=2, snapshots_s=2, precond="ssor",
                   method="aug_oblique")
    _check_parity(out)


@pytest.mark.parametrize("method,k,s", [("guess_project", 4, 4), ("guess_extrap3", 0, 3), ("defl_ls", 6, 8),
                                        ("defl_ortho", 6, 8)])
def test_ssor_other_rows(gpu_ctx, method, k, s):
    """The preconditioner under the section 4 guesses and the least-squares and orthogonal
    projectors (Table 1): the same bars, one step per cycle more for the orthogonal row."""
    print(f"[ssor] {method}", flush=True)
    out = run_pair(gpu_ctx, WL.C2_SMALL, 6, 1e-10, restart_m=30, recycle_k=k, snapshots_s=s, precond="ssor",
                   method=method, ortho="dcgs2")
    if method == "defl_ortho":
        _check_ortho(out)
    else:
        _check_parity(out)


@pytest.mark.parametrize("omega", [0.7, 1.5])
def test_ssor_relaxation(gpu_ctx, omega):
    print(f"[ssor] omega {omega}", flush=True)
    out = run_pair(gpu_ctx, WL.C3_SMALL, 4, 1e-10, restart_m=40, recycle_k=4, snapshots_s=4, precond="ssor",
                   ssor_omega=omega, method="aug_oblique")
    _check_parity(out)


def test_ssor_pattern_change(gpu_ctx):
    """One sequence solves a Q1 system and then a Q2 system of the same size: the second pattern
    is coloured afresh (9 colours in the place of 4)."""
    import torch
    from paper_1807_09467_amd import rsolve
    p1 = WL.Problem(p=1, N=32, eps=1e-2, dt=1e-2, beta="const")
    p2 = WL.Problem(p=2, N=16, eps=1e-2, dt=1e-2, beta="const")
    assert p1.n == p2.n
    a1, a2 = WL.Assembler(p1), WL.Assembler(p2)
    seq = rsolve.Sequence(p1.n, max(a1.pat.nnz, a2.pat.nnz), device=gpu_ctx, restart_m=30, precond="ssor",
                          method="plain")
    ocfg = O.Config(restart_m=30, method=O.PLAIN, precond=O.PRECOND_SSOR)
    for asm, prob in ((a1, p1), (a2, p2), (a1, p1)):
        print(f"[ssor] pattern p={prob.p}", flush=True)
        vals = asm.matrix_values(WL.initial_condition(prob, 1))
        b = asm.rhs(WL.initial_condition(prob, 1))
        A = asm.csr(vals)
        x, st, status = seq.solve(_t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx), _t(vals, gpu_ctx),
                                  _t(b, gpu_ctx), tol=1e-10)
        ores = O.solve(A, b, None, 1e-10, ocfg)
        xg = x.cpu().numpy()
        assert status == 0 and st["converged"] == 1
        assert np.linalg.norm(xg - ores.x) <= 1e-9 * np.linalg.norm(ores.x)
        assert abs(st["iterations"] - ores.iterations) <= 2
    seq.close()


def test_ssor_batch_routes_to_multikernel(gpu_ctx):
    """An SSOR sequence inside a batched call takes the multi-kernel path and gives the same
    solution and step count as its single call."""
    import torch
    from paper_1807_09467_amd import rsolve
    prob = WL.C3_SMALL
    asm, systems, _ = WL.march(prob, 2, 3)
    vals, b = systems[1]
    rp, ci = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx)
    res = []
    for batched in (False, True):
        seq = rsolve.Sequence(prob.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, precond="ssor", method="plain")
        if batched:
            out = rsolve.solve_batch([dict(seq=seq, row_ptr=rp, col_idx=ci, val=_t(vals, gpu_ctx), b=_t(b, gpu_ctx),
                                           tol=1e-10)])
            x, st, status = out[0]
        else:
            x, st, status = seq.solve(rp, ci, _t(vals, gpu_ctx), _t(b, gpu_ctx), tol=1e-10)
        res.append((x.cpu().numpy(), st["iterations"], status))
        seq.close()
    assert res[0][2] == 0 and res[1][2] == 0
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])


def test_ssor_config_limits(gpu_ctx):
    from paper_1807_09467_amd import rsolve
    bad = [dict(precision="fp32_ir"), dict(recycle_k=4, select="ritz"), dict(ssor_omega=2.0),
           dict(ssor_omega=-0.5)]
    for kw in bad:
        with pytest.raises(rsolve.RsolveError):
            rsolve.Sequence(1000, 5000, device=gpu_ctx, restart_m=30, precond="ssor", **kw)
    rsolve.Sequence(1000, 5000, device=gpu_ctx, restart_m=30, precond="ssor", ssor_omega=0.0).close()
