"""GPU parity of the batched one-block path (rsolve_solve_batch / rsolve_update_recycle_batch)
against the FP64 oracle, and its isolation properties: a sequence solved alone and inside a
batch of others gives bitwise the same answer, and a corrupt item fails alone."""
import numpy as np
import pytest

from oracle import rgmres as O
from paper_1807_09467_amd import workload as WL

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _ocfg(kw):
    return O.Config(restart_m=kw.get("restart_m", 30), recycle_k=kw.get("recycle_k", 0),
                    snapshots_s=kw.get("snapshots_s", 0), svd_interval=kw.get("svd_interval", 1),
                    method={"plain": O.PLAIN, "aug_oblique": O.AUG_OBLIQUE, "defl_oblique": O.DEFL_OBLIQUE}[
                        kw.get("method", "aug_oblique")],
                    precond=O.PRECOND_JACOBI if kw.get("precond") == "jacobi" else O.PRECOND_NONE)


class Stream:
    """One generated sequence driven through the batch calls, with the oracle beside it."""

    def __init__(self, dev, prob, steps, seed, tol, **kw):
        from paper_1807_09467_amd import rsolve
        import torch
        self.asm, self.systems, _ = WL.march(prob, steps, seed)
        pat = self.asm.pat
        self.rp, self.ci = _t(pat.row_ptr, dev), _t(pat.col_idx, dev)
        self.seq = rsolve.Sequence(pat.n, pat.nnz, device=dev, **kw)
        self.ocfg = _ocfg(kw)
        self.ost = O.RecycleState(pat.n, self.ocfg)
        self.tol = tol
        self.dev = dev
        self.x_prev = torch.zeros(pat.n, dtype=torch.float64, device=dev)
        self.xo_prev = np.zeros(pat.n)
        self.gpu_vals = [(_t(v, dev), _t(b, dev)) for v, b in self.systems]

    def job(self, i):
        vals, b = self.gpu_vals[i]
        return dict(seq=self.seq, row_ptr=self.rp, col_idx=self.ci, val=vals, b=b, x0=self.x_prev, tol=self.tol,
                    same_pattern=i > 0)

    def oracle(self, i):
        vals, b = self.systems[i]
        ores = O.solve(self.asm.csr(vals), b, self.xo_prev, self.tol, self.ocfg, self.ost.W)
        self.ost.update(ores.x)
        self.xo_prev = ores.x
        return ores


def _check(res, ores, rel_bar=1e-9, its_bar=2):
    x, st, status = res
    assert status == 0 and st["converged"] == 1
    xg = x.cpu().numpy()
    rel = np.linalg.norm(xg - ores.x) / np.linalg.norm(ores.x)
    assert rel <= rel_bar, rel
    assert abs(st["iterations"] - ores.iterations) <= its_bar, (st["iterations"], ores.iterations)
    assert st["k_eff"] == ores.k_eff, (st["k_eff"], ores.k_eff)


def test_batch_c1_full_sequence_vs_oracle(gpu_ctx):
    """Q1 32x32, 20 steps, GMRES(30), k=5, s=10, tol 1e-10, every solve and update batched."""
    from paper_1807_09467_amd import rsolve
    s = Stream(gpu_ctx, WL.C1, 20, 0, 1e-10, restart_m=30, recycle_k=5, snapshots_s=10)
    for i in range(20):
        [res] = rsolve.solve_batch([s.job(i)])
        ores = s.oracle(i)
        _check(res, ores)
        assert rsolve.update_batch([s.seq]) == [0]
        rec = s.seq.recycle()
        assert rec["k_eff"] == s.ost.W.shape[1] and rec["rank"] == s.ost.rank
        c = len(s.ost.sigma)
        assert np.all(np.abs(np.array(rec["sigma"][:c]) - s.ost.sigma) <= 1e-9 * s.ost.sigma[0])
        s.x_prev = res[0]
    s.seq.close()


@pytest.mark.parametrize("prob,m,k,sn", [(WL.C2_SMALL, 30, 10, 20), (WL.C3_SMALL, 50, 16, 32)])
def test_batch_jacobi_vs_oracle(gpu_ctx, prob, m, k, sn):
    from paper_1807_09467_amd import rsolve
    s = Stream(gpu_ctx, prob, 8, 1, 1e-10, restart_m=m, recycle_k=k, snapshots_s=sn, precond="jacobi")
    for i in range(8):
        [res] = rsolve.solve_batch([s.job(i)])
        _check(res, s.oracle(i))
        rsolve.update_batch([s.seq])
        s.x_prev = res[0]
    s.seq.close()


def test_batch_alone_equals_mixed_bitwise(gpu_ctx):
    """Six sequences of three sizes: each solved alone, then all in one batch, step by step.
    The one-block computation of an item does not depend on its neighbours."""
    import torch
    from paper_1807_09467_amd import rsolve
    specs = [(WL.C1, 0), (WL.C1, 3), (WL.C2_SMALL, 1), (WL.C1, 5), (WL.C3_SMALL, 2), (WL.C2_SMALL, 4)]
    kws = [dict(restart_m=30, recycle_k=5, snapshots_s=10) if p is WL.C1 else
           dict(restart_m=30, recycle_k=8, snapshots_s=12, precond="jacobi") for p, _ in specs]
    steps = 5
    alone = []
    for (p, seed), kw in zip(specs, kws):
        s = Stream(gpu_ctx, p, steps, seed, 1e-10, **kw)
        xs = []
        for i in range(steps):
            [res] = rsolve.solve_batch([s.job(i)])
            rsolve.update_batch([s.seq])
            s.x_prev = res[0]
            xs.append((res[0].clone(), res[1]["iterations"]))
        s.seq.close()
        alone.append(xs)
    streams = [Stream(gpu_ctx, p, steps, seed, 1e-10, **kw) for (p, seed), kw in zip(specs, kws)]
    for i in range(steps):
        out = rsolve.solve_batch([s.job(i) for s in streams])
        rsolve.update_batch([s.seq for s in streams])
        for q, (s, res) in enumerate(zip(streams, out)):
            assert torch.equal(res[0], alone[q][i][0]), (q, i)
            assert res[1]["iterations"] == alone[q][i][1]
            s.x_prev = res[0]
    for s in streams:
        s.seq.close()


def test_batch_routes_outside_limits_through_the_multikernel_path(gpu_ctx):
    """A mixed-precision sequence and a restart above the one-block limit share a batch with
    a one-block item; all three meet their oracle bars."""
    from paper_1807_09467_amd import rsolve
    small = Stream(gpu_ctx, WL.C1, 3, 0, 1e-10, restart_m=30, recycle_k=5, snapshots_s=10)
    mixed = Stream(gpu_ctx, WL.C3_SMALL, 3, 0, 1e-8, precision="fp32_ir", restart_m=50, recycle_k=16,
                   snapshots_s=32, precond="jacobi", inner_tol=1e-5)
    long_m = Stream(gpu_ctx, WL.C2_SMALL, 3, 0, 1e-10, restart_m=80, recycle_k=4, snapshots_s=8, precond="jacobi")
    for i in range(3):
        out = rsolve.solve_batch([small.job(i), mixed.job(i), long_m.job(i)])
        rsolve.update_batch([small.seq, mixed.seq, long_m.seq])
        _check(out[0], small.oracle(i))
        _check(out[2], long_m.oracle(i))
        om = mixed.oracle(i)
        x, st, status = out[1]
        assert status == 0 and st["converged"] == 1
        A, b = mixed.asm.csr(mixed.systems[i][0]), mixed.systems[i][1]
        xg = x.cpu().numpy()
        assert np.linalg.norm(b - A @ xg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)
        kappa = np.linalg.cond(A.toarray(), 1)
        assert np.linalg.norm(xg - om.x) / np.linalg.norm(om.x) <= max(1e-8, 2 * kappa * 1e-8)
        for s, res in zip((small, mixed, long_m), out):
            s.x_prev = res[0]
    for s in (small, mixed, long_m):
        s.seq.close()


def test_batch_corrupt_item_fails_alone(gpu_ctx):
    from paper_1807_09467_amd import rsolve
    good = Stream(gpu_ctx, WL.C1, 2, 0, 1e-10, restart_m=30)
    bad = Stream(gpu_ctx, WL.C1, 2, 1, 1e-10, restart_m=30)
    pat = bad.asm.pat
    for mutate in ("col_out_of_range", "unsorted", "row_ptr_overflow", "no_diagonal"):
        rp, ci = pat.row_ptr.copy(), pat.col_idx.copy()
        if mutate == "col_out_of_range":
            ci[100] = pat.n + 7
        elif mutate == "unsorted":
            a = rp[200]
            ci[a], ci[a + 1] = ci[a + 1], ci[a]
        elif mutate == "row_ptr_overflow":
            rp[300] = pat.nnz + 1000
        elif mutate == "no_diagonal":
            ci[rp[0]] = 1 if ci[rp[0]] != 1 else 2
        bj = bad.job(0)
        bj["row_ptr"], bj["col_idx"], bj["same_pattern"] = _t(rp, gpu_ctx), _t(ci, gpu_ctx), False
        out = rsolve.solve_batch([good.job(0), bj], check=False)
        assert out[1][2] == rsolve.E_INVALID, mutate
        _check(out[0], O.solve(good.asm.csr(good.systems[0][0]), good.systems[0][1], None, 1e-10, good.ocfg, None))
    # the corrupted sequence works again with its real pattern
    [res] = rsolve.solve_batch([bad.job(0)])
    _check(res, bad.oracle(0))
    good.seq.close()
    bad.seq.close()


def test_batch_zero_rhs_nonfinite_and_duplicates(gpu_ctx):
    import torch
    from paper_1807_09467_amd import rsolve
    s = Stream(gpu_ctx, WL.C1, 1, 0, 1e-10, restart_m=10)
    j = s.job(0)
    j["b"] = torch.zeros(s.seq.n, dtype=torch.float64, device=gpu_ctx)
    j["x0"] = torch.ones(s.seq.n, dtype=torch.float64, device=gpu_ctx)
    [(x, st, status)] = rsolve.solve_batch([j])
    assert status == 0 and st["iterations"] == 0 and not x.any()
    j = s.job(0)
    b = j["b"].clone()
    b[5] = float("nan")
    j["b"] = b
    [(_, _, status)] = rsolve.solve_batch([j], check=False)
    assert status == rsolve.E_NONFINITE
    # the same sequence twice in one batch: the second entry is refused, the first runs
    out = rsolve.solve_batch([s.job(0), s.job(0)], check=False)
    assert out[0][2] == 0 and out[1][2] == rsolve.E_INVALID
    s.seq.close()


@pytest.mark.parametrize("n,c,k", [(1089, 10, 5), (4000, 20, 10), (30000, 32, 16)])
def test_batch_update_subspace_against_lapack(gpu_ctx, n, c, k):
    """Push c synthetic snapshots with a graded spectrum; the one-block update's W spans the
    leading singular subspace of LAPACK's SVD, is orthonormal, and the rank rule agrees."""
    import torch
    from paper_1807_09467_amd import rsolve
    rng = np.random.default_rng(c + n)
    U, _ = np.linalg.qr(rng.standard_normal((n, c)))
    Vt, _ = np.linalg.qr(rng.standard_normal((c, c)))
    sig = 10.0 ** (-0.35 * np.arange(c))
    X = (U * sig) @ Vt.T
    seq = rsolve.Sequence(n, n, device=gpu_ctx, restart_m=max(c, 30), recycle_k=k, snapshots_s=c)
    cols = [_t(X[:, i], gpu_ctx) for i in range(c)]
    for i in range(c):
        assert rsolve.update_batch([seq], [cols[i]]) == [0]
    rec = seq.recycle(with_basis=True)
    s_ref = np.linalg.svd(X, compute_uv=False)
    rank_ref = int(np.sum(s_ref > s_ref[0] * max(n, c) * np.finfo(float).eps))
    assert rec["rank"] == rank_ref and rec["k_eff"] == min(k, rank_ref)
    assert np.all(np.abs(np.array(rec["sigma"][:c]) - s_ref) <= 64 * c * np.finfo(float).eps * s_ref[0])
    Wn = rec["W"].cpu().numpy().T
    keff = rec["k_eff"]
    assert np.abs(Wn.T @ Wn - np.eye(keff)).max() <= 1e-13
    Uk = np.linalg.svd(X, full_matrices=False)[0][:, :keff]
    cosines = np.linalg.svd(Uk.T @ Wn, compute_uv=False)
    gap = (s_ref[keff - 1] - s_ref[keff]) / s_ref[0] if keff < c else 1.0
    assert 1.0 - cosines.min() <= max(1e-24 / gap ** 2, 1e-14) * 100
    seq.close()


def test_batch_update_rank_deficient_ring(gpu_ctx):
    from paper_1807_09467_amd import rsolve
    rng = np.random.default_rng(9)
    n = 777
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    X = np.column_stack([x, y, x, 2 * y, x + y, 0 * x])
    seq = rsolve.Sequence(n, n, device=gpu_ctx, restart_m=10, recycle_k=4, snapshots_s=6)
    for i in range(6):
        rsolve.update_batch([seq], [_t(X[:, i], gpu_ctx)])
    rec = seq.recycle(with_basis=True)
    assert rec["rank"] == 2 and rec["k_eff"] == 2
    B, _ = np.linalg.qr(np.column_stack([x, y]))
    Wn = rec["W"].cpu().numpy().T
    assert np.linalg.svd(B.T @ Wn, compute_uv=False).min() >= 1 - 1e-12
    seq.close()


def test_batch_plan_matches_item_by_item_calls(gpu_ctx):
    """BatchPlan (vectorised pointer updates over a prebuilt item array) gives bitwise the same
    answers and statistics as solve_batch with per-call job dicts."""
    import torch
    from paper_1807_09467_amd import rsolve
    kw = dict(restart_m=30, recycle_k=5, snapshots_s=10)
    a = [Stream(gpu_ctx, WL.C1, 4, seed, 1e-10, **kw) for seed in (0, 1, 2)]
    b = [Stream(gpu_ctx, WL.C1, 4, seed, 1e-10, **kw) for seed in (0, 1, 2)]
    plan = rsolve.BatchPlan([s.seq for s in b], [s.rp for s in b], [s.ci for s in b], tol=1e-10)
    x_prev = [s.x_prev for s in b]
    for i in range(4):
        ref = rsolve.solve_batch([s.job(i) for s in a])
        rsolve.update_batch([s.seq for s in a])
        vals = [s.gpu_vals[i][0] for s in b]
        bs = [s.gpu_vals[i][1] for s in b]
        if i % 2 == 0:
            outs = plan.solve(vals, bs, x_prev, same_pattern=i > 0)
        else:   # address arrays and the previous round's outputs as starts
            outs = plan.solve(plan.pointers(vals), plan.pointers(bs), "previous", same_pattern=True,
                              nnz=np.array([v.numel() for v in vals]))
        plan.update()
        for q, s in enumerate(a):
            assert torch.equal(outs[q], ref[q][0])
            assert int(plan.view["iterations"][q]) == ref[q][1]["iterations"]
            assert int(plan.view["status"][q]) == 0
            s.x_prev = ref[q][0]
        x_prev = outs
    for s in a + b:
        s.seq.close()
