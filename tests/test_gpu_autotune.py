"""GPU tests of the SpMV shape autotuner: every candidate shape gives an oracle-matching solve
(each is a distinct kernel variant), the tuner ranks all of them, and the JSON cache is reused."""
import numpy as np
import pytest

from oracle import rgmres as O
from paper_1807_09467_amd import workload as WL

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_every_shape_solves_to_the_oracle(gpu_ctx, precision):
    from paper_1807_09467_amd import rsolve
    prob = WL.C3_SMALL
    asm = WL.Assembler(prob)
    u = WL.initial_condition(prob, 3)
    vals, b = asm.system(u)
    A = asm.csr(vals)
    rp, ci, v, bg = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx), _t(vals, gpu_ctx), _t(b, gpu_ctx)
    tol = 1e-10 if precision == "fp64" else 1e-8
    ref = O.solve(A, b, u, 1e-12, O.Config(restart_m=40, method=O.PLAIN, precond=O.PRECOND_JACOBI), None)
    seq = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=40, method="plain", precond="jacobi",
                          precision=precision, inner_tol=1e-5)
    res = seq.tune_spmv(rp, ci, v, reps=2)
    assert len(res) == 42
    assert all(a["us"] <= b2["us"] for a, b2 in zip(res, res[1:]))
    assert {(r["format"], r["lanes_per_row"], r["vec"], r["xcd_remap"]) for r in res} == {
        ("csr", l, e, m) for l in (2, 4, 8, 16, 32) for e in (1, 4, 8) for m in (0, 1)} | {
        ("banded", l, e, m) for l in (2, 4, 8) for e in (4, 8) for m in (0, 1)}
    kappa = np.linalg.cond(A.toarray(), 1)
    for r in res:
        seq.set_spmv_shape(r["lanes_per_row"], r["vec"], r["xcd_remap"], r["format"])
        x, st, status = seq.solve(rp, ci, v, bg, x0=_t(u, gpu_ctx), tol=tol)
        assert status == 0 and st["converged"] == 1
        rel = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
        assert rel <= (1e-9 if precision == "fp64" else max(1e-8, 2 * kappa * 1e-8)), (r, rel)
    sh = seq.spmv_shape()
    assert sh["user_set"] and (sh["lanes_per_row"], sh["vec"]) == (res[-1]["lanes_per_row"], res[-1]["vec"])
    seq.close()


def test_tuner_cache_roundtrip_and_bad_shapes(gpu_ctx, tmp_path):
    from paper_1807_09467_amd import autotune, rsolve
    asm = WL.Assembler(WL.C2_SMALL)
    vals, b = asm.system(WL.initial_condition(WL.C2_SMALL, 0))
    rp, ci, v = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx), _t(vals, gpu_ctx)
    path = str(tmp_path / "shapes.json")
    s1 = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, precond="jacobi")
    best, src, allres = autotune.tune_sequence(s1, rp, ci, v, cache_path=path, reps=3)
    assert src == "timed" and len(allres) == 42 and best["us"] == allres[0]["us"]
    s2 = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, precond="jacobi")
    best2, src2, _ = autotune.tune_sequence(s2, rp, ci, v, cache_path=path)
    assert src2 == "cache" and best2["lanes_per_row"] == best["lanes_per_row"] and best2["vec"] == best["vec"]
    got = s2.spmv_shape()
    assert (got["format"], got["lanes_per_row"]) == (best["format"], best["lanes_per_row"])
    for bad in ((3, 4, 0), (4, 2, 0), (4, 4, 2), (64, 4, 0), (16, 8, 0, "banded"), (4, 1, 0, "banded"),
                (4, 8, 0, 2)):
        with pytest.raises(rsolve.RsolveError):
            s2.set_spmv_shape(*bad)
    # a corrupt pattern is refused before any candidate runs
    bad_ci = asm.pat.col_idx.copy()
    bad_ci[10] = asm.pat.n + 3
    with pytest.raises(rsolve.RsolveError):
        s2.tune_spmv(rp, _t(bad_ci, gpu_ctx), v, reps=1)
    s1.close()
    s2.close()


def test_banded_format_needs_a_narrow_band(gpu_ctx):
    """A pattern with an entry 40,000 columns off the diagonal does not fit the 16-bit offsets: the
    default shape falls back to CSR, the tuner offers CSR shapes only, and a solve with the
    banded format set by hand is refused."""
    import scipy.sparse as sp
    from paper_1807_09467_amd import rsolve
    n = 50000
    rng = np.random.default_rng(5)
    A = sp.diags([np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -1.0)], [-1, 0, 1], format="lil")
    for _ in range(12):                     # enough entries per row for the banded default otherwise
        A.setdiag(rng.uniform(-0.05, 0.05, n - 3), 3 + _)     # diagonally dominant
        A.setdiag(rng.uniform(-0.05, 0.05, n - 3), -3 - _)
    A[0, 40000] = 0.01
    A = A.tocsr()
    A.sort_indices()
    rp, ci = _t(A.indptr.astype(np.int32), gpu_ctx), _t(A.indices.astype(np.int32), gpu_ctx)
    v, b = _t(A.data, gpu_ctx), _t(np.ones(n), gpu_ctx)
    seq = rsolve.Sequence(n, A.nnz, device=gpu_ctx, restart_m=30)
    x, st, status = seq.solve(rp, ci, v, b, tol=1e-10)
    assert status == 0 and seq.spmv_shape()["format"] == "csr"
    assert np.linalg.norm(A @ x.cpu().numpy() - 1.0) <= 1e-9 * np.sqrt(n)
    res = seq.tune_spmv(rp, ci, v, reps=1)
    assert len(res) == 30 and all(r["format"] == "csr" for r in res)
    seq.set_spmv_shape(4, 8, 0, "banded")
    with pytest.raises(rsolve.RsolveError):
        seq.solve(rp, ci, v, b, tol=1e-10)
    seq.close()


def _ragged_banded(n, seed):
    """Diagonally dominant matrix with row lengths from 1 to 70 (rows of one entry, rows shorter
    and longer than a chunk round) and every column within 2,000 of its row."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        L = int(rng.choice([0, 1, 3, 7, 8, 9, 16, 31, 33, 69]))
        c = np.unique(np.clip(i + rng.integers(-2000, 2001, L), 0, n - 1))
        c = c[c != i]
        v = rng.uniform(-1.0, 1.0, c.size)
        rows += [i] * (c.size + 1)
        cols += list(c) + [i]
        vals += list(v) + [np.abs(v).sum() + 1.0 + rng.uniform()]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_banded_shapes_on_ragged_rows(gpu_ctx, precision):
    """Every banded shape (chunks of 4 and 8, 2/4/8 lanes, both block orders) on ragged rows,
    with and without Jacobi, against a direct solve."""
    import scipy.sparse.linalg as sla
    from paper_1807_09467_amd import rsolve
    n = 20011
    A = _ragged_banded(n, 9)
    b = np.random.default_rng(1).standard_normal(n)
    xref = sla.spsolve(A.tocsc(), b)
    rp, ci = _t(A.indptr.astype(np.int32), gpu_ctx), _t(A.indices.astype(np.int32), gpu_ctx)
    v, bg = _t(A.data, gpu_ctx), _t(b, gpu_ctx)
    tol = 1e-10 if precision == "fp64" else 1e-8
    for precond in ("none", "jacobi"):
        seq = rsolve.Sequence(n, A.nnz, device=gpu_ctx, restart_m=30, precond=precond, precision=precision,
                              inner_tol=1e-5)
        for l in (2, 4, 8):
            for e in (4, 8):
                for m in (0, 1):
                    seq.set_spmv_shape(l, e, m, "banded")
                    x, st, status = seq.solve(rp, ci, v, bg, tol=tol)
                    assert status == 0 and st["converged"] == 1, (precond, l, e, m)
                    rel = np.linalg.norm(x.cpu().numpy() - xref) / np.linalg.norm(xref)
                    assert rel <= 50 * tol, (precond, l, e, m, rel)
        seq.close()
