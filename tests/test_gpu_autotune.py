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
    assert len(res) == 30
    assert all(a["us"] <= b2["us"] for a, b2 in zip(res, res[1:]))
    assert {(r["lanes_per_row"], r["vec"], r["xcd_remap"]) for r in res} == {
        (l, e, m) for l in (2, 4, 8, 16, 32) for e in (1, 4, 8) for m in (0, 1)}
    kappa = np.linalg.cond(A.toarray(), 1)
    for r in res:
        seq.set_spmv_shape(r["lanes_per_row"], r["vec"], r["xcd_remap"])
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
    assert src == "timed" and len(allres) == 30 and best["us"] == allres[0]["us"]
    s2 = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, precond="jacobi")
    best2, src2, _ = autotune.tune_sequence(s2, rp, ci, v, cache_path=path)
    assert src2 == "cache" and best2["lanes_per_row"] == best["lanes_per_row"] and best2["vec"] == best["vec"]
    assert s2.spmv_shape()["lanes_per_row"] == best["lanes_per_row"]
    for bad in ((3, 4, 0), (4, 2, 0), (4, 4, 2), (64, 4, 0)):
        with pytest.raises(rsolve.RsolveError):
            s2.set_spmv_shape(*bad)
    # a corrupt pattern is refused before any candidate runs
    bad_ci = asm.pat.col_idx.copy()
    bad_ci[10] = asm.pat.n + 3
    with pytest.raises(rsolve.RsolveError):
        s2.tune_spmv(rp, _t(bad_ci, gpu_ctx), v, reps=1)
    s1.close()
    s2.close()
