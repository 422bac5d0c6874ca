"""Captured Arnoldi chunks (hipGraph): the same sequence solved with graphs on and off gives
bitwise the same solutions and iteration counts.  Each graph is replayed many times (every
cycle of every solve), with the solver's own eager kernels, copies and synchronisations between
the replays, and every replayed solve is checked against the eager one."""
import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("kw", [
    dict(restart_m=30, recycle_k=8, snapshots_s=12, precond="jacobi"),
    dict(restart_m=50, recycle_k=16, snapshots_s=32, precond="jacobi", precision="fp32_ir", inner_tol=1e-5),
    dict(restart_m=10, recycle_k=4, snapshots_s=6, precond="none"),
    dict(restart_m=30, recycle_k=8, snapshots_s=12, precond="jacobi", ortho="dcgs2"),
    dict(restart_m=50, recycle_k=16, snapshots_s=32, precond="jacobi", precision="fp32_ir", inner_tol=1e-5,
         ortho="dcgs2"),
])
def test_graph_replay_equals_eager(gpu_ctx, kw):
    import torch
    from paper_1807_09467_amd import rsolve
    prob = WL.C3_SMALL
    asm, systems, _ = WL.march(prob, 6, 4)
    rp, ci = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx)
    gv = [(_t(v, gpu_ctx), _t(b, gpu_ctx)) for v, b in systems]
    tol = 1e-8 if kw.get("precision") == "fp32_ir" else 1e-10
    out = {}
    for on in (False, True):
        seq = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, **kw)
        seq.graphs(on)
        x_prev = torch.zeros(asm.pat.n, dtype=torch.float64, device=gpu_ctx)
        res = []
        for i, (v, b) in enumerate(gv):
            x, st, status = seq.solve(rp, ci, v, b, x0=x_prev, tol=tol, same_pattern=i > 0)
            assert status == 0 and st["converged"] == 1
            seq.update()
            res.append((x.clone(), st["iterations"], st["cycles"]))
            x_prev = x
        cap, launches = seq.graph_counts()
        if on:
            assert cap > 0 and launches > cap
        else:
            assert cap == 0 and launches == 0
        out[on] = res
        seq.close()
    for i, (a, b) in enumerate(zip(out[False], out[True])):
        assert torch.equal(a[0], b[0]), i
        assert a[1:] == b[1:], i


def test_graphs_requested_for_ssor_run_eagerly(gpu_ctx):
    """Multicolour SSOR sequences capture no graphs (their sweeps depend on the pattern's colour
    count); with graphs requested they run eagerly and give bitwise the eager results."""
    import torch
    from paper_1807_09467_amd import rsolve
    prob = WL.C3_SMALL
    asm, systems, _ = WL.march(prob, 3, 4)
    rp, ci = _t(asm.pat.row_ptr, gpu_ctx), _t(asm.pat.col_idx, gpu_ctx)
    out = {}
    for on in (False, True):
        seq = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=gpu_ctx, restart_m=30, recycle_k=6, snapshots_s=8,
                              precond="ssor")
        seq.graphs(on)
        x_prev = torch.zeros(asm.pat.n, dtype=torch.float64, device=gpu_ctx)
        res = []
        for i, (v, b) in enumerate(systems):
            x, st, status = seq.solve(rp, ci, _t(v, gpu_ctx), _t(b, gpu_ctx), x0=x_prev, tol=1e-10,
                                      same_pattern=i > 0)
            assert status == 0 and st["converged"] == 1
            seq.update()
            res.append((x.clone(), st["iterations"]))
            x_prev = x
        assert seq.graph_counts() == (0, 0)
        out[on] = res
        seq.close()
    for a, b in zip(out[False], out[True]):
        assert torch.equal(a[0], b[0]) and a[1] == b[1]
