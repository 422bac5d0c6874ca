"""GPU tests of the serving loop (rsolve_server_*): a sequence gives bitwise the same solutions
alone and in a mix of others of uneven size (batched and large paths, overlapping on the
device); admission refuses what the pool cannot hold and admits it once memory frees up; a
failing request does not disturb its neighbours; served solutions match the oracle."""
import numpy as np
import pytest

from oracle import rgmres as O
from paper_1807_09467_amd import workload as WL

pytestmark = pytest.mark.gpu

CFG = dict(restart_m=30, recycle_k=10, snapshots_s=20, precond="jacobi")


def _specs():
    from paper_1807_09467_amd.serve import SeqSpec
    # three one-block sizes and two multi-kernel sizes (n = 103,041 and 66,049), staggered arrivals
    return [SeqSpec(0, 0.000, 1, 32, 1e-2, 5, 11), SeqSpec(1, 0.002, 2, 160, 1e-3, 4, 12),
            SeqSpec(2, 0.004, 3, 24, 1e-4, 5, 13), SeqSpec(3, 0.006, 2, 128, 3e-2, 4, 14),
            SeqSpec(4, 0.008, 1, 64, 5e-3, 6, 15), SeqSpec(5, 0.010, 2, 32, 1e-3, 5, 16)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_serving_alone_equals_mixed_bitwise(gpu_ctx, precision):
    """precision fp32_ir: the large sequences run FP32 Arnoldi cycles inside FP64 refinement (as
    in the serving replay), the batched small ones stay FP64."""
    import torch
    from paper_1807_09467_amd import serve
    specs = _specs()
    cache = serve.AssemblerCache(gpu_ctx)
    keep = {s.idx for s in specs}
    cfg = dict(CFG, precision=precision, inner_tol=1e-4) if precision == "fp32_ir" else CFG
    _, summ, mixed = serve.run_serving(specs, cfg, 1e-8, gpu_ctx, 4 << 30, large_workers=2, cache=cache,
                                       keep_solutions=keep)
    assert summ["all_converged"] and summ["solves"] == sum(s.steps for s in specs)
    assert 0.0 < summ["batched_fraction"] < 1.0
    for sp in specs:
        alone_spec = serve.SeqSpec(sp.idx, 0.0, sp.p, sp.N, sp.eps, sp.steps, sp.seed)
        _, _, alone = serve.run_serving([alone_spec], cfg, 1e-8, gpu_ctx, 4 << 30, large_workers=2, cache=cache,
                                        keep_solutions={sp.idx})
        assert len(alone[sp.idx]) == sp.steps
        for i, (xa, xm) in enumerate(zip(alone[sp.idx], mixed[sp.idx])):
            assert torch.equal(xa, xm), (sp.idx, i)


def test_serving_matches_oracle_on_small_sequences(gpu_ctx):
    """Two Q1 32x32 sequences through the server (batched path) against the oracle's recycled
    FP64 GMRES(30) on the same trajectory (each step assembled from the served solution)."""
    from paper_1807_09467_amd import serve
    specs = [serve.SeqSpec(0, 0.0, 1, 32, 1e-2, 6, 21), serve.SeqSpec(1, 0.001, 1, 32, 1e-2, 6, 22)]
    cfg = dict(restart_m=30, recycle_k=5, snapshots_s=10)
    _, summ, kept = serve.run_serving(specs, cfg, 1e-10, gpu_ctx, 1 << 30, large_workers=1,
                                      keep_solutions={0, 1})
    assert summ["batched_fraction"] == 1.0
    for sp in specs:
        prob = sp.problem()
        asm = WL.Assembler(prob)
        ocfg = O.Config(restart_m=30, recycle_k=5, snapshots_s=10)
        st = O.RecycleState(asm.pat.n, ocfg)
        u = WL.initial_condition(prob, sp.seed)
        for i, xg in enumerate(kept[sp.idx]):
            vals, b = asm.system(u)
            ores = O.solve(asm.csr(vals), b, u, 1e-10, ocfg, st.W)
            st.update(ores.x)
            xg = xg.cpu().numpy()
            assert np.linalg.norm(xg - ores.x) <= 1e-9 * np.linalg.norm(ores.x), (sp.idx, i)
            u = xg          # the served trajectory drives the next system, as in the server run


def test_admission_by_pool_memory(gpu_ctx):
    from paper_1807_09467_amd import rsolve, serve
    n, nnz = 263169, 4198401
    need = rsolve.workspace_bytes(rsolve.make_config(**CFG), n, nnz)
    srv = serve.Server(int(need * 1.5), gpu_ctx, large_workers=1)
    a = srv.open(n, nnz, **CFG)
    assert a is not None
    assert srv.open(n, nnz, **CFG) is None            # no room for a second one
    info = srv.info()
    assert info["sequences"] == 1 and info["pool_used"] >= need
    small = srv.open(1089, 9409, restart_m=30, recycle_k=5, snapshots_s=10)
    assert small is not None                           # a small one still fits
    srv.close(a)
    b = srv.open(n, nnz, **CFG)                        # memory freed: admitted now
    assert b is not None
    srv.close(b)
    srv.close(small)
    assert srv.info()["pool_used"] == 0
    slots = serve.Server(1 << 28, gpu_ctx, large_workers=1, max_sequences=2)
    ids = [slots.open(1089, 9409, restart_m=30) for _ in range(3)]
    assert ids[0] is not None and ids[1] is not None and ids[2] is None
    srv.destroy()
    slots.destroy()


def test_failed_request_is_isolated(gpu_ctx):
    import torch
    from paper_1807_09467_amd import rsolve, serve
    srv = serve.Server(1 << 30, gpu_ctx, large_workers=1)
    prob = WL.C1
    asm = WL.Assembler(prob)
    gasm = WL.GpuAssembler(asm, gpu_ctx)
    pat = asm.pat
    u = torch.from_numpy(WL.initial_condition(prob, 0)).to(gpu_ctx)
    vals, b = gasm.system(u)
    torch.cuda.synchronize()
    bad_ci = gasm.col_idx.clone()
    bad_ci[100] = pat.n + 7                            # column out of range: refused by the check
    ids = [srv.open(pat.n, pat.nnz, restart_m=30, recycle_k=5, snapshots_s=10) for _ in range(3)]
    xs = [torch.empty(pat.n, dtype=torch.float64, device=gpu_ctx) for _ in range(3)]
    for q, sid in enumerate(ids):
        srv.submit(sid, gasm.row_ptr, bad_ci if q == 1 else gasm.col_idx, vals, b, u, xs[q], 1e-10, tag=q + 1)
    got = {}
    while len(got) < 3:
        for c in srv.poll(timeout_ms=100):
            got[c["tag"]] = c
    assert got[2]["status"] == rsolve.E_INVALID
    assert got[1]["status"] == 0 and got[3]["status"] == 0
    assert torch.equal(xs[0], xs[2])
    ref = O.solve(asm.csr(vals.cpu().numpy()), b.cpu().numpy(), u.cpu().numpy(), 1e-10,
                  O.Config(restart_m=30, recycle_k=5, snapshots_s=10), None)
    assert np.linalg.norm(xs[0].cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    # the sequence that failed serves its next request normally
    srv.submit(ids[1], gasm.row_ptr, gasm.col_idx, vals, b, u, xs[1], 1e-10, tag=9)
    c = []
    while not c:
        c = srv.poll(timeout_ms=100)
    assert c[0]["status"] == 0 and torch.equal(xs[1], xs[0])
    for sid in ids:
        srv.close(sid)
    srv.destroy()


def test_serving_ssor_sequences(gpu_ctx):
    """Sequences configured with multicolour SSOR are served on the multi-kernel path (none is
    batched) and give bitwise the same solutions alone and in the mix."""
    import torch
    from paper_1807_09467_amd import serve
    specs = [serve.SeqSpec(0, 0.000, 1, 32, 1e-2, 4, 31), serve.SeqSpec(1, 0.002, 2, 64, 1e-3, 3, 32),
             serve.SeqSpec(2, 0.004, 1, 96, 5e-3, 3, 33)]
    cfg = dict(restart_m=30, recycle_k=6, snapshots_s=8, precond="ssor")
    cache = serve.AssemblerCache(gpu_ctx)
    _, summ, mixed = serve.run_serving(specs, cfg, 1e-8, gpu_ctx, 2 << 30, large_workers=2, cache=cache,
                                       keep_solutions={s.idx for s in specs})
    assert summ["all_converged"] and summ["batched_fraction"] == 0.0
    for sp in specs:
        alone_spec = serve.SeqSpec(sp.idx, 0.0, sp.p, sp.N, sp.eps, sp.steps, sp.seed)
        _, _, alone = serve.run_serving([alone_spec], cfg, 1e-8, gpu_ctx, 2 << 30, large_workers=2, cache=cache,
                                        keep_solutions={sp.idx})
        for i, (xa, xm) in enumerate(zip(alone[sp.idx], mixed[sp.idx])):
            assert torch.equal(xa, xm), (sp.idx, i)
