"""The GPU assembler (qkgen) reproduces the CPU generator's systems."""
import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prob", [WL.C1, WL.C2_SMALL, WL.C3_SMALL])
def test_gpu_assembly_matches_host(gpu_ctx, prob):
    import torch
    asm = WL.Assembler(prob)
    gasm = WL.GpuAssembler(asm, gpu_ctx)
    rng = np.random.default_rng(1)
    u = WL.initial_condition(prob, 3) + 0.1 * rng.standard_normal(asm.pat.n)
    u[asm.pat.boundary] = 0.0
    vals, b = asm.system(u)
    gv, gb = gasm.system(torch.from_numpy(u).to(gpu_ctx))
    gv, gb = gv.cpu().numpy(), gb.cpu().numpy()
    assert np.abs(gv - vals).max() <= 1e-13 * np.abs(vals).max()
    assert np.abs(gb - b).max() <= 1e-13 * np.abs(b).max()
    assert np.array_equal(gasm.row_ptr.cpu().numpy(), asm.pat.row_ptr)
