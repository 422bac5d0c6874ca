"""The Gram product entry point that allocates nothing (rsolve_gram_tn_noalloc) against the one
that takes a workspace (rsolve_gram_tn): same kernels, so the same result, on two calls in a row
through the C-ABI, the second smaller than the first (the static scratch keeps the first call's
contents, which must not leak into the second); sizes beyond the scratch are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _pair(dev, n, p, q, seed):
    from paper_1807_09467_amd import rsolve
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((p, n))
    B = rng.standard_normal((q, n))
    At, Bt = _t(A, dev), _t(B, dev)
    print(f"[no_alloc] n={n} p={p} q={q}", flush=True)
    C_ws = rsolve.gram_tn(At, Bt)
    C_na, status = rsolve.gram_tn_noalloc(At, Bt)
    assert status == rsolve.OK
    ref = A @ B.T
    bound = 1e-14 * n * np.sqrt(np.outer((A * A).sum(1), (B * B).sum(1))) + 1e-300
    assert np.all(np.abs(C_na - ref) <= bound), np.abs(C_na - ref).max()
    # identical kernels, block counts and reduction order: the two entry points agree exactly
    assert np.array_equal(C_na, C_ws)


@pytest.mark.parametrize("first,second", [((200003, 64, 64), (1000, 5, 3)), ((70001, 16, 16), (63, 1, 1)),
                                          ((4097, 33, 40), (4096, 32, 40))])
def test_noalloc_gram_equals_workspace_gram_twice(gpu_ctx, first, second):
    _pair(gpu_ctx, *first, seed=1)
    _pair(gpu_ctx, *second, seed=2)


def test_noalloc_gram_rejects_sizes_beyond_scratch(gpu_ctx):
    import torch
    from paper_1807_09467_amd import rsolve
    A = torch.ones((65, 100), dtype=torch.float64, device=gpu_ctx)
    B = torch.ones((3, 100), dtype=torch.float64, device=gpu_ctx)
    C, status = rsolve.gram_tn_noalloc(A, B, check=False)
    assert C is None and status == rsolve.E_INVALID
    assert "at most 64" in rsolve.last_error()
    C, status = rsolve.gram_tn_noalloc(B, A, check=False)
    assert C is None and status == rsolve.E_INVALID
    # the entry point still works after the refusals
    C, status = rsolve.gram_tn_noalloc(B, B)
    assert status == rsolve.OK and np.allclose(C, 100.0)
