"""The library's SSOR colouring (host code behind RSOLVE_PRECOND_SSOR, exported as
rsolve_colour_first_fit) against the oracle's, which implements first fit over the symmetrised
pattern on its own: bit-exact colours on the workload meshes and on random nonsymmetric
patterns, and the library's own checks of its arguments.  CPU only: the colouring does not use
the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import rgmres as O
from paper_1807_09467_amd import rsolve
from paper_1807_09467_amd import workload as WL


def _pattern(prob):
    asm = WL.Assembler(prob)
    return asm.csr(asm.matrix_values(np.zeros(prob.n)))


@pytest.mark.parametrize("prob", [WL.PAPER_Q1[1e-2], WL.C3_SMALL, WL.C2_SMALL, WL.PAPER_SEM8],
                         ids=["q1_64", "c3_small", "c2_small", "sem8"])
def test_colouring_matches_the_oracle_on_meshes(prob):
    A = _pattern(prob)
    col, nc = rsolve.colour_first_fit(A.indptr, A.indices)
    ref = O.greedy_colouring(A)
    assert np.array_equal(col, ref) and nc == ref.max() + 1


@pytest.mark.parametrize("seed", range(6))
def test_colouring_matches_the_oracle_on_nonsymmetric_patterns(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    R = sp.random(n, n, density=float(rng.uniform(0.005, 0.2)), random_state=rng, format="csr")
    A = (R + sp.identity(n)).tocsr()
    A.sort_indices()
    col, nc = rsolve.colour_first_fit(A.indptr, A.indices)
    ref = O.greedy_colouring(A)
    assert np.array_equal(col, ref) and nc == ref.max() + 1
    coo = A.tocoo()
    off = coo.row != coo.col
    assert not np.any(col[coo.row[off]] == col[coo.col[off]])


def test_colouring_rejects_bad_patterns():
    rp = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(rsolve.RsolveError):
        rsolve.colour_first_fit(rp, np.array([0, 2], dtype=np.int32))     # column out of range
    with pytest.raises(rsolve.RsolveError):
        rsolve.colour_first_fit(np.array([0, 2, 1], dtype=np.int32), np.array([0, 1], dtype=np.int32))
