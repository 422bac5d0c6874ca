"""Generator checks: Q_p element matrices against closed forms and exact identities,
pattern sizes, Dirichlet rows.  CPU only."""
import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL


def test_q1_reference_matrices_closed_form():
    t = WL.element_tables(1)
    M = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
    K = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(t.mass_ref, M, atol=1e-15)
    assert np.allclose(t.stiff_ref, K, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reference_matrices_identities(p):
    t = WL.element_tables(p)
    # partition of unity: mass entries sum to the element area, stiffness annihilates constants
    assert abs(t.mass_ref.sum() - 1.0) < 1e-14
    assert np.abs(t.stiff_ref @ np.ones(t.nl)).max() < 1e-13
    # the 2-D matrices are tensor products of the 1-D ones (uniform tensor mesh)
    xq, wq = WL.gauss_01(p + 2)
    V, D = WL.lagrange_1d(p, xq)
    M1 = (V * wq[:, None]).T @ V
    K1 = (D * wq[:, None]).T @ D
    assert np.allclose(t.mass_ref, np.kron(M1, M1), atol=1e-15)
    assert np.allclose(t.stiff_ref, np.kron(K1, M1) + np.kron(M1, K1), atol=1e-13)
    # 1-D Lagrange basis is nodal
    Vn, _ = WL.lagrange_1d(p, np.linspace(0, 1, p + 1))
    assert np.allclose(Vn, np.eye(p + 1), atol=1e-14)


def _nnz_full_formula(p, N):
    s1 = (N - 1) * (2 * p + 1) + 2 * (p + 1) + N * (p - 1) * (p + 1)
    return s1 * s1


@pytest.mark.parametrize("prob,nnz", [(WL.C1, 8409), (WL.C2, 4159569)])
def test_pattern_sizes(prob, nnz):
    pat = WL.build_pattern(prob)
    assert pat.n == (prob.N * prob.p + 1) ** 2
    assert pat.nnz == nnz
    assert pat.row_ptr[0] == 0 and pat.row_ptr[-1] == nnz
    assert pat.col_idx.dtype == np.int32 and pat.row_ptr.dtype == np.int32


@pytest.mark.parametrize("prob", [WL.C1, WL.C2_SMALL, WL.C3_SMALL])
def test_pattern_against_assembled_coo(prob):
    """CSR pattern / element map agree with a plain COO assembly of the same element matrices."""
    import scipy.sparse as sp
    asm = WL.Assembler(prob)
    pat = asm.pat
    u = WL.initial_condition(prob, 1)
    ev = asm.element_values(u)
    E, nl = pat.elem_nodes.shape
    rows = np.repeat(pat.elem_nodes, nl, axis=1).ravel()
    cols = np.tile(pat.elem_nodes, (1, nl)).ravel()
    full = sp.coo_matrix((ev.ravel(), (rows, cols)), shape=(pat.n, pat.n)).tocsr()
    full.sum_duplicates()
    # Dirichlet elimination by hand
    inter = ~pat.boundary
    ref = full[inter][:, inter].toarray()
    A = asm.csr(asm.matrix_values(u)).toarray()
    assert np.allclose(A[np.ix_(inter, inter)], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    assert np.array_equal(A[pat.boundary], np.eye(pat.n)[pat.boundary])
    assert not A[np.ix_(inter, pat.boundary)].any()
    # sorted, unique columns with a stored diagonal
    rp = pat.row_ptr.astype(np.int64)
    for i in range(0, pat.n, max(1, pat.n // 50)):
        c = pat.col_idx[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


@pytest.mark.parametrize("prob", [WL.C1, WL.C3_SMALL])
def test_convection_is_skew_for_constant_coefficient(prob):
    """With u_prev = 1 and a solenoidal beta, (v, beta.grad u) is skew on interior nodes
    (integration by parts), so A - A^T = 2 C there; the symmetric part is M/dt + eps K."""
    asm = WL.Assembler(prob)
    pat = asm.pat
    one = np.ones(pat.n)
    A = asm.csr(asm.matrix_values(one)).toarray()
    inter = ~pat.boundary
    Ai = A[np.ix_(inter, inter)]
    zero = WL.Assembler(prob, pat).csr(asm.matrix_values(np.zeros(pat.n))).toarray()[np.ix_(inter, inter)]
    S = 0.5 * (Ai + Ai.T)
    assert np.allclose(S, zero, atol=1e-12 * np.abs(zero).max())


def test_rhs_and_mass():
    prob = WL.C2_SMALL
    asm = WL.Assembler(prob)
    u = WL.initial_condition(prob, 3)
    b = asm.rhs(u)
    assert not b[asm.pat.boundary].any()
    # mass matrix of the full space integrates constants: sum of all entries = area (interior part less)
    Mv = asm.mass_values()
    assert Mv.sum() < 1.0 and Mv.sum() > 0.9
    assert u[asm.pat.boundary].max() == 0.0 and abs(u.max() - 1.0) < 0.05


def test_march_is_deterministic_and_direct():
    _, s1, x1 = WL.march(WL.C1, 3, 5)
    _, s2, x2 = WL.march(WL.C1, 3, 5)
    for (v1, b1), (v2, b2) in zip(s1, s2):
        assert np.array_equal(v1, v2) and np.array_equal(b1, b2)
    asm = WL.Assembler(WL.C1)
    A = asm.csr(s1[2][0])
    assert np.linalg.norm(A @ x1[2] - s1[2][1]) <= 1e-12 * np.linalg.norm(s1[2][1])
