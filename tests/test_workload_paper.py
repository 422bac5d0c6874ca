"""Generator checks for the paper's own experiments (section 6.1): the vortex field, the random
low-mode forcing, the zero initial value and the Gauss-Lobatto support points of the order-23
Legendre spectral elements (section 6.3).  Closed forms and exact identities; CPU only."""
import math

import numpy as np
import pytest

from paper_1807_09467_amd import workload as WL


@pytest.mark.parametrize("p", [2, 5, 8, 23])
def test_gll_points_closed_form(p):
    """Interior GLL points are the roots of P_p', i.e. (1 - x^2) P_p'(x) vanishes at every point;
    they are symmetric about 1/2 and include the end points."""
    x = WL.support_points(p, "gll")
    assert x.size == p + 1 and x[0] == 0.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x + x[::-1], 1.0, atol=1e-14)
    t = 2 * x - 1
    dP = np.polynomial.legendre.Legendre.basis(p).deriv()(t)
    assert np.abs((1 - t * t) * dP).max() < 1e-11
    if p == 2:
        assert np.allclose(x, [0.0, 0.5, 1.0], atol=1e-15)


@pytest.mark.parametrize("p", [8, 23])
def test_gll_lagrange_basis_reproduces_polynomials(p):
    """On GLL points the order-p basis is nodal and reproduces x^p and its derivative exactly."""
    nodes = WL.support_points(p, "gll")
    V, D = WL.lagrange_1d(p, nodes, "gll")
    assert np.allclose(V, np.eye(p + 1), atol=1e-12)
    xq = np.linspace(0.0, 1.0, 37)
    V, D = WL.lagrange_1d(p, xq, "gll")
    f = nodes ** p
    assert np.allclose(V @ f, xq ** p, atol=1e-11)
    assert np.allclose(D @ f, p * xq ** (p - 1), atol=1e-8)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-12)


def test_sem_reference_matrices_identities():
    t = WL.element_tables(23, "gll")
    assert abs(t.mass_ref.sum() - 1.0) < 1e-12
    assert np.abs(t.stiff_ref @ np.ones(t.nl)).max() < 1e-9
    xq, wq = WL.gauss_01(25)
    V, D = WL.lagrange_1d(23, xq, "gll")
    M1 = (V * wq[:, None]).T @ V
    K1 = (D * wq[:, None]).T @ D
    assert np.allclose(t.mass_ref, np.kron(M1, M1), atol=1e-14)
    assert np.allclose(t.stiff_ref, np.kron(K1, M1) + np.kron(M1, K1), atol=1e-10)


def test_sem23_pattern_size():
    """2 x 2 elements of order 23: n = 47^2; rows of nodes on the shared element edges couple
    across both elements (47 node columns), the others to one element's 24."""
    pat = WL.build_pattern(WL.PAPER_SEM23)
    assert pat.n == 47 * 47
    lo, hi = WL._range_1d(23, 2)
    len1 = hi - lo + 1
    assert len1.sum() == 46 * 24 + 47          # 46 nodes inside one element's span, the shared vertex spans both
    assert pat.nnz == 1117433                   # full tensor pattern minus the Dirichlet rows / columns
    assert np.diff(pat.row_ptr).max() == 45 * 45   # the shared vertex row, boundary columns dropped


def test_vortex_field_and_convection_skew():
    """The vortex field is solenoidal and tangent to the boundary, so for u_prev = 1 the
    convection form (v, b.grad u) is skew on functions vanishing on the boundary: C + C^T = 0
    up to the quadrature error of the smooth field."""
    prob = WL.Problem(p=2, N=16, eps=0.0, dt=1e30, beta="vortex")
    asm = WL.Assembler(prob)
    x = np.linspace(0, 1, 101)
    X, Y = np.meshgrid(x, x)
    bx = -np.sin(math.pi * X) * np.cos(math.pi * Y)
    by = np.cos(math.pi * X) * np.sin(math.pi * Y)
    div = math.pi * (-np.cos(math.pi * X) * np.cos(math.pi * Y) + np.cos(math.pi * X) * np.cos(math.pi * Y))
    assert np.abs(div).max() == 0.0
    assert np.abs(bx[:, 0]).max() < 1e-15 and np.abs(by[0, :]).max() < 1e-15
    vals = asm.matrix_values(np.ones(asm.pat.n)) - asm.mass_values() / prob.dt
    C = asm.csr(vals).toarray()
    inner = ~asm.pat.boundary
    Ci = C[np.ix_(inner, inner)]
    assert np.abs(Ci + Ci.T).max() <= 1e-5 * np.abs(Ci).max()
    # the const field gives an exactly skew form (polynomial integrands)
    asm_c = WL.Assembler(WL.Problem(p=2, N=16, eps=0.0, dt=1e30, beta="const"))
    Cc = asm_c.csr(asm_c.matrix_values(np.ones(asm_c.pat.n))).toarray()[np.ix_(inner, inner)]
    assert np.abs(Cc + Cc.T).max() <= 1e-13 * np.abs(Cc).max()


@pytest.mark.parametrize("j", [1, 2, 3])
def test_forcing_load_closed_form_q1(j):
    """Q1 hats: the load of sin(w x) sin(w y), w = 2 j pi, at an interior node is
    sin(w x_i) sin(w y_i) (2 (1 - cos(w h)) / (w^2 h))^2, exact up to the Gauss rule's error."""
    prob = WL.PAPER_Q1[1e-2]
    asm = WL.Assembler(prob)
    L = asm.forcing_modes()[j - 1]
    h = 1.0 / prob.N
    w = 2 * j * math.pi
    xs = np.linspace(0, 1, prob.n1)
    X, Y = np.meshgrid(xs, xs)
    fac = 2 * (1 - math.cos(w * h)) / (w * w * h)
    exact = (np.sin(w * X) * np.sin(w * Y)).ravel() * fac * fac
    exact[asm.pat.boundary] = 0.0
    assert np.abs(L - exact).max() <= 1e-7 * np.abs(exact).max()


def test_forcing_coefficients_and_load():
    c = WL.forcing_coefficients(0, 50)
    assert c.shape == (50, 16)
    assert np.all(c[:, 0] == 1.0)
    assert np.all(np.abs(c[:, 1:]) <= 1.0)
    assert np.array_equal(c, WL.forcing_coefficients(0, 50))
    assert not np.array_equal(c[0], c[1])
    assert not np.array_equal(c, WL.forcing_coefficients(1, 50))
    # the load is linear in the coefficients with weights (C/2) exp(-j^2/20)
    asm = WL.Assembler(WL.PAPER_Q1[1e-1])
    e3 = np.zeros(16)
    e3[2] = 1.0
    assert np.allclose(asm.forcing_load(e3), 0.05 * math.exp(-9 / 20) * asm.forcing_modes()[2], rtol=0, atol=1e-18)


def test_paper_march_zero_start():
    """Zero initial value: the first right-hand side is the forcing load alone and the first
    matrix has no convection term; later steps convect with the previous solution."""
    prob = WL.PAPER_Q1[1e-2]
    asm, systems, states = WL.march(prob, 3, 0)
    c = WL.forcing_coefficients(0, 3)
    f0 = asm.forcing_load(c[0])
    f0[asm.pat.boundary] = 0.0
    assert np.allclose(systems[0][1], f0, rtol=0, atol=1e-18)
    A0 = asm.csr(systems[0][0])
    static = asm.csr(asm.matrix_values(np.zeros(prob.n)))
    assert abs(A0 - static).max() == 0.0
    r = systems[1][1] - (asm.csr(asm.mass_values()) @ states[0]) / prob.dt - asm.forcing_load(c[1])
    r[asm.pat.boundary] = 0.0
    assert np.abs(r).max() < 1e-14 * np.abs(systems[1][1]).max()
    assert all(np.linalg.norm(u) > 0 for u in states)


def test_device_assembler_refuses_paper_problems():
    import torch
    asm = WL.Assembler(WL.PAPER_Q1[1e-2])
    with pytest.raises(ValueError):
        WL.GpuAssembler(asm, torch.device("cpu"))


def _node_xy(prob):
    """Coordinates of the mesh nodes, node (I, J) at index J n1 + I."""
    s = WL.support_points(prob.p, prob.nodes)
    I = np.arange(prob.n1)
    e = np.minimum(I // prob.p, prob.N - 1)
    x1 = (e + s[I - e * prob.p]) / prob.N
    X, Y = np.meshgrid(x1, x1)
    return X.ravel(), Y.ravel()


@pytest.mark.parametrize("p,nodes", [(1, "equispaced"), (2, "equispaced"), (3, "gll")])
def test_l2_projection_reproduces_the_discrete_space(p, nodes):
    """Section 6.1's P_{V_h}: a function already in the continuous Q_p space (degree p in each
    variable) is its own projection, so the coefficients are its nodal values."""
    prob = WL.Problem(p=p, N=5, eps=1e-2, dt=0.5, beta="vortex", nodes=nodes)
    asm = WL.Assembler(prob)
    X, Y = _node_xy(prob)
    f = lambda x, y: (1.0 + x ** p) * (2.0 - 3.0 * y ** p) + x * y
    c = asm.l2_projection(f)
    assert np.abs(c - f(X, Y)).max() <= 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_l2_projection_of_the_vortex_converges_at_order_p_plus_one(p):
    """The L2 error of the projected vortex field falls as h^{p+1} (ratios near 2^{p+1} when h
    halves); the projection differs from the nodal interpolant by O(h^{p+1}) too but is not it."""
    errs = []
    for N in (8, 16, 32):
        prob = WL.Problem(p=p, N=N, eps=1e-2, dt=0.5, beta="vortex", beta_projected=True)
        asm = WL.Assembler(prob)
        bx, by = asm._beta_at_quad()
        x, y = asm.quad_points()
        fx, fy = WL.beta_field(prob)
        wq = (asm.h ** 2) * asm.tab.w[None, :]
        errs.append(math.sqrt(float(np.sum(((bx - fx(x, y)) ** 2 + (by - fy(x, y)) ** 2) * wq))))
        if N == 8:
            X, Y = _node_xy(prob)
            assert np.abs(asm.l2_projection(fx) - fx(X, Y)).max() > 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 2 ** (p + 1) * 0.8 <= a / b <= 2 ** (p + 1) * 1.25, errs


def test_paper_problems_project_the_velocity():
    assert all(prob.beta_projected for prob in WL.PAPER_Q1.values())
    assert WL.PAPER_SEM23.beta_projected and WL.PAPER_SEM8.beta_projected
