"""Seeded synthetic workload: sequences of convection-diffusion systems A_i x = b_i.

This module is the input generator shared by the tests, the benchmark and the
GPU solver's callers.  It holds finite-element assembly only, none of the
solver's arithmetic (no Krylov method, projector or SVD lives here).

What it builds (paper, section 2, eq. (def_Axb), and section 6.1): a scalar
equation u_t + div(0.5 u^2 beta) - eps Lap(u) = 0 on the unit square with a
solenoidal field beta, so the convection term is u beta.grad(u).  Time is
advanced by backward Euler and the non-linear term is linearised by lagging
its coefficient (Picard): step i solves

    (v, u^i)/dt + eps (grad v, grad u^i) + (v, u^{i-1} beta.grad u^i) = (v, u^{i-1})/dt

so every step yields one non-symmetric sparse system whose matrix and
right-hand side depend on the previous solution (section 2, the closing
paragraph of the problem definition).

Discretisation: continuous Q_p Lagrange elements (p = 1, 2, 3) on a uniform
N x N quad mesh, equispaced support points, Gauss-Legendre quadrature with
p + 2 points per direction, consistent mass.  Global nodes are numbered
lexicographically, index = J * (N p + 1) + I with I along x.  Homogeneous
Dirichlet data: boundary rows become identity rows, boundary columns are
dropped from interior rows, boundary right-hand-side entries are zero.

Matrices are CSR with int32 row pointers / column indices, sorted columns,
no duplicates and an explicit diagonal in every row.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

# ---------------------------------------------------------------------------
# Problem descriptions
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Problem:
    """One PDE / mesh / time-step setting.

    beta: 'const' uses beta_const everywhere; 'rotating' uses
    beta = 2 pi (-(y - 1/2), x - 1/2) (a rigid rotation about the centre);
    'vortex' uses beta = (-sin(pi x) cos(pi y), cos(pi x) sin(pi y)), the
    field of the paper's experiments (section 6.1).

    forcing: add the load (v, f) of the paper's random low-mode forcing
    (section 6.1): f = (C/2) sum_{j=1}^{16} c_j exp(-j^2/20) sin(2 j pi x)
    sin(2 j pi y) with C = 0.1, c_1 = 1 and c_2..c_16 drawn uniformly from
    [-1, 1] at every step (seeded; see forcing_coefficients).  Since v lies in
    the discrete space, (v, P f) = (v, f) for the L2 projection P of the paper.

    beta_projected: use the L2 projection of beta onto the continuous Lagrange space of
    the mesh (every node, no boundary condition) in the convection term, as the paper's
    discrete problem does (section 6.1, P_{V_h} b), instead of beta itself.

    u0: 'bump' (a seeded Gaussian bump) or 'zero' (the paper's zero initial value).

    nodes: support points of the 1-D Lagrange basis, 'equispaced' or 'gll'
    (Gauss-Lobatto-Legendre, the support points of Legendre spectral elements).
    """

    p: int
    N: int
    eps: float
    dt: float
    beta: str = "const"
    beta_const: tuple = (1.0, 0.5)
    forcing: bool = False
    u0: str = "bump"
    nodes: str = "equispaced"
    beta_projected: bool = False

    @property
    def n1(self) -> int:
        return self.N * self.p + 1

    @property
    def n(self) -> int:
        return self.n1 * self.n1


# Shapes and parameters of the five workload families (sizes as in the
# synthetic configurations this library is measured on).
C1 = Problem(p=1, N=32, eps=1e-2, dt=1e-2, beta="const")
C2 = Problem(p=2, N=256, eps=1e-3, dt=5e-3, beta="const")
C3 = Problem(p=3, N=512, eps=1e-4, dt=5e-3, beta="rotating")

# Reduced shapes of the same families, small enough for the CPU oracle.
C2_SMALL = Problem(p=2, N=32, eps=1e-3, dt=5e-3, beta="const")
C3_SMALL = Problem(p=3, N=16, eps=1e-4, dt=5e-3, beta="rotating")

# The paper's own experiments (section 6.1): vortex field, random low-mode
# forcing, zero initial value, dt = 0.5; first-order elements on a 64 x 64 grid
# for nu = 1e-1, 1e-2, 1e-3, and a 2 x 2 grid of order-23 Legendre spectral
# elements (section 6.3) for nu = 1e-2.
PAPER_Q1 = {nu: Problem(p=1, N=64, eps=nu, dt=0.5, beta="vortex", forcing=True, u0="zero", beta_projected=True)
            for nu in (1e-1, 1e-2, 1e-3)}
PAPER_SEM23 = Problem(p=23, N=2, eps=1e-2, dt=0.5, beta="vortex", forcing=True, u0="zero", nodes="gll",
                      beta_projected=True)
# reduced spectral-element shape for the CPU oracle (same family, lower order)
PAPER_SEM8 = Problem(p=8, N=2, eps=1e-2, dt=0.5, beta="vortex", forcing=True, u0="zero", nodes="gll",
                     beta_projected=True)

FORCING_MODES = 16
FORCING_C = 0.1


# ---------------------------------------------------------------------------
# 1-D Lagrange basis and quadrature
# ---------------------------------------------------------------------------


def support_points(p: int, kind: str = "equispaced") -> np.ndarray:
    """The p+1 support points on [0, 1]: equispaced, or Gauss-Lobatto-Legendre (the end
    points and the roots of the derivative of the Legendre polynomial of degree p)."""
    if kind == "equispaced":
        return np.linspace(0.0, 1.0, p + 1)
    if kind == "gll":
        if p == 1:
            return np.array([0.0, 1.0])
        inner = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
        return 0.5 * (np.concatenate([[-1.0], inner, [1.0]]) + 1.0)
    raise ValueError(kind)


def lagrange_1d(p: int, x: np.ndarray, kind: str = "equispaced"):
    """Values and derivatives of the p+1 Lagrange polynomials on [0, 1] with the support
    points of `support_points(p, kind)`.

    Returns (V, D) with V[q, a] = phi_a(x_q), D[q, a] = phi_a'(x_q).
    """
    nodes = support_points(p, kind)
    x = np.asarray(x, dtype=np.float64)
    V = np.ones((x.size, p + 1))
    D = np.zeros((x.size, p + 1))
    for a in range(p + 1):
        den = 1.0
        for b in range(p + 1):
            if b != a:
                den *= nodes[a] - nodes[b]
        for b in range(p + 1):
            if b != a:
                V[:, a] *= x - nodes[b]
        # derivative: sum over the dropped factor
        for c in range(p + 1):
            if c == a:
                continue
            term = np.ones_like(x)
            for b in range(p + 1):
                if b != a and b != c:
                    term *= x - nodes[b]
            D[:, a] += term
        V[:, a] /= den
        D[:, a] /= den
    return V, D


def gauss_01(nq: int):
    """Gauss-Legendre points and weights mapped to [0, 1]."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (xg + 1.0), 0.5 * wg


@dataclasses.dataclass
class ElementTables:
    """Reference-element tables for Q_p on the unit square.

    Local node i = b * (p+1) + a (a along x); quadrature point q = qy * nq1 + qx.
    """

    p: int
    nl: int
    nq: int
    xi: np.ndarray      # (nq,) reference x of each quadrature point
    eta: np.ndarray     # (nq,) reference y
    w: np.ndarray       # (nq,) weights (sum 1)
    phi: np.ndarray     # (nq, nl)
    dxi: np.ndarray     # (nq, nl) d/dxi
    deta: np.ndarray    # (nq, nl) d/deta
    mass_ref: np.ndarray    # (nl, nl) integral phi_i phi_j on the unit square
    stiff_ref: np.ndarray   # (nl, nl) integral grad phi_i . grad phi_j


def element_tables(p: int, kind: str = "equispaced") -> ElementTables:
    nq1 = p + 2
    xq, wq = gauss_01(nq1)
    V, D = lagrange_1d(p, xq, kind)
    nl = (p + 1) ** 2
    nq = nq1 * nq1
    qx = np.tile(np.arange(nq1), nq1)
    qy = np.repeat(np.arange(nq1), nq1)
    la = np.tile(np.arange(p + 1), p + 1)
    lb = np.repeat(np.arange(p + 1), p + 1)
    phi = V[qx][:, la] * V[qy][:, lb]
    dxi = D[qx][:, la] * V[qy][:, lb]
    deta = V[qx][:, la] * D[qy][:, lb]
    w = wq[qx] * wq[qy]
    mass_ref = (phi * w[:, None]).T @ phi
    stiff_ref = (dxi * w[:, None]).T @ dxi + (deta * w[:, None]).T @ deta
    return ElementTables(p, nl, nq, xq[qx], xq[qy], w, phi, dxi, deta, mass_ref, stiff_ref)


# ---------------------------------------------------------------------------
# Sparsity pattern (tensor product of 1-D element connectivity)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Pattern:
    problem: Problem
    n: int
    nnz: int
    row_ptr: np.ndarray   # int32 (n+1,)
    col_idx: np.ndarray   # int32 (nnz,)
    boundary: np.ndarray  # bool (n,)
    diag_pos: np.ndarray  # int64 (n,) CSR index of each diagonal entry
    emap: np.ndarray      # int64 (E, nl*nl): CSR index of each element-matrix entry, -1 if dropped
    elem_nodes: np.ndarray  # int64 (E, nl) global node of each local node
    elem_origin: np.ndarray  # (E, 2) lower-left corner (x, y) of each element

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64, nnz)."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr.astype(np.int64)))


def _range_1d(p: int, N: int):
    """For each 1-D node, the contiguous range [lo, hi] of nodes sharing an element."""
    n1 = N * p + 1
    I = np.arange(n1)
    e = I // p
    vertex = (I % p) == 0
    lo = np.where(vertex, np.maximum(I - p, 0), e * p)
    hi = np.where(vertex, np.minimum(I + p, n1 - 1), (e + 1) * p)
    return lo.astype(np.int64), hi.astype(np.int64)


def build_pattern(prob: Problem) -> Pattern:
    p, N = prob.p, prob.N
    n1 = prob.n1
    n = n1 * n1
    lo, hi = _range_1d(p, N)
    len1 = hi - lo + 1
    # full (no Dirichlet elimination) pattern: row (I, J) couples to I' in [lo(I), hi(I)], J' in [lo(J), hi(J)]
    Jg, Ig = np.divmod(np.arange(n, dtype=np.int64), n1)
    rowlen_full = len1[Ig] * len1[Jg]
    rp_full = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(rowlen_full, out=rp_full[1:])
    nnz_full = int(rp_full[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), rowlen_full)
    off = np.arange(nnz_full, dtype=np.int64) - rp_full[rows]
    Ir, Jr = Ig[rows], Jg[rows]
    L = len1[Ir]
    cI = lo[Ir] + off % L
    cJ = lo[Jr] + off // L
    del off, L
    cols = cJ * n1 + cI
    boundary1 = np.zeros(n1, dtype=bool)
    boundary1[0] = boundary1[-1] = True
    bnd = (boundary1[Ig] | boundary1[Jg])
    keep = np.where(bnd[rows], cols == rows, ~(boundary1[cI] | boundary1[cJ]))
    del cI, cJ, Ir, Jr
    newidx = np.cumsum(keep, dtype=np.int64) - 1
    newidx[~keep] = -1
    col_idx = cols[keep].astype(np.int32)
    rowlen = np.bincount(rows[keep], minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(rowlen, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    # diagonal positions
    diag_full = rp_full[:-1] + (Jg - lo[Jg]) * len1[Ig] + (Ig - lo[Ig])
    diag_pos = newidx[diag_full]
    assert np.all(diag_pos >= 0)
    # element -> CSR map
    ex, ey = np.meshgrid(np.arange(N), np.arange(N))
    ex = ex.ravel().astype(np.int64)
    ey = ey.ravel().astype(np.int64)
    la = np.tile(np.arange(p + 1), p + 1)
    lb = np.repeat(np.arange(p + 1), p + 1)
    Iloc = ex[:, None] * p + la[None, :]       # (E, nl)
    Jloc = ey[:, None] * p + lb[None, :]
    elem_nodes = Jloc * n1 + Iloc
    nl = (p + 1) ** 2
    # entry (i, j): row node (Iloc[i], Jloc[i]), col node (Iloc[j], Jloc[j])
    Ri, Rj = Iloc[:, :, None], Jloc[:, :, None]
    Ci, Cj = Iloc[:, None, :], Jloc[:, None, :]
    full_pos = rp_full[Rj * n1 + Ri] + (Cj - lo[Rj]) * len1[Ri] + (Ci - lo[Ri])
    emap = newidx[full_pos].reshape(N * N, nl * nl)
    h = 1.0 / N
    origin = np.stack([ex * h, ey * h], axis=1)
    return Pattern(prob, n, nnz, row_ptr.astype(np.int32), col_idx, bnd, diag_pos,
                   emap, elem_nodes, origin)


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------


class Assembler:
    """Assembles A(u_prev) and b(u_prev) for one Problem on one Pattern."""

    def __init__(self, prob: Problem, pattern: Optional[Pattern] = None):
        self.prob = prob
        self.pat = pattern if pattern is not None else build_pattern(prob)
        self.tab = element_tables(prob.p, prob.nodes)
        h = 1.0 / prob.N
        self.h = h
        t = self.tab
        mass_e = (h * h) * t.mass_ref
        # static element matrix: M/dt + eps K  (the same on every element of a uniform mesh)
        self.static_e = (mass_e / prob.dt + prob.eps * t.stiff_ref).ravel()
        self.mass_e = mass_e.ravel()
        # B_x[q, i*nl + j] = phi_i(q) dphi_j/dxi(q) (low orders; high orders contract per element)
        nl = t.nl
        self._tensor_b = t.nq * nl * nl <= (1 << 22)
        if self._tensor_b:
            self.Bx = (t.phi[:, :, None] * t.dxi[:, None, :]).reshape(t.nq, nl * nl)
            self.By = (t.phi[:, :, None] * t.deta[:, None, :]).reshape(t.nq, nl * nl)
        pat = self.pat
        keep = pat.emap >= 0
        self._keep = keep
        self._map = pat.emap[keep]
        self._mass_vals = None

    def _beta_at_quad(self):
        """beta_x, beta_y at every (element, quadrature point); with `beta_projected`, those of its
        L2 projection onto the mesh's continuous Lagrange space."""
        t, prob = self.tab, self.prob
        if prob.beta == "const":
            bx, by = prob.beta_const
            return float(bx), float(by)
        if prob.beta_projected:
            if getattr(self, "_beta_proj", None) is None:
                fx, fy = beta_field(prob)
                cx, cy = self.l2_projection(fx), self.l2_projection(fy)
                en = self.pat.elem_nodes
                self._beta_proj = (cx[en] @ t.phi.T, cy[en] @ t.phi.T)
            return self._beta_proj
        x, y = self.quad_points()
        fx, fy = beta_field(prob)
        return fx(x, y), fy(x, y)

    def full_mass(self):
        """The consistent mass matrix of the whole continuous Lagrange space (every node, no
        boundary condition), CSC."""
        if getattr(self, "_full_mass", None) is None:
            import scipy.sparse as sp
            en = self.pat.elem_nodes
            E, nl = en.shape
            rows = np.repeat(en, nl, axis=1).ravel()
            cols = np.tile(en, (1, nl)).ravel()
            vals = np.broadcast_to(self.mass_e[None, :], (E, nl * nl)).ravel()
            self._full_mass = sp.csc_matrix((vals, (rows, cols)), shape=(self.pat.n, self.pat.n))
        return self._full_mass

    def l2_projection(self, f) -> np.ndarray:
        """Nodal coefficients c of the L2 projection of f(x, y) onto the mesh's continuous
        Lagrange space: M c = F with F_a the integral of phi_a f by the element quadrature."""
        from scipy.sparse.linalg import spsolve
        t, pat = self.tab, self.pat
        x, y = self.quad_points()
        fq = f(x, y) * (self.h * self.h) * t.w[None, :]
        F = np.bincount(pat.elem_nodes.ravel(), weights=(fq @ t.phi).ravel(), minlength=pat.n)
        return spsolve(self.full_mass(), F)

    def quad_points(self):
        """Physical x, y of every (element, quadrature point)."""
        t = self.tab
        org = self.pat.elem_origin
        return org[:, 0:1] + self.h * t.xi[None, :], org[:, 1:2] + self.h * t.eta[None, :]

    def element_values(self, u_prev: np.ndarray) -> np.ndarray:
        """(E, nl*nl) element matrices of A(u_prev)."""
        t = self.tab
        U = u_prev[self.pat.elem_nodes]            # (E, nl)
        Uq = U @ t.phi.T                           # (E, nq)
        bx, by = self._beta_at_quad()
        scale = self.h * t.w[None, :] * Uq         # dx = h^2 dxi, grad = grad_ref / h
        ax = scale * bx
        ay = scale * by
        if self._tensor_b:
            vals = ax @ self.Bx
            vals += ay @ self.By
        else:
            # (E, nl, nq) @ (nq, nl): sum_q phi_i(q) (ax dphi_j/dxi + ay dphi_j/deta)(q)
            phit = t.phi.T[None, :, :]
            vals = ((phit * ax[:, None, :]) @ t.dxi + (phit * ay[:, None, :]) @ t.deta).reshape(len(U), -1)
        vals += self.static_e[None, :]
        return vals

    def matrix_values(self, u_prev: np.ndarray) -> np.ndarray:
        """CSR values of A(u_prev) (float64, nnz)."""
        ev = self.element_values(u_prev)
        vals = np.bincount(self._map, weights=ev[self._keep], minlength=self.pat.nnz)
        pat = self.pat
        bdiag = pat.diag_pos[pat.boundary]
        vals[bdiag] = 1.0
        return vals

    def mass_values(self) -> np.ndarray:
        """CSR values of the (Dirichlet-eliminated) consistent mass matrix; boundary rows zero."""
        if self._mass_vals is None:
            E = self.pat.emap.shape[0]
            ev = np.broadcast_to(self.mass_e[None, :], (E, self.mass_e.size))
            vals = np.bincount(self._map, weights=ev[self._keep], minlength=self.pat.nnz)
            vals[self.pat.diag_pos[self.pat.boundary]] = 0.0
            self._mass_vals = vals
        return self._mass_vals

    def forcing_modes(self) -> np.ndarray:
        """(16, n) loads L_j[i] = integral of phi_i sin(2 j pi x) sin(2 j pi y), j = 1..16,
        by the element quadrature; boundary entries zero."""
        if getattr(self, "_fmodes", None) is None:
            t, pat = self.tab, self.pat
            x, y = self.quad_points()
            L = np.zeros((FORCING_MODES, pat.n))
            wq = (self.h * self.h) * t.w[None, :]
            for j in range(1, FORCING_MODES + 1):
                fq = np.sin(2 * j * math.pi * x) * np.sin(2 * j * math.pi * y) * wq   # (E, nq)
                L[j - 1] = np.bincount(pat.elem_nodes.ravel(), weights=(fq @ t.phi).ravel(), minlength=pat.n)
            L[:, pat.boundary] = 0.0
            self._fmodes = L
        return self._fmodes

    def forcing_load(self, coeffs: np.ndarray) -> np.ndarray:
        """(v, f) for one step's coefficients c_1..c_16 (section 6.1)."""
        j = np.arange(1, FORCING_MODES + 1)
        a = 0.5 * FORCING_C * np.asarray(coeffs, dtype=np.float64) * np.exp(-(j * j) / 20.0)
        return a @ self.forcing_modes()

    def rhs(self, u_prev: np.ndarray, coeffs: Optional[np.ndarray] = None) -> np.ndarray:
        """b(u_prev) = M u_prev / dt (+ the forcing load of `coeffs`) on interior rows, 0 on
        the boundary."""
        import scipy.sparse as sp
        pat = self.pat
        if getattr(self, "_mass_csr", None) is None:
            self._mass_csr = sp.csr_matrix((self.mass_values(), pat.col_idx, pat.row_ptr), shape=(pat.n, pat.n))
        b = (self._mass_csr @ u_prev) / self.prob.dt
        if coeffs is not None:
            b += self.forcing_load(coeffs)
        b[pat.boundary] = 0.0
        return b

    def csr(self, vals: np.ndarray):
        import scipy.sparse as sp
        pat = self.pat
        return sp.csr_matrix((vals, pat.col_idx, pat.row_ptr), shape=(pat.n, pat.n))

    def system(self, u_prev: np.ndarray, coeffs: Optional[np.ndarray] = None):
        """(vals, b) of step i given u^{i-1} (and step i's forcing coefficients)."""
        return self.matrix_values(u_prev), self.rhs(u_prev, coeffs)


def beta_field(prob: Problem):
    """(beta_x, beta_y) of a non-constant velocity field as functions of (x, y)."""
    if prob.beta == "rotating":
        return (lambda x, y: -2.0 * math.pi * (y - 0.5)), (lambda x, y: 2.0 * math.pi * (x - 0.5))
    if prob.beta == "vortex":
        return ((lambda x, y: -np.sin(math.pi * x) * np.cos(math.pi * y)),
                (lambda x, y: np.cos(math.pi * x) * np.sin(math.pi * y)))
    raise ValueError(prob.beta)


def forcing_coefficients(seed: int, steps: int) -> np.ndarray:
    """(steps, 16) forcing coefficients: c_1 = 1, c_2..c_16 ~ U[-1, 1] drawn afresh at every
    step from one seeded stream (section 6.1)."""
    rng = np.random.default_rng([seed, 6101])
    c = np.ones((steps, FORCING_MODES))
    c[:, 1:] = rng.uniform(-1.0, 1.0, size=(steps, FORCING_MODES - 1))
    return c


def initial_condition(prob: Problem, seed: int, pattern: Optional[Pattern] = None) -> np.ndarray:
    """Gaussian bump of amplitude 1 and width 0.1, centre ~ U[0.25, 0.75]^2, zero on the
    boundary; or zero everywhere for u0 = 'zero'."""
    if prob.u0 == "zero":
        return np.zeros(prob.n)
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.25, 0.75, size=2)
    n1 = prob.n1
    xs = np.linspace(0.0, 1.0, n1)
    X, Y = np.meshgrid(xs, xs)          # Y rows -> J, X cols -> I: ravel gives J*n1+I
    u = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * 0.1 ** 2)).ravel()
    bnd = np.zeros((n1, n1), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    u[bnd.ravel()] = 0.0
    return u


def direct_solver(asm: Assembler):
    """Sparse direct solve (SuperLU) used only to advance the generator's own trajectory."""
    import scipy.sparse.linalg as spla

    def solve(vals, b):
        return spla.spsolve(asm.csr(vals).tocsc(), b)

    return solve


def march(prob: Problem, steps: int, seed: int,
          advance: Optional[Callable[[np.ndarray, np.ndarray], np.ndarray]] = None,
          asm: Optional[Assembler] = None):
    """Generate `steps` systems along a trajectory.

    The trajectory u^0, u^1, ... is advanced with `advance(vals, b) -> u`
    (default: a sparse direct solve), so the systems are the same whichever
    iterative solver is later run on them.  Returns (asm, list of (vals, b),
    list of trajectory states u^1..u^steps).
    """
    asm = asm if asm is not None else Assembler(prob)
    adv = advance if advance is not None else direct_solver(asm)
    u = initial_condition(prob, seed, asm.pat)
    coeffs = forcing_coefficients(seed, steps) if prob.forcing else [None] * steps
    systems, states = [], []
    for i in range(steps):
        vals, b = asm.system(u, coeffs[i])
        systems.append((vals, b))
        u = adv(vals, b)
        states.append(u)
    return asm, systems, states


# ---------------------------------------------------------------------------
# GPU assembly (qkgen library): the same systems, built in device memory
# ---------------------------------------------------------------------------

_QKGEN = None


def _qkgen():
    """Load libqkgen.so (built next to this file by build.py)."""
    global _QKGEN
    if _QKGEN is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqkgen.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built")
        lib = ctypes.CDLL(path)
        c = ctypes
        lib.qkgen_element_values.argtypes = [c.c_int64, c.c_int32, c.c_int32] + [c.c_void_p] * 7 + [
            c.c_int32, c.c_double, c.c_double, c.c_void_p, c.c_void_p, c.c_int32, c.c_double, c.c_void_p,
            c.c_void_p]
        lib.qkgen_gather.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
        lib.qkgen_set_value.argtypes = [c.c_int64, c.c_void_p, c.c_double, c.c_void_p, c.c_void_p]
        lib.qkgen_spmv_scaled.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p, c.c_double,
                                          c.c_void_p, c.c_void_p]
        for f in (lib.qkgen_element_values, lib.qkgen_gather, lib.qkgen_set_value, lib.qkgen_spmv_scaled):
            f.restype = c.c_int
        _QKGEN = lib
    return _QKGEN


class GpuAssembler:
    """Device-side twin of Assembler: A(u_prev) and b(u_prev) assembled on the GPU.

    The contribution list of every CSR entry (element entries that add into
    it) is built once on the host and sorted by element index, so the device
    sum runs in a fixed order.
    """

    def __init__(self, asm: Assembler, device):
        import torch
        if asm.prob.beta not in ("const", "rotating") or asm.prob.forcing:
            raise ValueError("the device assembler builds the constant and rotating-field families without "
                             "forcing; assemble this problem with the host Assembler")
        self.asm = asm
        self.dev = torch.device(device)
        pat, t = asm.pat, asm.tab
        T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(self.dev)
        self.row_ptr = T(pat.row_ptr, np.int32)
        self.col_idx = T(pat.col_idx, np.int32)
        self.elem_nodes = T(pat.elem_nodes, np.int32)
        em = pat.emap.ravel()
        keep = np.flatnonzero(em >= 0)
        key = em[keep]
        order = np.argsort(key, kind="stable")
        cnt = np.bincount(key, minlength=pat.nnz)
        cptr = np.zeros(pat.nnz + 1, dtype=np.int64)
        np.cumsum(cnt, out=cptr[1:])
        self.cptr = T(cptr, np.int32)
        self.cidx = T(keep[order], np.int32)
        del em, keep, key, order, cnt, cptr
        self.phi = T(t.phi, np.float64)
        self.wq = T(t.w, np.float64)
        self.Bx = T(asm.Bx, np.float64)
        self.By = T(asm.By, np.float64)
        self.static_e = T(asm.static_e, np.float64)
        self.qxi = T(t.xi, np.float64)
        self.qeta = T(t.eta, np.float64)
        self.mass = T(asm.mass_values(), np.float64)
        self.bdiag = T(pat.diag_pos[pat.boundary], np.int32)
        E = pat.elem_nodes.shape[0]
        self.E = E
        self.ev = torch.empty(E * t.nl * t.nl, dtype=torch.float64, device=self.dev)

    def variant(self, prob: Problem) -> "GpuAssembler":
        """An assembler for another Problem on the same mesh and degree (other eps, dt or velocity):
        shares every pattern-level device array and the element-value scratch (so its systems must
        be assembled on the same stream as this one's)."""
        import copy
        import torch
        if (prob.p, prob.N) != (self.asm.prob.p, self.asm.prob.N):
            raise ValueError("a variant must keep the degree and the mesh")
        v = copy.copy(self)
        v.asm = Assembler(prob, self.asm.pat)
        v.asm._mass_vals = self.asm._mass_vals
        v.static_e = torch.from_numpy(np.ascontiguousarray(v.asm.static_e, dtype=np.float64)).to(self.dev)
        return v

    def system(self, u_prev, vals_out=None, b_out=None, stream=None):
        """Fill vals_out (nnz) and b_out (n) with A(u_prev), b(u_prev); u_prev is a device tensor."""
        import torch
        pat, t, prob = self.asm.pat, self.asm.tab, self.asm.prob
        lib = _qkgen()
        if vals_out is None:
            vals_out = torch.empty(pat.nnz, dtype=torch.float64, device=self.dev)
        if b_out is None:
            b_out = torch.empty(pat.n, dtype=torch.float64, device=self.dev)
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream(self.dev).cuda_stream
        rot = 1 if prob.beta == "rotating" else 0
        bx, by = (0.0, 0.0) if rot else prob.beta_const
        p = lambda x: x.data_ptr()
        rc = lib.qkgen_element_values(self.E, t.nl, t.nq, p(self.elem_nodes), p(u_prev), p(self.phi), p(self.wq),
                                      p(self.Bx), p(self.By), p(self.static_e), rot, float(bx), float(by),
                                      p(self.qxi), p(self.qeta), prob.N, self.asm.h, p(self.ev), s)
        rc |= lib.qkgen_gather(pat.nnz, p(self.cptr), p(self.cidx), p(self.ev), p(vals_out), s)
        rc |= lib.qkgen_set_value(int(self.bdiag.numel()), p(self.bdiag), 1.0, p(vals_out), s)
        rc |= lib.qkgen_spmv_scaled(pat.n, p(self.row_ptr), p(self.col_idx), p(self.mass), p(u_prev),
                                    1.0 / prob.dt, p(b_out), s)
        if rc:
            raise RuntimeError(f"qkgen launch failed ({rc})")
        return vals_out, b_out
