"""Oracle: plain, slow FP64 CPU reference for restarted GMRES(m) with an SVD recycle space.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
imports, calls or links it, and it shares no code with the GPU library.

Method (Pitton & Heltai, "Accelerating the iterative solution of
convection-diffusion problems using singular value decomposition"):

* Krylov projection template and GMRES as the minimal-residual choice of the
  constraint space (section 3, the search-space template and the paragraph
  that picks C_k = A S_k for GMRES).
* Recycle basis W (the paper's V_s, n x k, orthonormal columns), with
  E = W^T A W (section 3.2, the definition of E_s) and the oblique projector
  P = I - A W E^{-1} W^T (section 3.2, eq. (left_deflation), and the second
  projector choice in section 3.3).
* Initial guess by Galerkin projection onto span(W): x0 = W E^{-1} W^T b
  (section 4.2, eqs. (projection_guess), (projection_t_s)); generalised here
  to a caller-supplied x0 as x0 + W E^{-1} W^T (b - A x0).
* Krylov operator P A and initial vector r0 = P r0 (Table 1, rows
  "augmented oblique" and "deflated oblique"; with the projected guess the two
  rows start from the same vector, eq. (equivalence_oblique)).
* The orthogonal projector P_o = I - W W^T in its place (Table 1, rows
  "augmented orthogonal" and "deflated orthogonal"; section 3.3, the first
  projector choice): operator P_o A, initial vector r0 (augmented) or P_o r0
  (deflated).  GMRES then minimises the projected residual ||P_o r||; the
  cycle-end correction below makes W^T r = 0, after which P_o r = r.
* The least-squares projector P_LS = I - A W (W^T A^T A W)^{-1} W^T A^T in
  its place (Table 1, rows "augmented LS" and "deflated LS"; section 3.3, the
  third projector choice): operator P_LS A, initial vector r0 (augmented) or
  P_LS r0 (deflated; the inner iteration of GCRO).  P_LS is the orthogonal
  projector onto the complement of range(A W), so GMRES minimises ||P_LS r||,
  and the cycle-end correction is the least-squares one,
  x += W c, r <- r - A W c with c = argmin ||r - A W c||, after which
  P_LS r = r: the true residual is the minimised one.
* Initial-guess-only strategies (section 4): the Galerkin projection guess
  onto span(W) followed by plain GMRES (section 4.2, eqs. (projection_guess),
  (projection_t_s), (iteration_projection)), and Lagrange extrapolation of
  order 2, 3 or 4 from the most recent solutions (section 4.1, eqs. (ext2),
  (ext3), (ext4)) followed by plain GMRES.
* Recycle space = leading left singular vectors of the last s solutions,
  recomputed every ell solves (section 5.2, Algorithm 1, eqs. (best_rank_s),
  (opt_svd)).
* Or, in its place, Ritz or harmonic Ritz vectors of A (section 5.1, eqs.
  (def_Ritz_pair), (eigenvalues_hessenberg), (eigenvalues_harmonic)) with
  respect to the search space of the solve just finished: span(W) plus the
  x-space directions D^{-1} V of its last cycle; the k pairs of smallest
  |theta| are kept (the small eigenvalues the deflation targets), a complex
  pair as the real and imaginary parts of its vector.

* Or the paper's SSOR preconditioner (section 6.1), in its multicolour form:
  symmetric SOR on the matrix permuted so that rows of one colour come
  together, the colouring first-fit in natural row order over the
  symmetrised pattern (rows of one colour never couple, so each half-sweep
  is a sequence of independent colour steps).

Readings where the paper is silent (each also listed in the design notes):
* right preconditioning, Jacobi D^{-1} or multicolour SSOR M (operator
  P A M^{-1}, x = x0 + M^{-1} V y), so the GMRES residual is the true
  deflated residual;
* Arnoldi orthogonalisation is classical Gram-Schmidt applied twice (CGS2);
* every cycle ends with the correction x += W E^{-1} W^T r, r <- P r, so the
  explicit stop test ||b - A x|| <= tol ||b|| applies to the true residual
  (the stopping rule of section 6.1);
* E is factorised with partial pivoting; if its 1-norm condition number
  exceeds 1e13 recycling is dropped for that solve (section 5.2 notes E may
  be singular and takes no measure);
* the snapshot ring holds the s most recent solutions; the numerical rank
  uses sigma_i > sigma_1 * max(n, c) * eps64 and k_eff = min(k, rank);
* Ritz and harmonic Ritz spaces: the search space is orthonormalised (its
  numerical rank cut as for the ring), the k values of smallest modulus are
  kept, a complex conjugate pair only whole (a pair that would exceed k is
  left out), and the kept vectors are orthonormalised with the same rank cut.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg

PLAIN, AUG_OBLIQUE, DEFL_OBLIQUE, AUG_ORTHO, DEFL_ORTHO = 0, 1, 2, 3, 4
GUESS_PROJECT, GUESS_EXTRAP2, GUESS_EXTRAP3, GUESS_EXTRAP4 = 5, 6, 7, 8
AUG_LS, DEFL_LS = 9, 10
ORTHO_METHODS = (AUG_ORTHO, DEFL_ORTHO)
LS_METHODS = (AUG_LS, DEFL_LS)
PROJECTED_START_METHODS = (DEFL_ORTHO, DEFL_LS)   # deflated rows: Krylov initial vector P r
EXTRAP_ORDER = {GUESS_EXTRAP2: 2, GUESS_EXTRAP3: 3, GUESS_EXTRAP4: 4}
GUESS_ONLY_METHODS = (GUESS_PROJECT, GUESS_EXTRAP2, GUESS_EXTRAP3, GUESS_EXTRAP4)
PRECOND_NONE, PRECOND_JACOBI, PRECOND_SSOR = 0, 1, 2

SPACE_SVD, SPACE_RITZ, SPACE_HARMONIC = "svd", "ritz", "harmonic_ritz"

FLAG_RECYCLE_DROPPED = 1
FLAG_BREAKDOWN_LUCKY = 2
FLAG_NONFINITE = 4

EPS64 = np.finfo(np.float64).eps
E_COND_MAX = 1e13
LUCKY_REL = 1e-14


@dataclasses.dataclass
class Config:
    restart_m: int = 30
    recycle_k: int = 0
    snapshots_s: int = 0
    svd_interval: int = 1
    method: int = AUG_OBLIQUE
    precond: int = PRECOND_NONE
    max_iters: int = 10000
    select_smallest: bool = False
    recycle_space: str = SPACE_SVD   # SPACE_SVD (Algorithm 1), SPACE_RITZ or SPACE_HARMONIC (section 5.1)
    ssor_omega: float = 1.0          # relaxation factor of PRECOND_SSOR, 0 < omega < 2


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iterations: int
    cycles: int
    k_eff: int
    converged: bool
    flags: int
    rel_res_true: float
    res_history: List[float]        # explicit ||r||/||b|| at the end of every cycle
    implicit_history: List[float]   # |g_{j+1}|/||b|| after every Arnoldi step
    krylov_x: Optional[np.ndarray] = None   # M^{-1} V_j of the last cycle: its x-space directions


# ---------------------------------------------------------------------------
# Building blocks
# ---------------------------------------------------------------------------


def jacobi_inverse(A) -> np.ndarray:
    """1 / diag(A): the diagonal (Jacobi) preconditioner, applied on the right."""
    d = A.diagonal().astype(np.float64)
    return 1.0 / d


def greedy_colouring(A) -> np.ndarray:
    """First-fit colouring of the symmetrised sparsity pattern of A in natural row order: row i
    takes the smallest colour held by none of its neighbours j < i (j couples to i when a_ij or
    a_ji is stored).  Rows of one colour never couple."""
    import scipy.sparse as sp
    n = A.shape[0]
    S = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    S = (S + S.T).tocsr()
    colour = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        used = set(colour[nb[nb < i]].tolist())
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


class MulticolourSSOR:
    """Symmetric SOR with relaxation omega as a preconditioner (the paper's SSOR, section 6.1),
    on the ordering that takes the colours of `greedy_colouring` one after the other.  With D
    the diagonal and L, U the couplings of each row to rows of lower and of higher colour,

        M = (D + omega L) D^{-1} (D + omega U) / (omega (2 - omega)),

    and M^{-1} r is one forward SOR sweep over the colours in increasing order from a zero
    start followed by one backward sweep in decreasing order: here the two triangular solves
    (D + omega L) y = omega (2 - omega) r and (D + omega U) z = D y on the permuted matrix, whose
    strict lower triangle is L because rows of one colour do not couple."""

    def __init__(self, A, omega: float = 1.0):
        import scipy.sparse as sp
        if not 0.0 < omega < 2.0:
            raise ValueError("SSOR needs 0 < omega < 2")
        self.omega = float(omega)
        self.colour = greedy_colouring(A)
        self.perm = np.argsort(self.colour, kind="stable")
        Ap = A.tocsr()[self.perm][:, self.perm].tocsr()
        self.d = Ap.diagonal().astype(np.float64)
        Dm = sp.diags(self.d)
        self.lower = (Dm + self.omega * sp.tril(Ap, -1)).tocsr()
        self.upper = (Dm + self.omega * sp.triu(Ap, 1)).tocsr()

    def __call__(self, r: np.ndarray) -> np.ndarray:
        from scipy.sparse.linalg import spsolve_triangular
        w = self.omega
        y = spsolve_triangular(self.lower, w * (2.0 - w) * r[self.perm], lower=True)
        z = spsolve_triangular(self.upper, self.d * y, lower=False)
        out = np.empty_like(z)
        out[self.perm] = z
        return out


def preconditioner(A, cfg: Config):
    """M^{-1} as a function of a vector: identity, Jacobi D^{-1} or multicolour SSOR; applied on
    the right (operator A M^{-1}, x = x0 + M^{-1} V y)."""
    if cfg.precond == PRECOND_JACOBI:
        dinv = jacobi_inverse(A)
        return lambda v: dinv * v
    if cfg.precond == PRECOND_SSOR:
        return MulticolourSSOR(A, cfg.ssor_omega)
    return lambda v: v


def recycle_setup(A, W: np.ndarray):
    """Z = A W and E = W^T A W (section 3.2, E_s = V_s^T A V_s).

    Returns (Z, E, cond1) with cond1 the 1-norm condition number of E.
    Z is formed one column at a time with the sparse matvec.
    """
    k = W.shape[1]
    Z = np.empty_like(W)
    for i in range(k):
        Z[:, i] = A @ W[:, i]
    E = W.T @ Z
    cond1 = float(np.linalg.cond(E, 1)) if k > 0 else 1.0
    return Z, E, cond1


def oblique_project(W, Z, E, v):
    """P v = v - A W E^{-1} W^T v  (section 3.2, the deflation projector M_D)."""
    return v - Z @ np.linalg.solve(E, W.T @ v)


def extrapolation_weights(order: int):
    """Weights of x_{i-1}, ..., x_{i-order} in the Lagrange extrapolation to the next equispaced
    time (section 4.1): the interpolating polynomial through the last `order` solutions, taken one
    step ahead, is sum_j (-1)^(j+1) C(order, j) x_{i-j} (eqs. (ext2): 2, -1; (ext3): 3, -3, 1;
    (ext4): 4, -6, 4, -1)."""
    from math import comb
    return [(-1) ** (j + 1) * comb(order, j) for j in range(1, order + 1)]


def extrapolate(history: List[np.ndarray], order: int) -> np.ndarray:
    """The extrapolated guess from the most recent solutions (history[-1] = x_{i-1}); with fewer
    than `order` solutions the highest order they allow."""
    q = min(order, len(history))
    wts = extrapolation_weights(q)
    return sum(w * history[-1 - j] for j, w in enumerate(wts))


def orthogonal_project(W, v):
    """P_o v = v - W W^T v  (section 3.3, the orthogonal projector onto the complement of span(W))."""
    return v - W @ (W.T @ v)


def ls_coefficients(Z, v):
    """c = argmin ||v - Z c||_2 = (Z^T Z)^{-1} Z^T v, with Z = A W (section 3.3, the third
    projector choice), by a library least-squares solve."""
    return np.linalg.lstsq(Z, v, rcond=None)[0]


def ls_project(Z, v):
    """P_LS v = v - A W (W^T A^T A W)^{-1} W^T A^T v: v minus its orthogonal projection onto
    range(A W) (section 3.3, the third projector; Table 1 LS rows)."""
    return v - Z @ ls_coefficients(Z, v)


def ls_correction(W, Z, x, r):
    """x <- x + W c, r <- r - A W c with c the least-squares coefficients of r on A W: the
    minimal-residual correction in span(W), after which (A W)^T r = 0."""
    c = ls_coefficients(Z, r)
    return x + W @ c, r - Z @ c


def projection_correction(W, Z, E, x, r):
    """x <- x + W E^{-1} W^T r, r <- r - A W E^{-1} W^T r  (section 4.2, eq. (projection_t_s)).

    With x = 0, r = b this is exactly the Galerkin projection guess of the
    paper; applied to a later residual it solves for the span(W) component.
    """
    c = np.linalg.solve(E, W.T @ r)
    return x + W @ c, r - Z @ c


def krylov_update(x, minv, V, y):
    """x <- x + M^{-1} V y: the Krylov correction of one cycle mapped back through the
    right preconditioner (section 3, right preconditioning A M^{-1} u = b, x = M^{-1} u)."""
    return x + minv(V @ y)


def is_lucky_breakdown(h_next: float, colnorm: float) -> bool:
    """The Krylov space has become invariant: the new Hessenberg subdiagonal entry is zero up to
    rounding, relative to the norm of its column (scale-free, so a matrix multiplied by any
    constant breaks down at the same step).  The minimal-residual iterate over the current space
    is then the exact solution of the projected system (section 3: the search space stops growing
    once it contains the solution)."""
    return h_next <= LUCKY_REL * colnorm


def givens(a: float, b: float):
    """Rotation (c, s) with [c s; -s c] [a; b] = [rho; 0], rho = hypot(a, b)."""
    rho = float(np.hypot(a, b))
    if rho == 0.0:
        return 1.0, 0.0, 0.0
    return a / rho, b / rho, rho


@dataclasses.dataclass
class Cycle:
    """Result of one GMRES cycle: basis V (n x (j+1)), Hessenberg H ((j+1) x j),
    triangularised R, rotated rhs g, steps taken j, flags."""
    V: np.ndarray
    H: np.ndarray
    R: np.ndarray
    g: np.ndarray
    steps: int
    lucky: bool
    implicit: List[float]


def arnoldi_cycle(op, r0: np.ndarray, m: int, stop_abs: float, max_steps: int) -> Cycle:
    """One restart cycle of GMRES on the operator `op` starting from r0.

    Arnoldi with classical Gram-Schmidt applied twice, Hessenberg least
    squares by Givens rotations (section 3: minimal residual over the Krylov
    space K_j(op, r0)).  Stops after m steps, when the rotated residual
    |g_{j+1}| <= stop_abs, on a lucky breakdown, or after max_steps steps.
    """
    n = r0.size
    beta = float(np.linalg.norm(r0))
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    R = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[:, 0] = r0 / beta
    implicit = []
    j = 0
    lucky = False
    while j < m and j < max_steps:
        w = op(V[:, j])
        h1 = V[:, : j + 1].T @ w
        w = w - V[:, : j + 1] @ h1
        h2 = V[:, : j + 1].T @ w
        w = w - V[:, : j + 1] @ h2
        hcol = np.zeros(j + 2)
        hcol[: j + 1] = h1 + h2
        hcol[j + 1] = np.linalg.norm(w)
        H[: j + 2, j] = hcol
        colnorm = float(np.linalg.norm(hcol))
        rcol = hcol.copy()
        for i in range(j):
            t = cs[i] * rcol[i] + sn[i] * rcol[i + 1]
            rcol[i + 1] = -sn[i] * rcol[i] + cs[i] * rcol[i + 1]
            rcol[i] = t
        c, s, rho = givens(rcol[j], rcol[j + 1])
        cs[j], sn[j] = c, s
        rcol[j] = rho
        rcol[j + 1] = 0.0
        R[: j + 2, j] = rcol
        g[j + 1] = -s * g[j]
        g[j] = c * g[j]
        implicit.append(abs(g[j + 1]))
        steps = j + 1
        if is_lucky_breakdown(hcol[j + 1], colnorm):
            lucky = True
            j = steps
            break
        V[:, j + 1] = w / hcol[j + 1]
        j = steps
        if abs(g[j]) <= stop_abs or steps >= max_steps:
            break
    return Cycle(V[:, : j + 1], H[: j + 1, :j], R[: j + 1, :j], g[: j + 1], j, lucky, implicit)


# ---------------------------------------------------------------------------
# One solve
# ---------------------------------------------------------------------------


def solve(A, b: np.ndarray, x0: Optional[np.ndarray], tol: float, cfg: Config,
          W: Optional[np.ndarray] = None, history: Optional[List[np.ndarray]] = None) -> Result:
    """Solve A x = b to ||b - A x||_2 <= tol ||b||_2 with recycled GMRES(m).

    A: scipy CSR matrix (used only for A @ v and its diagonal).  W: recycle
    basis (n x k_eff, orthonormal columns) or None.  history: previous solutions,
    most recent last (the extrapolation methods' input; x0 is used while it is
    empty).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    bnorm = float(np.linalg.norm(b))
    if not np.isfinite(bnorm):
        return Result(np.full(n, np.nan), 0, 0, 0, False, FLAG_NONFINITE, float("nan"), [], [])
    if bnorm == 0.0:
        return Result(np.zeros(n), 0, 0, 0, True, 0, 0.0, [0.0], [])
    flags = 0
    minv = preconditioner(A, cfg)
    use_w = cfg.method != PLAIN and W is not None and W.shape[1] > 0
    Z = E = None
    k_eff = 0
    if use_w:
        Z, E, cond1 = recycle_setup(A, W)
        if not np.isfinite(cond1) or cond1 > E_COND_MAX:
            flags |= FLAG_RECYCLE_DROPPED
            use_w = False
        else:
            k_eff = W.shape[1]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if cfg.method in EXTRAP_ORDER and history:
        x = extrapolate(history, EXTRAP_ORDER[cfg.method])
    r = b - A @ x
    if use_w:
        x, r = projection_correction(W, Z, E, x, r)
    # guess-only projection: span(W) enters the initial guess alone; the Krylov part is plain GMRES
    guess_only = cfg.method in GUESS_ONLY_METHODS
    use_w_krylov = use_w and not guess_only

    ortho = cfg.method in ORTHO_METHODS
    lsq = cfg.method in LS_METHODS

    def op(v):
        w = A @ minv(v)
        if use_w_krylov:
            if lsq:
                w = ls_project(Z, w)
            else:
                w = orthogonal_project(W, w) if ortho else oblique_project(W, Z, E, w)
        return w

    def correct(x, r):
        # cycle-end correction in span(W): least squares for the LS rows, Galerkin otherwise
        return ls_correction(W, Z, x, r) if lsq else projection_correction(W, Z, E, x, r)

    stop_abs = tol * bnorm
    its = 0
    cycles = 0
    last_kx = None
    hist: List[float] = []
    implicit: List[float] = []
    rnorm = float(np.linalg.norm(r))
    if not np.isfinite(rnorm):
        return Result(x, 0, 0, k_eff, False, flags | FLAG_NONFINITE, float("nan"), [], [])
    while True:
        if rnorm <= stop_abs:
            return Result(x, its, cycles, k_eff, True, flags, rnorm / bnorm, hist, implicit, last_kx)
        if its >= cfg.max_iters:
            return Result(x, its, cycles, k_eff, False, flags, rnorm / bnorm, hist, implicit, last_kx)
        # deflated rows: the Krylov initial vector is the projected residual (P_o r equals r once
        # W^T r = 0; P_LS r equals r once (A W)^T r = 0, i.e. after the first cycle's correction)
        r_start = r
        if use_w_krylov and cfg.method in PROJECTED_START_METHODS:
            r_start = ls_project(Z, r) if lsq else orthogonal_project(W, r)
        cyc = arnoldi_cycle(op, r_start, cfg.restart_m, stop_abs, cfg.max_iters - its)
        cycles += 1
        its += cyc.steps
        implicit += [v / bnorm for v in cyc.implicit]
        if cyc.lucky:
            flags |= FLAG_BREAKDOWN_LUCKY
        j = cyc.steps
        y = scipy.linalg.solve_triangular(cyc.R[:j, :j], cyc.g[:j], lower=False)
        x = krylov_update(x, minv, cyc.V[:, :j], y)
        last_kx = krylov_directions(minv, cyc.V[:, :j])
        r = b - A @ x
        if use_w_krylov:
            x, r = correct(x, r)
        rnorm = float(np.linalg.norm(r))
        hist.append(rnorm / bnorm)
        if not np.isfinite(rnorm):
            return Result(x, its, cycles, k_eff, False, flags | FLAG_NONFINITE, float("nan"), hist, implicit)


# ---------------------------------------------------------------------------
# Recycle-space update (Algorithm 1)
# ---------------------------------------------------------------------------


def svd_basis(X: np.ndarray, k: int, smallest: bool = False):
    """Leading (or trailing) left singular vectors of the snapshot matrix X.

    Returns (W, sigma, rank): W has k_eff = min(k, rank) orthonormal columns,
    rank = #{sigma_i > sigma_1 * max(n, c) * eps64} (no direction below the
    numerical rank is ever kept).  Section 5.2, eqs. (best_rank_s), (opt_svd).
    """
    n, c = X.shape
    if c == 0:
        return np.zeros((n, 0)), np.zeros(0), 0
    U, sig, _ = np.linalg.svd(X, full_matrices=False)
    if sig[0] == 0.0 or not np.isfinite(sig[0]):
        return np.zeros((n, 0)), sig, 0
    rank = int(np.sum(sig > sig[0] * max(n, c) * EPS64))
    k_eff = min(k, rank)
    if smallest:
        return U[:, rank - k_eff: rank].copy(), sig, rank
    return U[:, :k_eff].copy(), sig, rank


def orthonormal_basis(U: np.ndarray) -> np.ndarray:
    """Orthonormal basis of span(U) from its SVD, with the numerical-rank cut of the ring
    (sigma_i > sigma_1 * max(n, c) * eps64)."""
    n, c = U.shape
    if c == 0:
        return np.zeros((n, 0))
    Q, sig, _ = np.linalg.svd(U, full_matrices=False)
    if sig[0] == 0.0 or not np.isfinite(sig[0]):
        return np.zeros((n, 0))
    return Q[:, : int(np.sum(sig > sig[0] * max(n, c) * EPS64))].copy()


def ritz_pairs(A, Q: np.ndarray, harmonic: bool):
    """Ritz (or harmonic Ritz) pairs of A with respect to span(Q), Q with orthonormal columns:
    theta and z with Q^T A Q z = theta z (section 5.1, eq. (eigenvalues_hessenberg); Q^T Q = I), or
    (A Q)^T (A Q) z = theta (A Q)^T Q z (eq. (eigenvalues_harmonic)).  The vectors are y = Q z.
    A Q is formed one column at a time with the sparse product."""
    AQ = np.empty_like(Q)
    for i in range(Q.shape[1]):
        AQ[:, i] = A @ Q[:, i]
    if harmonic:
        theta, Z = scipy.linalg.eig(AQ.T @ AQ, AQ.T @ Q)
    else:
        theta, Z = scipy.linalg.eig(Q.T @ AQ)
    return theta, Z


def ritz_order(theta: np.ndarray):
    """Indices of the finite values, smallest modulus first (the eigenvalues that deflation removes,
    section 3.2; harmonic Ritz values approximate those nearest the origin, section 5.1)."""
    return [i for i in np.argsort(np.abs(theta), kind="stable") if np.isfinite(theta[i])]


def pair_basis(y: np.ndarray):
    """Real vectors spanning the same space as a complex Ritz vector and its conjugate."""
    return [y.real.copy(), y.imag.copy()]


def krylov_directions(minv, V: np.ndarray) -> np.ndarray:
    """The x-space directions of a cycle's Krylov basis under right preconditioning: M^{-1} V."""
    if V.shape[1] == 0:
        return V.copy()
    return np.column_stack([minv(V[:, i]) for i in range(V.shape[1])])


def ritz_basis(A, U: np.ndarray, k: int, harmonic: bool):
    """Recycle basis from the Ritz or harmonic Ritz vectors of A over span(U) (section 5.1): the k
    pairs of smallest |theta| (finite values only), a complex pair as the real and imaginary parts
    of its vector and only whole, orthonormalised.  Returns (W, selected theta)."""
    n = U.shape[0]
    Q = orthonormal_basis(U)
    if Q.shape[1] == 0 or k == 0:
        return np.zeros((n, 0)), np.zeros(0, dtype=complex)
    theta, Z = ritz_pairs(A, Q, harmonic)
    order = ritz_order(theta)
    cols, picked, used = [], [], set()
    for i in order:
        if i in used:
            continue
        if abs(theta[i].imag) > 0.0:
            # the conjugate partner: the other index of equal modulus and opposite imaginary part
            partner = min((j for j in order if j not in used and j != i),
                          key=lambda j: abs(theta[j] - np.conj(theta[i])), default=None)
            if len(cols) + 2 > k:
                break
            cols += pair_basis(Q @ Z[:, i])
            picked += [theta[i], np.conj(theta[i])]
            used.update({i, partner})
        else:
            if len(cols) + 1 > k:
                break
            cols.append((Q @ Z[:, i]).real)
            picked.append(theta[i])
            used.add(i)
    if not cols:
        return np.zeros((n, 0)), np.zeros(0, dtype=complex)
    return orthonormal_basis(np.column_stack(cols)), np.array(picked)


class RecycleState:
    """Snapshot ring and recycle basis of one sequence (section 5.2, Algorithm 1)."""

    def __init__(self, n: int, cfg: Config):
        self.n = n
        self.cfg = cfg
        self.ring: List[np.ndarray] = []
        self.count = 0
        self.W = np.zeros((n, 0))
        self.sigma = np.zeros(0)
        self.theta = np.zeros(0, dtype=complex)
        self.rank = 0

    def update(self, x: np.ndarray, A=None, result: Optional[Result] = None):
        """Store x among the s most recent solutions; every ell solves recompute W (the
        extrapolation methods keep the ring only).  With a Ritz or harmonic Ritz recycle space, W
        is instead recomputed after every solve from A and the solve's search space: the W it
        used plus its last cycle's directions (result.krylov_x)."""
        if self.cfg.recycle_space != SPACE_SVD:
            self.count += 1
            if self.cfg.recycle_k <= 0 or result is None or result.krylov_x is None:
                return
            U = np.column_stack([self.W, result.krylov_x])
            self.W, self.theta = ritz_basis(A, U, self.cfg.recycle_k,
                                            self.cfg.recycle_space == SPACE_HARMONIC)
            self.rank = self.W.shape[1]
            return
        s = self.cfg.snapshots_s
        extrap = self.cfg.method in EXTRAP_ORDER
        if s <= 0 or (self.cfg.recycle_k <= 0 and not extrap):
            self.count += 1
            return
        self.ring.append(np.array(x, dtype=np.float64))
        if len(self.ring) > s:
            self.ring.pop(0)
        self.count += 1
        if extrap:
            return
        if self.count % max(1, self.cfg.svd_interval) == 0:
            X = np.stack(self.ring, axis=1)
            self.W, self.sigma, self.rank = svd_basis(X, self.cfg.recycle_k, self.cfg.select_smallest)


def run_sequence(A_list, b_list, tol: float, cfg: Config, x_init=None):
    """Solve a sequence with x0 = previous solution, updating the recycle space after each solve."""
    n = b_list[0].size
    st = RecycleState(n, cfg)
    x_prev = np.zeros(n) if x_init is None else x_init
    results = []
    for A, b in zip(A_list, b_list):
        res = solve(A, b, x_prev, tol, cfg, st.W, st.ring)
        results.append(res)
        st.update(res.x, A, res)
        x_prev = res.x
    return results, st
