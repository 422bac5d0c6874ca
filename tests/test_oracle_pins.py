"""Pins for the FP64 oracle: each check ties it to the paper or to mathematics,
never to itself (dense direct solves, brute-force minimal residuals over an
explicit Krylov basis, exact algebraic identities, closed-form special cases,
and library SVD properties).  CPU only."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import rgmres as O
from paper_1807_09467_amd import workload as WL


def rand_system(n, seed, density=0.2, shift=4.0):
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=density, random_state=rng, format="csr")
    R.data = rng.standard_normal(R.nnz)
    A = (sp.identity(n, format="csr") * shift + R).tocsr()
    A.sort_indices()
    b = rng.standard_normal(n)
    return A, b


def orthonormal(n, k, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return Q


def c1_system(step=3, seed=0):
    asm, systems, states = WL.march(WL.C1, step, seed)
    vals, b = systems[-1]
    return asm.csr(vals), b, states[-1]


# -- GMRES core -------------------------------------------------------------


@pytest.mark.parametrize("precond", [O.PRECOND_NONE, O.PRECOND_JACOBI])
def test_unrestarted_gmres_equals_dense_solve(precond):
    """m >= n: GMRES is a direct method (section 1); compare with LU."""
    A, b = rand_system(40, 1)
    cfg = O.Config(restart_m=60, method=O.PLAIN, precond=precond)
    res = O.solve(A, b, None, 1e-13, cfg)
    xd = np.linalg.solve(A.toarray(), b)
    kappa = np.linalg.cond(A.toarray())
    assert res.converged
    assert np.linalg.norm(res.x - xd) / np.linalg.norm(xd) <= kappa * 1e-13
    assert res.iterations <= 40


def test_restarted_gmres_matches_scipy():
    """GMRES(m) with m < n: same solution as SciPy's restarted GMRES (independent implementation)."""
    A, b, _ = c1_system()
    cfg = O.Config(restart_m=10, method=O.PLAIN)
    res = O.solve(A, b, None, 1e-12, cfg)
    xs, info = spla.gmres(A, b, rtol=1e-12, atol=0.0, restart=10, maxiter=500)
    assert info == 0
    xd = spla.spsolve(A.tocsc(), b)
    kappa = np.linalg.cond(A.toarray())
    assert np.linalg.norm(res.x - xd) / np.linalg.norm(xd) <= kappa * 1e-12
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xd) <= 2 * kappa * 1e-12


def krylov_min_residual(op, r0, j):
    """min_z ||r0 - op-Krylov(z)|| over z in K_j(op, r0) by brute force (power basis + QR + lstsq)."""
    K = np.empty((r0.size, j))
    v = r0 / np.linalg.norm(r0)
    for i in range(j):
        K[:, i] = v
        v = op(v)
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    AQ = np.column_stack([op(Q[:, i]) for i in range(j)])
    y, *_ = np.linalg.lstsq(AQ, r0, rcond=None)
    return np.linalg.norm(r0 - AQ @ y)


@pytest.mark.parametrize("recycle", [False, True])
def test_implicit_residual_is_krylov_minimum(recycle):
    """|g_{j+1}| after j steps equals the minimal residual over K_j (minimal-residual condition, section 3)."""
    A, b, x_true = c1_system(step=4)
    n = b.size
    dinv = O.jacobi_inverse(A)
    if recycle:
        W = orthonormal(n, 3, 7)
        Z, E, _ = O.recycle_setup(A, W)
        _, r0 = O.projection_correction(W, Z, E, np.zeros(n), b.copy())
        op = lambda v: O.oblique_project(W, Z, E, A @ (dinv * v))
    else:
        r0 = b.copy()
        op = lambda v: A @ (dinv * v)
    cyc = O.arnoldi_cycle(op, r0, 8, 0.0, 8)
    for j in range(1, 9):
        ref = krylov_min_residual(op, r0, j)
        assert abs(cyc.implicit[j - 1] - ref) <= 1e-9 * np.linalg.norm(r0) + 1e-8 * ref


@pytest.mark.parametrize("recycle", [False, True])
def test_arnoldi_relation_and_orthogonality(recycle):
    """op V_m = V_{m+1} H_m and V^T V = I for the CGS2 Arnoldi basis."""
    A, b, _ = c1_system()
    n = b.size
    dinv = O.jacobi_inverse(A)
    if recycle:
        W = orthonormal(n, 4, 3)
        Z, E, _ = O.recycle_setup(A, W)
        op = lambda v: O.oblique_project(W, Z, E, A @ (dinv * v))
        _, r0 = O.projection_correction(W, Z, E, np.zeros(n), b.copy())
    else:
        op = lambda v: A @ (dinv * v)
        r0 = b
    m = 25
    cyc = O.arnoldi_cycle(op, r0, m, 0.0, m)
    V, H = cyc.V, cyc.H
    assert V.shape[1] == m + 1 and H.shape == (m + 1, m)
    OV = np.column_stack([op(V[:, i]) for i in range(m)])
    anorm = spla.norm(A) * np.abs(dinv).max()
    assert np.linalg.norm(OV - V @ H) <= 1e-13 * anorm * m
    assert np.abs(V.T @ V - np.eye(m + 1)).max() <= 1e-14 * m
    if recycle:
        # range(P) = ker(W^T): the first Krylov vectors carry no W component (later ones pick up
        # rounding amplified by 1/h_{j+1,j}, which does not change the iterates measurably)
        assert np.abs(W.T @ V[:, :3]).max() <= 1e-12


def test_residual_history_monotone():
    A, b, _ = c1_system()
    cfg = O.Config(restart_m=5, method=O.PLAIN)
    res = O.solve(A, b, None, 1e-11, cfg)
    imp = np.array(res.implicit_history)
    # within a cycle the minimal residual never grows; across restarts the explicit one never grows
    for c in range(0, imp.size, 5):
        seg = imp[c:c + 5]
        assert np.all(np.diff(seg) <= 1e-14)
    hist = np.array(res.res_history)
    assert np.all(np.diff(hist) <= 1e-12 * hist[:-1])


# -- projector and projection guess ----------------------------------------------


def test_oblique_projector_identities():
    """P^2 = P, P A W = 0 (section 3.2: M_D A V_s = 0), W^T P = 0."""
    A, b = rand_system(60, 2)
    W = orthonormal(60, 5, 11)
    Z, E, _ = O.recycle_setup(A, W)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((60, 7))
    P = lambda v: O.oblique_project(W, Z, E, v)
    PV = np.column_stack([P(V[:, i]) for i in range(7)])
    PPV = np.column_stack([P(PV[:, i]) for i in range(7)])
    assert np.abs(PPV - PV).max() <= 1e-12 * np.abs(V).max()
    PAW = np.column_stack([P(A @ W[:, i]) for i in range(5)])
    assert np.abs(PAW).max() <= 1e-12 * spla.norm(A)
    assert np.abs(W.T @ PV).max() <= 1e-12 * np.abs(V).max()


def test_projection_guess_exact_when_solution_in_span():
    """x* in span(W) -> x0 = W E^{-1} W^T b = x* and no Arnoldi step (section 4.2)."""
    A, _ = rand_system(50, 3)
    W = orthonormal(50, 4, 5)
    c = np.array([1.0, -2.0, 0.5, 3.0])
    x_star = W @ c
    b = A @ x_star
    cfg = O.Config(restart_m=20, recycle_k=4, snapshots_s=4)
    res = O.solve(A, b, None, 1e-12, cfg, W)
    assert res.iterations == 0 and res.converged
    assert np.linalg.norm(res.x - x_star) <= 1e-13 * np.linalg.norm(x_star) * np.linalg.cond(A.toarray())


def test_correction_leaves_residual_orthogonal_to_W():
    A, b, _ = c1_system()
    W = orthonormal(b.size, 5, 9)
    res = O.solve(A, b, None, 1e-9, O.Config(restart_m=10, recycle_k=5, snapshots_s=5), W)
    r = b - A @ res.x
    assert np.abs(W.T @ r).max() <= 1e-13 * np.linalg.norm(b) * 100
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)


def test_augmented_and_deflated_oblique_coincide_without_preconditioner():
    """(I - A W E^{-1} W^T)^2 b = (I - A W E^{-1} W^T) b, eq. (equivalence_oblique): the two Table 1
    rows then run the same iteration."""
    A, b, _ = c1_system()
    W = orthonormal(b.size, 5, 21)
    Z, E, _ = O.recycle_setup(A, W)
    Pb = O.oblique_project(W, Z, E, b)
    PPb = O.oblique_project(W, Z, E, Pb)
    assert np.linalg.norm(PPb - Pb) <= 1e-13 * np.linalg.norm(b)
    ra = O.solve(A, b, None, 1e-10, O.Config(restart_m=20, recycle_k=5, snapshots_s=5, method=O.AUG_OBLIQUE), W)
    rd = O.solve(A, b, None, 1e-10, O.Config(restart_m=20, recycle_k=5, snapshots_s=5, method=O.DEFL_OBLIQUE), W)
    assert ra.iterations == rd.iterations
    assert np.array_equal(ra.x, rd.x)


def test_invariant_subspace_reduces_to_complement_block():
    """W spanning an invariant subspace of A (block-diagonal A, W = first block's coordinates):
    the residual has no component left in span(W) and the recycled solve is plain GMRES on the
    second block (section 3.2, the invariant-subspace estimate)."""
    A1, b1 = rand_system(12, 4)
    A2, b2 = rand_system(30, 5)
    A = sp.block_diag([A1, A2], format="csr")
    b = np.concatenate([b1, b2])
    W = np.zeros((42, 12))
    W[:12, :] = orthonormal(12, 12, 2)
    res = O.solve(A, b, None, 1e-11, O.Config(restart_m=50, recycle_k=12, snapshots_s=12), W)
    res2 = O.solve(A2, b2, None, 1e-11 * np.linalg.norm(b) / np.linalg.norm(b2), O.Config(restart_m=50, method=O.PLAIN))
    assert res.converged
    assert res.iterations == res2.iterations
    r = b - A @ res.x
    assert np.linalg.norm(r[:12]) <= 1e-13 * np.linalg.norm(b)
    assert np.linalg.norm(res.x[:12] - np.linalg.solve(A1.toarray(), b1)) <= 1e-12 * np.linalg.norm(b1) * 100


def test_recycling_reduces_iterations_on_sequence():
    """The method's purpose (section 6): recycling the SVD space of previous solutions cuts
    Arnoldi steps on a slowly varying sequence."""
    asm, systems, _ = WL.march(WL.C3_SMALL, 10, 0)
    A_list = [asm.csr(v) for v, _ in systems]
    b_list = [b for _, b in systems]
    plain, _ = O.run_sequence(A_list, b_list, 1e-10, O.Config(restart_m=50, method=O.PLAIN, precond=1))
    rec, _ = O.run_sequence(A_list, b_list, 1e-10, O.Config(restart_m=50, recycle_k=16, snapshots_s=32, precond=1))
    assert sum(r.iterations for r in rec[5:]) < 0.75 * sum(r.iterations for r in plain[5:])
    for r, p in zip(rec, plain):
        assert r.converged and p.converged
        assert np.linalg.norm(r.x - p.x) <= 1e-8 * np.linalg.norm(p.x)


# -- SVD recycle space ----------------------------------------------------------------


def test_svd_basis_eckart_young_and_rank():
    rng = np.random.default_rng(3)
    n, c, k = 300, 12, 5
    X = rng.standard_normal((n, c)) @ np.diag(2.0 ** -np.arange(c)) @ orthonormal(c, c, 1).T
    W, sig, rank = O.svd_basis(X, k)
    assert rank == c and W.shape == (n, k)
    assert np.abs(W.T @ W - np.eye(k)).max() <= 1e-14
    # Eckart-Young (eqs. best_rank_s / opt_svd): the residual of the rank-k projection
    res = np.linalg.norm(X - W @ (W.T @ X), "fro") ** 2
    assert abs(res - np.sum(sig[k:] ** 2)) <= 1e-12 * np.sum(sig ** 2)
    # singular values are those of X (X^T X eigenvalues, an independent route)
    ev = np.sort(np.linalg.eigvalsh(X.T @ X))[::-1]
    assert np.allclose(sig ** 2, ev, rtol=1e-10, atol=1e-12 * ev[0])
    # span is invariant under a permutation of the snapshot columns
    Wp, _, _ = O.svd_basis(X[:, rng.permutation(c)], k)
    s = np.linalg.svd(W.T @ Wp, compute_uv=False)
    assert s.min() >= 1 - 1e-12


def test_svd_basis_rank_cut_on_duplicate_snapshots():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(100)
    y = rng.standard_normal(100)
    X = np.column_stack([x, y, x, 2 * y, x + y])
    W, sig, rank = O.svd_basis(X, 4)
    assert rank == 2 and W.shape[1] == 2
    B, _ = np.linalg.qr(np.column_stack([x, y]))
    assert np.linalg.svd(W.T @ B, compute_uv=False).min() >= 1 - 1e-12
    W0, _, r0 = O.svd_basis(np.zeros((50, 3)), 2)
    assert r0 == 0 and W0.shape == (50, 0)


def test_ring_keeps_most_recent_s_and_interval():
    cfg = O.Config(recycle_k=2, snapshots_s=3, svd_interval=2)
    st = O.RecycleState(10, cfg)
    e = np.eye(10)
    st.update(e[0])
    assert st.W.shape[1] == 0           # no SVD before the first interval boundary
    st.update(e[1])
    assert st.W.shape[1] == 2
    for i in range(2, 6):
        st.update(e[i])
    assert len(st.ring) == 3 and np.array_equal(st.ring[0], e[3])
    # span of W is within the span of the 3 most recent snapshots
    assert np.abs(st.W[:3]).max() == 0.0


# -- degenerate and failure cases -----------------------------------------------------


def test_zero_rhs_and_nonfinite():
    A, b = rand_system(20, 6)
    res = O.solve(A, np.zeros(20), np.ones(20), 1e-8, O.Config())
    assert res.converged and res.iterations == 0 and not res.x.any()
    bn = b.copy()
    bn[3] = np.nan
    res = O.solve(A, bn, None, 1e-8, O.Config())
    assert not res.converged and res.flags & O.FLAG_NONFINITE


def test_singular_E_drops_recycling():
    A, b = rand_system(30, 7)
    w = orthonormal(30, 1, 0)
    W = np.column_stack([w, w])          # duplicate columns -> E singular
    res = O.solve(A, b, None, 1e-10, O.Config(restart_m=30, recycle_k=2, snapshots_s=2), W)
    assert res.flags & O.FLAG_RECYCLE_DROPPED and res.k_eff == 0 and res.converged


def invariant_krylov_system(n=60, d=3, seed=11, scale=1.0):
    """A system whose Krylov space from b is a d-dimensional invariant subspace of A:
    A = Pi diag(B, C) Pi^T (B d x d nonsymmetric, C a random shifted sparse block, Pi a random
    permutation that scatters the subspace over the index range) and b = Pi [b1; 0].  The exact
    solution is Pi [B^{-1} b1; 0], and K_j(A, b) stops growing at j = d.  Products with vectors
    supported on the subspace are exact outside it, so the Hessenberg entry that signals the
    breakdown is zero up to rounding of the subspace's own arithmetic."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((d, d)) + 3.0 * np.eye(d)
    C, _ = rand_system(n - d, seed + 1)
    M = sp.block_diag([sp.csr_matrix(B), C]).tocsr()
    perm = rng.permutation(n)
    P = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    A = (scale * (P @ M @ P.T)).tocsr()
    A.sort_indices()
    b1 = rng.standard_normal(d)
    b = P @ np.concatenate([b1, np.zeros(n - d)])
    xs = P @ np.concatenate([np.linalg.solve(B, b1) / scale, np.zeros(n - d)])
    return A, b, xs


@pytest.mark.parametrize("scale", [1.0, 1e20, 1e-20])
def test_lucky_breakdown_exit(scale):
    """Krylov space invariant after d steps: the cycle ends at exactly step d with the lucky
    flag (even with the residual stop switched off), at any scale of A, and the iterate is the
    exact solution; a generic system never raises the flag."""
    for d in (1, 3, 5):
        A, b, xs = invariant_krylov_system(d=d, scale=scale)
        cyc = O.arnoldi_cycle(lambda v: A @ v, b, 20, 0.0, 20)
        assert cyc.lucky and cyc.steps == d, (d, cyc.lucky, cyc.steps)
        y = scipy.linalg.solve_triangular(cyc.R[:d, :d], cyc.g[:d])
        assert np.linalg.norm(cyc.V[:, :d] @ y - xs) <= 1e-12 * np.linalg.norm(xs)
        res = O.solve(A, b, None, 1e-12, O.Config(restart_m=20, method=O.PLAIN))
        assert res.flags & O.FLAG_BREAKDOWN_LUCKY and res.iterations == d and res.cycles == 1, (d, res.flags)
        assert res.converged and np.linalg.norm(res.x - xs) <= 1e-12 * np.linalg.norm(xs)
        # nearly invariant: b leaves the subspace by 1e-11 relative, so the subdiagonal entry at
        # step d is small (about 1e-11 to 1e-9 of its column) but far above rounding: no
        # breakdown, and the iteration goes on to the full solution
        c = np.random.default_rng(5).standard_normal(b.size)
        c[b != 0] = 0.0
        b2 = b + 1e-11 * np.linalg.norm(b) * c / np.linalg.norm(c)
        res = O.solve(A, b2, None, 1e-12, O.Config(restart_m=20, method=O.PLAIN))
        assert res.converged and not res.flags & O.FLAG_BREAKDOWN_LUCKY and res.iterations > d, (d, res.flags)
        x2 = np.linalg.solve(A.toarray(), b2)
        assert np.linalg.norm(res.x - x2) <= 1e-10 * np.linalg.norm(x2)
    # generic systems: restarted cycles, no invariant subspace reached, no flag
    for seed in range(4):
        A, b = rand_system(60, seed)
        A = (scale * A).tocsr()
        res = O.solve(A, b, None, 1e-10, O.Config(restart_m=10, method=O.PLAIN))
        assert res.converged and not res.flags & O.FLAG_BREAKDOWN_LUCKY, seed


def test_max_iters_not_converged():
    A, b, _ = c1_system()
    res = O.solve(A, b, None, 1e-12, O.Config(restart_m=30, method=O.PLAIN, max_iters=3))
    assert not res.converged and res.iterations == 3
    assert res.rel_res_true > 1e-12


# -- orthogonal projector variants (Table 1 rows 1 and 4) and the smallest modes -------


@pytest.mark.parametrize("method", [O.AUG_ORTHO, O.DEFL_ORTHO])
def test_orthogonal_variant_minimises_projected_residual(method):
    """Inside the solve, each step's implicit residual equals the brute-force minimum of
    ||(I - W W^T)(r0 - A D^{-1} K z)|| over the Krylov space of the operator (I - W W^T) A D^{-1}
    started from the projected-guess residual (Table 1, orthogonal rows; section 3.3)."""
    A, b, _ = c1_system(step=4)
    n = b.size
    dinv = O.jacobi_inverse(A)
    W = orthonormal(n, 3, 11)
    # the guess: x0 = W (W^T A W)^{-1} W^T b, by dense algebra
    Wd = W
    E = Wd.T @ (A @ Wd)
    x0 = Wd @ np.linalg.solve(E, Wd.T @ b)
    r0 = b - A @ x0
    Pmat = np.eye(n) - Wd @ Wd.T
    op_ref = lambda v: Pmat @ (A @ (dinv * v))
    res = O.solve(A, b, None, 1e-30, O.Config(restart_m=10, method=method, precond=O.PRECOND_JACOBI,
                                                 max_iters=10), W)
    bnorm = np.linalg.norm(b)
    for j in range(1, 11):
        ref = krylov_min_residual(op_ref, Pmat @ r0, j)
        assert abs(res.implicit_history[j - 1] * bnorm - ref) <= 1e-9 * np.linalg.norm(r0) + 1e-8 * ref, j


def test_orthogonal_equals_oblique_on_invariant_subspace():
    """For symmetric A and W spanning an invariant subspace, A W = W L, so E = L and the oblique
    projector I - A W E^{-1} W^T reduces to I - W W^T: the two methods give the same iterates."""
    n = 60
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(1.0, 30.0, n)
    A = sp.csr_matrix((Q * lam) @ Q.T)
    W = Q[:, :5]
    b = rng.standard_normal(n)
    cfg = dict(restart_m=8, max_iters=200)
    ro = O.solve(A, b, None, 1e-12, O.Config(method=O.AUG_ORTHO, **cfg), W)
    rb = O.solve(A, b, None, 1e-12, O.Config(method=O.AUG_OBLIQUE, **cfg), W)
    assert ro.iterations == rb.iterations
    assert np.linalg.norm(ro.x - rb.x) <= 1e-10 * np.linalg.norm(rb.x)
    # and on a nonsymmetric matrix the two differ (the variant is not silently the oblique one)
    An, bn = rand_system(60, 5)
    Wn = orthonormal(60, 5, 6)
    r1 = O.solve(An, bn, None, 1e-12, O.Config(method=O.AUG_ORTHO, restart_m=8, max_iters=3), Wn)
    r2 = O.solve(An, bn, None, 1e-12, O.Config(method=O.AUG_OBLIQUE, restart_m=8, max_iters=3), Wn)
    assert np.linalg.norm(r1.x - r2.x) > 1e-6 * np.linalg.norm(r2.x)


def test_orthogonal_solves_a_sequence_to_tolerance():
    """The orthogonal variants converge on the generator sequence to the explicit tolerance, with
    W^T r = 0 after every cycle's correction (so the projected and true residuals coincide)."""
    asm, systems, _ = WL.march(WL.C1, 8, 1)
    for method in (O.AUG_ORTHO, O.DEFL_ORTHO):
        cfg = O.Config(restart_m=30, recycle_k=5, snapshots_s=10, method=method)
        results, st = O.run_sequence([asm.csr(v) for v, _ in systems], [b for _, b in systems], 1e-10, cfg)
        assert st.W.shape[1] == 5
        for (v, b), r in zip(systems, results):
            assert r.converged and np.linalg.norm(b - asm.csr(v) @ r.x) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)


def test_svd_basis_smallest_modes():
    """select smallest: W spans the left singular vectors of the k smallest singular values above
    the rank cut (Algorithm 1 with the trailing modes), on a matrix built from known factors."""
    rng = np.random.default_rng(8)
    n, c, k = 500, 12, 4
    U, _ = np.linalg.qr(rng.standard_normal((n, c)))
    Vt, _ = np.linalg.qr(rng.standard_normal((c, c)))
    sig = 10.0 ** (-0.5 * np.arange(c))
    sig[-2:] = 0.0                                   # rank 10
    X = (U * sig) @ Vt.T
    W, s, rank = O.svd_basis(X, k, smallest=True)
    assert rank == 10 and W.shape[1] == k
    cos = np.linalg.svd(U[:, rank - k:rank].T @ W, compute_uv=False)
    assert cos.min() >= 1 - 1e-10


# -- initial-guess strategies (section 4) ----------------------------------------------


def test_extrapolation_weights_are_the_printed_ones():
    """Eqs. (ext2), (ext3), (ext4) print the coefficients of the linear, quadratic and cubic
    extrapolations."""
    assert O.extrapolation_weights(2) == [2, -1]
    assert O.extrapolation_weights(3) == [3, -3, 1]
    assert O.extrapolation_weights(4) == [4, -6, 4, -1]
    assert O.extrapolation_weights(1) == [1]


def _poly_history(deg, count, n=40, seed=0):
    """x(t) = sum_{d<=deg} c_d t^d at t = 0..count (the last one is the value to predict)."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((deg + 1, n))
    return [sum(C[d] * float(t) ** d for d in range(deg + 1)) for t in range(count + 1)]


@pytest.mark.parametrize("order", [2, 3, 4])
def test_extrapolation_exact_for_polynomials_in_time(order):
    """Lagrange extrapolation through `order` equispaced points reproduces every polynomial of
    degree < order (section 4.1); one degree more it does not."""
    xs = _poly_history(order - 1, 6)
    pred = O.extrapolate(xs[:-1], order)
    assert np.linalg.norm(pred - xs[-1]) <= 1e-10 * np.linalg.norm(xs[-1])
    xs = _poly_history(order, 6, seed=1)
    pred = O.extrapolate(xs[:-1], order)
    assert np.linalg.norm(pred - xs[-1]) > 1e-3 * np.linalg.norm(xs[-1])


@pytest.mark.parametrize("order", [2, 3, 4])
def test_extrapolated_guess_then_no_iteration_on_polynomial_sequence(order):
    """A fixed matrix and solutions polynomial in the step index (degree order-1): from exact
    previous solutions the guess is the solution and GMRES takes no step; along a solved
    sequence (previous solutions exact to the tolerance only) the guess is off by the propagated
    solve errors, so a step or two remain; the guess itself is the closed-form extrapolation."""
    A, _ = rand_system(40, 11)
    xs = _poly_history(order - 1, 9, n=40, seed=2)
    method = {2: O.GUESS_EXTRAP2, 3: O.GUESS_EXTRAP3, 4: O.GUESS_EXTRAP4}[order]
    cfg = O.Config(restart_m=20, snapshots_s=order, method=method)
    for i in range(order, 10):
        res = O.solve(A, A @ xs[i], None, 1e-10, cfg, None, xs[i - order:i])
        assert res.converged and res.iterations == 0, (i, res.iterations)
        assert np.linalg.norm(res.x - xs[i]) <= 1e-9 * np.linalg.norm(xs[i])
    results, st = O.run_sequence([A] * 10, [A @ x for x in xs], 1e-10, cfg)
    first = results[1].iterations
    assert first > 4
    for i, res in enumerate(results):
        assert res.converged
        if i >= order:
            assert res.iterations <= 2, (i, res.iterations)
    assert len(st.ring) == order and st.W.shape[1] == 0
    # with max_iters = 0 the returned iterate is the guess: the printed combination of the history
    hist = [np.array(x) for x in _poly_history(order, 5, n=40, seed=3)[:-1]]
    cfg0 = O.Config(restart_m=20, snapshots_s=order, method=method, max_iters=0)
    res = O.solve(A, A @ hist[0], None, 1e-10, cfg0, None, hist)
    want = {2: 2 * hist[-1] - hist[-2],
            3: 3 * hist[-1] - 3 * hist[-2] + hist[-3],
            4: 4 * hist[-1] - 6 * hist[-2] + 4 * hist[-3] - hist[-4]}[order]
    assert np.allclose(res.x, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_projection_guess_satisfies_the_galerkin_conditions():
    """Eq. (projection_guess): x0 lies in span(W) and its residual is orthogonal to W; the two
    conditions fix x0 (max_iters = 0 returns the guess itself)."""
    A, b = rand_system(60, 21)
    W = orthonormal(60, 5, 22)
    cfg = O.Config(restart_m=20, recycle_k=5, snapshots_s=5, method=O.GUESS_PROJECT, max_iters=0)
    res = O.solve(A, b, None, 1e-10, cfg, W)
    x = res.x
    assert np.linalg.norm(x - W @ (W.T @ x)) <= 1e-13 * np.linalg.norm(x)
    assert np.abs(W.T @ (b - A @ x)).max() <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x) > 0.0


def test_projection_guess_then_plain_gmres():
    """Eq. (iteration_projection): after the guess the Krylov iteration is the unmodified one: its
    implicit residuals are the brute-force minima over K_j(A D^-1, r0) of the plain operator."""
    A, b, _ = c1_system(step=4)
    n = b.size
    W = orthonormal(n, 4, 23)
    dinv = O.jacobi_inverse(A)
    cfg0 = O.Config(restart_m=8, recycle_k=4, snapshots_s=4, method=O.GUESS_PROJECT,
                    precond=O.PRECOND_JACOBI, max_iters=0)
    xg = O.solve(A, b, None, 0.0, cfg0, W).x
    r0 = b - A @ xg
    cfg = O.Config(restart_m=8, recycle_k=4, snapshots_s=4, method=O.GUESS_PROJECT,
                   precond=O.PRECOND_JACOBI, max_iters=8)
    res = O.solve(A, b, None, 0.0, cfg, W)
    bn = np.linalg.norm(b)
    op = lambda v: A @ (dinv * v)
    for j in range(1, 9):
        ref = krylov_min_residual(op, r0, j)
        assert abs(res.implicit_history[j - 1] * bn - ref) <= 1e-9 * np.linalg.norm(r0) + 1e-8 * ref


def test_projection_beats_extrapolation_off_polynomial_trajectory():
    """Solutions in a fixed two-dimensional space with non-polynomial coefficients: once W spans
    it (after two solves) the projection guess is exact up to the previous solves' tolerance (a
    step or two remain), while linear extrapolation leaves a residual that needs a full solve;
    with exact previous solutions the projection guess is the solution."""
    A, _ = rand_system(50, 31)
    U = orthonormal(50, 2, 32)
    xs = [U @ np.array([np.cos(0.7 * i), np.sin(1.3 * i) + 2.0]) for i in range(8)]
    bs = [A @ x for x in xs]
    proj, _ = O.run_sequence([A] * 8, bs, 1e-10,
                             O.Config(restart_m=20, recycle_k=2, snapshots_s=2, method=O.GUESS_PROJECT))
    ext, _ = O.run_sequence([A] * 8, bs, 1e-10,
                            O.Config(restart_m=20, snapshots_s=2, method=O.GUESS_EXTRAP2))
    assert all(r.iterations <= 2 for r in proj[2:])
    assert all(r.iterations >= proj[0].iterations // 2 for r in ext[2:])
    W = np.linalg.qr(np.column_stack(xs[:2]))[0]
    cfg = O.Config(restart_m=20, recycle_k=2, snapshots_s=2, method=O.GUESS_PROJECT)
    for i in range(2, 8):
        res = O.solve(A, bs[i], None, 1e-10, cfg, W)
        assert res.iterations == 0 and np.linalg.norm(res.x - xs[i]) <= 1e-9 * np.linalg.norm(xs[i])


# -- least-squares projector rows (Table 1 rows 3 and 6) -------------------------------


def _galerkin_guess(A, W, b):
    """x0 = W (W^T A W)^{-1} W^T b (eq. (projection_t_s)) by dense algebra, and its residual."""
    E = W.T @ (A @ W)
    x0 = W @ np.linalg.solve(E, W.T @ b)
    return x0, b - A @ x0


def _krylov_basis(op, r0, j):
    """Orthonormal basis of K_j(op, r0) from the normalised power sequence and a library QR."""
    K = np.empty((r0.size, j))
    v = r0 / np.linalg.norm(r0)
    for i in range(j):
        K[:, i] = v
        v = op(v)
        v = v / np.linalg.norm(v)
    return np.linalg.qr(K)[0]


def _ls_case():
    A, b, _ = c1_system(step=4)
    n = b.size
    dinv = O.jacobi_inverse(A)
    W = orthonormal(n, 3, 12)
    AW = np.asarray(A @ W)
    Qz = np.linalg.qr(AW)[0]
    Pm = np.eye(n) - Qz @ Qz.T          # orthogonal projector onto range(A W)^perp, by a dense QR
    x0, r0 = _galerkin_guess(A, W, b)
    return A, b, dinv, W, AW, Pm, r0


def test_deflated_ls_is_minimal_residual_over_the_sum_space():
    """Deflated LS (Table 1 row 6, the inner iteration of GCRO): after j steps the implicit
    residual, and the true residual of the returned iterate after the least-squares correction,
    equal the brute-force minimum of ||r0 - A W c - A D^{-1} K z|| over c and over z in
    K_j(P A D^{-1}, P r0), with P built from a dense QR of A W and r0 the residual of the
    projection guess; the final residual is orthogonal to A W."""
    A, b, dinv, W, AW, Pm, r0 = _ls_case()
    op_ref = lambda v: Pm @ (A @ (dinv * v))
    bnorm = np.linalg.norm(b)
    for j in (1, 3, 6, 10):
        res = O.solve(A, b, None, 1e-30, O.Config(restart_m=10, method=O.DEFL_LS, precond=O.PRECOND_JACOBI,
                                                     max_iters=j), W)
        K = _krylov_basis(op_ref, Pm @ r0, j)
        M = np.column_stack([AW, A @ (dinv[:, None] * K)])
        c, *_ = np.linalg.lstsq(M, r0, rcond=None)
        ref = np.linalg.norm(r0 - M @ c)
        rfin = b - A @ res.x
        assert res.iterations == j and res.k_eff == 3
        assert abs(res.implicit_history[j - 1] * bnorm - ref) <= 1e-9 * np.linalg.norm(r0), j
        assert abs(np.linalg.norm(rfin) - ref) <= 1e-9 * np.linalg.norm(r0), j
        assert np.linalg.norm(AW.T @ rfin) <= 1e-10 * np.linalg.norm(AW) * np.linalg.norm(r0), j


def test_augmented_ls_minimises_from_the_unprojected_residual():
    """Augmented LS (Table 1 row 3): the Krylov space K_j(P A D^{-1}, r0) starts from the
    unprojected residual, so the implicit residual is the brute-force minimum of
    ||r0 - P A D^{-1} K z|| and never falls below ||(I - P) r0|| (why the paper saw this row fail
    to converge); after the least-squares correction the true residual is the minimum of
    ||r0 - A W c - A D^{-1} K z|| over the same space, and the two differ by exactly that floor."""
    A, b, dinv, W, AW, Pm, r0 = _ls_case()
    op_ref = lambda v: Pm @ (A @ (dinv * v))
    bnorm = np.linalg.norm(b)
    floor = np.linalg.norm(r0 - Pm @ r0)
    assert floor > 1e-3 * np.linalg.norm(r0)          # the case is not degenerate
    for j in (2, 5, 9):
        res = O.solve(A, b, None, 1e-30, O.Config(restart_m=10, method=O.AUG_LS, precond=O.PRECOND_JACOBI,
                                                     max_iters=j), W)
        imp = res.implicit_history[j - 1] * bnorm
        assert abs(imp - krylov_min_residual(op_ref, r0, j)) <= 1e-9 * np.linalg.norm(r0), j
        assert imp >= floor * (1 - 1e-12)
        K = _krylov_basis(op_ref, r0, j)
        M = np.column_stack([AW, A @ (dinv[:, None] * K)])
        c, *_ = np.linalg.lstsq(M, r0, rcond=None)
        ref = np.linalg.norm(r0 - M @ c)
        fin = np.linalg.norm(b - A @ res.x)
        assert abs(fin - ref) <= 1e-9 * np.linalg.norm(r0), j
        assert abs(imp ** 2 - floor ** 2 - fin ** 2) <= 1e-8 * np.linalg.norm(r0) ** 2, j


def test_ls_rows_equal_oblique_on_invariant_subspace():
    """If A W = W L (W spans an invariant subspace of a nonsymmetric A), range(A W) = range(W) and
    the least-squares, orthogonal and oblique projectors coincide, as do the least-squares and
    Galerkin corrections: all rows give the same iterates.  On a generic matrix they differ."""
    n, k = 60, 5
    rng = np.random.default_rng(21)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    T = np.triu(rng.standard_normal((n, n)), 1) * 0.3 + np.diag(np.linspace(2.0, 20.0, n))
    T[k:, :k] = 0.0                                  # block upper triangular: span(Q[:, :k]) invariant
    A = sp.csr_matrix(Q @ T @ Q.T)
    W = Q[:, :k]
    b = rng.standard_normal(n)
    cfg = dict(restart_m=8, max_iters=300)
    ref = O.solve(A, b, None, 1e-12, O.Config(method=O.AUG_OBLIQUE, **cfg), W)
    for m in (O.AUG_LS, O.DEFL_LS):
        r = O.solve(A, b, None, 1e-12, O.Config(method=m, **cfg), W)
        assert r.converged and r.iterations == ref.iterations, (m, r.iterations, ref.iterations)
        assert np.linalg.norm(r.x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    An, bn = rand_system(60, 5)
    Wn = orthonormal(60, 5, 6)
    xs = [O.solve(An, bn, None, 1e-12, O.Config(method=m, restart_m=8, max_iters=3), Wn).x
          for m in (O.AUG_OBLIQUE, O.AUG_LS, O.DEFL_LS)]
    assert np.linalg.norm(xs[1] - xs[0]) > 1e-6 * np.linalg.norm(xs[0])
    assert np.linalg.norm(xs[2] - xs[1]) > 1e-6 * np.linalg.norm(xs[0])


def test_ls_rows_solve_a_sequence_to_tolerance():
    """Both LS rows converge on the generator sequence with the SVD recycle space (augmented LS
    through a restart: its first cycle's estimate is floored, the correction then removes the
    floor), and deflated LS takes no more Arnoldi steps than plain GMRES on any system."""
    asm, systems, _ = WL.march(WL.C1, 8, 1)
    As = [asm.csr(v) for v, _ in systems]
    bs = [b for _, b in systems]
    plain, _ = O.run_sequence(As, bs, 1e-10, O.Config(restart_m=30, method=O.PLAIN))
    for method in (O.AUG_LS, O.DEFL_LS):
        cfg = O.Config(restart_m=30, recycle_k=5, snapshots_s=10, method=method)
        results, st = O.run_sequence(As, bs, 1e-10, cfg)
        assert st.W.shape[1] == 5
        for A, b, r, p in zip(As, bs, results, plain):
            assert r.converged and np.linalg.norm(b - A @ r.x) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
            if method == O.DEFL_LS:
                assert r.iterations <= p.iterations


# -- Ritz and harmonic Ritz recycle spaces (section 5.1) -------------------------------


def small_eigen_system(n=64, seed=21):
    """A = Pi [[B, K], [0, C]] Pi^T: B (4 x 4) holds the four eigenvalues of smallest modulus,
    0.01 +- 0.02i, 0.03 and 0.05 (a rotation block and two diagonal entries), C is a shifted random
    sparse block whose field of values stays far from the origin, K a sparse coupling (so the
    invariant subspace of B, the columns Pi e_0..e_3, has no invariant orthogonal complement and
    its left and right eigenvectors differ); Pi scatters it over the index range."""
    rng = np.random.default_rng(seed)
    B = np.array([[0.01, 0.02, 0, 0], [-0.02, 0.01, 0, 0], [0, 0, 0.03, 0], [0, 0, 0, 0.05]])
    C, _ = rand_system(n - 4, seed + 1, density=0.08, shift=4.0)
    K = sp.random(4, n - 4, density=0.2, random_state=rng) * 0.5
    M = sp.bmat([[sp.csr_matrix(B), K], [None, C]]).tocsr()
    perm = rng.permutation(n)
    P = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    A = (P @ M @ P.T).tocsr()
    A.sort_indices()
    X_B = P.toarray()[:, :4]          # orthonormal basis of B's invariant subspace
    return A, X_B, np.array([0.01 + 0.02j, 0.01 - 0.02j, 0.03, 0.05])


def _max_angle_sin(X, Y):
    """sin of the largest principal angle between span(X) and span(Y) (equal dimensions)."""
    Qx, Qy = np.linalg.qr(X)[0], np.linalg.qr(Y)[0]
    return float(np.linalg.norm(Qy - Qx @ (Qx.T @ Qy), 2))


@pytest.mark.parametrize("harmonic", [False, True])
def test_ritz_space_recovers_an_invariant_subspace(harmonic):
    """A search space that contains an invariant subspace gives its eigenpairs exactly: the four
    smallest (harmonic) Ritz values are B's eigenvalues, the complex pair included, and W spans
    the subspace; with k = 3 the pair and 0.03 are kept; with k = 1 the pair does not fit and
    nothing is kept before it."""
    A, X_B, lam = small_eigen_system()
    rng = np.random.default_rng(3)
    U = np.column_stack([X_B @ rng.standard_normal((4, 4)), rng.standard_normal((64, 3))])
    W, theta = O.ritz_basis(A, U, 4, harmonic)
    assert W.shape[1] == 4 and np.abs(W.T @ W - np.eye(4)).max() <= 1e-13
    assert _max_angle_sin(W, X_B) <= 1e-10
    assert np.allclose(np.sort_complex(theta), np.sort_complex(lam), atol=1e-11)
    W3, theta3 = O.ritz_basis(A, U, 3, harmonic)
    assert W3.shape[1] == 3 and np.allclose(np.sort(np.abs(theta3)), np.sort(np.abs(lam[:3])), atol=1e-11)
    assert _max_angle_sin(W3, X_B[:, :3]) <= 1e-10
    W1, theta1 = O.ritz_basis(A, U, 1, harmonic)
    assert W1.shape[1] == 0


def test_harmonic_ritz_values_are_inverse_ritz_values_of_the_inverse():
    """Eq. (harmonic_ritz_inverse): the harmonic Ritz values of A over span(U) are the reciprocals of
    the Ritz values of A^{-1} over A span(U) (computed here with a dense inverse)."""
    rng = np.random.default_rng(8)
    n = 40
    Ad = rng.standard_normal((n, n)) + 6.0 * np.eye(n)
    A = sp.csr_matrix(Ad)
    U = rng.standard_normal((n, 7))
    Q = O.orthonormal_basis(U)
    theta, _ = O.ritz_pairs(A, Q, harmonic=True)
    P = np.linalg.qr(Ad @ Q)[0]
    mu = np.linalg.eigvals(P.T @ np.linalg.inv(Ad) @ P)
    assert np.allclose(np.sort_complex(theta), np.sort_complex(1.0 / mu), rtol=1e-10)
    # and they differ from the (plain) Ritz values on the same space
    ritz, _ = O.ritz_pairs(A, Q, harmonic=False)
    assert not np.allclose(np.sort_complex(theta), np.sort_complex(ritz), rtol=1e-3)


@pytest.mark.parametrize("harmonic", [False, True])
def test_ritz_values_of_a_symmetric_matrix_lie_in_its_spectrum(harmonic):
    """Symmetric positive definite A: (harmonic) Ritz values are real and inside [lambda_min,
    lambda_max] (Courant-Fischer; harmonic ones are inverted Ritz values of A^{-1}), and the pairs
    satisfy their Galerkin (Petrov-Galerkin) conditions."""
    rng = np.random.default_rng(5)
    n = 50
    G = rng.standard_normal((n, n))
    Ad = G @ G.T / n + 0.05 * np.eye(n)
    lam = np.linalg.eigvalsh(Ad)
    A = sp.csr_matrix(Ad)
    Q = O.orthonormal_basis(rng.standard_normal((n, 9)))
    theta, Z = O.ritz_pairs(A, Q, harmonic)
    assert np.abs(theta.imag).max() <= 1e-10 * lam[-1]
    assert theta.real.min() >= lam[0] * (1 - 1e-10) and theta.real.max() <= lam[-1] * (1 + 1e-10)
    for i in range(theta.size):
        y = Q @ Z[:, i]
        res = Ad @ y - theta[i] * y
        T = Ad @ Q if harmonic else Q
        assert np.linalg.norm(T.T @ res) <= 1e-10 * lam[-1] * np.linalg.norm(y)


def test_krylov_directions_carry_the_last_cycle_update():
    """Right Jacobi, one cycle: the returned solution minus the starting guess lies in the span of
    the cycle's x-space directions D^{-1} V (and not in the span of V itself)."""
    A, b = rand_system(40, 12, shift=4.0)
    A = (A + sp.diags(np.linspace(1.0, 30.0, 40))).tocsr()   # a diagonal far from constant
    x0 = np.random.default_rng(1).standard_normal(40)
    res = O.solve(A, b, x0, 1e-10, O.Config(restart_m=40, method=O.PLAIN, precond=O.PRECOND_JACOBI))
    assert res.cycles == 1
    K = res.krylov_x
    d = res.x - x0
    coef = np.linalg.lstsq(K, d, rcond=None)[0]
    assert np.linalg.norm(K @ coef - d) <= 1e-10 * np.linalg.norm(d)
    V = K / (1.0 / A.diagonal())[:, None]
    coef = np.linalg.lstsq(V[:, : K.shape[1] - 2], d, rcond=None)[0]
    assert np.linalg.norm(V[:, : K.shape[1] - 2] @ coef - d) > 1e-6 * np.linalg.norm(d)


@pytest.mark.parametrize("space", [O.SPACE_RITZ, O.SPACE_HARMONIC])
def test_ritz_recycling_deflates_small_eigenvalues(space):
    """GMRES(20) crawls on the four small eigenvalues; recycling the (harmonic) Ritz vectors of each
    solve's search space converges onto their invariant subspace within a few solves of the
    sequence (the same matrix, new right-hand sides), and the later solves take a small fraction of
    plain GMRES(20)'s steps on the same systems."""
    A, X_B, _ = small_eigen_system()
    rng = np.random.default_rng(9)
    bs = [rng.standard_normal(64) for _ in range(6)]
    plain = [O.solve(A, b, None, 1e-8, O.Config(restart_m=20, method=O.PLAIN)).iterations for b in bs]
    cfg = O.Config(restart_m=20, recycle_k=4, method=O.AUG_OBLIQUE, recycle_space=space)
    st = O.RecycleState(64, cfg)
    its = []
    for b in bs:
        r = O.solve(A, b, None, 1e-8, cfg, st.W)
        assert r.converged
        st.update(r.x, A, r)
        its.append(r.iterations)
    assert sum(its[3:]) <= 0.25 * sum(plain[3:]), (its, plain)
    assert st.W.shape[1] == 4 and _max_angle_sin(st.W, X_B) <= 0.05


# -- multicolour SSOR (the paper's preconditioner, section 6.1) ---------------------------


def _sor_sweeps(A, r, omega, order):
    """One forward SOR sweep over `order` from a zero start, then one backward sweep over it
    reversed: each row in turn takes the SOR update from the current values, in place."""
    Ad = A.toarray()
    z = np.zeros(len(r))
    for seq in (order, order[::-1]):
        for i in seq:
            s = r[i] - Ad[i] @ z + Ad[i, i] * z[i]
            z[i] = (1.0 - omega) * z[i] + omega * s / Ad[i, i]
    return z


@pytest.mark.parametrize("omega", [1.0, 1.4, 0.6])
def test_ssor_is_one_symmetric_sor_sweep(omega):
    """M^{-1} r equals one forward and one backward SOR sweep from zero in the colour order,
    written as plain loops over the rows of a nonsymmetric matrix (where forward-then-backward
    and backward-then-forward differ)."""
    A, _ = rand_system(40, 31, density=0.12, shift=3.0)
    ssor = O.MulticolourSSOR(A, omega)
    r = np.random.default_rng(2).standard_normal(40)
    z = _sor_sweeps(A, r, omega, list(np.argsort(ssor.colour, kind="stable")))
    assert np.abs(ssor(r) - z).max() <= 1e-12 * np.abs(z).max()


def test_ssor_rows_of_one_colour_are_independent():
    """Any order of the rows inside each colour gives the same sweeps (rows of one colour never
    couple), and the colouring has no coupled pair inside a colour."""
    A, _ = rand_system(40, 32, density=0.12, shift=3.0)
    col = O.greedy_colouring(A)
    coo = A.tocoo()
    off = coo.row != coo.col
    assert not np.any(col[coo.row[off]] == col[coo.col[off]])
    r = np.random.default_rng(3).standard_normal(40)
    rng = np.random.default_rng(4)
    base = _sor_sweeps(A, r, 1.2, list(np.argsort(col, kind="stable")))
    for _ in range(3):
        order = [i for c in range(col.max() + 1) for i in rng.permutation(np.flatnonzero(col == c))]
        assert np.abs(_sor_sweeps(A, r, 1.2, order) - base).max() <= 1e-13 * np.abs(base).max()
    assert np.abs(O.MulticolourSSOR(A, 1.2)(r) - base).max() <= 1e-12 * np.abs(base).max()


def test_first_fit_colouring_of_the_q1_grid():
    """The 9-point pattern of first-order elements, Dirichlet rows decoupled: first fit in
    natural order gives boundary nodes colour 0 and interior node (I, J) the colour
    2 ((J - 1) mod 2) + (I - 1) mod 2, four colours in all; a path gives red-black colours."""
    prob = WL.Problem(p=1, N=12, eps=1e-2, dt=0.5, beta="vortex")
    asm = WL.Assembler(prob)
    A = asm.csr(asm.matrix_values(np.zeros(prob.n)))
    col = O.greedy_colouring(A)
    J, I = np.divmod(np.arange(prob.n), prob.n1)
    expect = 2 * ((J - 1) % 2) + (I - 1) % 2
    expect[asm.pat.boundary] = 0
    assert np.array_equal(col, expect)
    path = sp.diags([np.ones(9), 4 * np.ones(10), np.ones(9)], [-1, 0, 1], format="csr")
    assert np.array_equal(O.greedy_colouring(path), np.arange(10) % 2)


@pytest.mark.parametrize("upper", [False, True])
def test_ssor_is_exact_on_a_colour_triangular_matrix(upper):
    """Couplings of odd rows to their even neighbours only (path colouring: even 0, odd 1) make
    A = D + L in the colour order, so with omega = 1 M = (D + L) D^{-1} D = A; the couplings of
    even rows to odd neighbours make A = D + U and M = D D^{-1} (D + U) = A.  M^{-1} A is the
    identity and GMRES with this preconditioner stops after one step."""
    rng = np.random.default_rng(12)
    n = 21
    A = sp.lil_matrix((n, n))
    for i in range(n):
        A[i, i] = 2.0 + rng.random()
        if (i % 2 == 0) == upper:
            for j in (i - 1, i + 1):
                if 0 <= j < n:
                    A[i, j] = rng.standard_normal()
    A = A.tocsr()
    ssor = O.MulticolourSSOR(A, 1.0)
    assert np.array_equal(ssor.colour, np.arange(n) % 2)
    v = rng.standard_normal(n)
    assert np.abs(ssor(A @ v) - v).max() <= 1e-13 * np.abs(v).max()
    b = rng.standard_normal(n)
    res = O.solve(A, b, None, 1e-12, O.Config(restart_m=10, method=O.PLAIN, precond=O.PRECOND_SSOR))
    assert res.converged and res.iterations == 1
    assert np.linalg.norm(A @ res.x - b) <= 1e-12 * np.linalg.norm(b)


def test_ssor_preconditioned_gmres_solves_and_helps():
    """Right SSOR: the solve meets the true-residual tolerance, and on a convection-diffusion
    system of the paper's family it takes fewer steps than Jacobi."""
    prob = WL.Problem(p=1, N=24, eps=1e-2, dt=0.5, beta="vortex", forcing=True, u0="zero", beta_projected=True)
    asm, systems, _ = WL.march(prob, 3, 0)
    A, b = asm.csr(systems[2][0]), systems[2][1]
    its = {}
    for pc in (O.PRECOND_JACOBI, O.PRECOND_SSOR):
        r = O.solve(A, b, None, 1e-10, O.Config(restart_m=30, method=O.PLAIN, precond=pc))
        assert r.converged and np.linalg.norm(b - A @ r.x) <= 1e-10 * np.linalg.norm(b)
        its[pc] = r.iterations
    assert its[O.PRECOND_SSOR] < 0.75 * its[O.PRECOND_JACOBI], its


# -- planted mistakes: each plausible error in the oracle is caught by a pin ----------


def _pins_pass():
    try:
        test_unrestarted_gmres_equals_dense_solve(O.PRECOND_JACOBI)
        test_oblique_projector_identities()
        test_projection_guess_exact_when_solution_in_span()
        test_implicit_residual_is_krylov_minimum(True)
        test_correction_leaves_residual_orthogonal_to_W()
        test_orthogonal_variant_minimises_projected_residual(O.AUG_ORTHO)
        test_orthogonal_equals_oblique_on_invariant_subspace()
        test_extrapolated_guess_then_no_iteration_on_polynomial_sequence(3)
        test_projection_guess_satisfies_the_galerkin_conditions()
        test_projection_guess_then_plain_gmres()
        test_deflated_ls_is_minimal_residual_over_the_sum_space()
        test_augmented_ls_minimises_from_the_unprojected_residual()
        test_lucky_breakdown_exit(1e20)
        test_lucky_breakdown_exit(1e-20)
        test_ritz_space_recovers_an_invariant_subspace(False)
        test_ritz_space_recovers_an_invariant_subspace(True)
        test_harmonic_ritz_values_are_inverse_ritz_values_of_the_inverse()
        test_krylov_directions_carry_the_last_cycle_update()
        test_ssor_is_one_symmetric_sor_sweep(1.4)
        test_ssor_rows_of_one_colour_are_independent()
        test_first_fit_colouring_of_the_q1_grid()
        test_ssor_is_exact_on_a_colour_triangular_matrix(False)
    except AssertionError:
        return False
    return True


def test_pins_pass_on_unmodified_oracle():
    assert _pins_pass()


@pytest.mark.parametrize("mutation", ["projector_uses_W", "guess_transposed_E", "givens_sign",
                                      "update_without_preconditioner", "operator_perturbed",
                                      "correction_sign", "ortho_projector_missing", "ortho_projector_half",
                                      "extrap_weights_reversed", "extrap_off_by_one",
                                      "guess_only_projects_krylov", "ls_projector_missing",
                                      "ls_correction_galerkin", "ls_coefficients_unnormalised",
                                      "ls_deflated_start_unprojected", "lucky_never", "lucky_absolute",
                                      "lucky_loose", "ritz_largest_first", "harmonic_as_plain_ritz",
                                      "ritz_pair_real_part_only", "ritz_left_eigenvectors",
                                      "krylov_directions_unpreconditioned", "ssor_sweeps_swapped",
                                      "ssor_middle_diagonal_dropped", "ssor_scale_dropped",
                                      "colouring_by_parity", "ssor_colours_reversed"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    if mutation == "ssor_sweeps_swapped":
        def swapped(self, r):
            from scipy.sparse.linalg import spsolve_triangular
            w = self.omega
            y = spsolve_triangular(self.upper, w * (2.0 - w) * r[self.perm], lower=False)
            z = spsolve_triangular(self.lower, self.d * y, lower=True)
            out = np.empty_like(z)
            out[self.perm] = z
            return out
        monkeypatch.setattr(O.MulticolourSSOR, "__call__", swapped)
    elif mutation == "ssor_middle_diagonal_dropped":
        def nodiag(self, r):
            from scipy.sparse.linalg import spsolve_triangular
            w = self.omega
            y = spsolve_triangular(self.lower, w * (2.0 - w) * r[self.perm], lower=True)
            z = spsolve_triangular(self.upper, y, lower=False)
            out = np.empty_like(z)
            out[self.perm] = z
            return out
        monkeypatch.setattr(O.MulticolourSSOR, "__call__", nodiag)
    elif mutation == "ssor_scale_dropped":
        orig_call = O.MulticolourSSOR.__call__
        monkeypatch.setattr(O.MulticolourSSOR, "__call__",
                            lambda self, r: orig_call(self, r) / (self.omega * (2.0 - self.omega)))
    elif mutation == "colouring_by_parity":
        monkeypatch.setattr(O, "greedy_colouring", lambda A: np.arange(A.shape[0]) % 2)
    elif mutation == "ssor_colours_reversed":
        orig_col = O.greedy_colouring
        monkeypatch.setattr(O, "greedy_colouring", lambda A: (lambda c: c.max() - c)(orig_col(A)))
    elif mutation == "ritz_largest_first":
        orig_o = O.ritz_order
        monkeypatch.setattr(O, "ritz_order", lambda th: orig_o(th)[::-1])
    elif mutation == "harmonic_as_plain_ritz":
        orig_p = O.ritz_pairs
        monkeypatch.setattr(O, "ritz_pairs", lambda A, Q, harmonic: orig_p(A, Q, False))
    elif mutation == "ritz_pair_real_part_only":
        monkeypatch.setattr(O, "pair_basis", lambda y: [y.real.copy(), y.real.copy()])
    elif mutation == "ritz_left_eigenvectors":
        def left(A, Q, harmonic):
            AQ = np.column_stack([A @ Q[:, i] for i in range(Q.shape[1])])
            if harmonic:
                return scipy.linalg.eig((AQ.T @ AQ).T, (AQ.T @ Q).T)
            return scipy.linalg.eig((Q.T @ AQ).T)
        monkeypatch.setattr(O, "ritz_pairs", left)
    elif mutation == "krylov_directions_unpreconditioned":
        monkeypatch.setattr(O, "krylov_directions", lambda dinv, V: V.copy())
    elif mutation == "lucky_never":
        monkeypatch.setattr(O, "is_lucky_breakdown", lambda h, c: False)
    elif mutation == "lucky_absolute":
        monkeypatch.setattr(O, "is_lucky_breakdown", lambda h, c: h <= O.LUCKY_REL)
    elif mutation == "lucky_loose":
        monkeypatch.setattr(O, "is_lucky_breakdown", lambda h, c: h <= 1e-10 * c)
    elif mutation == "extrap_weights_reversed":
        orig_w = O.extrapolation_weights
        monkeypatch.setattr(O, "extrapolation_weights", lambda q: orig_w(q)[::-1])
    elif mutation == "extrap_off_by_one":
        monkeypatch.setattr(O, "extrapolate",
                            lambda h, q: sum(w * h[-2 - j] if len(h) > j + 1 else w * h[0]
                                             for j, w in enumerate(O.extrapolation_weights(min(q, len(h))))))
    elif mutation == "guess_only_projects_krylov":
        monkeypatch.setattr(O, "GUESS_ONLY_METHODS", ())
    elif mutation == "ls_projector_missing":
        monkeypatch.setattr(O, "ls_project", lambda Z, v: v)
    elif mutation == "ls_correction_galerkin":
        monkeypatch.setattr(O, "ls_correction",
                            lambda W, Z, x, r: O.projection_correction(W, Z, W.T @ Z, x, r))
    elif mutation == "ls_coefficients_unnormalised":
        monkeypatch.setattr(O, "ls_coefficients", lambda Z, v: Z.T @ v)
    elif mutation == "ls_deflated_start_unprojected":
        monkeypatch.setattr(O, "PROJECTED_START_METHODS", (O.DEFL_ORTHO,))
    if mutation == "ortho_projector_missing":
        monkeypatch.setattr(O, "orthogonal_project", lambda W, v: v)
    elif mutation == "ortho_projector_half":
        monkeypatch.setattr(O, "orthogonal_project", lambda W, v: v - 0.5 * W @ (W.T @ v))
    elif mutation == "projector_uses_W":
        monkeypatch.setattr(O, "oblique_project", lambda W, Z, E, v: v - W @ np.linalg.solve(E, W.T @ v))
    elif mutation == "guess_transposed_E":
        def bad(W, Z, E, x, r):
            c = np.linalg.solve(E.T, W.T @ r)
            return x + W @ c, r - Z @ c
        monkeypatch.setattr(O, "projection_correction", bad)
    elif mutation == "correction_sign":
        def bad(W, Z, E, x, r):
            c = np.linalg.solve(E, W.T @ r)
            return x - W @ c, r - Z @ c
        monkeypatch.setattr(O, "projection_correction", bad)
    elif mutation == "givens_sign":
        orig = O.givens
        monkeypatch.setattr(O, "givens", lambda a, b: (lambda c, s, r: (c, -s, r))(*orig(a, b)))
    elif mutation == "update_without_preconditioner":
        monkeypatch.setattr(O, "krylov_update", lambda x, dinv, V, y: x + V @ y)
    elif mutation == "operator_perturbed":
        orig_cycle = O.arnoldi_cycle

        def cycle(op, r0, m, stop_abs, max_steps):
            return orig_cycle(lambda v: op(v) + 1e-3 * v, r0, m, stop_abs, max_steps)
        monkeypatch.setattr(O, "arnoldi_cycle", cycle)
    assert not _pins_pass()
