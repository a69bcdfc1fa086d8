"""Pins of the oracle's solve phase (CPU only): l1-Jacobi, K-cycle, outer flexible CG.

Independent references: dense linear algebra (numpy), a textbook CG written here,
the two-grid error operator written as a matrix product, and the limit of the
K-cycle when its inner Krylov iteration is run to convergence.
"""
import numpy as np
import pytest

import oracle
from paper_1302_2547_amd import inputs


def dense(rp, ci, va):
    return inputs.csr_to_dense(rp, ci, va)


def prolongation(agg, nc):
    p = np.zeros((len(agg), nc))
    p[np.arange(len(agg)), agg] = 1.0
    return p


def kcycle_matrix(h, n):
    return np.column_stack([h.kcycle(e) for e in np.eye(n)])


def two_grid_matrix(a, minv, p, ac_inv):
    """Preconditioner of Alg. 1's cycle on two levels, as a matrix:
    x1 = M^-1 r;  x2 = x1 + P Ac^-1 P^T (r - A x1);  x3 = x2 + M^-1 (r - A x2)."""
    n = a.shape[0]
    m = np.diag(minv)
    x2 = m + p @ ac_inv @ p.T @ (np.eye(n) - a @ m)
    return x2 + m @ (np.eye(n) - a @ x2)


def test_smoother_is_convergent_on_spd():
    """l1-Jacobi (Sec. 4.1): rho(I - M^-1 A) < 1 for SPD A."""
    for dims, jit in (((10, 10), 0.0), ((6, 5, 4), 0.5)):
        rp, ci, va = inputs.grid_laplacian(dims, jitter=jit, seed=3)
        a = dense(rp, ci, va)
        minv = oracle.l1_inverse_diagonal(rp, ci, va)
        rho = max(abs(np.linalg.eigvals(np.eye(len(minv)) - np.diag(minv) @ a)))
        assert rho < 1.0


def test_two_level_kcycle_is_the_symmetric_two_grid_operator():
    rp, ci, va = inputs.grid_laplacian((12, 12), jitter=0.2, seed=5)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=100)
    assert h.num_levels == 2
    l0, l1 = h.level(0), h.level(1)
    a = dense(rp, ci, va)
    p = prolongation(l0.agg, l1.n)
    b = kcycle_matrix(h, l0.n)
    expect = two_grid_matrix(a, l0.minv, p, np.linalg.inv(p.T @ a @ p))
    np.testing.assert_allclose(b, expect, rtol=0, atol=1e-12 * np.abs(expect).max())
    np.testing.assert_allclose(b, b.T, atol=1e-12 * np.abs(b).max())   # symmetric smoother pair
    rho = max(abs(np.linalg.eigvals(np.eye(l0.n) - b @ a)))
    assert rho < 1.0


def test_kcycle_with_converged_inner_krylov_tends_to_two_grid():
    """With many inner flexible-CG steps the coarse equation is solved to high
    accuracy, so the K-cycle approaches the exact two-grid preconditioner."""
    rp, ci, va = inputs.grid_laplacian((16, 16), jitter=0.2, seed=6)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=8, kcycle_inner=60)
    assert h.num_levels >= 3
    l0, l1 = h.level(0), h.level(1)
    a = dense(rp, ci, va)
    p = prolongation(l0.agg, l1.n)
    two = two_grid_matrix(a, l0.minv, p, np.linalg.inv(p.T @ a @ p))
    r = inputs.rhs(l0.n, 9)
    np.testing.assert_allclose(h.kcycle(r), two @ r, rtol=1e-8, atol=1e-10)
    # with nu = 1 or 2 it is a different (nonlinear, inexact) cycle
    h2 = oracle.Hierarchy(rp, ci, va, coarsest_size=8, kcycle_inner=2)
    assert np.abs(h2.kcycle(r) - two @ r).max() > 1e-6


def textbook_cg(a, b, iters):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    hist = [np.linalg.norm(r) / np.linalg.norm(b)]
    for _ in range(iters):
        q = a @ p
        alpha = (r @ r) / (p @ q)
        x += alpha * p
        rn = r - alpha * q
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
        hist.append(np.linalg.norm(r) / np.linalg.norm(b))
    return x, np.array(hist)


def test_flexible_cg_with_identity_is_textbook_cg():
    rp, ci, va = inputs.grid_laplacian((9, 8), jitter=0.3, seed=2)
    h = oracle.Hierarchy(rp, ci, va)
    b = inputs.rhs(len(rp) - 1, 4)
    x, st, it, rel, _, hist = h.solve(b, tol=1e-300, max_iters=8, precond=False, history=True)
    assert it == 8
    x_ref, hist_ref = textbook_cg(dense(rp, ci, va), b, 8)
    np.testing.assert_allclose(hist, hist_ref, rtol=1e-9)
    np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-12)


def test_two_level_fcg_equals_pcg_with_the_fixed_preconditioner():
    """On two levels the K-cycle is a fixed SPD matrix B, and flexible CG with a
    fixed SPD preconditioner produces the PCG iterates."""
    rp, ci, va = inputs.grid_laplacian((11, 10), jitter=0.2, seed=8)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=100)
    assert h.num_levels == 2
    a = dense(rp, ci, va)
    bmat = kcycle_matrix(h, a.shape[0])
    b = inputs.rhs(a.shape[0], 3)
    x, st, it, rel, _, hist = h.solve(b, tol=1e-300, max_iters=6, history=True)
    # PCG (textbook form)
    xr = np.zeros_like(b); r = b.copy(); z = bmat @ r; p = z.copy(); ref = [1.0]
    for _ in range(6):
        q = a @ p
        alpha = (r @ z) / (p @ q)
        xr += alpha * p
        rn = r - alpha * q
        zn = bmat @ rn
        p = zn + (rn @ zn) / (r @ z) * p
        r, z = rn, zn
        ref.append(np.linalg.norm(r) / np.linalg.norm(b))
    np.testing.assert_allclose(hist, ref, rtol=1e-7)
    np.testing.assert_allclose(x, xr, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("case", range(5))
def test_solve_reaches_direct_solution(case):
    if case < 3:
        rp, ci, va = inputs.random_graph_laplacian(60 + 40 * case, p=0.08, seed=case, integer_weights=False,
                                                   shift=1e-3)
    elif case == 3:
        rp, ci, va = inputs.grid_laplacian((20, 20), jitter=0.1, seed=1)
    else:
        rp, ci, va = inputs.grid_laplacian((8, 7, 6), jitter=0.1, seed=1)
    a = dense(rp, ci, va)
    b = inputs.rhs(a.shape[0], 10 + case)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=10)
    assert h.num_levels >= 2
    x, st, it, rel, _ = h.solve(b, tol=1e-12, max_iters=300)
    assert st == oracle.OK
    x_ref = np.linalg.solve(a, b)
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())
    assert rel <= 1e-12
    assert abs(rel - np.linalg.norm(b - a @ x) / np.linalg.norm(b)) < 1e-13


def test_iteration_count_uniform_in_problem_size():
    """Sec. 5.2: the K-cycle method converges uniformly with respect to the size."""
    its = []
    for n in (32, 64, 128):
        rp, ci, va = inputs.grid_laplacian((n, n))
        h = oracle.Hierarchy(rp, ci, va)
        _, st, it, rel, _ = h.solve(inputs.rhs(n * n, 1), tol=1e-8)
        assert st == oracle.OK and rel <= 1e-8
        its.append(it)
    assert max(its) - min(its) <= 3 and max(its) <= 30, its


def test_not_converged_and_single_level():
    rp, ci, va = inputs.grid_laplacian((16, 16))
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=10)
    b = inputs.rhs(256, 1)
    _, st, it, rel, _ = h.solve(b, tol=1e-12, max_iters=1)
    assert st == oracle.ERR_NOT_CONVERGED and it == 1 and rel > 1e-12
    # one level: the coarsest (direct) solve is the whole preconditioner
    h1 = oracle.Hierarchy(rp, ci, va, coarsest_size=1000)
    assert h1.num_levels == 1
    x, st, it, rel, _ = h1.solve(b, tol=1e-10)
    assert st == oracle.OK and it == 1
    # b = 0 gives x = 0 in zero iterations
    x, st, it, rel, _ = h.solve(np.zeros(256))
    assert st == oracle.OK and it == 0 and not x.any()


def test_indefinite_input_is_detected():
    """A positive diagonal does not make A SPD; the method must not return a
    'converged' answer for an indefinite matrix: either the coarsest Cholesky
    or a Krylov step (p^T A p <= 0) reports the breakdown."""
    rp, ci, va = inputs.grid_laplacian((10, 10))
    va = va.copy()
    diag = ci == np.repeat(np.arange(100), np.diff(rp))
    va[diag] -= 1.0                                                # L - I: indefinite, diagonal 2..3
    with pytest.raises(RuntimeError, match="status 6"):
        oracle.Hierarchy(rp, ci, va, coarsest_size=1000)           # coarsest Cholesky fails
    try:
        h = oracle.Hierarchy(rp, ci, va, coarsest_size=4)
    except RuntimeError as e:
        assert "status 6" in str(e)
        return
    _, st, _, _, _ = h.solve(inputs.rhs(100, 2), tol=1e-10)
    assert st == oracle.ERR_BREAKDOWN


# --- exact pins of the inner flexible-CG steps of the K-cycle (Sec. 4.3) -------------------
#
# Two flexible-CG steps from zero on A_c e = g, the second direction A_c-orthogonalised
# against the first (truncation 1), leave e equal to the A_c-Galerkin solution on the
# span of the two preconditioned vectors: e = V (V^T A_c V)^-1 V^T g with V = [c1, c2],
# c1 = B g and c2 = B (g - alpha A_c c1), alpha = (c1, g) / (c1, A_c c1).  The
# references below use that characterisation (a 2 x 2 dense solve) instead of the
# CG recurrences, so a wrong or missing orthogonalisation, a sign error in the inner
# residual or a wrong step length changes the result.

def dense_hierarchy(h):
    levels = [h.level(l) for l in range(h.num_levels)]
    mats = [dense(L.row_ptr, L.col, L.val) for L in levels]
    prols = [prolongation(L.agg, levels[l + 1].n) for l, L in enumerate(levels[:-1])]
    return levels, mats, prols


def kcycle_galerkin(levels, mats, prols, k, r, nu):
    """K-cycle on level k written with the Galerkin characterisation of its inner steps."""
    a, m = mats[k], levels[k].minv
    last = len(levels) - 1
    if k == last:
        return np.linalg.solve(a, r)
    p = prols[k]
    x = m * r
    g = p.T @ (r - a @ x)
    ac = mats[k + 1]
    if k + 1 == last:
        e = np.linalg.solve(ac, g)
    else:
        c1 = kcycle_galerkin(levels, mats, prols, k + 1, g, nu)
        if nu == 1:
            e = (c1 @ g) / (c1 @ ac @ c1) * c1
        else:
            alpha = (c1 @ g) / (c1 @ ac @ c1)
            c2 = kcycle_galerkin(levels, mats, prols, k + 1, g - alpha * (ac @ c1), nu)
            v = np.column_stack([c1, c2])
            e = v @ np.linalg.solve(v.T @ ac @ v, v.T @ g)
    x = x + p @ e
    return x + m * (r - a @ x)


def test_three_level_nu2_kcycle_is_galerkin_on_the_krylov_pair():
    """Three levels: K(1, .) is the fixed two-grid matrix B1, so the two inner steps
    give the A1-Galerkin solution on span{B1 g, B1 A1 B1 g} (a Krylov space)."""
    rp, ci, va = inputs.grid_laplacian((12, 12), jitter=0.2, seed=5)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=20, kcycle_inner=2)
    assert h.num_levels == 3
    levels, (a0, a1, a2), (p0, p1) = dense_hierarchy(h)
    b1 = two_grid_matrix(a1, levels[1].minv, p1, np.linalg.inv(a2))
    m0 = np.diag(levels[0].minv)
    for seed in (3, 4):
        r = inputs.rhs(levels[0].n, seed)
        x1 = m0 @ r
        g = p0.T @ (r - a0 @ x1)
        v = np.column_stack([b1 @ g, b1 @ a1 @ b1 @ g])
        e = v @ np.linalg.solve(v.T @ a1 @ v, v.T @ g)
        x2 = x1 + p0 @ e
        expect = x2 + m0 @ (r - a0 @ x2)
        got = h.kcycle(r)
        np.testing.assert_allclose(got, expect, rtol=0, atol=1e-12 * np.abs(expect).max())
        # one inner step only would be a different vector
        e1 = (v[:, 0] @ g) / (v[:, 0] @ a1 @ v[:, 0]) * v[:, 0]
        x2b = x1 + p0 @ e1
        assert np.abs(x2b + m0 @ (r - a0 @ x2b) - expect).max() > 1e-6 * np.abs(expect).max()


@pytest.mark.parametrize("dims,coarsest,nu", [((10, 9, 8), 10, 2), ((20, 20), 4, 2), ((20, 20), 4, 1),
                                              ((16, 16), 8, 2)])
def test_deep_kcycle_matches_the_galerkin_recursion(dims, coarsest, nu):
    """Four to six levels: the oracle's K-cycle equals the recursion whose inner
    steps are Galerkin solutions on the span of the recursive directions."""
    rp, ci, va = inputs.grid_laplacian(dims, jitter=0.2, seed=5)
    h = oracle.Hierarchy(rp, ci, va, coarsest_size=coarsest, kcycle_inner=nu)
    assert h.num_levels >= 4
    levels, mats, prols = dense_hierarchy(h)
    for seed in (1, 2):
        r = inputs.rhs(levels[0].n, seed)
        expect = kcycle_galerkin(levels, mats, prols, 0, r, nu)
        np.testing.assert_allclose(h.kcycle(r), expect, rtol=0, atol=1e-12 * np.abs(expect).max())


def kcycle_galerkin_threshold(levels, mats, prols, k, r, theta, skips):
    """As kcycle_galerkin with nu = 2, except that the second inner direction is
    dropped when the inner residual after the first step satisfies
    ||g - alpha A c1|| < theta ||g||; skips counts those visits."""
    a, m = mats[k], levels[k].minv
    last = len(levels) - 1
    p = prols[k]
    x = m * r
    g = p.T @ (r - a @ x)
    ac = mats[k + 1]
    if k + 1 == last:
        e = np.linalg.solve(ac, g)
    else:
        c1 = kcycle_galerkin_threshold(levels, mats, prols, k + 1, g, theta, skips)
        alpha = (c1 @ g) / (c1 @ ac @ c1)
        rt = g - alpha * (ac @ c1)
        if rt @ rt < theta * theta * (g @ g):
            skips[0] += 1
            e = alpha * c1
        else:
            c2 = kcycle_galerkin_threshold(levels, mats, prols, k + 1, rt, theta, skips)
            v = np.column_stack([c1, c2])
            e = v @ np.linalg.solve(v.T @ ac @ v, v.T @ g)
    x = x + p @ e
    return x + m * (r - a @ x)


def test_kcycle_threshold_readings():
    """K-cycle threshold theta (Sec. 4.3's cycle, in the form that tests whether a
    second inner step pays): theta = 0 is the default cycle bit for bit; a huge theta
    always stops after one step, i.e. nu = 1 bit for bit; in between the oracle takes
    the second step exactly where the Galerkin recursion with the same test does."""
    rp, ci, va = inputs.grid_laplacian((10, 9, 8), jitter=0.2, seed=5)
    r = inputs.rhs(len(rp) - 1, 3)
    base = oracle.Hierarchy(rp, ci, va, coarsest_size=10).kcycle(r)
    zero = oracle.Hierarchy(rp, ci, va, coarsest_size=10, kcycle_threshold=0.0).kcycle(r)
    assert np.array_equal(base, zero)
    one = oracle.Hierarchy(rp, ci, va, coarsest_size=10, kcycle_inner=1).kcycle(r)
    huge = oracle.Hierarchy(rp, ci, va, coarsest_size=10, kcycle_threshold=1e300).kcycle(r)
    assert np.array_equal(one, huge)
    levels, mats, prols = dense_hierarchy(oracle.Hierarchy(rp, ci, va, coarsest_size=10))
    assert [L.n for L in levels] == [720, 284, 56, 15, 4]   # inner pairs on levels 1-3: at most 7 tests
    for theta in (0.1, 0.3, 0.7):
        h = oracle.Hierarchy(rp, ci, va, coarsest_size=10, kcycle_threshold=theta)
        skips = [0]
        expect = kcycle_galerkin_threshold(levels, mats, prols, 0, r, theta, skips)
        np.testing.assert_allclose(h.kcycle(r), expect, rtol=0, atol=1e-12 * np.abs(expect).max())
        assert 0 < skips[0] < 7   # both branches of the test are taken


def test_kcycle_threshold_is_validated():
    rp, ci, va = inputs.grid_laplacian((8, 8))
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(RuntimeError, match="status 1"):
            oracle.Hierarchy(rp, ci, va, kcycle_threshold=bad)
