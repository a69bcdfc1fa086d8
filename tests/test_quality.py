"""||Q||_A^2, the energy norm of the l2 projection onto the coarse space (Sec. 5.1),
computed by oracle.quality: pinned to closed forms, then compared with the values
the paper prints for its aggregations (Tables 5.1, 5.2, 5.3 and 5.6)."""
import numpy as np
import pytest

import oracle
from oracle import quality
from paper_1302_2547_amd import inputs


def dense(rp, ci, va):
    return inputs.csr_to_dense(rp, ci, va)


def one_aggregate_norm(a):
    """Q = 1 1^T / n: Q A Q = (1^T A 1 / n^2) 1 1^T has rank one, so the largest
    eigenvalue of the pencil is (1^T A 1)(1^T A^-1 1) / n^2."""
    n = a.shape[0]
    one = np.ones(n)
    return (one @ a @ one) * (one @ np.linalg.solve(a, one)) / n ** 2


def test_singletons_give_the_identity():
    rp, ci, va = inputs.random_graph_laplacian(80, 0.1, seed=3, integer_weights=False, shift=0.5)
    assert abs(quality.energy_norm_q(rp, ci, va, np.arange(80)) - 1.0) < 1e-10


@pytest.mark.parametrize("n", [50, 700])  # dense and Lanczos paths
def test_one_aggregate_closed_form(n):
    rp, ci, va = inputs.random_graph_laplacian(n, 8.0 / n, seed=5, integer_weights=False, shift=0.3)
    got = quality.energy_norm_q(rp, ci, va, np.zeros(n, np.int64))
    assert abs(got - one_aggregate_norm(dense(rp, ci, va))) < 1e-8 * got


def test_disconnected_blocks_take_the_larger_norm():
    """Two components, one aggregate each: Q is block diagonal and its norm is the
    larger of the two blocks' closed forms."""
    r1, c1, v1 = inputs.random_graph_laplacian(40, 0.2, seed=1, integer_weights=False, shift=0.2)
    r2, c2, v2 = inputs.random_graph_laplacian(30, 0.2, seed=2, integer_weights=False, shift=2.0)
    rp = np.concatenate([r1, r2[1:] + r1[-1]]).astype(np.int32)
    ci = np.concatenate([c1, c2 + 40]).astype(np.int32)
    va = np.concatenate([v1, v2])
    agg = np.concatenate([np.zeros(40, np.int64), np.ones(30, np.int64)])
    expect = max(one_aggregate_norm(dense(r1, c1, v1)), one_aggregate_norm(dense(r2, c2, v2)))
    assert abs(quality.energy_norm_q(rp, ci, va, agg) - expect) < 1e-9 * expect


def test_neumann_constants_give_zero():
    """A graph Laplacian with one aggregate: Q maps onto the constants, the null
    space, so the seminorm vanishes."""
    rp, ci, va = inputs.grid_laplacian((12, 11), bc="neumann")
    assert abs(quality.energy_norm_q(rp, ci, va, np.zeros(132, np.int64), singular=True)) < 1e-8


def test_lanczos_path_matches_a_dense_pencil():
    rp, ci, va = inputs.grid_laplacian((25, 24), jitter=0.3, seed=4)
    agg, nc = quality.aggregate(rp, ci, cap=4)
    a = dense(rp, ci, va)
    q = quality.projection(agg).toarray()
    import scipy.linalg as la
    expect = la.eigh(q @ a @ q, a, eigvals_only=True)[-1]
    assert abs(quality.energy_norm_q(rp, ci, va, agg) - expect) < 1e-8 * expect


def test_tables_5_1_and_5_2_at_128(golden):
    """Level-0 aggregates of the 128^2 grid do not depend on the random part of
    eq. (3.2) (128 mod 12 = 8), so the printed norms are reproduced digit for digit."""
    rows = [r for r in golden("table_5_1_5_2_energy_norms.txt") if r[1] == 128]
    rpd, cid, vad = inputs.grid_laplacian((128, 128))
    rpn, cin, van = inputs.grid_laplacian((128, 128), bc="neumann")
    for bc, n, t, paper in rows:
        agg, _ = quality.aggregate(rpd, cid, cap=t)
        mat = (rpn, cin, van) if bc else (rpd, cid, vad)
        got = quality.energy_norm_q(*mat, agg, singular=bool(bc))
        assert round(got, 2) == paper, (bc, t, got, paper)


def test_table_5_3_seed_independent_rows(golden):
    """Rows n = 126..130 with the Dirichlet matrix (see the fixture's note); the
    n = 128, t = 4 entry prints 2.47 where Table 5.1 prints 2.46 for the same case."""
    for n in (126, 127, 129, 130):
        rp, ci, va = inputs.grid_laplacian((n, n))
        for _, t, paper in [r for r in golden("table_5_3_energy_norms.txt") if r[0] == n]:
            agg, _ = quality.aggregate(rp, ci, cap=t)
            got = quality.energy_norm_q(rp, ci, va, agg)
            assert round(got, 2) == paper, (n, t, got, paper)


def test_table_5_6_multilevel_norms(golden):
    """Norms between any two levels of the t = 5 hierarchy of 128^2.  The entries
    that involve only levels 0-2 are reproduced to the printed digits (the Neumann
    0-1 entry prints 3.23 where Table 5.2 prints 3.24); deeper levels depend on
    the random part of eq. (3.2) (their coarsening ratios differ from the paper's
    by up to 6 %), and their norms are within 15 %."""
    rpd, cid, vad = inputs.grid_laplacian((128, 128))
    rpn, cin, van = inputs.grid_laplacian((128, 128), bc="neumann")
    h = oracle.Hierarchy(rpd, cid, vad, max_aggregate=5, coarsest_size=100)
    assert h.num_levels == 6
    aggs = [h.level(l).agg for l in range(5)]
    mats = {0: [(rpd, cid, vad)] + [(h.level(l).row_ptr, h.level(l).col, h.level(l).val) for l in range(1, 6)],
            1: [(rpn, cin, van)]}
    for l in range(5):
        mats[1].append(oracle.coarse_operator(*mats[1][-1], aggs[l], h.level(l + 1).n)[:3])
    for bc, i, j, paper in golden("table_5_6_energy_norms.txt"):
        got = quality.energy_norm_q(*mats[bc][i], quality.compose(aggs[i:j]), singular=bool(bc))
        if j <= 2:
            assert abs(got - paper) <= 0.011, (bc, i, j, got, paper)
        else:
            assert abs(got - paper) <= 0.15 * paper, (bc, i, j, got, paper)
