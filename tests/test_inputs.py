"""Seeded input generators: structure of the synthetic workloads (CPU only)."""
import numpy as np

from paper_1302_2547_amd import inputs


def test_grid_laplacian_structure_3d_jitter():
    n = 12
    rp, ci, va = inputs.grid_laplacian((n, n, n), jitter=0.1, seed=2)
    assert rp[-1] == 7 * n**3 - 6 * n**2                            # 7-point stencil, Dirichlet interior
    a = inputs.csr_to_dense(rp, ci, va)
    np.testing.assert_array_equal(a, a.T)                           # symmetric
    off = -a[~np.eye(n**3, dtype=bool)]
    w = off[off != 0]
    assert w.min() >= 0.9 and w.max() <= 1.1 and w.std() > 0.03     # 1 + 0.1 U[-1, 1]
    # diagonal = sum of all 6 incident edge weights (boundary edges eliminated)
    rowsum = a.sum(axis=1)
    interior = np.nonzero(np.diff(rp) == 7)[0]
    boundary = np.nonzero(np.diff(rp) < 7)[0]
    assert (rowsum[boundary] > 0.8).all()
    np.testing.assert_allclose(rowsum[interior], 0.0, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(a) > 0)                        # SPD
    for i in range(n**3):                                           # strictly ascending, diagonal present
        c = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    rp2, ci2, va2 = inputs.grid_laplacian((n, n, n), jitter=0.1, seed=2)
    assert np.array_equal(va, va2)                                  # deterministic
    assert not np.array_equal(va, inputs.grid_laplacian((n, n, n), jitter=0.1, seed=3)[2])


def test_grid_laplacian_2d_unit_and_neumann():
    rp, ci, va = inputs.grid_laplacian((64, 64))
    assert len(rp) - 1 == 4096 and rp[-1] == 20224                  # the 64x64 workload
    assert set(np.unique(va)) == {-1.0, 4.0}
    rp, ci, va = inputs.grid_laplacian((5, 4), bc="neumann")
    np.testing.assert_allclose(inputs.csr_to_dense(rp, ci, va).sum(axis=1), 0.0)


def test_rgg_laplacian():
    n = 20000
    rp, ci, va = inputs.rgg_laplacian(n, mean_degree=8.0, seed=3, weight_range=(0.5, 1.5), shift=1e-6)
    deg = np.diff(rp) - 1
    assert abs(deg.mean() - 8.0) < 0.4                              # boundary effect lowers it a little
    rows = np.repeat(np.arange(n), np.diff(rp))
    offd = rows != ci
    w = -va[offd]
    assert w.min() >= 0.5 and w.max() < 1.5
    # symmetric: (i, j, w) pairs match (j, i, w)
    key = rows[offd].astype(np.int64) * n + ci[offd]
    tkey = ci[offd].astype(np.int64) * n + rows[offd]
    o1, o2 = np.argsort(key), np.argsort(tkey)
    np.testing.assert_array_equal(key[o1], tkey[o2])
    np.testing.assert_array_equal(w[o1], w[o2])
    diag = va[~offd]
    np.testing.assert_allclose(diag, np.bincount(rows[offd], weights=w, minlength=n) + 1e-6)
    for i in range(0, n, 997):
        c = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    assert (deg == 0).sum() > 0                                     # isolated vertices exist (~n e^-8)


def test_rhs_range_and_determinism():
    b = inputs.rhs(100000, 7)
    assert b.min() >= -1 and b.max() < 1 and abs(b.mean()) < 0.02
    assert np.array_equal(b, inputs.rhs(100000, 7))
