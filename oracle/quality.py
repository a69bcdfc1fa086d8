"""Energy norm of the l2 projection onto a piecewise-constant coarse space (Sec. 5.1).

TEST INFRASTRUCTURE, like the rest of ``oracle``: a slow, plain reference used by
the test suite to compare the aggregations of the library with the quality
figures the paper prints (Tables 5.1-5.3 and 5.6).

For a partition of the vertices into aggregates, P is the piecewise-constant
prolongation (one column per aggregate) and Q = P (P^T P)^-1 P^T the l2
projection onto its range; (Q v)_i is the mean of v over the aggregate of i.
The paper measures the quality of an aggregation by ||Q||_A^2, the square of
the norm of Q in the energy (semi-)norm |v|_A = (A v, v)^1/2:

    ||Q||_A^2 = max_v (A Q v, Q v) / (A v, v),

the largest eigenvalue of the pencil (Q A Q, A).  For a singular A whose null
space is the constants (Neumann problems, graph Laplacians) Q maps constants to
constants, so the quotient is taken on the complement of the constants; a
shift eps I of the right-hand matrix removes the constant vector (its quotient
becomes 0) and changes every other quotient by a relative O(eps / lambda_min).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def aggregate(rp, ci, cap=0, seed=0x5EED5EED, level=0):
    """One aggregation of the oracle (eq. (3.2) priorities, Alg. 2 with size limit
    cap, ascending numbering) without building the rest of a hierarchy; returns
    (agg, number of aggregates)."""
    from . import number, paa, priorities
    owner, _, _ = paa(rp, ci, priorities(rp, ci, seed, level), cap)
    return number(owner)


def compose(aggs):
    """Aggregate index on the last level of every vertex of the first, for the
    aggregation maps of consecutive levels (agg[l][vertex of level l] = vertex of
    level l + 1)."""
    out = np.asarray(aggs[0], dtype=np.int64)
    for a in aggs[1:]:
        out = np.asarray(a, dtype=np.int64)[out]
    return out


def projection(agg, nc=None):
    """Q = P (P^T P)^-1 P^T as a sparse matrix, for the partition agg."""
    agg = np.asarray(agg, dtype=np.int64)
    n = len(agg)
    nc = int(agg.max()) + 1 if nc is None else nc
    p = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))
    sizes = np.bincount(agg, minlength=nc).astype(float)
    return (p @ sp.diags(1.0 / sizes) @ p.T).tocsr()


def energy_norm_q(rp, ci, va, agg, singular=False, tol=1e-10):
    """||Q||_A^2 of the partition agg (seminorm on the complement of the
    constants when singular)."""
    n = len(rp) - 1
    a = sp.csr_matrix((np.asarray(va, float), np.asarray(ci), np.asarray(rp)), shape=(n, n))
    q = projection(agg)
    qaq = (q @ a @ q).tocsc()
    b = a.tocsc()
    if singular:
        eps = 1e-10 * abs(a.diagonal()).max()
        b = (b + eps * sp.identity(n, format="csc")).tocsc()
    if n <= 400:  # small: dense generalized eigenproblem
        import scipy.linalg as la
        return float(la.eigh(qaq.toarray(), b.toarray(), eigvals_only=True)[-1])
    lu = sla.splu(b)
    minv = sla.LinearOperator((n, n), matvec=lu.solve, dtype=float)
    v0 = np.cos(np.arange(n) * 0.37) + 1.5  # deterministic start vector
    lam = sla.eigsh(qaq, k=1, M=b, Minv=minv, which="LA", tol=tol, v0=v0, return_eigenvectors=False)
    return float(lam[0])
