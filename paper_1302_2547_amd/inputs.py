"""Seeded synthetic inputs: graph Laplacians in CSR and right-hand sides.

This module is the one piece shared by the HIP library's callers and by the CPU
oracle's tests: it builds problems, it holds none of the method's arithmetic.
Every array is a deterministic function of its arguments (numpy only).

Problems follow the paper's model problem (Sec. 2): a weighted graph Laplacian
(A u, v) = sum_{(i,j) in E} w_ij (u_i - u_j)(v_i - v_j) + sum_{j in S} w^D_j u_j v_j
with positive weights, stored as CSR with strictly ascending columns and the
diagonal present.

Random numbers come from SplitMix64 used as a counter-based generator:
``u(seed, k) = (splitmix64_k(seed) >> 11) * 2^-53`` in [0, 1).
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k) -> np.ndarray:
    """k-th output (k >= 0, array) of SplitMix64 seeded with ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & (2**64 - 1)) + _GAMMA * (k + np.uint64(1))
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, k) -> np.ndarray:
    """Uniform [0, 1) doubles for counters k (53-bit mantissas)."""
    return (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side with entries uniform in [-1, 1)."""
    return 2.0 * uniform(seed, np.arange(n, dtype=np.uint64)) - 1.0


# ---------------------------------------------------------------------------------------
# Structured grids: 2D 5-point / 3D 7-point finite-difference Laplacians.
# ---------------------------------------------------------------------------------------

def grid_laplacian(dims, jitter: float = 0.0, seed: int = 0, bc: str = "dirichlet"):
    """(2d+1)-point Laplacian on the interior nodes of a tensor grid.

    Unknowns are numbered x fastest: i = x + nx*(y + ny*z).  Each grid edge has
    weight w_e = 1 + jitter*(2u_e - 1), with u_e drawn from a counter equal to
    (index of the edge's lower endpoint on the (n+2)^d grid that includes the
    boundary nodes) * d + (edge direction).  With bc="dirichlet" the edges to
    the eliminated boundary nodes add their weights to the diagonal (the set S of
    the model problem); with bc="neumann" they are dropped (a singular matrix,
    useful for pattern-only experiments).

    Returns (row_ptr int32[n+1], col int32[nnz], val float64[nnz]).
    """
    dims = tuple(int(d) for d in dims)
    d = len(dims)
    if d not in (1, 2, 3) or min(dims) < 1:
        raise ValueError("dims must have 1 to 3 positive sizes")
    n = int(np.prod(dims))
    ext = tuple(s + 2 for s in dims)
    # interior coordinates, x fastest
    coords = np.indices(dims[::-1], dtype=np.int64).reshape(d, -1)[::-1]  # coords[0] = x
    ext_stride = [1] * d
    for a in range(1, d):
        ext_stride[a] = ext_stride[a - 1] * ext[a - 1]
    stride = [1] * d
    for a in range(1, d):
        stride[a] = stride[a - 1] * dims[a - 1]
    ext_index = sum((coords[a] + 1) * ext_stride[a] for a in range(d))

    def weight(lower_ext_index, direction):
        if jitter == 0.0:
            return np.ones(lower_ext_index.shape)
        u = uniform(seed, (lower_ext_index * d + direction).astype(np.uint64))
        return 1.0 + jitter * (2.0 * u - 1.0)

    # weights of the edge in direction a from each node to its +a neighbour (and -a)
    w_plus = [weight(ext_index, a) for a in range(d)]
    w_minus = [weight(ext_index - ext_stride[a], a) for a in range(d)]
    valid_minus = [coords[a] > 0 for a in range(d)]
    valid_plus = [coords[a] < dims[a] - 1 for a in range(d)]
    # slots in ascending column order: -z, -y, -x, diagonal, +x, +y, +z
    slots = [(valid_minus[a], -stride[a], w_minus[a]) for a in reversed(range(d))] + [None] + \
            [(valid_plus[a], stride[a], w_plus[a]) for a in range(d)]
    # diagonal: incident edge weights added in slot order (boundary edges only for Dirichlet)
    diag = np.zeros(n)
    counts = np.ones(n, np.int64)
    for slot in slots:
        if slot is not None:
            m, _, w = slot
            diag += w if bc == "dirichlet" else np.where(m, w, 0.0)
            counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), np.int32)
    val = np.empty(int(row_ptr[-1]), np.float64)
    cursor = row_ptr[:-1].copy()
    ids = np.arange(n, dtype=np.int32)
    for slot in slots:
        if slot is None:
            col[cursor] = ids
            val[cursor] = diag
            cursor += 1
            continue
        m, off, w = slot
        at = cursor[m]
        col[at] = ids[m] + off
        val[at] = -w[m]
        cursor[m] += 1
    return row_ptr.astype(np.int32), col, val


# ---------------------------------------------------------------------------------------
# Random geometric graphs in the unit square.
# ---------------------------------------------------------------------------------------

def rgg_laplacian(npoints: int, mean_degree: float = 8.0, seed: int = 3, weight_range=None,
                  shift: float = 1e-6, chunk: int = 1 << 19):
    """Graph Laplacian of a random geometric graph plus ``shift`` * I.

    Points are uniform in [0,1)^2 (x_k = u(seed, 2k), y_k = u(seed, 2k+1)); an
    edge joins two points closer than r = sqrt(mean_degree / (pi * npoints)).
    Vertices are numbered by cell of a grid of side 1/floor(1/r) (cells row-major
    by (cy, cx)), ties by generation index, which gives mesh-like locality.
    Edge weights are 1, or uniform in ``weight_range`` = (lo, hi) with the counter
    lo_vertex * npoints + hi_vertex (final numbering) on stream seed + 1.

    Returns (row_ptr int32[n+1], col int32[nnz], val float64[nnz]).
    """
    n = int(npoints)
    r = math.sqrt(mean_degree / (math.pi * n))
    m = max(1, int(math.floor(1.0 / r)))
    k = np.arange(n, dtype=np.uint64)
    px = uniform(seed, 2 * k)
    py = uniform(seed, 2 * k + np.uint64(1))
    cx = np.minimum((px * m).astype(np.int64), m - 1)
    cy = np.minimum((py * m).astype(np.int64), m - 1)
    cell = cy * m + cx
    order = np.argsort(cell, kind="stable")
    px, py, cx, cy, cell = px[order], py[order], cx[order], cy[order], cell[order]
    cell_start = np.searchsorted(cell, np.arange(m * m + 1))
    r2 = r * r
    rows, cols = [], []
    offsets = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]  # ascending cell order
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        idx = np.arange(lo, hi)
        starts = np.empty((hi - lo, 9), np.int64)
        lens = np.empty((hi - lo, 9), np.int64)
        for o, (dy, dx) in enumerate(offsets):
            ny_, nx_ = cy[idx] + dy, cx[idx] + dx
            ok = (ny_ >= 0) & (ny_ < m) & (nx_ >= 0) & (nx_ < m)
            c = np.where(ok, ny_ * m + nx_, 0)
            s = cell_start[c]
            e = cell_start[c + 1]
            starts[:, o] = s
            lens[:, o] = np.where(ok, e - s, 0)
        lens_f = lens.ravel()
        total = int(lens_f.sum())
        src = np.repeat(np.repeat(idx, 9), lens_f)
        base = np.repeat(starts.ravel(), lens_f)
        first = np.repeat(np.cumsum(lens_f) - lens_f, lens_f)
        dst = base + (np.arange(total) - first)
        dxs = px[src] - px[dst]
        dys = py[src] - py[dst]
        keep = ((dxs * dxs + dys * dys) < r2) | (src == dst)
        rows.append(src[keep])
        cols.append(dst[keep])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    offd = rows != cols
    lo_v = np.minimum(rows, cols).astype(np.uint64)
    hi_v = np.maximum(rows, cols).astype(np.uint64)
    if weight_range is None:
        w = np.ones(rows.shape[0])
    else:
        a, b = weight_range
        w = a + (b - a) * uniform(seed + 1, lo_v * np.uint64(n) + hi_v)
    val = np.where(offd, -w, 0.0)
    degsum = np.bincount(rows[offd], weights=w[offd], minlength=n)
    val[~offd] = degsum + shift
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32), val


def path_laplacian(n: int):
    """1D path graph Laplacian with Dirichlet ends (tridiagonal 2, -1)."""
    return grid_laplacian((n,))


def csr_to_dense(row_ptr, col, val, n=None):
    n = len(row_ptr) - 1 if n is None else n
    a = np.zeros((n, n))
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    np.add.at(a, (rows, col), val)
    return a


def random_graph_laplacian(n: int, p: float, seed: int, integer_weights: bool = True, shift: float = 1.0):
    """Small Erdos-Renyi graph Laplacian + shift*I (for tests on tiny graphs).

    Edge (i<j) present when u(seed, i*n+j) < p; weight 1..4 (integer) or
    uniform [0.5, 1.5) from stream seed + 1.
    """
    iu, ju = np.triu_indices(n, 1)
    keys = (iu * n + ju).astype(np.uint64)
    present = uniform(seed, keys) < p
    iu, ju, keys = iu[present], ju[present], keys[present]
    if integer_weights:
        w = 1.0 + np.floor(4.0 * uniform(seed + 1, keys))
    else:
        w = 0.5 + uniform(seed + 1, keys)
    a = np.zeros((n, n))
    a[iu, ju] = -w
    a[ju, iu] = -w
    a[np.arange(n), np.arange(n)] = -a.sum(axis=1) + shift
    # the diagonal is kept even where it is zero (isolated vertex, shift 0); nonzero() sorts by row, col
    rows, cols = np.nonzero((a != 0.0) | np.eye(n, dtype=bool))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32), a[rows, cols]
