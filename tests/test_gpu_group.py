"""GPU: grouped solves (amg_solve_group / amg_kcycle_group) against the oracle.

One launch carries jobs on different hierarchies (grids, random graphs, a hub row,
the K-cycle variants: threshold, one inner step, damped Jacobi, level skipping, a
single coarse unknown, and a finest level of more than 100k rows); each job's
K-cycle must match the oracle's
element by element and each solve must reach the tolerance with the oracle's
iteration count (+-1).  A job gives the same bits alone and in any group.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1302_2547_amd import inputs  # noqa: E402
from test_gpu_parity import hub_graph  # noqa: E402  (row 0 holds n entries)


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_2547_amd import amg as mod
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "grid2d_64": (lambda: inputs.grid_laplacian((64, 64)), {}),
    "grid2d_77x50_jitter": (lambda: inputs.grid_laplacian((77, 50), jitter=0.3, seed=5), {}),
    "grid3d_24_jitter": (lambda: inputs.grid_laplacian((24, 24, 24), jitter=0.1, seed=2), {}),
    "grid3d_31x17x9": (lambda: inputs.grid_laplacian((31, 17, 9), jitter=0.1, seed=7), {}),
    "rgg_20k": (lambda: inputs.rgg_laplacian(20000, seed=3, weight_range=(0.5, 1.5)), {}),
    "random_int_300": (lambda: inputs.random_graph_laplacian(300, 0.02, seed=4, integer_weights=True, shift=1.0),
                       {}),
    "hub_6000": (hub_graph, {}),
    "grid3d_24_theta": (lambda: inputs.grid_laplacian((24, 24, 24), jitter=0.1, seed=2), {"kcycle_threshold": 0.25}),
    "grid2d_64_nu1": (lambda: inputs.grid_laplacian((64, 64)), {"kcycle_inner": 1}),
    "grid3d_24_jacobi": (lambda: inputs.grid_laplacian((24, 24, 24), jitter=0.1, seed=2),
                         {"smoother": 1, "jacobi_weight": 0.7}),
    "grid3d_31x17x9_skip": (lambda: inputs.grid_laplacian((31, 17, 9), jitter=0.1, seed=7), {"skip_ratio": 2.0}),
    "grid2d_64_single": (lambda: inputs.grid_laplacian((64, 64)), {"coarsest_size": 1}),
    "grid2d_256": (lambda: inputs.grid_laplacian((256, 256), jitter=0.1, seed=11), {}),
    "grid3d_40": (lambda: inputs.grid_laplacian((40, 40, 40), jitter=0.1, seed=12), {}),
    # a finest level of more than 100k rows: it also holds a sliced copy, and its
    # entries have no per-entry coarse index (the group path reads the CSR arrays)
    "grid3d_50": (lambda: inputs.grid_laplacian((50, 50, 50), jitter=0.1, seed=13), {}),
}

ORACLE_KEYS = ("coarsest_size", "kcycle_inner", "kcycle_threshold", "skip_ratio", "jacobi_weight")


@pytest.fixture(scope="module")
def problems(amg):
    out = {}
    for name, (make, opt) in CASES.items():
        rp, ci, va = make()
        print(f"[group] {name}: n={len(rp) - 1} nnz={len(ci)} opt={opt}", flush=True)
        h = amg.Hierarchy(dev(rp), dev(ci), dev(va), max_rhs=4, **opt)
        oopt = {k: v for k, v in opt.items() if k in ORACLE_KEYS}
        if opt.get("smoother") == 1:
            oopt["smoother"] = "jacobi"
        ref = oracle.Hierarchy(rp, ci, va, **oopt)
        assert h.num_levels == ref.num_levels >= 2
        out[name] = (rp, ci, va, h, ref)
    yield out
    for rp, ci, va, h, ref in out.values():
        h.close()
        ref.close()


def test_kcycle_group_matches_oracle(amg, problems):
    """One launch applies every hierarchy's K-cycle; each equals the oracle's
    K-cycle element by element."""
    jobs, want = [], []
    for k, (name, (rp, ci, va, h, ref)) in enumerate(problems.items()):
        r = inputs.rhs(len(rp) - 1, 40 + k)
        z = torch.full((len(r),), np.nan, dtype=torch.float64, device="cuda")
        jobs.append((h, 0, dev(r), z))
        want.append((name, ref.kcycle(r)))
    status = amg.kcycle_group(jobs)
    assert status == [amg.AMG_OK] * len(jobs)
    for (name, zo), (_, _, _, z) in zip(want, jobs):
        np.testing.assert_allclose(z.cpu().numpy(), zo, rtol=0, atol=1e-10 * np.abs(zo).max(), err_msg=name)


def test_solve_group_matches_oracle(amg, problems):
    """One launch solves every problem to 1e-10: true residual within the tolerance
    and the oracle's iteration count +-1."""
    jobs, meta = [], []
    for k, (name, (rp, ci, va, h, ref)) in enumerate(problems.items()):
        b = inputs.rhs(len(rp) - 1, 60 + k)
        jobs.append((h, 1, dev(b), torch.zeros(len(b), dtype=torch.float64, device="cuda")))
        meta.append((name, rp, ci, va, ref, b))
    st, status, infos = amg.solve_group(jobs, tol=1e-10)
    assert st == amg.AMG_OK and status == [amg.AMG_OK] * len(jobs)
    for (name, rp, ci, va, ref, b), (_, _, _, x), info in zip(meta, jobs, infos):
        xo, st_o, it_o, rel_o, _ = ref.solve(b, tol=1e-10)
        xg = x.cpu().numpy()
        rel = np.linalg.norm(b - oracle.spmv(rp, ci, va, xg)) / np.linalg.norm(b)
        print(f"[group] {name}: {info.iterations} iterations (oracle {it_o}), true rel {rel:.2e}, "
              f"reported {info.rel_residual:.2e}", flush=True)
        assert rel <= 1e-10, name
        # the residual near 1e-10 ||b|| is a difference of terms of size |A||x| (large
        # where the diagonal shift is small): two summation orders agree to a few %
        assert abs(info.rel_residual - rel) <= 0.05 * rel, name
        assert abs(info.iterations - it_o) <= 1, name
    print(f"[group] {len(jobs)} solves in one launch: {infos[0].solve_ms:.1f} ms", flush=True)


def test_group_alone_equals_in_mix(amg, problems):
    """A job's solution and iteration count are the same bits alone, in a group,
    and at another place in the group."""
    names = list(problems)
    rhs = {name: inputs.rhs(problems[name][3].n, 80 + k) for k, name in enumerate(names)}

    def run(order):
        jobs = [(problems[n][3], 2, dev(rhs[n]), torch.zeros(problems[n][3].n, dtype=torch.float64, device="cuda"))
                for n in order]
        st, status, infos = amg.solve_group(jobs, tol=1e-8)
        assert st == amg.AMG_OK
        return {n: (j[3].cpu().numpy(), i.iterations) for n, j, i in zip(order, jobs, infos)}

    mix = run(names)
    rev = run(names[::-1])
    for name in ("grid3d_24_jitter", "rgg_20k", "hub_6000"):
        alone = run([name])[name]
        for other in (mix[name], rev[name]):
            assert alone[1] == other[1], name
            np.testing.assert_array_equal(alone[0], other[0], err_msg=name)


def test_columns_of_one_hierarchy(amg, problems):
    """Several right-hand sides of one hierarchy in one launch (distinct columns):
    each equals its job alone bit for bit and agrees with amg_solve."""
    rp, ci, va, h, ref = problems["grid3d_24_jitter"]
    n = h.n
    B = [inputs.rhs(n, 100 + c) for c in range(4)]
    jobs = [(h, c, dev(B[c]), torch.zeros(n, dtype=torch.float64, device="cuda")) for c in range(4)]
    st, status, infos = amg.solve_group(jobs, tol=1e-9)
    assert st == amg.AMG_OK
    for c in range(4):
        x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        st1, _, inf1 = amg.solve_group([(h, 3 - c, dev(B[c]), x1)], tol=1e-9)
        assert st1 == amg.AMG_OK and inf1[0].iterations == infos[c].iterations
        np.testing.assert_array_equal(x1.cpu().numpy(), jobs[c][3].cpu().numpy())
        xs = torch.zeros(n, dtype=torch.float64, device="cuda")
        _, info = h.solve(dev(B[c]), xs, tol=1e-9)
        assert abs(info.iterations - infos[c].iterations) <= 1
        xg, xr = jobs[c][3].cpu().numpy(), xs.cpu().numpy()
        assert np.linalg.norm(xg - xr) <= 1e-6 * np.linalg.norm(xr)


def test_group_edge_cases(amg, problems):
    rp, ci, va, h, ref = problems["grid2d_64"]
    n = h.n
    b = inputs.rhs(n, 7)
    # zero right-hand side: x = 0 at once; an exact start: no iteration
    x0 = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    xs = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, _, info = amg.solve_group([(h, 0, torch.zeros(n, dtype=torch.float64, device="cuda"), x0)], tol=1e-8)
    assert st == amg.AMG_OK and info[0].iterations == 0 and float(x0.abs().max()) == 0.0
    st, _ = h.solve(dev(b), xs, tol=1e-12)
    st, _, info = amg.solve_group([(h, 0, dev(b), xs)], tol=1e-8)
    assert st == amg.AMG_OK and info[0].iterations == 0
    # the iteration limit: not converged, with the true residual of the last iterate
    hl = amg.Hierarchy(dev(rp), dev(ci), dev(va), max_iters=2)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, status, info = amg.solve_group([(hl, 0, dev(b), x)], tol=1e-14, raise_on_error=False)
    assert st == amg.AMG_ERR_NOT_CONVERGED and status == [st] and info[0].iterations == 2
    rel = np.linalg.norm(b - oracle.spmv(rp, ci, va, x.cpu().numpy())) / np.linalg.norm(b)
    assert abs(info[0].rel_residual - rel) <= 1e-6 * rel
    # a non-finite right-hand side fails its own job only
    bad = dev(b)
    bad[5] = float("nan")
    x2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    x3 = torch.zeros(n, dtype=torch.float64, device="cuda")
    hj = problems["grid2d_64_nu1"][3]  # the same grid, another hierarchy
    st, status, info = amg.solve_group([(h, 0, bad, x2), (hj, 0, dev(b), x3)], tol=1e-6, raise_on_error=False)
    assert status[0] == amg.AMG_ERR_INVALID_ARGUMENT and status[1] == amg.AMG_OK and st == status[0]
    # refused before any launch
    with pytest.raises(amg.AmgError) as e:
        amg.solve_group([(h, 0, dev(b), x2), (h, 0, dev(b), x3)])
    assert e.value.status == amg.AMG_ERR_INVALID_ARGUMENT
    with pytest.raises(amg.AmgError) as e:
        amg.solve_group([(hl, 1, dev(b), x2)])  # max_rhs 1
    assert e.value.status == amg.AMG_ERR_INVALID_ARGUMENT
    hm = amg.Hierarchy(dev(rp), dev(ci), dev(va), precision=amg.AMG_PREC_FP32_INNER)
    with pytest.raises(amg.AmgError) as e:
        amg.solve_group([(hm, 0, dev(b), x2)])
    assert e.value.status == amg.AMG_ERR_UNSUPPORTED
    r1, c1, v1 = inputs.grid_laplacian((6, 6))
    h1 = amg.Hierarchy(dev(r1), dev(c1), dev(v1))  # 36 unknowns: a single level
    assert h1.num_levels == 1
    with pytest.raises(amg.AmgError) as e:
        amg.solve_group([(h1, 0, dev(inputs.rhs(36, 1)), torch.zeros(36, dtype=torch.float64, device="cuda"))])
    assert e.value.status == amg.AMG_ERR_UNSUPPORTED
    for hh in (hl, hm, h1):
        hh.close()
