"""GPU against the oracle at the two largest benchmark configurations:

* the 256^3 unit-weight 7-point Laplacian (16.8M unknowns) at tolerance 1e-10, in
  FP64 and with the FP32 K-cycle inside the FP64 outer flexible CG: the hierarchy
  must equal the oracle's bit for bit, both solves must reach the tolerance on the
  true residual, and each solution's distance to the oracle's is reported;
* the 4M-point random geometric graph Laplacian (weights U[0.5, 1.5], shift 1e-6)
  with 32 right-hand sides solved in one batch with the FP32 K-cycle: the hierarchy
  equals the oracle's, every column reaches 1e-8, and four columns are compared
  with oracle solves of the same right-hand sides.

The oracle's work here (a serial FP64 setup and solve of 16.8M unknowns, four
solves on 4M unknowns) takes a minute or two on one host core; progress goes to
the terminal as it runs.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1302_2547_amd import inputs  # noqa: E402


def note(request, msg):
    """Progress line on the terminal, past pytest's output capture."""
    capman = request.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        print(f"[headline] {msg}", flush=True)


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_2547_amd import amg as mod
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_hierarchy(h, ref):
    assert h.num_levels == ref.num_levels
    for l in range(h.num_levels):
        g, o = h.export_level(l), ref.level(l)
        assert (g.n, g.nnz, g.passes) == (o.n, o.nnz, o.passes), l
        np.testing.assert_array_equal(g.agg, o.agg)
        np.testing.assert_array_equal(g.row_ptr, o.row_ptr)
        np.testing.assert_array_equal(g.col, o.col)
        np.testing.assert_array_equal(g.val, o.val)


def true_rel(rp, ci, va, b, x):
    return np.linalg.norm(b - oracle.spmv(rp, ci, va, x)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cube256(request):
    t = time.perf_counter()
    rp, ci, va = inputs.grid_laplacian((256, 256, 256))
    b = inputs.rhs(len(rp) - 1, 1)
    note(request, f"256^3: generated n={len(rp) - 1} nnz={len(ci)} in {time.perf_counter() - t:.1f} s; oracle setup")
    ref = oracle.Hierarchy(rp, ci, va)
    note(request, f"256^3: oracle setup {ref.setup_ms / 1e3:.1f} s, {ref.num_levels} levels; oracle solve to 1e-10")
    t = time.perf_counter()
    x_o, st, it_o, rel_o, _ = ref.solve(b, tol=1e-10)
    note(request, f"256^3: oracle solve {time.perf_counter() - t:.1f} s, {it_o} iterations, rel {rel_o:.2e}")
    assert st == 0
    yield rp, ci, va, b, ref, x_o, it_o
    ref.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_inner"])
def test_cube256_tol_1e10_against_oracle(amg, cube256, precision, request):
    rp, ci, va, b, ref, x_o, it_o = cube256
    prec = amg.AMG_PREC_FP64 if precision == "fp64" else amg.AMG_PREC_FP32_INNER
    note(request, f"256^3 {precision}: GPU setup")
    h = amg.Hierarchy(dev(rp), dev(ci), dev(va), precision=prec)
    same_hierarchy(h, ref)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    st, info = h.solve(dev(b), x, tol=1e-10)
    xg = x.cpu().numpy()
    rel = true_rel(rp, ci, va, b, xg)
    err = np.linalg.norm(xg - x_o) / np.linalg.norm(x_o)
    note(request, f"256^3 {precision}: {info.iterations} iterations (oracle {it_o}), true rel {rel:.3e}, "
         f"||x - x_oracle|| / ||x_oracle|| = {err:.3e}, setup {info.setup_ms:.1f} ms solve {info.solve_ms:.1f} ms")
    assert st == amg.AMG_OK and rel <= 1e-10
    assert abs(info.iterations - it_o) <= 2
    # both solutions satisfy ||b - A x|| <= 1e-10 ||b||, so their distance is at most
    # cond(A) * 2e-10 relative; cond(A) = 12 / (12 sin^2(pi / 514)) ~ 2.7e4 at 256^3
    assert err <= 6e-6
    h.close()


COLUMNS = (0, 9, 22, 31)


def test_rgg4m_batch32_fp32_inner_against_oracle(amg, request):
    t = time.perf_counter()
    rp, ci, va = inputs.rgg_laplacian(4_000_000, seed=4, weight_range=(0.5, 1.5))
    n = len(rp) - 1
    B = np.stack([inputs.rhs(n, 500 + k) for k in range(32)])
    note(request, f"4M graph: generated n={n} nnz={len(ci)} in {time.perf_counter() - t:.1f} s; GPU setup + 32-column solve")
    h = amg.Hierarchy(dev(rp), dev(ci), dev(va), precision=amg.AMG_PREC_FP32_INNER, max_rhs=32)
    X = torch.zeros((32, n), dtype=torch.float64, device="cuda")
    st, infos = h.solve_batch(dev(B), X, tol=1e-8)
    assert st == amg.AMG_OK
    assert max(i.rel_residual for i in infos) <= 1e-8
    note(request, f"4M graph: batch of 32 in {infos[0].solve_ms:.0f} ms, iterations {min(i.iterations for i in infos)}-"
         f"{max(i.iterations for i in infos)}; oracle setup")
    ref = oracle.Hierarchy(rp, ci, va)
    same_hierarchy(h, ref)
    Xg = X.cpu().numpy()
    for c in COLUMNS:
        t = time.perf_counter()
        x_o, st_o, it_o, rel_o, _ = ref.solve(B[c], tol=1e-8)
        rel = true_rel(rp, ci, va, B[c], Xg[c])
        err = np.linalg.norm(Xg[c] - x_o) / np.linalg.norm(x_o)
        note(request, f"4M graph column {c}: GPU {infos[c].iterations} iterations, true rel {rel:.3e}; oracle {it_o} "
             f"iterations ({time.perf_counter() - t:.1f} s), ||x - x_oracle|| / ||x_oracle|| = {err:.3e}")
        assert st_o == 0 and rel <= 1e-8
        assert abs(infos[c].iterations - it_o) <= 3
        # A = L + 1e-6 I with L positive semidefinite, so two solutions of relative
        # residual <= 1e-8 differ by at most 2e-8 ||b|| / 1e-6 (~23); the ~1,300
        # isolated vertices (x_i = b_i / 1e-6) alone make ||x|| ~2e7: <= ~1.1e-6
        assert err <= 5e-6
    ref.close()
    h.close()
