"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
setup, aggregation, coarse operators, K-cycle and solves on grids, random graphs,
a star, a disconnected graph and the size-limited / level-skipping / threshold
variants, in a child process with the sanitizer runtime preloaded.  Any report
aborts the child."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

SCRIPT = r"""
import numpy as np
import oracle
from paper_1302_2547_amd import inputs

cases = [inputs.grid_laplacian((12, 11), jitter=0.3, seed=1),
         inputs.grid_laplacian((7, 6, 5), jitter=0.1, seed=2),
         inputs.grid_laplacian((300,), jitter=0.2, seed=3),
         inputs.random_graph_laplacian(150, 0.05, seed=4, integer_weights=True, shift=1.0),
         inputs.rgg_laplacian(3000, seed=5, weight_range=(0.5, 1.5))]
opts = [{}, dict(max_aggregate=2, skip_ratio=2.5), dict(kcycle_threshold=0.4, kcycle_inner=2),
        dict(coarsest_size=1), dict(coarsest_size=10000), dict(smoother="jacobi", kcycle_inner=1)]
for rp, ci, va in cases:
    n = len(rp) - 1
    b = inputs.rhs(n, 7)
    for o in opts:
        h = oracle.Hierarchy(rp, ci, va, **o)
        for l in range(h.num_levels):
            h.level(l)
        h.kcycle(b)
        x, st, it, rel, _ = h.solve(b, tol=1e-9, max_iters=100)
        assert st in (oracle.OK, oracle.ERR_NOT_CONVERGED), st
        h.close()
    key = oracle.priorities(rp, ci, 3, 0)
    owner, pass_of, passes = oracle.paa(rp, ci, key, cap=3)
    agg, nc = oracle.number(owner)
    oracle.coarse_operator(rp, ci, va, agg, nc)
print("sanitized oracle run ok")
"""


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(600)
def test_oracle_under_asan_and_ubsan():
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    import oracle
    lib = oracle.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=runtime, UA_AMG_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               PYTHONPATH=ROOT)
    p = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, cwd=ROOT)
    assert p.returncode == 0 and "sanitized oracle run ok" in p.stdout, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
