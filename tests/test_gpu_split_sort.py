"""The whole-chip sort of long coarse rows on a problem whose rows are shorter than
its default threshold (2^17 padded keys): AMG_SPLIT_MIN_KEYS lowers it to 4096 or
8192 keys.  On the 128^3 jittered Laplacian 15 (4096) or 6 (8192) of the 33 rows of
one coarse level that go to whole blocks are then sorted by the grid-wide passes
(a stage trace with AMG_TRACE=1 lists them), the others by their blocks.  The keys
(coarse column, position) are unique, so the hierarchy must still equal the oracle's
bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1302_2547_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def amg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_2547_amd import amg as mod
    return mod


def same_hierarchy(amg, rp, ci, va):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = amg.Hierarchy(d(rp), d(ci), d(va))
    ref = oracle.Hierarchy(rp, ci, va)
    try:
        assert h.num_levels == ref.num_levels
        for l in range(h.num_levels):
            g, o = h.export_level(l), ref.level(l)
            assert (g.n, g.nnz, g.passes) == (o.n, o.nnz, o.passes), l
            np.testing.assert_array_equal(g.agg, o.agg)
            np.testing.assert_array_equal(g.row_ptr, o.row_ptr)
            np.testing.assert_array_equal(g.col, o.col)
            np.testing.assert_array_equal(g.val, o.val)
    finally:
        h.close()
        ref.close()


@pytest.mark.parametrize("keys", [4096, 8192])
def test_grid_128cubed_split_rows(amg, keys, monkeypatch):
    monkeypatch.setenv("AMG_SPLIT_MIN_KEYS", str(keys))
    print(f"[split] 128^3 jittered, split at {keys} keys", flush=True)
    rp, ci, va = inputs.grid_laplacian((128, 128, 128), jitter=0.1, seed=2)
    same_hierarchy(amg, rp, ci, va)

