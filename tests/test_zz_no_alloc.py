"""The grid generator for callers that cannot allocate (amg_grid_laplacian_noalloc):
bit-identical to the allocating amg_grid_laplacian on two calls in a row (the second
smaller, so it runs on the scratch the first one left behind), and grids beyond its
static scratch are refused before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _arrays(dims):
    from paper_1302_2547_amd import amg
    d = len(dims)
    arr = (ctypes.c_int32 * 3)(*dims, *([1] * (3 - d)))
    nnz = amg.amg_grid_laplacian_nnz(d, arr)
    n = int(np.prod(dims))
    dev = torch.device("cuda:0")
    out = (torch.full((n + 1,), -7, dtype=torch.int32, device=dev),
           torch.full((nnz,), -7, dtype=torch.int32, device=dev),
           torch.full((nnz,), np.nan, dtype=torch.float64, device=dev))
    return d, arr, out


def test_noalloc_generator_equals_allocating_one_twice():
    from paper_1302_2547_amd import amg
    stream = torch.cuda.Stream()
    for dims, jitter, seed in [((41, 37, 33), 0.1, 7), ((50, 41), 0.05, 3)]:
        print(f"[no-alloc] grid {dims} jitter {jitter} seed {seed}", flush=True)
        d, arr, ref = _arrays(dims)
        _, _, got = _arrays(dims)
        st = amg.amg_grid_laplacian(d, arr, jitter, seed, *(t.data_ptr() for t in ref), None)
        assert st == amg.AMG_OK, st
        st = amg.amg_grid_laplacian_noalloc(d, arr, jitter, seed, *(t.data_ptr() for t in got),
                                            stream.cuda_stream)
        assert st == amg.AMG_OK, st
        stream.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a.cpu(), b.cpu())
        # and equal to the host generator of the package (independent of both)
        from paper_1302_2547_amd import inputs
        rp, ci, va = inputs.grid_laplacian(dims, jitter=jitter, seed=seed)
        np.testing.assert_array_equal(got[0].cpu().numpy(), rp)
        np.testing.assert_array_equal(got[1].cpu().numpy(), ci)
        np.testing.assert_array_equal(got[2].cpu().numpy(), va)


def test_noalloc_generator_refuses_grids_beyond_its_scratch():
    from paper_1302_2547_amd import amg
    d, arr, small = _arrays((4, 4))
    big = (ctypes.c_int32 * 3)(1024, 1024, 129)  # 135,266,304 unknowns > 2^27
    assert amg.amg_grid_laplacian_nnz(3, big) > 0  # a valid grid for the allocating call
    st = amg.amg_grid_laplacian_noalloc(3, big, 0.0, 1, *(t.data_ptr() for t in small), None)
    assert st == amg.AMG_ERR_UNSUPPORTED
    host = np.zeros(4, np.float64)
    st = amg.amg_grid_laplacian_noalloc(2, arr, 0.0, 1, small[0].data_ptr(), small[1].data_ptr(),
                                        host.ctypes.data, None)
    assert st == amg.AMG_ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
