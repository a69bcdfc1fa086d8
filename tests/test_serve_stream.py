"""The serving request stream (host logic, no GPU)."""
import math

from paper_1302_2547_amd import serve


def test_stream_is_deterministic_and_shaped():
    a = serve.make_requests(count=400, seed=6)
    b = serve.make_requests(count=400, seed=6)
    assert [(r.t_arrival, r.dims, r.jitter_seed, r.rhs_seeds) for r in a] == \
           [(r.t_arrival, r.dims, r.jitter_seed, r.rhs_seeds) for r in b]
    t = [r.t_arrival for r in a]
    assert all(x < y for x, y in zip(t, t[1:]))
    mean_gap = t[-1] / len(t)
    assert 0.8 / 200 < mean_gap < 1.2 / 200  # Poisson at 200 per second
    keys = [r.key for r in a]
    reused = sum(1 for i, k in enumerate(keys) if k in keys[:i])
    assert 0.2 < reused / len(a) < 0.4  # about 30 % reuse
    assert {len(r.rhs_seeds) for r in a} == set(range(1, 9))
    for r in a:
        assert len(r.dims) in (2, 3)
        lo, hi = (1e4, 2e6) if len(r.dims) == 2 else (1e4, 4e6)
        assert lo / 2 <= r.n <= hi * 1.5
        assert len(set(r.dims)) == 1
    assert abs(sum(len(r.dims) == 2 for r in a) / len(a) - 0.5) < 0.15
