"""Host checks of the seeded serving stream: every query's library (a subset of
whole reactions) has a compound count inside the requested range, also where a
single reaction is larger than the range's upper end."""
import math

import numpy as np

import workloads.gen as gen


def _sizes(stream, counts):
    return [sum(int(counts[r]) for r in q.reactions) for _, q in stream]


def _c3_counts():
    n_slots, sizes = gen.config_c3_shape(2)
    counts, off = [], 0
    for n in n_slots:
        c = 1
        for j in range(n):
            c *= int(sizes[off + j])
        counts.append(c)
        off += n
    return np.array(counts, dtype=np.int64)


def test_stream_sizes_within_range_large_library():
    counts = _c3_counts()
    assert counts.max() > 1e9  # single reactions above the range exist in this library
    st = gen.serving_stream(5, 400, 5.0, counts, 1e6, 1e9, lambda h, q: 0.0)
    sz = _sizes(st, counts)
    assert min(sz) >= 1e6 and max(sz) <= 1e9
    # the draw is log-uniform over the range: the median sits near its geometric middle
    assert 1e7 < float(np.median(sz)) < 1e8


def test_stream_arrivals_and_queries():
    counts = np.array([10, 20, 5000, 40, 7, 10 ** 7, 300, 64, 900, 12], dtype=np.int64)
    st = gen.serving_stream(3, 200, 4.0, counts, 50, 2000, lambda h, q: float(q))
    t = np.array([a for a, _ in st])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 4.0) < 1.5  # Poisson rate 4/s over 200 arrivals
    sz = _sizes(st, counts)
    assert min(sz) >= 50 and max(sz) <= 2000  # the 5000- and 1e7-compound reactions never enter
    for _, q in st:
        assert len(set(q.reactions)) == len(q.reactions) and q.reactions == sorted(q.reactions)
        assert 2 <= len(q.constraints) <= 6 and q.k in (100, 1000, 10000)
        assert len({c.head for c in q.constraints}) == len(q.constraints)
        for c in q.constraints:
            assert math.isinf(c.lo) != math.isinf(c.hi)  # one-sided


def test_stream_falls_back_to_smallest_reaction():
    counts = np.array([5000, 700, 90000], dtype=np.int64)  # every reaction is above the range
    st = gen.serving_stream(1, 5, 1.0, counts, 10, 100, lambda h, q: 0.0)
    assert all(q.reactions == [1] for _, q in st)
