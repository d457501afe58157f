"""Host-side logic of the serving loop (no GPU): batch formation and the
Poisson arrival process."""
import numpy as np


def test_batch_end_stays_in_ring_and_reservation():
    """Host logic of batch formation (no launch): batches never wrap the ring
    and never exceed the reserved byte size unless one document alone does."""
    from paper_1902_08318_amd.serve import Ring
    offs = np.array([0, 10, 30, 60, 100, 150, 210], dtype=np.int64)
    r = Ring.__new__(Ring)
    r.offs_h, r.ndocs, r.total, r.max_batch_bytes = offs, 6, 210, 70
    assert r.batch_end(0, 100) == 3          # 10+20+30 = 60 <= 70, +40 > 70
    assert r.batch_end(3, 100) == 4          # 40, then 90 > 70
    assert r.batch_end(5, 100) == 6          # stops at the ring end
    assert r.batch_end(6, 100) == 9          # slot 0.. again: 10+20+30
    assert r.batch_end(4, 5) == 5            # only what has arrived
    r.max_batch_bytes = 5
    assert r.batch_end(0, 100) == 1          # one oversized document still goes alone


def test_poisson_arrivals_rate():
    from paper_1902_08318_amd.serve import poisson_arrivals
    a = poisson_arrivals(np.random.default_rng(0), 1e6, 200_000)
    assert np.all(np.diff(a) >= 0)
    assert abs(a[-1] - 0.2) < 0.01   # 200k arrivals at 1M/s take about 0.2 s
