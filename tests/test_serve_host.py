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


def test_admission_fits_the_budget():
    """Host logic of admission by device memory: the admitted prefix's held
    bytes (5 per input byte) fit in what the budget leaves; one request goes
    alone when nothing is held; none is admitted when nothing fits."""
    from paper_1902_08318_amd.serve import REQUEST_BYTES_PER_BYTE as K, Ring, admit
    offs = np.array([0, 10, 30, 60, 100, 150, 210], dtype=np.int64)
    r = Ring.__new__(Ring)
    r.offs_h, r.ndocs, r.total, r.max_batch_bytes = offs, 6, 210, 1000
    assert admit(r, 0, 6, 0, K * 60) == 3        # 10+20+30 fit exactly
    assert admit(r, 0, 6, 0, K * 59) == 2
    assert admit(r, 0, 2, 0, K * 1000) == 2      # never past what was asked
    assert admit(r, 0, 6, K * 50, K * 60) == 1   # 10 left
    assert admit(r, 1, 6, K * 50, K * 60) == 1   # 20 > 10 left: wait
    assert admit(r, 4, 6, 0, K * 10) == 5        # 50 > budget, nothing held: alone
    assert admit(r, 6, 9, 0, K * 30) == 8        # second turn of the ring: slots 0, 1


def test_serving_loop_admission_without_a_device():
    """The loop's admission bookkeeping with a stand-in for the device (every
    batch completes at once): held bytes never pass the budget, waits are
    counted, and every request is served exactly once."""
    import sys
    import types
    from paper_1902_08318_amd import serve as sv

    class Ev:
        def record(self, stream):
            pass

        def query(self):
            return True

    fake = types.SimpleNamespace(cuda=types.SimpleNamespace(Event=Ev))
    real = sys.modules.get("torch")
    sys.modules["torch"] = fake
    try:
        offs = np.cumsum(np.r_[0, np.random.default_rng(1).integers(1, 100, 400)]).astype(np.int64)
        r = sv.Ring.__new__(sv.Ring)
        r.offs_h, r.ndocs, r.total, r.max_batch_bytes = offs, 400, int(offs[-1]), 1 << 20
        r.streams = [None, None]
        launched = []
        r.launch = lambda d0, nd, k: launched.append((d0, nd))
        st = sv.Admission(0)
        budget = sv.REQUEST_BYTES_PER_BYTE * 300
        lat, el, served, batches = sv.serve(r, np.zeros(1200), budget, st)
        assert served == 3 * r.total and batches == len(launched)
        assert sum(nd for _, nd in launched) == 1200
        assert 0 < st.peak_held_bytes <= budget
        assert st.budget_cut_batches > 0
    finally:
        if real is not None:
            sys.modules["torch"] = real
        else:
            del sys.modules["torch"]
