"""The continuous-batching serving loop on three streams: every request
completes, latencies are positive, and each request's result in the mix (its
ring slot, written by that request only) equals the result of indexing the
document alone (jsidx_build on its own buffer) and the oracle's."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_each_result_is_the_same_alone_and_in_the_mix():
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import serve, synth
    data, offs = synth.gen_c4(7, ring_bytes=24 << 20, hi=2 << 20, pool=60)
    nd = offs.size - 1
    _say(f"case: serving mix, ring {len(data)} bytes, {nd} docs, 3 streams")
    streams = [torch.cuda.Stream() for _ in range(3)]
    ring = serve.Ring(data, offs, 4 << 20, streams)
    sat = serve.saturated_rate(ring, seconds=0.05)
    assert sat > 0
    ring.out.fill_(-1)
    ring.cnt.fill_(-1)
    ring.err.fill_(-1)
    torch.cuda.synchronize()
    # one turn of the ring at 90% of saturation: every slot holds exactly one
    # request's result, computed while other batches ran beside it
    rate = 0.9 * sat / (len(data) / nd)
    arr = serve.poisson_arrivals(np.random.default_rng(5), rate, nd)
    lat, el, served, batches = serve.serve(ring, arr)
    torch.cuda.synchronize()
    assert served == len(data) and batches > 1
    assert np.all(lat > 0)
    mix_n = ring.cnt.cpu().numpy().view(np.uint32)
    mix_e = ring.err.cpu().numpy().view(np.uint32)
    mix_i = ring.out[:len(data)].cpu().numpy().view(np.uint32)
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert np.array_equal(mix_n, on) and np.array_equal(mix_e, oe)
    _say("case: each document alone")
    for d in range(nd):
        a, b = int(offs[d]), int(offs[d + 1])
        alone, n, e = jx.index(ring.bufs[a:b].clone())
        assert n == mix_n[d] and e == mix_e[d], f"doc {d}: alone ({n}, {e:#x}) vs mix ({mix_n[d]}, {mix_e[d]:#x})"
        al = alone.cpu().numpy().view(np.uint32)
        assert np.array_equal(al, mix_i[a:a + n]), f"doc {d}: positions differ alone vs in the mix"
        assert np.array_equal(al, oi[a:a + on[d]]), f"doc {d}: positions differ from the oracle"
    for st in streams:
        assert jx.diag(st) == 0


def test_serving_loop_over_many_turns_of_the_ring():
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import serve, synth
    data, offs = synth.gen_c4(8, ring_bytes=8 << 20, hi=1 << 20, pool=40)
    _say(f"case: serving loop, ring {len(data)} bytes, {offs.size - 1} docs, many turns")
    streams = [torch.cuda.Stream() for _ in range(2)]
    ring = serve.Ring(data, offs, 2 << 20, streams)
    sat = serve.saturated_rate(ring, seconds=0.05)
    res = serve.run_load(ring, sat, 0.5, 0.2, 6, min_requests=5 * ring.ndocs)
    torch.cuda.synchronize()
    assert res.requests >= 5 * ring.ndocs and res.batches > 0
    assert 0 < res.p50_us <= res.p99_us <= res.max_us
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert np.array_equal(ring.cnt.cpu().numpy().view(np.uint32), on)
    assert np.array_equal(ring.err.cpu().numpy().view(np.uint32), oe)
    gi = ring.out[:len(data)].cpu().numpy().view(np.uint32)
    for d in range(ring.ndocs):
        a, n = int(offs[d]), int(on[d])
        assert np.array_equal(gi[a:a + n], oi[a:a + n]), f"slot {d} differs"
    for st in streams:
        assert jx.diag(st) == 0


def test_forced_small_budget_binds_and_results_hold():
    """Admission by device memory with a budget far below one turn of the
    ring (room for about five of its largest requests): held bytes never pass
    the budget, the loop waits for completions and cuts batches, and every
    slot still holds the result of indexing its document alone and the
    oracle's."""
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import serve, synth
    data, offs = synth.gen_c4(9, ring_bytes=6 << 20, hi=256 << 10, pool=40)
    nd = offs.size - 1
    biggest = int(np.diff(offs.astype(np.int64)).max())
    budget = serve.REQUEST_BYTES_PER_BYTE * 5 * biggest
    assert budget < serve.REQUEST_BYTES_PER_BYTE * len(data)
    _say(f"case: forced budget {budget} bytes, ring {len(data)} bytes, {nd} docs, 3 streams")
    streams = [torch.cuda.Stream() for _ in range(3)]
    ring = serve.Ring(data, offs, 4 << 20, streams)
    ring.cnt.fill_(-1)
    ring.err.fill_(-1)
    torch.cuda.synchronize()
    st = serve.Admission(budget)
    arr = np.zeros(2 * nd)  # everything waiting at once: the budget is the only limit
    lat, el, served, batches = serve.serve(ring, arr, budget, st)
    torch.cuda.synchronize()
    _say(f"peak held {st.peak_held_bytes}, waits {st.admission_waits}, cut batches {st.budget_cut_batches}")
    assert served == 2 * len(data) and np.all(lat > 0)
    assert 0 < st.peak_held_bytes <= budget
    assert st.admission_waits > 0 and st.budget_cut_batches > 0
    on_n = ring.cnt.cpu().numpy().view(np.uint32)
    on_e = ring.err.cpu().numpy().view(np.uint32)
    gi = ring.out[:len(data)].cpu().numpy().view(np.uint32)
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert np.array_equal(on_n, on) and np.array_equal(on_e, oe)
    for d in range(nd):
        a, b = int(offs[d]), int(offs[d + 1])
        assert np.array_equal(gi[a:a + on[d]], oi[a:a + on[d]]), f"slot {d} differs from the oracle"
        if d % 7 == 0:
            alone, n, e = jx.index(ring.bufs[a:b].clone())
            assert n == on_n[d] and e == on_e[d]
            assert np.array_equal(alone.cpu().numpy().view(np.uint32), gi[a:a + n]), f"doc {d}: alone vs mix"
    for s in streams:
        assert jx.diag(s) == 0
