"""The continuous-batching serving loop: every request completes, latencies are
positive, and the outputs of every ring slot equal the oracle's for that
document (each slot is rewritten by every request that maps to it)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_serving_loop_completes_and_matches_oracle():
    import torch
    from paper_1902_08318_amd import serve, synth
    data, offs = synth.gen_c4(7, ring_bytes=24 << 20, hi=2 << 20, pool=60)
    print(f"case: serving loop ring {len(data)} bytes, {offs.size - 1} docs", flush=True)
    sys.stdout.flush()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ring = serve.Ring(data, offs, 4 << 20, s)
        sat = serve.saturated_rate(ring, seconds=0.05)
        assert sat > 0
        res = serve.run_load(ring, sat, 0.5, 0.2, 5, min_requests=3 * ring.ndocs)
    s.synchronize()
    assert res.requests >= 3 * ring.ndocs
    assert res.served_bytes > 0 and res.batches > 0
    assert 0 < res.p50_us <= res.p99_us <= res.max_us
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    gn = ring.cnt.cpu().numpy().view(np.uint32)
    ge = ring.err.cpu().numpy().view(np.uint32)
    assert np.array_equal(gn, on)
    assert np.array_equal(ge, oe)
    gi = ring.out[:len(data)].cpu().numpy().view(np.uint32)
    for d in range(ring.ndocs):
        a, n = int(offs[d]), int(on[d])
        assert np.array_equal(gi[a:a + n], oi[a:a + n]), f"slot {d} differs"
    import paper_1902_08318_amd as jx
    assert jx.diag(s) == 0
