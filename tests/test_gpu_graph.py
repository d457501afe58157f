"""The batched and single-document launches captured in a HIP graph.

After jsidx_reserve on a stream, jsidx_build_batch and jsidx_build on that
stream allocate nothing, copy nothing to the host and record no memset: the
kernel itself resets its ticket counter and bumps its launch epoch when the
last workgroup leaves, so one captured launch can be replayed.  Each replay
gets new input bytes (and new offsets, same document count) written by eager
work between replays, and every replay is checked against an eager launch on
the same input and against the CPU oracle.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batches(ndocs, cap, seeds):
    from paper_1902_08318_amd import synth
    out = []
    for s in seeds:
        data, offs, _ = synth.gen_c3(s, ndocs=ndocs, pool=80, median=1024, hi=16384, corrupt_frac=0.05)
        assert int(offs[-1]) <= cap
        out.append((data, offs))
    return out


def test_batched_launch_replayed_from_graph():
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    ndocs, cap = 700, 4 << 20
    batches = _batches(ndocs, cap, [31, 32, 33, 34])
    s = torch.cuda.Stream()
    bufs = torch.zeros(cap, dtype=torch.uint8, device=dev)
    offs = torch.zeros(ndocs + 1, dtype=torch.int64, device=dev)
    out = torch.zeros(cap, dtype=torch.int32, device=dev)
    cnt = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    err = torch.zeros(ndocs, dtype=torch.int32, device=dev)

    def load(k):
        data, o = batches[k]
        bufs[:len(data)].copy_(torch.frombuffer(bytearray(data), dtype=torch.uint8))
        offs.copy_(torch.from_numpy(o.astype(np.int64)))
        out.fill_(-1)
        cnt.fill_(-1)
        err.fill_(-1)

    with torch.cuda.stream(s):
        jx.reserve(cap, s)
        load(0)
        jx.build_batch(bufs, offs, out, cnt, err, s)  # eager warm-up on the capture stream
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        jx.build_batch(bufs, offs, out, cnt, err, s)
    for r in range(6):
        k = r % len(batches)
        data, o = batches[k]
        _say(f"case: batch graph replay {r} (batch {k}, {len(data)} bytes)")
        with torch.cuda.stream(s):
            load(k)
            jx.build_batch(bufs, offs, out, cnt, err, s)
        s.synchronize()
        e_out, e_cnt, e_err = out.clone(), cnt.clone(), err.clone()
        with torch.cuda.stream(s):
            out.fill_(-1)
            cnt.fill_(-1)
            err.fill_(-1)
        s.synchronize()
        g.replay()
        s.synchronize()
        assert torch.equal(cnt, e_cnt) and torch.equal(err, e_err), f"replay {r}: counts/flags differ from eager"
        tot = int(o[-1])
        gi = out[:tot].cpu().numpy().view(np.uint32)
        ei = e_out[:tot].cpu().numpy().view(np.uint32)
        oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), o)
        assert np.array_equal(cnt.cpu().numpy().view(np.uint32), on)
        assert np.array_equal(err.cpu().numpy().view(np.uint32), oe)
        for d in range(ndocs):
            a, n = int(o[d]), int(on[d])
            assert np.array_equal(gi[a:a + n], oi[a:a + n]), f"replay {r}: doc {d} differs from the oracle"
            assert np.array_equal(gi[a:a + n], ei[a:a + n]), f"replay {r}: doc {d} differs from eager"
    assert jx.diag(s) == 0


def test_single_document_launch_replayed_from_graph():
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    dev = torch.device("cuda:0")
    n = 3 << 20
    docs = [synth.gen_c1(41 + k, n, pool=64).data[:n] for k in range(3)]
    s = torch.cuda.Stream()
    buf = torch.zeros(n, dtype=torch.uint8, device=dev)
    out = torch.zeros(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.stream(s):
        jx.reserve(n, s)
        buf.copy_(torch.frombuffer(bytearray(docs[0]), dtype=torch.uint8))
        jx.build(buf, out, cnt, err, s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        jx.build(buf, out, cnt, err, s)
    for r in range(5):
        d = docs[r % len(docs)]
        _say(f"case: single-document graph replay {r}")
        with torch.cuda.stream(s):
            buf.copy_(torch.frombuffer(bytearray(d), dtype=torch.uint8))
            out.fill_(-1)
            cnt.fill_(-1)
        s.synchronize()
        g.replay()
        s.synchronize()
        oi, oe = oracle.index(d)
        k = int(cnt.item())
        assert k == len(oi) and (int(err.item()) & 0xFFFFFFFF) == oe
        assert np.array_equal(out[:k].cpu().numpy().view(np.uint32), oi)
    assert jx.diag(s) == 0
