"""GPU tape (jsidx_tape on the index and links jsidx_build and jsidx_scopes
wrote) against the oracle's tape, bit-exact: words, string buffer, flags."""
import json
import os
import random
import struct
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_tape(data: bytes):
    import torch
    import paper_1902_08318_amd as jx
    dev = torch.device("cuda:0")
    n = len(data)
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev) if n else torch.zeros(1, dtype=torch.uint8,
                                                                                                device=dev)
    idx = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    jx.build(buf, idx, cnt, err, length=n)
    k = int(cnt.item())
    match = torch.empty(max(1, k), dtype=torch.int32, device=dev)
    serr = torch.empty(1, dtype=torch.int32, device=dev)
    jx.scopes(buf, idx, match, serr, n=k, length=n)
    words = torch.full((2 * k + 2,), -1, dtype=torch.int64, device=dev)
    sbuf = torch.full((n + 2 * k + 4,), 0xA5, dtype=torch.uint8, device=dev)
    tn = torch.full((1,), -1, dtype=torch.int64, device=dev)
    sn = torch.full((1,), -1, dtype=torch.int64, device=dev)
    terr = torch.full((1,), -1, dtype=torch.int32, device=dev)
    jx.tape(buf, idx, match, words, tn, sbuf, sn, terr, n=k, length=n)
    torch.cuda.synchronize()
    nt, ns = int(tn.item()), int(sn.item())
    return (words[:nt].cpu().numpy().view(np.uint64), sbuf[:ns].cpu().numpy().tobytes(),
            int(terr.item()) & 0xFFFFFFFF, int(serr.item()) & 0xFFFFFFFF)


def assert_tape_matches(data: bytes, label: str):
    words, sbuf, flags, serr = gpu_tape(data)
    idx, _ = oracle.index(data)
    ow, osb, of = oracle.tape(data, idx)
    assert flags == of, f"{label}: flags {flags:#x} != {of:#x}"
    if of == 0 and ow.size:
        assert serr == 0, f"{label}: scope flags {serr:#x}"
        assert words.size == ow.size, f"{label}: {words.size} words != {ow.size}"
        bad = np.nonzero(words != ow)[0]
        assert bad.size == 0, f"{label}: {bad.size} words differ, first at {bad[0] if bad.size else -1}"
        assert sbuf == osb, f"{label}: string buffers differ"


def test_tape_fig1_and_small_cases():
    _say("case: tape Fig. 1 and small cases")
    assert_tape_matches(open(os.path.join(GOLDEN, "paper_fig1_document.json"), "rb").read(), "Fig. 1")
    for t in ("1", "-0", "0.5", '"x"', "true", "null", "[]", "{}", '{"a":[1,2,{"b":null}],"c":"\\u00e9\\ud83d\\ude00"}',
              "[01]", "[1.]", '["\\x"]', "[tru]", "[1e309]", '["a\\u12"]', '["\\ud800"]', "[-]", "[9223372036854775808]",
              "[-9223372036854775808, 9223372036854775807]", '"unclosed', "[1, 2", '["a\\u0000b", "\\/\\b"]'):
        assert_tape_matches(t.encode(), t)


def test_tape_numbers_in_bulk():
    """Random numbers over the double range, 17-digit doubles, and exact
    halfway points (taken by the exact conversion)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 1200
    rng = random.Random(21)
    nums = []
    for _ in range(20000):
        digits = "".join(rng.choice("0123456789") for _ in range(rng.randrange(1, 30))).lstrip("0") or "0"
        frac = "" if rng.random() < 0.3 else "." + "".join(rng.choice("0123456789")
                                                          for _ in range(rng.randrange(1, 25)))
        exp = "" if rng.random() < 0.3 else "e" + rng.choice(["", "+", "-"]) + str(rng.randrange(0, 340))
        nums.append(rng.choice(["", "-"]) + digits + frac + exp)
    for _ in range(20000):
        x = struct.unpack("<d", struct.pack("<Q", rng.getrandbits(63)))[0]
        if np.isfinite(x):
            nums.append(repr(x))
    for _ in range(500):
        x = struct.unpack("<d", struct.pack("<Q", rng.getrandbits(63)))[0]
        y = float(np.nextafter(x, np.inf))
        if np.isfinite(x) and np.isfinite(y) and x > 0:
            mid = (Decimal(x) + Decimal(y)) / 2
            nums += [str(mid), str(mid + (Decimal(y) - Decimal(x)) / 10 ** 30)]
    _say(f"case: tape {len(nums)} numbers")
    assert_tape_matches(("[" + ",".join(nums) + "]").encode(), "numbers")


def test_tape_random_and_generated_documents():
    rng = random.Random(6)

    def val(d):
        r = rng.random()
        if d > 5 or r < 0.45:
            k = rng.randrange(5)
            if k == 0:
                return rng.randrange(-(1 << 63), 1 << 63)
            if k == 1:
                return rng.choice([True, False, None])
            if k == 2:
                return rng.uniform(-1e300, 1e300) * rng.choice([1, 1e-300, 1e-10])
            return "".join(rng.choice(["a", " ", '"', "\\", "\n", "\x01", "é", "\U0001F600", "/"])
                           for _ in range(rng.randrange(0, 8)))
        if r < 0.7:
            return [val(d + 1) for _ in range(rng.randrange(0, 6))]
        return {f"k{i}é": val(d + 1) for i in range(rng.randrange(0, 6))}

    text = json.dumps([val(0) for _ in range(30000)], ensure_ascii=False)
    _say("case: tape random nested JSON")
    assert_tape_matches(text.encode(), "random")
    assert_tape_matches(json.dumps(json.loads(text), ensure_ascii=True, indent=1).encode(), "random ascii")
    from paper_1902_08318_amd import synth
    for name, doc in (("C0", synth.gen_c0(0, 1 << 20).data), ("C1 8 MiB", synth.gen_c1(1, 8 << 20, pool=256).data),
                      ("C2 8 MiB", synth.gen_c2(2, 8 << 20, pool=16).data)):
        _say(f"case: tape {name}")
        assert_tape_matches(doc, name)


def test_tape_full_size_c1_and_c2():
    from paper_1902_08318_amd import synth
    for name, doc in (("C1", synth.gen_c1(1).data), ("C2", synth.gen_c2(2).data)):
        _say(f"case: tape {name} full size {len(doc)}")
        assert_tape_matches(doc, name)


def test_tape_strings_above_2_23_bytes():
    """Strings of more than 2^23 bytes in one chunk: the chunk scans take their
    64-bit form (one document, and a batch of such documents)."""
    rng = random.Random(29)

    def big(k):
        body = "".join(rng.choice(["a", "b", " ", "\\n", "\\u00e9", "\\\""]) for _ in range(200))
        return body * k

    doc = ('[' + '"' + big(50000) + '", 1, {"k": "' + big(48000) + '", "v": [2.5, true, null]}, "z"]').encode()
    assert len(doc) > 2 * (1 << 23)
    _say(f"case: tape strings above 2^23 bytes, {len(doc)} bytes")
    assert_tape_matches(doc, "big strings")
    docs = [doc, b'["x", 3]', ('{"s": "' + big(45000) + '"}').encode()]
    data = b"".join(docs)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in docs], out=offs[1:])
    _say(f"case: tape batch with strings above 2^23 bytes, {len(data)} bytes")
    b = _Batch(data, offs)
    b.run()
    assert b.check("big strings batch") == 3


def test_tape_flags_on_corrupted_atoms():
    """One corruption per document, inserted as a new first element of a
    random array of a generated document: a number with a stray letter, a
    leading zero or an out-of-range value, a misspelled literal, a string with
    an unknown escape, a control byte or a lone surrogate.  The flags must
    equal the oracle's."""
    from paper_1902_08318_amd import synth
    rng = random.Random(13)
    base = synth.gen_c0(5, 1 << 19).data
    inserts = [b"7x, ", b"012, ", b"99999999999999999999, ", b"1e400, ", b"tru, ", b"nulll, ", b'"a\\qb", ',
               b'"a\x01b", ', b'"\\ud800x", ']
    idx, _ = oracle.index(base)
    starts = [int(p) + 1 for p in idx if base[int(p)] == 0x5B]  # just after a '['
    for k, ins in enumerate(inserts):
        p = rng.choice(starts)
        doc = base[:p] + ins + base[p:]
        _say(f"case: tape corrupted atom {k}")
        assert_tape_matches(doc, f"corruption {k}")


class _Batch:
    """A batch on the device: index, counts and links (jsidx_build_batch and
    jsidx_scopes_batch), and the outputs of jsidx_tape_batch."""

    def __init__(self, data: bytes, offs: np.ndarray, stream=None, reserve=True, tape_cap=None):
        import torch
        import paper_1902_08318_amd as jx
        dev = torch.device("cuda:0")
        self.data, self.offs = data, offs
        total, nd = int(offs[-1]), offs.size - 1
        self.buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
        self.o = torch.from_numpy(offs.astype(np.int64)).to(dev)
        self.idx = torch.empty(max(1, total), dtype=torch.int32, device=dev)
        self.cnt = torch.empty(nd, dtype=torch.int32, device=dev)
        err = torch.empty(nd, dtype=torch.int32, device=dev)
        jx.build_batch(self.buf, self.o, self.idx, self.cnt, err, stream)
        torch.cuda.synchronize()
        ent = int(self.cnt.to(torch.int64).sum().item())
        jx.scopes_reserve(ent, nd, stream)
        self.match = torch.empty(max(1, total), dtype=torch.int32, device=dev)
        self.serr = torch.empty(nd, dtype=torch.int32, device=dev)
        jx.scopes_batch(self.buf, self.o, self.idx, self.cnt, self.match, self.serr, stream)
        if reserve:
            jx.tape_reserve(ent, nd, stream)
        self.words = torch.full((tape_cap or 2 * (ent + nd),), -1, dtype=torch.int64, device=dev)
        self.sbuf = torch.full((total + 2 * ent + 4,), 0xA5, dtype=torch.uint8, device=dev)
        self.pos = torch.full((4 * nd,), -1, dtype=torch.int64, device=dev)
        self.terr = torch.full((nd,), -1, dtype=torch.int32, device=dev)

    def run(self, stream=None):
        import paper_1902_08318_amd as jx
        jx.tape_batch(self.buf, self.o, self.idx, self.cnt, self.match, self.words, self.sbuf, self.pos, self.terr,
                      stream)

    def check(self, label: str):
        """Every document's flags, and words and strings where the tape is
        defined, against the oracle's tape of that document alone."""
        import torch
        torch.cuda.synchronize()
        oi, on, _ = oracle.index_batch(np.frombuffer(self.data, dtype=np.uint8), self.offs)
        assert np.array_equal(self.cnt.cpu().numpy().view(np.uint32), on), f"{label}: counts"
        words = self.words.cpu().numpy().view(np.uint64)
        sbuf = self.sbuf.cpu().numpy().tobytes()
        pos = self.pos.cpu().numpy().view(np.uint64).reshape(-1, 4)
        terr = self.terr.cpu().numpy().view(np.uint32)
        serr = self.serr.cpu().numpy().view(np.uint32)
        compared = 0
        for d in range(self.offs.size - 1):
            a, b = int(self.offs[d]), int(self.offs[d + 1])
            doc = self.data[a:b]
            ow, osb, of = oracle.tape(doc, oi[a:a + on[d]])
            assert terr[d] == of, f"{label}: document {d} flags {terr[d]:#x} != {of:#x}"
            if of == 0 and serr[d] == 0:
                w0, nw, s0, ns = (int(x) for x in pos[d])
                assert nw == ow.size and np.array_equal(words[w0:w0 + nw], ow), f"{label}: document {d} words"
                assert sbuf[s0:s0 + ns] == osb, f"{label}: document {d} strings"
                compared += 1
        return compared


def test_tape_batch_mixed_documents():
    """Numbers (exact-path ones too), strings with escapes, literals, errors,
    empty documents and documents of more than a chunk, in one batch."""
    rng = random.Random(23)
    singles = ["1", "-0", "0.5", '"x"', "true", "null", "[]", "{}", '{"a":[1,2,{"b":null}],"c":"\\u00e9\\ud83d\\ude00"}',
               "[01]", "[1.]", '["\\x"]', "[tru]", "[1e309]", '["a\\u12"]', '["\\ud800"]', "[-]",
               "[9223372036854775808]", "[-9223372036854775808, 9223372036854775807]", '"unclosed', "[1, 2", "",
               "  ", "[2.2250738585072011e-308, 1.7976931348623157e308, 0.1, 123456789012345678901234567890]"]

    def val(dp):
        r = rng.random()
        if dp > 5 or r < 0.45:
            return rng.choice([1, -7, 2.5e-7, 1e300, "s\\\"q", "café", None, True, False, 12345678901234])
        if r < 0.7:
            return [val(dp + 1) for _ in range(rng.randrange(0, 5))]
        return {f"k{i}": val(dp + 1) for i in range(rng.randrange(0, 5))}

    docs = []
    for k in range(4000):
        docs.append(rng.choice(singles).encode() if k % 4 == 0 else json.dumps(val(0), ensure_ascii=k % 3 == 0).encode())
    for p in (7, 2000, 3999):
        docs.insert(p, json.dumps([val(0) for _ in range(3000)]).encode())
    data = b"".join(docs)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in docs], out=offs[1:])
    _say(f"case: tape batch mixed, {len(docs)} documents, {len(data)} bytes")
    b = _Batch(data, offs)
    b.run()
    assert b.check("mixed") > 2500


def test_tape_batch_full_c3():
    """The whole C3 batch (100,000 documents, 1% corrupted)."""
    from paper_1902_08318_amd import synth
    data, offs, _ = synth.gen_c3(3)
    _say(f"case: tape batch C3, {offs.size - 1} documents, {len(data)} bytes")
    b = _Batch(data, offs)
    b.run()
    assert b.check("C3") > 90000


def test_tape_batch_capacity_flag():
    docs = [b"[1,2]", b'{"a":"b"}', b"[[[]]]"]
    data = b"".join(docs)
    offs = np.array([0, 5, 14, 20], dtype=np.uint64)
    _say("case: tape batch over its output capacity")
    b = _Batch(data, offs, tape_cap=4)
    b.run()
    import torch
    torch.cuda.synchronize()
    assert np.all(b.terr.cpu().numpy().view(np.uint32) == 0x80000000)


def test_tape_batch_replayed_from_graph():
    """After jsidx_tape_reserve the batched tape is captured in a HIP graph and
    replayed on new batches (index and links rebuilt eagerly between replays,
    same document count); every replay equals an eager call and the oracle."""
    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    dev = torch.device("cuda:0")
    ndocs, cap = 500, 4 << 20
    batches = []
    for sd in (51, 52, 53):
        data, o, _ = synth.gen_c3(sd, ndocs=ndocs, pool=80, median=1024, hi=16384, corrupt_frac=0.05)
        assert int(o[-1]) <= cap
        batches.append((data, o))
    s = torch.cuda.Stream()
    b = _Batch.__new__(_Batch)
    b.buf = torch.zeros(cap, dtype=torch.uint8, device=dev)
    b.o = torch.zeros(ndocs + 1, dtype=torch.int64, device=dev)
    b.idx = torch.zeros(cap, dtype=torch.int32, device=dev)
    b.cnt = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    b.match = torch.zeros(cap, dtype=torch.int32, device=dev)
    b.serr = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    b.words = torch.zeros(2 * (cap + ndocs), dtype=torch.int64, device=dev)
    b.sbuf = torch.zeros(3 * cap + 4, dtype=torch.uint8, device=dev)
    b.pos = torch.zeros(4 * ndocs, dtype=torch.int64, device=dev)
    b.terr = torch.zeros(ndocs, dtype=torch.int32, device=dev)
    err = torch.zeros(ndocs, dtype=torch.int32, device=dev)

    def load(k):
        data, o = batches[k]
        b.data, b.offs = data, o
        b.buf[:len(data)].copy_(torch.frombuffer(bytearray(data), dtype=torch.uint8))
        b.o.copy_(torch.from_numpy(o.astype(np.int64)))
        jx.build_batch(b.buf, b.o, b.idx, b.cnt, err, s)
        jx.scopes_batch(b.buf, b.o, b.idx, b.cnt, b.match, b.serr, s)
        b.words.fill_(-1)
        b.terr.fill_(-1)
        b.pos.fill_(-1)

    with torch.cuda.stream(s):
        jx.reserve(cap, s)
        jx.scopes_reserve(cap, ndocs, s)
        jx.tape_reserve(cap, ndocs, s)
        load(0)
        b.run(s)  # eager warm-up on the capture stream
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(s)
    for r in range(4):
        k = r % len(batches)
        _say(f"case: tape batch graph replay {r} (batch {k})")
        with torch.cuda.stream(s):
            load(k)
            b.run(s)
        s.synchronize()
        e_w, e_p, e_e = b.words.clone(), b.pos.clone(), b.terr.clone()
        with torch.cuda.stream(s):
            b.words.fill_(-1)
            b.terr.fill_(-1)
            b.pos.fill_(-1)
        s.synchronize()
        g.replay()
        s.synchronize()
        assert torch.equal(b.terr, e_e) and torch.equal(b.pos, e_p), f"replay {r}"
        last = e_p.view(-1, 4)[-1]
        tw = int(last[0].item() + last[1].item())
        assert torch.equal(b.words[:tw], e_w[:tw]), f"replay {r}: words"
        assert b.check(f"replay {r}") > 0
