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
