"""The tape kernels (jsidx_tape.h), run on the CPU through the emulated
primitives, against the oracle's tape: words, string buffer and flags."""
import json
import os
import random
import struct

import numpy as np

import emu
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(data: bytes, exact_groups: int = 2, doc_shift: int = 0, str_shift: int = 0, paths=None) -> int:
    """Returns how many numbers took the exact conversion."""
    idx, _ = oracle.index(data)
    match, serr = oracle.scopes(data, idx)
    words, sbuf, flags, viol, nexact = emu.tape(data, idx, match, exact_groups, doc_shift, str_shift, paths)
    ow, osb, of = oracle.tape(data, idx)
    assert viol == 0
    assert flags == of, (hex(flags), hex(of), data[:80])
    if of == 0 and serr == 0 and oracle.structure(data, idx) == 0:
        assert words.size == ow.size, (words.size, ow.size)
        bad = np.nonzero(words != ow)[0]
        assert bad.size == 0, (int(bad[0]), hex(int(words[bad[0]])), hex(int(ow[bad[0]])), data[:80])
        assert sbuf == osb
    return nexact


def test_fig1_document():
    _check(open(os.path.join(GOLDEN, "paper_fig1_document.json"), "rb").read())


def test_small_values_and_errors():
    for t in ("1", "-0", "0.5", '"x"', "true", "null", "[]", "{}", '{"a":[1,2,{"b":null}],"c":"\\u00e9\\ud83d\\ude00"}',
              "[01]", "[1.]", '["\\x"]', "[tru]", "[1e309]", '["a\\u12"]', '["\\ud800"]', "[-]", "[9223372036854775808]",
              "[-9223372036854775808, 9223372036854775807]", '"unclosed', "[1, 2"):
        _check(t.encode())


def _numbers(rng, count):
    out = []
    for _ in range(count):
        digits = "".join(rng.choice("0123456789") for _ in range(rng.randrange(1, 30))).lstrip("0") or "0"
        frac = "" if rng.random() < 0.3 else "." + "".join(rng.choice("0123456789")
                                                          for _ in range(rng.randrange(1, 25)))
        exp = "" if rng.random() < 0.3 else "e" + rng.choice(["", "+", "-"]) + str(rng.randrange(0, 340))
        out.append(rng.choice(["", "-"]) + digits + frac + exp)
    return out


def test_numbers_in_bulk():
    """Numbers of every shape in arrays (several chunks): random digit counts
    and exponents over the whole double range, doubles printed with 17
    digits, and inputs whose rounding the fast conversion cannot decide
    (halfway points, subnormals, very long mantissas)."""
    rng = random.Random(21)
    nums = _numbers(rng, 2500)
    nums += [repr(struct.unpack("<d", struct.pack("<Q", rng.getrandbits(63)))[0]) for _ in range(1500)]
    nums = [x for x in nums if x not in ("nan", "inf")]
    hard = ["9007199254740993", "9007199254740993.0", "2.2250738585072011e-308", "2.2250738585072012e-308",
            "4.9406564584124654e-324", "2.4703282292062327e-324", "2.4703282292062328e-324", "1e-400",
            "1.7976931348623157e308", "1.7976931348623158e308", "1.7976931348623159e308", "1e23", "0.1",
            "123456789012345678901234567890e-10", "7.2057594037927933e16", "1" + "0" * 400 + "e-400",
            "0." + "0" * 400 + "1e400", "9007199254740992.5", "9007199254740993.000000000000000000001",
            "2.470328229206232720882e-324", "5e-324", "3e-324", "1.00000000000000011102230246251565404236316680908203125",
            "1.00000000000000011102230246251565404236316680908203124", "1.00000000000000011102230246251565404236316680908203126",
            "7.9228162514264337593543950335e28", "8.98846567431157953864652595394512366e307"]
    for k in range(0, 60):  # exact halfway points between consecutive doubles
        x = struct.unpack("<d", struct.pack("<Q", rng.getrandbits(62) + (1 << 61)))[0]
        y = np.nextafter(x, np.inf)
        from decimal import Decimal, getcontext
        getcontext().prec = 1000
        hard.append(str((Decimal(x) + Decimal(float(y))) / 2))
    data = ("[" + ",".join(nums + hard) + "]").encode()
    assert _check(data, exact_groups=3) >= 30  # most halfway points need the exact path
    assert _check(("[" + ",".join(hard) + "]").encode()) >= 30


def test_random_documents_across_chunks():
    rng = random.Random(4)

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
                           for _ in range(rng.randrange(0, 6)))
        if r < 0.7:
            return [val(d + 1) for _ in range(rng.randrange(0, 6))]
        return {f"k{i}é": val(d + 1) for i in range(rng.randrange(0, 6))}

    items = []
    while True:
        items.append(val(0))
        text = json.dumps(items, ensure_ascii=rng.random() < 0.5)
        if oracle.index(text.encode())[0].size > 2 * 4096 + 200:
            break
    _check(text.encode())
    _check(text.replace("true", "tru", 1).encode())
    _check(text.replace('"', '"\\q', 1).encode())


def test_number_conversions_against_python_float():
    """Both device conversions on their own, number by number: the fast one
    must be exact whenever it decides, the exact one always (CPython's float()
    is correctly rounded)."""
    rng = random.Random(77)
    texts = _numbers(rng, 4000)
    texts += [repr(struct.unpack("<d", struct.pack("<Q", rng.getrandbits(63)))[0]) for _ in range(2000)]
    texts = [t for t in texts if t not in ("nan", "inf")]
    from decimal import Decimal, getcontext
    getcontext().prec = 1200
    for _ in range(300):  # halfway points and their neighbours, subnormal ones too
        x = struct.unpack("<d", struct.pack("<Q", rng.getrandbits(63)))[0]
        if not np.isfinite(x) or x == 0:
            continue
        y = float(np.nextafter(x, np.inf))
        if not np.isfinite(y):
            continue
        mid = (Decimal(x) + Decimal(y)) / 2
        ulp = Decimal(y) - Decimal(x)
        texts += [str(mid), str(mid + ulp / 10 ** 30), str(mid - ulp / 10 ** 30)]
    for b in range(1, 200):  # subnormals
        texts.append(str(Decimal(struct.unpack("<d", struct.pack("<Q", rng.randrange(1, 1 << 52)))[0])))
    undecided = 0
    for t in texts:
        f = float(t)
        want = struct.unpack("<Q", struct.pack("<d", abs(f)))[0]
        r, bits = emu.number(t, exact=True)
        if np.isinf(f):
            assert r == 1, t
        else:
            assert r == 0 and bits == want, (t, hex(bits), hex(want))
        r, bits = emu.number(t, exact=False)
        if r == 2:
            undecided += 1
        elif np.isinf(f):
            assert r == 1, t
        else:
            assert r == 0 and bits == want, ("fast", t, hex(bits), hex(want))
    assert undecided >= 300


def test_long_strings_finished_by_the_wave():
    """Strings longer than a thread's budget (finished by the whole wave),
    with escapes, \\u sequences and surrogate pairs at every offset, errors
    deep inside, and a long string left open at the end."""
    rng = random.Random(31)
    pieces = ["a", "bc", " ", "\\\"", "\\\\", "\\n", "\\u00e9", "\\ud83d\\ude00", "é", "日本", "x" * 20, "\\/"]
    strs = []
    for _ in range(70):
        strs.append('"' + "".join(rng.choice(pieces) for _ in range(rng.randrange(1, 120))) + '"')
    doc = "[" + ",".join(strs) + "]"
    _check(doc.encode())
    bad = strs[:]
    bad[7] = bad[7][:-10] + "\x01" + bad[7][-10:]     # a control byte deep inside
    bad[11] = bad[11][:-5] + "\\q" + bad[11][-5:]    # an unknown escape
    _check(("[" + ",".join(bad) + "]").encode())
    _check(("[" + ",".join(strs[:50]) + ', "' + "y" * 300).encode())  # never closed


def test_string_sizes_around_2_16_bytes():
    """Strings whose buffer bytes (4 + decoded length) lie just below, at and
    above 2^16, with and without escapes."""
    strs = ['"' + "a" * k + '"' for k in (65530, 65531, 65532, 70000)]
    strs.insert(2, '"' + "\\u00e9" * 2 + "é" * 32764 + '"')   # 65532 bytes decoded
    strs.append('"' + "\\n" * 70000 + '"')                     # escapes: 70000 bytes decoded
    doc = "[" + ", ".join(strs + ['"short"', "1", "true"]) + "]"
    _check(doc.encode())


def test_strings_staged_at_every_alignment():
    """The string passes stage each group's bytes and output in LDS with
    16-byte blocks: documents and string buffers at every offset from a
    16-byte boundary, strings starting on the document's first bytes, groups
    whose bytes (and output) run past what is staged, strings longer than
    the staged bytes, an escape or a surrogate pair across a block edge."""
    rng = random.Random(33)
    pieces = ["a", "bc", "\\\"", "\\\\", "\\n", "\\u00e9", "\\ud83d\\ude00", "é", "日本", "x" * 13, "\\/", "\\t"]

    def s(lo, hi):
        return '"' + "".join(rng.choice(pieces) for _ in range(rng.randrange(lo, hi))) + '"'

    docs = [
        s(0, 40),                                                            # a lone string at byte 0
        "[" + ",".join(s(0, 12) for _ in range(300)) + "]",                  # many short strings per group
        "[" + ",".join(s(300, 900) for _ in range(12)) + "]",                # groups far longer than staged
        "{" + ",".join(f"{s(1, 4)}:{s(0, 60)}" for _ in range(200)) + "}",   # keys and values
        "[" + ",".join(s(0, 8) if i % 5 else str(i * 7) for i in range(400)) + "]",
    ]
    for k, d in enumerate(docs):
        for shift in (0, 3, 9, 15):
            _check(d.encode(), doc_shift=shift, str_shift=(shift * 5 + k) % 16)


def test_strings_byte_parallel_and_per_string_paths():
    """Runs of valid strings take the byte-parallel path, also with \\u
    sequences and surrogate pairs running across 16-byte lanes and 1 KiB
    steps; a run holding a control byte, a bad escape or an unclosed string
    takes the per-string path; both give the oracle's tape.  Backslash runs
    of every length across lane and step edges, escaped quotes, UTF-8 and
    strings crossing steps take the fast path."""
    rng = random.Random(35)
    words = ["a", "bc", "\\\"", "\\\\", "\\n", "é", "日本", "x" * 13, "\\/", "\\t", "\\" * 7 + "\"", "😀"]

    def s(lo, hi):
        return '"' + " ".join(rng.choice(words) for _ in range(rng.randrange(lo, hi))) + '"'

    valid = "[" + ",".join(s(0, 8) if i % 7 else s(100, 400) for i in range(700)) + "]"
    paths = []
    _check(valid.encode(), paths=paths)
    fast, slow = paths[-1]
    assert fast > 0 and slow == 0, paths[-1]
    # \u escapes and surrogate pairs at every offset from a lane edge
    uni = "[" + ",".join('"' + "ab" * rng.randrange(0, 9) + "\\u00e9" + "c" * rng.randrange(0, 7) + "\\ud83d\\ude00"
                         + "\\u4e2d" * rng.randrange(0, 3) + '"' for _ in range(600)) + "]"
    _check(uni.encode(), paths=paths)
    assert paths[-1][0] > 0 and paths[-1][1] == 0, paths[-1]
    for bad_u in ("\\ud83d\\u0041", "\\ude00", "\\u12g4"):  # a high surrogate alone, a low one alone, bad hex
        _check(uni.replace("\\u00e9", bad_u, 1).encode(), paths=paths)
        assert paths[-1][1] >= 1, paths[-1]
    for bad in (valid.replace("bc", "b\x01c", 1), valid.replace("\\n", "\\q", 1), valid[:-2]):
        _check(bad.encode(), paths=paths)
        assert paths[-1][1] >= 1, paths[-1]


def _check_batch(docs, **kw):
    """The batched tape kernels against the oracle's tape of each document
    alone: flags always, words and strings for documents whose tape is
    defined (valid structure, no flag)."""
    data = b"".join(docs)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in docs], out=offs[1:])
    oi, on, _ = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    match = np.full(max(1, int(offs[-1])), 0xFFFFFFFF, dtype=np.uint32)
    valid = []
    for d in range(len(docs)):
        a = int(offs[d])
        ix = oi[a:a + on[d]]
        m, se = oracle.scopes(docs[d], ix)
        match[a:a + on[d]] = m
        valid.append(se == 0 and oracle.structure(docs[d], ix) == 0)
    words, sbuf, pos, err, viol = emu.tape_batch(data, offs, oi, on, match, **kw)
    assert viol == 0
    for d in range(len(docs)):
        a = int(offs[d])
        ow, osb, of = oracle.tape(docs[d], oi[a:a + on[d]])
        assert err[d] == of, (d, hex(err[d]), hex(of), docs[d][:60])
        if of == 0 and valid[d]:
            w0, nw, s0, ns = (int(x) for x in pos[d])
            assert nw == ow.size, (d, nw, ow.size)
            assert np.array_equal(words[w0:w0 + nw], ow), (d, docs[d][:60])
            assert sbuf[s0:s0 + ns] == osb, d
    return pos


def test_batch_of_documents():
    """Documents of every kind in one batch: numbers (with exact-path ones),
    strings with escapes, literals, errors, empty documents and one larger
    than a chunk of 4096 entries; fewer workgroups than chunks."""
    rng = random.Random(21)
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
    for k in range(120):
        if k % 4 == 0:
            docs.append(rng.choice(singles).encode())
        else:
            docs.append(json.dumps(val(0), ensure_ascii=k % 3 == 0).encode())
    docs.insert(50, json.dumps([val(0) for _ in range(1500)]).encode())
    pos = _check_batch(docs, chunk_groups=2, doc_groups=3, exact_groups=2)
    assert int(pos[:, 1].sum()) > 4096


def test_batch_capacity_flag():
    docs = [b"[1,2]", b'{"a":"b"}', b"[[[]]]"]
    data = b"".join(docs)
    offs = np.array([0, 5, 14, 20], dtype=np.uint64)
    oi, on, _ = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    match = np.full(20, 0xFFFFFFFF, dtype=np.uint32)
    _, _, _, err, viol = emu.tape_batch(data, offs, oi, on, match, tape_cap=4)
    assert viol == 0 and np.all(err == 0x80000000)
    _, _, _, err, viol = emu.tape_batch(data, offs, oi, on, match, cap=int(on.sum()) - 1)
    assert viol == 0 and np.all(err == 0x80000000)


def test_batch_of_many_documents():
    """More documents than one workgroup of the per-document scan takes (2048),
    empty ones (a placeholder entry each) among them."""
    rng = random.Random(22)
    pool = [b"", b"1", b"[]", b"[1,[2.5]]", b'{"a":{"b":"c\\n"}}', b"tru", b'"x"', b"  ", b"[1e400]"]
    _check_batch([rng.choice(pool) for _ in range(5000)], chunk_groups=2, doc_groups=4, exact_groups=2)
