"""Pins of the oracle's tape (Sec. 3, Fig. 2; stage 2, Sec. 3.2).

From outside the oracle: Fig. 2 prints the tape of the Fig. 1 document word by
word; Python's json module parses the same texts (a tape read back into Python
values must equal json.loads, floats bit for bit, since CPython's float() is
correctly rounded); the number and string rules of the paper decide the error
cases json.loads accepts (integers outside int64, 1e309, lone surrogates).
"""
import json
import math
import os
import random
import struct

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M56 = (1 << 56) - 1


def read_tape(words: np.ndarray, sbuf: bytes):
    """Python value of a tape (a reader written from the figure's layout)."""
    w = [int(x) for x in words]
    assert chr(w[0] >> 56) == "r" and (w[0] & M56) == len(w) - 1
    assert chr(w[-1] >> 56) == "r" and (w[-1] & M56) == 0

    def string(k):
        off = w[k] & M56
        n = struct.unpack_from("<I", sbuf, off)[0]
        return sbuf[off + 4:off + 4 + n].decode("utf-8")

    def value(k):  # (value, next word)
        tag = chr(w[k] >> 56)
        if tag == '"':
            return string(k), k + 1
        if tag == "l":
            return struct.unpack("<q", struct.pack("<Q", w[k + 1]))[0], k + 2
        if tag == "d":
            return struct.unpack("<d", struct.pack("<Q", w[k + 1]))[0], k + 2
        if tag in "tfn":
            return {"t": True, "f": False, "n": None}[tag], k + 1
        if tag in "[{":
            end = (w[k] & M56) - 1
            assert chr(w[end] >> 56) == ("]" if tag == "[" else "}") and (w[end] & M56) == k
            j = k + 1
            if tag == "[":
                out = []
                while j < end:
                    v, j = value(j)
                    out.append(v)
            else:
                out = {}
                while j < end:
                    key = string(j)
                    v, j = value(j + 1)
                    out[key] = v
            assert j == end
            return out, end + 1
        raise AssertionError(f"bad tag {tag!r} at {k}")

    v, k = value(1)
    assert k == len(w) - 1
    return v


def tape_of(text):
    data = text.encode("utf-8") if isinstance(text, str) else text
    idx, _ = oracle.index(data)
    return oracle.tape(data, idx)


def same(a, b):
    """Equal as JSON values, floats bit for bit (and never int == float)."""
    if isinstance(a, float) or isinstance(b, float):
        return type(a) is type(b) and struct.pack("<d", a) == struct.pack("<d", b)
    if isinstance(a, list):
        return isinstance(b, list) and len(a) == len(b) and all(same(x, y) for x, y in zip(a, b))
    if isinstance(a, dict):
        return isinstance(b, dict) and list(a) == list(b) and all(same(a[k], b[k]) for k in a)
    return type(a) is type(b) and a == b


def test_fig2_tape_of_the_fig1_document():
    text = open(os.path.join(GOLDEN, "paper_fig1_document.json"), encoding="utf-8").read()
    words, sbuf, flags = tape_of(text)
    assert flags == 0
    w = [int(x) for x in words]
    rows = [ln.split(" ", 2) for ln in open(os.path.join(GOLDEN, "paper_fig2_tape_words.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(w) == int(rows[-1][0]) + 1
    for pos, kind, *rest in rows:
        k = int(pos)
        word = w[k]
        arg = rest[0].strip() if rest else ""
        if kind in ("r", "{", "}", "[", "]"):
            assert chr(word >> 56) == kind and (word & M56) == int(arg), (k, kind)
        elif kind == "string":
            off = word & M56
            n = struct.unpack_from("<I", sbuf, off)[0]
            assert chr(word >> 56) == '"' and sbuf[off + 4:off + 4 + n].decode() == arg
        elif kind == "integer":
            assert chr(word >> 56) == "l" and w[k + 1] == int(arg)
        else:
            assert word == ord(kind[0]) << 56, (k, kind)
    # the string buffer: a 32-bit length, then the bytes, entry after entry
    assert sbuf[:9] == struct.pack("<I", 5) + b"Width"


def _value(rng, depth=0):
    r = rng.random()
    if depth > 4 or r < 0.45:
        k = rng.randrange(7)
        if k == 0:
            return rng.randrange(-(1 << 63), 1 << 63)
        if k == 1:
            return rng.choice([True, False, None])
        if k == 2:
            return struct.unpack("<d", struct.pack("<Q", rng.getrandbits(64)))[0]
        if k == 3:
            return rng.uniform(-1e6, 1e6)
        pieces = ["a", "b c", '"', "\\", "/", "\b", "\f", "\n", "\r", "\t", "\x01", "\x1f", "é", "日本", "\U0001F600",
                  " ", "\x7f", "\U0010FFFF"]
        return "".join(rng.choice(pieces) for _ in range(rng.randrange(0, 8)))
    if r < 0.7:
        return [_value(rng, depth + 1) for _ in range(rng.randrange(0, 6))]
    return {f"k{i}" + rng.choice(["", "é", "\\q", "\U0001F600"]): _value(rng, depth + 1)
            for i in range(rng.randrange(0, 6))}


def test_tapes_read_back_as_json_loads():
    rng = random.Random(12)
    checked = 0
    for trial in range(500):
        obj = _value(rng)
        for kw in ({"ensure_ascii": True}, {"ensure_ascii": False, "indent": 1}):
            try:
                text = json.dumps(obj, allow_nan=False, **kw)
            except ValueError:
                continue  # a random 64-bit pattern that is NaN or infinite
            words, sbuf, flags = tape_of(text)
            assert flags == 0, (trial, text[:100])
            assert same(read_tape(words, sbuf), json.loads(text)), (trial, text[:200])
            checked += 1
    assert checked > 900


def _number_texts(rng):
    for _ in range(3000):
        digits = "".join(rng.choice("0123456789") for _ in range(rng.randrange(1, 40))).lstrip("0") or "0"
        frac = "" if rng.random() < 0.3 else "." + "".join(rng.choice("0123456789")
                                                          for _ in range(rng.randrange(1, 25)))
        exp = "" if rng.random() < 0.3 else rng.choice("eE") + rng.choice(["", "+", "-"]) + str(rng.randrange(0, 400))
        yield rng.choice(["", "-"]) + digits + frac + exp
    # near halfway between doubles, subnormals, limits
    for t in ("9007199254740993", "9007199254740993.0", "2.2250738585072011e-308", "2.2250738585072012e-308",
              "4.9406564584124654e-324", "2.4703282292062327e-324", "2.4703282292062328e-324", "1e-400",
              "0.1e-999", "1.7976931348623157e308", "1.7976931348623158e308", "1e23", "8.98846567431158e307",
              "0.1", "0.2", "0.3", "123456789012345678901234567890e-10", "7.2057594037927933e16", "-0.0", "0e5",
              "1" + "0" * 400 + "e-400", "0." + "0" * 400 + "1e400"):
        yield t


def test_numbers_match_python_float_and_int():
    rng = random.Random(3)
    for t in _number_texts(rng):
        words, sbuf, flags = tape_of(t)
        is_int = all(c not in t for c in ".eE")
        if is_int:
            v = int(t)
            if -(1 << 63) <= v < (1 << 63):
                assert flags == 0 and chr(int(words[1]) >> 56) == "l", t
                assert struct.unpack("<q", struct.pack("<Q", int(words[2])))[0] == v, t
            else:
                assert flags == oracle.ERR_NUMBER, t
            continue
        f = float(t)
        if math.isinf(f):
            assert flags == oracle.ERR_NUMBER, t
        else:
            assert flags == 0 and chr(int(words[1]) >> 56) == "d", t
            assert int(words[2]) == struct.unpack("<Q", struct.pack("<d", f))[0], t


def test_integer_bounds_and_invalid_numbers():
    for t, ok in (("9223372036854775807", True), ("9223372036854775808", False), ("-9223372036854775808", True),
                  ("-9223372036854775809", False), ("-0", True), ("0", True), ("1e309", False), ("-1e309", False),
                  ("012", False), ("1E+", False), (".1", False), ("1.", False), ("-", False), ("--1", False),
                  ("1.5e+", False), ("1a", False), ("0x10", False), ("+1", False), ("1e5", True), ("-1.5E-3", True),
                  ("abc", False), ("1.e5", False), ("01.5", False)):
        _, _, flags = tape_of(t)
        assert (flags == 0) == ok, t
        if not ok:
            assert flags == oracle.ERR_NUMBER, t
    words, _, _ = tape_of("-0")
    assert chr(int(words[1]) >> 56) == "l" and int(words[2]) == 0


def test_strings_and_their_errors():
    for s in ('"plain"', r'"\"\\\/\b\f\n\r\t"', r'"Aé日😀"', '"é日本😀"', r'"\u0000x"',
              r'"a b"', '""'):
        words, sbuf, flags = tape_of(s)
        assert flags == 0, s
        assert read_tape(words, sbuf) == json.loads(s), s
    for s in ('"a\x01b"', '"\x1f"', r'"\x"', r'"\u12"', r'"\u12g4"', r'"\ud800"', r'"\udc00"', r'"\ud800A"',
              r'"\ud800x"', '"unclosed', '"ends with backslash\\'):
        _, _, flags = tape_of(s)
        assert flags == oracle.ERR_STRING, s


def test_literals():
    for t in ("true", "false", "null", "[true,false,null]", '{"a":null}'):
        words, sbuf, flags = tape_of(t)
        assert flags == 0 and same(read_tape(words, sbuf), json.loads(t)), t
    for t in ("tru", "truex", "nul", "nulll", "fals", "t", "[true1]"):
        _, _, flags = tape_of(t)
        assert flags == oracle.ERR_LITERAL, t


def test_flags_collect_every_atom_and_the_tape_needs_valid_structure():
    _, _, flags = tape_of('[tru, 01, "\\x", 5]')
    assert flags == oracle.ERR_LITERAL | oracle.ERR_NUMBER | oracle.ERR_STRING
    words, sbuf, flags = tape_of("[1, 2")      # structure invalid, atoms fine
    assert flags == 0 and words.size == 0 and sbuf == b""
    words, sbuf, flags = tape_of("7")
    assert flags == 0 and same(read_tape(words, sbuf), 7)
