"""Pins of the oracle's minify (the paper's minified form: white-space
characters outside quotes omitted, dataset-size table of the evaluation).

The pins come from outside the oracle: Python's json module writes the same
value compact and indented, and only white space outside strings differs
between the two, so minifying the indented text must give the compact text
exactly; json.loads of a minified valid document equals that of the original.
"""
import itertools
import json
import random

import numpy as np

import oracle


def _value(rng: random.Random, depth: int = 0):
    r = rng.random()
    if depth > 4 or r < 0.3:
        k = rng.randrange(6)
        if k == 0:
            return rng.randrange(-10**12, 10**12)
        if k == 1:
            return rng.choice([True, False, None])
        if k == 2:
            return rng.uniform(-1e6, 1e6)
        pieces = [" ", "  ", "a", "b c", '"', "\\", "\t", "\n", "é", "日本", "\U0001F600", "x y\tz", ":", ",", "{", "]"]
        return "".join(rng.choice(pieces) for _ in range(rng.randrange(0, 8)))
    if r < 0.65:
        return [_value(rng, depth + 1) for _ in range(rng.randrange(0, 6))]
    return {("k " + str(i) + rng.choice(["", " \"q\"", "\\"])): _value(rng, depth + 1) for i in range(rng.randrange(0, 6))}


def test_indented_json_minifies_to_compact_json():
    rng = random.Random(7)
    for trial in range(400):
        obj = _value(rng)
        for ascii_only in (False, True):
            compact = json.dumps(obj, separators=(",", ":"), ensure_ascii=ascii_only).encode()
            for kw in ({"indent": 2}, {"indent": "\t"}, {}, {"indent": 1, "separators": (" ,  ", " :\r\n")}):
                text = json.dumps(obj, ensure_ascii=ascii_only, **kw).encode()
                assert oracle.minify(text) == (compact, 0), (trial, kw, text[:200])
            assert oracle.minify(compact) == (compact, 0)


def test_minified_documents_parse_to_the_same_value():
    from paper_1902_08318_amd import synth
    for seed in range(6):
        doc = synth.gen_c0(seed, 20000 + 5000 * seed).data
        m, flags = oracle.minify(doc)
        assert flags == 0
        assert json.loads(m) == json.loads(doc)
        assert len(m) < len(doc)
    doc = synth.gen_c1(3, 1 << 18, pool=32).data   # generated minified already
    assert oracle.minify(doc) == (doc, 0)


def test_strings_keep_their_white_space_and_escapes_decide_where_they_end():
    assert oracle.minify(b'"a \t\n b"') == (b'"a \t\n b"', 0)
    assert oracle.minify(b'"a\\" b" c') == (b'"a\\" b"c', 0)        # escaped quote: still inside
    assert oracle.minify(b'"a\\\\" b') == (b'"a\\\\"b', 0)          # even run: the quote closes
    assert oracle.minify(b'[1, "x y" , 2 ]') == (b'[1,"x y",2]', 0)
    assert oracle.minify(b" \t\r\n ")[0] == b""
    assert oracle.minify(b"")[0] == b""
    assert oracle.minify(b'\\ a')[0] == b"\\a"                      # outside strings every space goes


def test_flags_equal_the_index_flags():
    """Minify reports the index's flags; EMPTY coincides because the first
    byte outside strings that is not white space is always indexed."""
    alpha = [b'"', b"\\", b" ", b"a", b"[", b"\t", b"\xc3", b"\xa9"]
    for n in range(0, 6):
        for t in itertools.product(alpha, repeat=n):
            d = b"".join(t)
            assert oracle.minify(d)[1] == oracle.index(d)[1], d


def test_batch_equals_single_documents():
    rng = np.random.default_rng(3)
    docs = []
    for _ in range(200):
        a = np.frombuffer(b'"\\[]{},: \tax1\n\xc3\xa9', dtype=np.uint8)
        docs.append(a[rng.integers(0, a.size, int(rng.integers(0, 300)))].tobytes())
    offs = np.concatenate([[0], np.cumsum([len(d) for d in docs])]).astype(np.uint64)
    out, n, err = oracle.minify_batch(b"".join(docs), offs)
    for d, doc in enumerate(docs):
        m, f = oracle.minify(doc)
        a = int(offs[d])
        assert n[d] == len(m) and err[d] == f
        assert out[a:a + n[d]].tobytes() == m
