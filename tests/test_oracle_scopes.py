"""Pins of the oracle's scope matching over the structural index (the scope
links of the paper's tape, Fig. 2).

From outside the oracle: Python's json decoder, started at an opening bracket,
returns the end of that value, so the closing bracket of the scope is the byte
before it; a generator that builds bracket sequences knows the pairs it built.
"""
import json
import os
import random

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNLINKED = 0xFFFFFFFF


def _pairs_by_decoder(text: str, idx: np.ndarray) -> dict:
    """Opening-bracket entry -> closing-bracket entry, from json's raw_decode
    (text is ASCII, so character and byte offsets agree)."""
    pos_to_entry = {int(p): i for i, p in enumerate(idx)}
    dec = json.JSONDecoder()
    out = {}
    for i, p in enumerate(idx):
        if text[int(p)] in "{[":
            _, end = dec.raw_decode(text, int(p))
            out[i] = pos_to_entry[end - 1]
    return out


def _value(rng, depth=0):
    r = rng.random()
    if depth > 5 or r < 0.35:
        return rng.choice([1, -2.5, True, None, "a]b", "{[", "x\"y}", "\\]"])
    if r < 0.7:
        return [_value(rng, depth + 1) for _ in range(rng.randrange(0, 5))]
    return {f"k{i}]": _value(rng, depth + 1) for i in range(rng.randrange(0, 5))}


def test_scope_links_agree_with_the_json_decoder():
    rng = random.Random(11)
    for trial in range(300):
        obj = _value(rng)
        for kw in ({"separators": (",", ":")}, {"indent": 2}):
            text = json.dumps(obj, ensure_ascii=True, **kw)
            data = text.encode()
            idx, _ = oracle.index(data)
            match, err = oracle.scopes(data, idx)
            assert err == 0
            pairs = _pairs_by_decoder(text, idx)
            for i, k in pairs.items():
                assert match[i] == k and match[k] == i, (trial, text[:80])
            linked = set(pairs) | set(pairs.values())
            for i in range(idx.size):
                if i not in linked:
                    assert match[i] == UNLINKED


def test_fig1_document_scopes():
    text = open(os.path.join(GOLDEN, "paper_fig1_document.json"), encoding="utf-8").read()
    data = text.encode()
    idx, _ = oracle.index(data)
    match, err = oracle.scopes(data, idx)
    assert err == 0
    # the document is ASCII, so the decoder's offsets are byte offsets
    pairs = _pairs_by_decoder(text, idx)
    assert len(pairs) == 3   # the root object, Thumbnail, IDs
    for i, k in pairs.items():
        assert match[i] == k and match[k] == i


def test_generated_bracket_sequences():
    """Sequences built as balanced trees (the builder records each pair),
    with atoms between; the oracle must find exactly the built pairs."""
    rng = random.Random(5)
    for trial in range(300):
        toks, pairs = [], []

        def build(depth):
            for _ in range(rng.randrange(0, 4)):
                if depth < 6 and rng.random() < 0.5:
                    kind = rng.choice("{[")
                    a = len(toks)
                    toks.append(kind)
                    build(depth + 1)
                    pairs.append((a, len(toks)))
                    toks.append("}" if kind == "{" else "]")
                else:
                    toks.append("1")
        build(0)
        data = " ".join(toks).encode()
        idx, _ = oracle.index(data)
        assert idx.size == len(toks)
        match, err = oracle.scopes(data, idx)
        assert err == 0
        for a, b in pairs:
            assert match[a] == b and match[b] == a


def test_unbalanced_and_mismatched():
    def run(d):
        idx, _ = oracle.index(d)
        return oracle.scopes(d, idx)
    m, e = run(b"[}")
    assert e == oracle.ERR_MISMATCHED and list(m) == [1, 0]
    m, e = run(b"]")
    assert e == oracle.ERR_UNBALANCED and list(m) == [UNLINKED]
    m, e = run(b"[[")
    assert e == oracle.ERR_UNBALANCED and list(m) == [UNLINKED, UNLINKED]
    m, e = run(b"[ ] ]")
    assert e == oracle.ERR_UNBALANCED and list(m) == [1, 0, UNLINKED]
    m, e = run(b'"[" ]')                      # a bracket inside a string is not indexed
    assert e == oracle.ERR_UNBALANCED and list(m) == [UNLINKED, UNLINKED]
    m, e = run(b"{ [ } ]")
    assert e == oracle.ERR_MISMATCHED and list(m) == [3, 2, 1, 0]
    m, e = run(b"")
    assert e == 0 and m.size == 0
