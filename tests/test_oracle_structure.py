"""Pins of the oracle's structure check (the index entries' tokens must form one
JSON value; token contents are not checked).

Python's json parser decides: over every sequence of up to 5 tokens from
{ } [ ] : , "s" 1 true, separated by spaces (so that token contents are always
valid and never merge), json.loads accepts exactly the sequences the oracle
accepts; the same holds for structural edits of generated documents.
"""
import itertools
import json
import random

import oracle

TOKENS = ["{", "}", "[", "]", ":", ",", '"s"', "1", "true"]


def _json_ok(text: str) -> bool:
    try:
        json.loads(text)
        return True
    except ValueError:
        return False


def _structure_ok(data: bytes) -> bool:
    idx, _ = oracle.index(data)
    return oracle.structure(data, idx) == 0


def test_every_short_token_sequence():
    for n in range(0, 6):
        for seq in itertools.product(TOKENS, repeat=n):
            text = " ".join(seq)
            assert _structure_ok(text.encode()) == _json_ok(text), text


def test_structural_edits_of_generated_documents():
    rng = random.Random(17)

    def val(d):
        r = rng.random()
        if d > 5 or r < 0.4:
            return rng.choice([1, 25, True, None, "a b", "{x:[y,]}"])
        if r < 0.7:
            return [val(d + 1) for _ in range(rng.randrange(0, 5))]
        return {f"k{i}": val(d + 1) for i in range(rng.randrange(0, 5))}

    agree = 0
    for trial in range(400):
        text = json.dumps(val(0), indent=1)
        assert _structure_ok(text.encode())
        idx, _ = oracle.index(text.encode())
        # edit one token position outside strings: delete a structural byte,
        # replace it, or insert one (with spaces, so atoms never merge)
        p = int(rng.choice(list(idx))) if len(idx) else 0
        op = rng.randrange(3)
        ch = rng.choice("{}[]:,")
        if op == 0 and text[p] in "{}[]:,":
            edited = text[:p] + " " + text[p + 1:]
        elif op == 1 and text[p] in "{}[]:,":
            edited = text[:p] + ch + text[p + 1:]
        else:
            edited = text[:p] + " " + ch + " " + text[p:]
        ok = _json_ok(edited)
        assert _structure_ok(edited.encode()) == ok, (trial, edited[:120])
        agree += 1
    assert agree == 400


def test_hand_cases():
    for text, ok in (('{"a":1}', True), ("[1,2]", True), ("1", True), ("", False), ("1 2", False),
                     ("[1,]", False), ('{"a" 1}', False), ("{1:2}", False), ("[,1]", False), ('{"a":}', False),
                     ("[[]]", True), ('{"a":[{}]}', True), ('"s"', True), (":", False), ("[}", False),
                     ('{"a":1,}', False), ('{"a":1 "b":2}', False), ("]", False), ("[", False)):
        assert _structure_ok(text.encode()) == ok, text
