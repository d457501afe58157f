"""The scope-link kernels (jsidx_scopes.h), run on the CPU through the
emulated primitives, against the oracle's bracket stack and structure check."""
import itertools
import json
import random

import numpy as np

import emu
import oracle


def _check(data: bytes, far_groups: int = 2):
    idx, _ = oracle.index(data)
    m, e, v = emu.scopes(data, idx, far_groups)
    om, oe = oracle.scopes(data, idx)
    oe |= oracle.structure(data, idx)
    assert v == 0
    assert e == oe, (e, oe)
    assert np.array_equal(m, om)


def test_small_and_invalid():
    for d in (b"", b"1", b"[]", b"{}", b"[}", b"]", b"[[", b"[ ] ]", b'{"a":[1,{"b":[]}]}', b"{ [ } ]",
              b"]]]][[[[", b"[" * 50 + b"]" * 49):
        _check(d)


def test_scopes_across_chunks():
    """Documents with more than 4096 index entries, so that scopes leave their
    chunk (the root always does), deep nesting and unbalanced tails."""
    rng = random.Random(3)

    def val(d):
        r = rng.random()
        if d > 7 or r < 0.4:
            return rng.choice([1, "s]", None])
        if r < 0.7:
            return [val(d + 1) for _ in range(rng.randrange(0, 6))]
        return {f"k{i}": val(d + 1) for i in range(rng.randrange(0, 6))}

    items = []
    while True:  # a few chunks of 4096 entries (the emulation runs one thread per lane)
        items.append(val(0))
        big = json.dumps(items, separators=(",", ":")).encode()
        if oracle.index(big)[0].size > 3 * 4096 + 100:
            break
    _check(big, far_groups=3)
    _check(big[:-1])                    # the root never closes
    _check(big + b"]")                  # one closer too many
    _check(big.replace(b"}", b"]", 1))  # a mismatch somewhere early
    _check(b"[" * 2100 + b"1" + b"]" * 2100)   # depth 2100, the openers' closers in the next chunk
    _check(b"[" * 4200 + b"]" * 4000, far_groups=3)


TOKENS = ["{", "}", "[", "]", ":", ",", '"s"', "1"]


def test_structure_of_short_token_sequences():
    """Every sequence of up to two tokens, and a sample of longer ones."""
    for n in range(0, 3):
        for seq in itertools.product(TOKENS, repeat=n):
            _check(" ".join(seq).encode(), far_groups=1)
    rng = random.Random(23)
    for _ in range(12):
        seq = [rng.choice(TOKENS) for _ in range(rng.randrange(3, 8))]
        _check(" ".join(seq).encode(), far_groups=1)


def test_structure_edits_across_chunks():
    """A valid document of several chunks, then one structural edit at a time
    (a comma's scope is found outside its chunk, keys and values after it)."""
    rng = random.Random(8)
    items = []
    while True:
        items.append({f"k{i}": [i, {"x": "y"}] for i in range(rng.randrange(1, 5))})
        big = json.dumps(items, separators=(",", ":"))
        if oracle.index(big.encode())[0].size > 2 * 4096 + 300:
            break
    _check(big.encode(), far_groups=2)
    for at, old, new in ((0.3, ",", " "), (0.2, ":", ","), (0.9, ",", ":"), (0.01, "{", "[")):
        p = big.index(old, int(at * len(big)))
        _check((big[:p] + new + big[p + 1:]).encode(), far_groups=2)
    _check((big + " 1").encode())
