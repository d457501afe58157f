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


def _oracle_batch(data: bytes, offs: np.ndarray):
    """The oracle per document: (index in batch layout, counts, expected links
    in batch layout, expected flags)."""
    oi, on, _ = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    em = np.full(max(1, int(offs[-1])), 0xFFFFFFFF, dtype=np.uint32)
    ee = np.zeros(offs.size - 1, dtype=np.uint32)
    for d in range(offs.size - 1):
        a, b = int(offs[d]), int(offs[d + 1])
        ix = oi[a:a + on[d]]
        m, e = oracle.scopes(data[a:b], ix)
        ee[d] = e | oracle.structure(data[a:b], ix)
        em[a:a + on[d]] = m
    return oi, on, em, ee


def _check_batch(docs, **kw):
    data = b"".join(docs)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in docs], out=offs[1:])
    oi, on, em, ee = _oracle_batch(data, offs)
    m, e, v = emu.scopes_batch(data, offs, oi, on, **kw)
    assert v == 0
    assert np.array_equal(e, ee), [(d, hex(e[d]), hex(ee[d])) for d in np.nonzero(e != ee)[0][:5]]
    for d in range(len(docs)):
        a = int(offs[d])
        assert np.array_equal(m[a:a + on[d]], em[a:a + on[d]]), d
    return data, offs, on


def test_batch_of_documents():
    """A batch in the batched scope kernels: small valid and invalid
    documents, empty ones, documents that straddle chunk edges of the
    virtual sequence, one of more than a chunk (its scopes leave their
    chunk), unclosed openers whose search must stop at their document's
    end, and fewer workgroups than chunks and documents."""
    rng = random.Random(11)
    small = [b"", b"1", b"[]", b"{}", b"[}", b"]", b"[[", b"[ ] ]", b'{"a":[1,{"b":[]}]}', b"{ [ } ]",
             b"]]]][[[[", b"[" * 50 + b"]" * 49, b'{"a":1,"b":[2,3]}', b'[1,2', b'{"k" 1}', b",", b'"s"', b"  "]

    def val(dp):
        r = rng.random()
        if dp > 6 or r < 0.4:
            return rng.choice([1, "s]", None, True])
        if r < 0.7:
            return [val(dp + 1) for _ in range(rng.randrange(0, 5))]
        return {f"k{i}": val(dp + 1) for i in range(rng.randrange(0, 5))}

    docs = []
    for k in range(160):
        if k % 3 == 0:
            docs.append(rng.choice(small))
        else:
            d = json.dumps(val(0), separators=(",", ":")).encode()
            if k % 7 == 0 and len(d) > 2:
                d = d[:-1]  # unclosed
            docs.append(d)
    big = json.dumps([val(0) for _ in range(900)], separators=(",", ":")).encode()
    docs.insert(40, big)
    docs.insert(90, big[:-1])
    _, _, on = _check_batch(docs, chunk_groups=2, doc_groups=3, far_groups=2)
    assert int(on.sum()) > 3 * 4096 and int(on.max()) > 4096


def test_batch_capacity_flag():
    docs = [b"[1,2]", b'{"a":[]}', b"[[[]]]"]
    data = b"".join(docs)
    offs = np.array([0, 5, 13, 19], dtype=np.uint64)
    oi, on, _, _ = _oracle_batch(data, offs)
    m, e, v = emu.scopes_batch(data, offs, oi, on, cap=int(on.sum()) - 1)
    assert v == 0 and np.all(e == 0x80000000)


def test_batch_of_many_documents():
    """More documents than one workgroup of the per-document scan takes (2048):
    the scan's group sums and bases, with empty documents among them."""
    rng = random.Random(12)
    pool = [b"", b"1", b"[]", b"[1,[2]]", b'{"a":{}}', b"]", b"[[", b'"x"']
    docs = [rng.choice(pool) for _ in range(5000)]
    _check_batch(docs, chunk_groups=2, doc_groups=4, far_groups=2)
