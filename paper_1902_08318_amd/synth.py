"""Seeded synthetic JSON workloads (inputs only; no indexing arithmetic here).

The paper measures on public JSON files (twitter, canada, mesh, ...) that are
not available here; these generators produce documents with the same shapes:
minified record arrays rich in strings, escapes and non-ASCII text
(twitter-like), pretty-printed coordinate arrays of 17-digit doubles
(canada / mesh.pretty-like), and batches of small documents.

Every generator also returns the number of structural characters, strings
(keys included) and atoms (numbers, true, false, null) it emitted: for a valid
document, that sum is the size of its stage-1 index (one position per
structural character, per string start and per atom start).
"""
from __future__ import annotations

import json
from dataclasses import dataclass

import numpy as np

ASCII_WORDS = ["alpha", "beta", "gamma", "delta", "view", "from", "my", "room", "http://ex.com/img.png",
               "user", "name", "text", "id", "lorem", "ipsum", "dolor", "sit", "amet", "json", "stage"]
UTF8_WORDS = ["é", "ü", "ß", "€", "日本語", "中文", "한국어", "Ελληνικά", "русский", "\U0001F600",
              "\U0001D11E", "\U00010348", "ﬁ", "ñandú"]
ESCAPES = ['\\"', "\\\\", "\\n", "\\t", "\\/", "\\u00e9", "\\uD834\\uDD1E", "\\r", "\\b"]


@dataclass
class Doc:
    data: bytes
    expected_index: int  # structural + strings + atoms (valid documents)


class _Emitter:
    def __init__(self, rng: np.random.Generator, indent: int | None):
        self.rng = rng
        self.parts: list[str] = []
        self.size = 0
        self.count = 0  # structural + strings + atoms
        self.indent = indent

    def put(self, s: str, n_index: int = 0):
        self.parts.append(s)
        self.size += len(s.encode("utf-8")) if not s.isascii() else len(s)
        self.count += n_index

    def newline(self, depth: int):
        if self.indent is not None:
            self.put("\n" + " " * (self.indent * depth))

    # ---- values
    def string_body(self, p_escape: float, p_utf8: float, max_words: int = 6) -> str:
        rng = self.rng
        k = int(rng.integers(0, max_words + 1))
        words = []
        for _ in range(k):
            r = rng.random()
            if r < p_utf8:
                words.append(UTF8_WORDS[int(rng.integers(0, len(UTF8_WORDS)))])
            else:
                words.append(ASCII_WORDS[int(rng.integers(0, len(ASCII_WORDS)))])
        if rng.random() < p_escape:
            pos = int(rng.integers(0, len(words) + 1))
            words.insert(pos, ESCAPES[int(rng.integers(0, len(ESCAPES)))])
        return " ".join(words)

    def number(self) -> str:
        rng = self.rng
        if rng.random() < 0.5:
            return str(int(rng.integers(-(2**62), 2**62)))
        v = float(rng.normal()) * 10.0 ** int(rng.integers(-20, 20))
        s = repr(v)
        if rng.random() < 0.3 and "e" not in s:
            s = f"{v:.6e}"
        return s


def gen_c0(seed: int = 0, target: int = 1 << 20) -> Doc:
    """Pretty-printed (2-space) document, root object, depth <= 8, arrays of 0-50
    elements; values 40% strings (5% with escapes, 10% with 2-4 byte UTF-8),
    30% numbers (int64 and doubles with exponents), 15% true/false/null, 15%
    nested.  Grows until `target` bytes, then closes its scopes."""
    rng = np.random.default_rng(seed)
    em = _Emitter(rng, indent=2)
    # stack entries: [kind ('{' or '['), remaining elements, emitted count]
    em.put("{", 1)
    stack = [["{", 10**9, 0]]
    while stack:
        top = stack[-1]
        depth = len(stack)
        if top[1] <= 0 or em.size >= target:
            stack.pop()
            em.newline(depth - 1)
            em.put("}" if top[0] == "{" else "]", 1)
            continue
        if top[2] > 0:
            em.put(",", 1)
        em.newline(depth)
        if top[0] == "{":
            key = em.string_body(0.05, 0.1, 2) or "k"
            em.put('"' + key + '"', 1)
            em.put(": ", 1)
        top[1] -= 1
        top[2] += 1
        r = rng.random()
        if r < 0.40:
            em.put('"' + em.string_body(0.05, 0.10) + '"', 1)
        elif r < 0.70:
            em.put(em.number(), 1)
        elif r < 0.85:
            em.put(["true", "false", "null"][int(rng.integers(0, 3))], 1)
        elif depth < 8:
            kind = "{" if rng.random() < 0.5 else "["
            em.put(kind, 1)
            stack.append([kind, int(rng.integers(0, 51)), 0])
        else:
            em.put("null", 1)
    data = "".join(em.parts).encode("utf-8")
    return Doc(data, em.count)


def _expected_from_value(v) -> int:
    """Index size of a value serialised by json.dumps (separators given)."""
    if isinstance(v, dict):
        return 2 + sum(1 + 1 + _expected_from_value(x) for x in v.values()) + max(0, len(v) - 1)
    if isinstance(v, list):
        return 2 + sum(_expected_from_value(x) for x in v) + max(0, len(v) - 1)
    return 1


def _record(rng: np.random.Generator, rid: int) -> dict:
    def text(n_max: int) -> str:
        parts = []
        total = 0
        lim = int(rng.integers(0, n_max + 1))
        while total < lim:
            r = rng.random()
            if r < 0.25:
                w = UTF8_WORDS[int(rng.integers(0, len(UTF8_WORDS)))]
            elif r < 0.32:
                w = '"quoted"'
            elif r < 0.38:
                w = "\\" * int(rng.integers(1, 6)) + ("x" if rng.random() < 0.5 else '"')
            else:
                w = ASCII_WORDS[int(rng.integers(0, len(ASCII_WORDS)))]
            parts.append(w)
            total += len(w) + 1
        return " ".join(parts)
    user = {
        "id": int(rng.integers(0, 2**63 - 1)),
        "name": text(20),
        "screen_name": text(12),
        "location": text(30),
        "description": text(160),
        "followers_count": int(rng.integers(0, 10**7)),
        "verified": bool(rng.random() < 0.1),
        "url": None if rng.random() < 0.5 else "http://ex.com/" + str(int(rng.integers(0, 10**6))),
    }
    rec = {
        "id": rid * 7919 + int(rng.integers(0, 7919)),
        "id_str": str(rid),
        "created_at": "Sun Aug 31 00:29:15 +0000 2014",
        "text": text(280),
        "source": '<a href="http://ex.com" rel="nofollow">client</a>',
        "truncated": bool(rng.random() < 0.5),
        "in_reply_to_status_id": None if rng.random() < 0.7 else int(rng.integers(0, 2**62)),
        "in_reply_to_user_id": None,
        "in_reply_to_screen_name": None,
        "user": user,
        "geo": None,
        "coordinates": None,
        "place": None,
        "contributors": None,
        "retweet_count": int(rng.integers(0, 10**5)),
        "favorite_count": int(rng.integers(0, 10**5)),
        "favorited": False,
        "retweeted": bool(rng.random() < 0.3),
        "lang": ["ja", "en", "zh", "es"][int(rng.integers(0, 4))],
        "hashtags": [text(10) for _ in range(int(rng.integers(0, 3)))],
        "possibly_sensitive": False,
        "score": float(rng.normal()),
        "quoted": text(40),
        "tags": [int(x) for x in rng.integers(0, 1000, int(rng.integers(0, 5)))],
        "metadata": {"iso_language_code": "ja", "result_type": "recent"},
        "filter_level": "low",
        "timestamp_ms": str(int(rng.integers(10**12, 10**13))),
        "reply": text(40),
        "extra": None,
    }
    return rec


def _pool_join(pieces: list[tuple[bytes, int]], rng: np.random.Generator, target: int,
               open_b: bytes, close_b: bytes, sep: bytes) -> Doc:
    sizes = np.array([len(p[0]) for p in pieces])
    mean = float(sizes.mean()) + len(sep)
    n = int(target / mean) + 1
    picks = rng.integers(0, len(pieces), n)
    chosen = [pieces[int(i)] for i in picks]
    data = open_b + sep.join(c[0] for c in chosen) + close_b
    expected = 2 + sum(c[1] for c in chosen) + (len(chosen) - 1)
    return Doc(data, expected)


def gen_c1(seed: int = 1, target: int = 256 << 20, pool: int = 4096) -> Doc:
    """Minified array of twitter-like records (~30 keys, nested user object,
    strings up to 280 chars, 25% non-ASCII words incl. 4-byte, escaped quotes
    and backslash runs of 1-5, int64 ids, booleans, nulls); valid UTF-8."""
    rng = np.random.default_rng(seed)
    pieces = []
    for i in range(pool):
        rec = _record(rng, i)
        s = json.dumps(rec, ensure_ascii=False, separators=(",", ":")).encode("utf-8")
        pieces.append((s, _expected_from_value(rec)))
    return _pool_join(pieces, rng, target, b"[", b"]", b",")


def gen_c2(seed: int = 2, target: int = 256 << 20, pool: int = 48) -> Doc:
    """Pretty-printed GeoJSON-like polygons of [lon, lat] doubles with 17
    significant digits (negatives, exponents), 100-10k points each, little
    string content."""
    rng = np.random.default_rng(seed)
    pieces = []
    for _ in range(pool):
        npts = int(rng.integers(100, 10001))
        lon = rng.uniform(-180, 180, npts)
        lat = rng.uniform(-90, 90, npts)
        small = rng.random(npts) < 0.05
        lat[small] *= 1e-7
        rows = [f"          [{a:.17g}, {b:.17g}]" for a, b in zip(lon, lat)]
        body = ",\n".join(rows)
        feat = ('    {\n      "type": "Feature",\n      "properties": {"name": "region"},\n'
                '      "geometry": {\n        "type": "Polygon",\n        "coordinates": [\n'
                "        [\n" + body + "\n        ]\n        ]\n      }\n    }")
        expected = _expected_from_value({"type": "Feature", "properties": {"name": "region"},
                                         "geometry": {"type": "Polygon",
                                                      "coordinates": [[[0.0, 0.0]] * npts]}})
        pieces.append((feat.encode(), expected))
    head = b'{\n  "type": "FeatureCollection",\n  "features": [\n'
    doc = _pool_join(pieces, rng, target - len(head), head, b"\n  ]\n}\n", b",\n")
    # the head holds { "type" : "FeatureCollection" , "features" : [ (8 entries)
    # and the tail ] } (2): 10 in place of the 2 brackets _pool_join counted
    return Doc(doc.data, doc.expected_index - 2 + 10)


def lognormal_sizes(rng: np.random.Generator, n: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    s = np.exp(np.log(median) + sigma * rng.standard_normal(n))
    return np.clip(s, lo, hi).astype(np.int64)


CORRUPT_UTF8, CORRUPT_UNCLOSED, CORRUPT_BACKSLASH = 1, 2, 3


def corrupt(doc: bytes, kind: int, rng: np.random.Generator) -> bytes:
    """Break a valid document in one of three ways a stage-1 flag can see."""
    if kind == CORRUPT_UTF8:
        i = int(rng.integers(0, len(doc)))
        return doc[:i] + b"\xff" + doc[i + 1:]
    if kind == CORRUPT_UNCLOSED:
        j = doc.rfind(b'"')
        return doc[:j] + doc[j + 1:] if j >= 0 else doc + b'"'
    return doc + b"\\"


def gen_c3(seed: int = 3, ndocs: int = 100_000, median: int = 2048, sigma: float = 0.9,
           lo: int = 200, hi: int = 65536, corrupt_frac: float = 0.01, pool: int = 1500):
    """Batch of `ndocs` independent documents generated as gen_c0, sizes
    log-normal (median 2 KB, clipped to 200 B..64 KB), `corrupt_frac` of them
    corrupted (invalid UTF-8 byte, unterminated string, stray backslash at the
    end).  Returns (concatenated bytes, offsets[ndocs+1], corruption kind per
    doc (0 = none))."""
    rng = np.random.default_rng(seed)
    psizes = np.unique(np.geomspace(lo, hi, pool).astype(np.int64))
    pool_docs = [gen_c0(seed * 100003 + i, int(t)).data for i, t in enumerate(psizes)]
    plen = np.array([len(d) for d in pool_docs])
    want = lognormal_sizes(rng, ndocs, median, sigma, lo, hi)
    pick = np.clip(np.searchsorted(plen, want), 0, len(pool_docs) - 1)
    kinds = np.zeros(ndocs, dtype=np.int8)
    nc = int(round(ndocs * corrupt_frac))
    if nc:
        idx = rng.choice(ndocs, nc, replace=False)
        kinds[idx] = (np.arange(nc) % 3) + 1
    docs = []
    for i in range(ndocs):
        d = pool_docs[int(pick[i])]
        if kinds[i]:
            d = corrupt(d, int(kinds[i]), rng)
        docs.append(d)
    lens = np.fromiter((len(d) for d in docs), dtype=np.uint64, count=ndocs)
    offsets = np.zeros(ndocs + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    return b"".join(docs), offsets, kinds


def gen_c4(seed: int = 4, ring_bytes: int = 1 << 30, median: int = 4096, sigma: float = 2.0,
           lo: int = 100, hi: int = 16 << 20, pool: int = 160):
    """Request stream for the serving loop: documents with log-normal sizes
    (median 4 KB, sigma 2, clipped to 100 B..16 MB), up to 64 KB generated as
    gen_c0 (pretty-printed mixed values) and above as gen_c1 (minified
    twitter-like records), laid end to end until `ring_bytes`.  Request r of
    a run is document r mod ndocs of this ring.  Returns (bytes, offsets)."""
    rng = np.random.default_rng(seed)
    psizes = np.unique(np.geomspace(lo, hi, pool).astype(np.int64))
    pool_docs = []
    for i, t in enumerate(psizes):
        s = seed * 100003 + i
        pool_docs.append(gen_c0(s, int(t)).data if t <= 65536 else gen_c1(s, int(t), pool=64).data)
    plen = np.array([len(d) for d in pool_docs])
    mean = float(np.exp(np.log(median) + sigma * sigma / 2))
    n = int(ring_bytes / mean * 1.5) + 16
    want = lognormal_sizes(rng, n, median, sigma, lo, hi)
    pick = np.clip(np.searchsorted(plen, want), 0, len(pool_docs) - 1)
    lens = plen[pick]
    keep = int(np.searchsorted(np.cumsum(lens), ring_bytes, side="right"))
    keep = max(1, keep)
    pick, lens = pick[:keep], lens[:keep]
    offsets = np.zeros(keep + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    return b"".join(pool_docs[int(i)] for i in pick), offsets
