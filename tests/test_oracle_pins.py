"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the rows the
paper prints for its worked example (Figs. 3-5), the tape of Fig. 2, the small
examples in the text, an independent transcription of the paper's block
formulas (brute force over all short strings), and Python's strict UTF-8
decoder (a library routine) for the paper's table of code points.
"""
import codecs
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import paper_blocks as pb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows():
    rows = {}
    with open(os.path.join(GOLDEN, "paper_fig3_5_rows.txt"), encoding="utf-8") as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.rstrip("\n").split("\t")
            rows[k] = v
    return rows


def _mask(bits):
    return sum(1 << i for i, c in enumerate(bits) if c == "1")


def _bits(m, n=64):
    return "".join("1" if (m >> i) & 1 else "_" for i in range(n))


# ---------------------------------------------------------------- Sec. 3.1.2
def test_nibble_tables_give_desired_classes():
    """The two printed nibble tables classify all 256 byte values exactly as
    the 'desired value' column of the classification table says."""
    desired = {0x2C: 1, 0x3A: 2, 0x5B: 4, 0x5D: 4, 0x7B: 4, 0x7D: 4,
               0x09: 8, 0x0A: 8, 0x0D: 8, 0x20: 16}
    for b in range(256):
        assert pb.nibble_class(b) == desired.get(b, 0), hex(b)


# ---------------------------------------------------------- Figs. 3, 4 and 5
def test_block_transcription_reproduces_every_printed_row():
    rows = _rows()
    inp = rows["INPUT"].encode()
    assert len(inp) == 64
    C = sum(1 << i for i, b in enumerate(inp) if pb.nibble_class(b) & 7)
    W = sum(1 << i for i, b in enumerate(inp) if pb.nibble_class(b) & 0x18)
    Q = sum(1 << i for i, b in enumerate(inp) if b == 0x22)
    B = sum(1 << i for i, b in enumerate(inp) if b == 0x5C)
    one = (1 << 64) - 1
    assert _bits(B) == rows["B.fig3"]
    assert _bits(Q) == rows["Q.fig4"]
    assert _bits(C) == rows["S.fig5"]
    assert _bits(W) == rows["W.fig5"]
    # Fig. 3 intermediate rows, formula by formula.
    E = pb.even_bits(64)
    O = one & ~E
    S = B & ~(B << 1) & one
    assert _bits(S) == rows["S.fig3"]
    ES = S & E
    assert _bits(ES) == rows["ES.fig3"]
    EC = (B + ES) & one
    assert _bits(EC) == rows["EC.fig3"]
    ECE = EC & ~B
    assert _bits(ECE) == rows["ECE.fig3"]
    assert _bits(ECE & ~E) == rows["OD1.fig3"]
    OS = S & O
    assert _bits(OS) == rows["OS.fig3"]
    OC = (B + OS) & one
    assert _bits(OC) == rows["OC.fig3"]
    OCE = OC & ~B
    assert _bits(OCE) == rows["OCE.fig3"]
    assert _bits(OCE & E) == rows["OD2.fig3"]
    # Whole block step: Fig. 3 result, Fig. 4 and Fig. 5 rows.
    F, r, _ = pb.block_step(C, W, Q, B, 64, (0, 0, 0), 0)
    assert _bits(r["OD"]) == rows["OD.fig3"] == rows["OD.fig4"]
    assert _bits(r["Q_UNESC"]) == rows["Q_UNESC.fig4"] == rows["Q.fig5"]
    assert _bits(r["R"]) == rows["R.fig4"] == rows["R.fig5"]
    Rm = r["R"]
    Qu = r["Q_UNESC"]
    assert _bits(C & ~Rm) == rows["S_NOT_R.fig5"]
    assert _bits(r["S_OR_Q"]) == rows["S_OR_Q.fig5"]
    P = (r["S_OR_Q"] | W) & one
    assert _bits(P) == rows["P_SW.fig5"]
    assert _bits((P << 1) & one) == rows["P_SHL.fig5"]
    assert _bits(r["P_MASKED"]) == rows["P_MASKED.fig5"]
    assert _bits(r["S_OR_Q"] | r["P_MASKED"]) == rows["S_OR_P.fig5"]
    assert _bits(F) == rows["FINAL.fig5"]
    del Qu


def test_oracle_matches_fig5_final_row():
    rows = _rows()
    idx, err = oracle.index(rows["INPUT"].encode())
    assert _mask(rows["FINAL.fig5"]) == sum(1 << int(i) for i in idx)
    assert list(idx) == [0, 2, 13, 15, 17, 20, 21, 28, 30, 33, 35, 41, 43, 49, 50,
                         52, 55, 56, 63]
    assert err == 0


# ------------------------------------------------------------ Figs. 1 and 2
def test_fig1_document_node_order_matches_fig2_tape():
    doc = open(os.path.join(GOLDEN, "paper_fig1_document.json"), "rb").read()
    tape = [l.strip() for l in open(os.path.join(GOLDEN, "paper_fig2_tape.txt"))
            if l.strip() and not l.startswith("#")]
    idx, err = oracle.index(doc)
    assert err == 0
    kinds = []
    for i in idx:
        ch = chr(doc[int(i)])
        if ch in ":,":
            continue
        if ch in "{}[]":
            kinds.append(ch)
        elif ch == '"':
            end = doc.index(b'"', int(i) + 1)
            kinds.append("string " + doc[int(i) + 1:end].decode())
        elif ch in "-0123456789":
            j = int(i)
            while j < len(doc) and chr(doc[j]) in "-0123456789":
                j += 1
            kinds.append("integer " + doc[int(i):j].decode())
        elif ch == "f":
            kinds.append("false")
        elif ch == "n":
            kinds.append("null")
        else:
            kinds.append("?" + ch)
    assert kinds == tape
    assert len(idx) == 51
    # A trailing newline adds nothing.
    idx2, err2 = oracle.index(doc + b"\n")
    assert list(idx2) == list(idx) and err2 == 0


# --------------------------------------------------------- examples in text
@pytest.mark.parametrize("doc,expected", [
    # Sec. 3 two-stage example: braces, the four string starts, two colons and
    # the comma (the prose list omits the comma, but commas are structural).
    (b'{"key1":"val1", "key2":"val2"}', [0, 1, 7, 8, 14, 16, 22, 23, 29]),
    # Sec. 3 item 1: a quoted "[1,2]" is one string.
    (b'"[1,2]"', [0]),
    # Sec. 3.1.3: the dangling atom in [12 a] is exposed.
    (b"[12 a]", [0, 1, 4, 5]),
    # Sec. 3.1.1: quote range 0b100010000 -> 0b011110000 (bits 4..7 inside).
    (b',,,,",,,",', [0, 1, 2, 3, 4, 9]),
    # Sec. 3.1.1: \" is an escaped quote, \\" is not.
    (b'["\\"",1]', [0, 1, 5, 6, 7]),
    (b'["\\\\",1]', [0, 1, 5, 6, 7]),
    (b'["\\\\"],1', [0, 1, 5, 6, 7]),
    # A scalar root value is indexed (predecessor of byte 0 is white space).
    (b"123", [0]),
    (b" 1 ", [1]),
])
def test_text_examples(doc, expected):
    idx, _ = oracle.index(doc)
    assert list(idx) == expected


def test_escaped_quote_parity():
    # "\\\"x" : three backslashes then a quote -> escaped; still inside string.
    idx, err = oracle.index(b'["\\\\\\"x"]')
    assert list(idx) == [0, 1, 8] and err == 0
    idx, err = oracle.index(b'["\\\\\\\\"]')  # four backslashes then quote
    assert list(idx) == [0, 1, 7] and err == 0


def test_flags_on_constructed_errors():
    assert oracle.index(b'{"a":1}')[1] == 0
    assert oracle.index(b'{"a:1}')[1] & oracle.ERR_UNCLOSED_STRING
    assert oracle.index(b'{"a":1}\\')[1] & oracle.ERR_TRAILING_ESCAPE
    assert oracle.index(b"")[1] == oracle.ERR_EMPTY
    assert oracle.index(b" \t\r\n ")[1] == oracle.ERR_EMPTY
    assert oracle.index(b'{"a":"\xff"}')[1] & oracle.ERR_UTF8
    assert oracle.index(b'{"a":"\x80"}')[1] & oracle.ERR_UTF8
    # Sec. 4 parser-conformance example: B1 87 is not valid UTF-8.
    assert oracle.index(b'["\xb1\x87"]')[1] == oracle.ERR_UTF8
    # Truncated multi-byte sequence at the end of the document.
    assert oracle.index(b'"\xe2\x82')[1] & oracle.ERR_UTF8


# ------------------------------------------------- brute force vs Figs. 3-5
ALPHABET = [0x22, 0x5C, 0x5B, 0x3A, 0x2C, 0x61, 0x20, 0xC3, 0xA9]


@pytest.mark.parametrize("width", [1, 2, 4, 63])
def test_oracle_equals_block_formulas_all_short_strings(width):
    """All strings of length <= 6 over {quote, backslash, bracket, colon,
    comma, letter, space, 0xC3, 0xA9}: the byte-at-a-time oracle equals the
    paper's block formulas evaluated with explicit carries at several block
    widths (index, unclosed-string and trailing-escape flags)."""
    alpha = np.array(ALPHABET, dtype=np.uint8)
    for L in range(1, 7):
        grid = np.array(list(itertools.product(range(len(alpha)), repeat=L)), dtype=np.int64)
        X = alpha[grid]
        mask, unclosed, trailing = pb.index_strings(X, width)
        n = X.shape[0]
        offs = np.arange(n + 1, dtype=np.uint64) * np.uint64(L)
        out_idx, out_n, out_err = oracle.index_batch(X.reshape(-1), offs)
        # Rebuild the oracle's index as a bit mask per string.
        region = out_idx.reshape(n, L).astype(np.uint64)
        valid = np.arange(L)[None, :] < out_n[:, None]
        om = np.bitwise_or.reduce(np.where(valid, np.uint64(1) << region, np.uint64(0)), axis=1)
        assert np.array_equal(om, mask), (L, width)
        assert np.array_equal((out_err & oracle.ERR_UNCLOSED_STRING) != 0, unclosed != 0)
        assert np.array_equal((out_err & oracle.ERR_TRAILING_ESCAPE) != 0, trailing != 0)
        assert np.array_equal((out_err & oracle.ERR_EMPTY) != 0, mask == 0)


def test_oracle_equals_block_formulas_long_backslash_runs():
    """Random 48-byte strings rich in backslash runs and quotes, block widths
    1..17 (runs cross many block boundaries)."""
    rng = np.random.default_rng(7)
    X = rng.choice(np.array([0x5C] * 6 + [0x22, 0x22, 0x5B, 0x61, 0x20, 0x2C], dtype=np.uint8),
                   size=(20000, 48))
    offs = np.arange(X.shape[0] + 1, dtype=np.uint64) * np.uint64(48)
    out_idx, out_n, out_err = oracle.index_batch(X.reshape(-1), offs)
    region = out_idx.reshape(X.shape[0], 48).astype(np.uint64)
    valid = np.arange(48)[None, :] < out_n[:, None]
    om = np.bitwise_or.reduce(np.where(valid, np.uint64(1) << region, np.uint64(0)), axis=1)
    for width in range(1, 18):
        mask, unclosed, trailing = pb.index_strings(X, width)
        assert np.array_equal(om, mask), width
        assert np.array_equal((out_err & 2) != 0, unclosed != 0)
        assert np.array_equal((out_err & 4) != 0, trailing != 0)


# ------------------------------------------------------ UTF-8, Sec. 3.1.5
def _py_valid(b: bytes) -> bool:
    try:
        codecs.utf_8_decode(b, "strict", True)
        return True
    except UnicodeDecodeError:
        return False


def _batch_utf8_flags(strings, L):
    X = np.frombuffer(b"".join(strings), dtype=np.uint8)
    offs = np.arange(len(strings) + 1, dtype=np.uint64) * np.uint64(L)
    _, _, err = oracle.index_batch(X, offs)
    return (err & oracle.ERR_UTF8) == 0


@pytest.mark.parametrize("L", [1, 2])
def test_utf8_exhaustive_short(L):
    strings = [bytes(t) for t in itertools.product(range(256), repeat=L)]
    got = _batch_utf8_flags(strings, L)
    want = np.array([_py_valid(s) for s in strings])
    assert np.array_equal(got, want)


def test_utf8_exhaustive_three_bytes():
    X = np.array(list(itertools.product(range(256), repeat=2)), dtype=np.uint8)
    for a in range(256):
        strings = [bytes((a, int(b), int(c))) for b, c in X]
        got = _batch_utf8_flags(strings, 3)
        want = np.array([_py_valid(s) for s in strings])
        assert np.array_equal(got, want), hex(a)


def test_utf8_four_byte_boundary_alphabet():
    alpha = [0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF,
             0xE0, 0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xFF,
             0x41, 0x22]
    strings = [bytes(t) for t in itertools.product(alpha, repeat=4)]
    got = _batch_utf8_flags(strings, 4)
    want = np.array([_py_valid(s) for s in strings])
    assert np.array_equal(got, want)


def test_utf8_every_scalar_value_is_valid_and_count():
    cps = [cp for cp in range(0x110000) if not 0xD800 <= cp <= 0xDFFF]
    assert len(cps) == 1112064
    enc = [chr(cp).encode("utf-8") for cp in cps]
    blob = b"".join(enc)
    assert oracle.utf8_valid(blob)
    lens = np.array([len(e) for e in enc], dtype=np.uint64)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    _, _, err = oracle.index_batch(np.frombuffer(blob, dtype=np.uint8), offs)
    assert not np.any(err & oracle.ERR_UTF8)
    # Surrogates encoded in the 3-byte form are not well formed.
    for cp in (0xD800, 0xDBFF, 0xDC00, 0xDFFF):
        b = bytes([0xE0 | (cp >> 12), 0x80 | ((cp >> 6) & 0x3F), 0x80 | (cp & 0x3F)])
        assert not oracle.utf8_valid(b)


# ------------------------------------------------- soundness of the flags
def test_valid_json_has_no_flags():
    rng = np.random.default_rng(3)
    words = ["a", "é", "日本", "\U0001D11E", 'q"q', "b\\s", "\n", "/"]
    for _ in range(300):
        def val(depth):
            k = rng.integers(0, 7 if depth < 3 else 4)
            if k == 0:
                return int(rng.integers(-10**18, 10**18))
            if k == 1:
                return float(rng.normal()) * 10 ** int(rng.integers(-30, 30))
            if k == 2:
                return "".join(rng.choice(words, size=int(rng.integers(0, 5))))
            if k == 3:
                return [True, False, None][int(rng.integers(0, 3))]
            if k == 4:
                return [val(depth + 1) for _ in range(int(rng.integers(0, 4)))]
            return {f"k{i}{rng.choice(words)}": val(depth + 1) for i in range(int(rng.integers(0, 4)))}
        v = val(0)
        for indent in (None, 2):
            doc = json.dumps(v, ensure_ascii=bool(rng.integers(0, 2)), indent=indent).encode()
            idx, err = oracle.index(doc)
            assert err == 0, doc
            assert len(idx) > 0


# ------------------------------------------- the generators' closed form
@pytest.mark.parametrize("name,seed,target", [("c0", 0, 1 << 20), ("c0", 3, 300_000), ("c1", 1, 4 << 20),
                                              ("c1", 5, 1 << 20), ("c2", 2, 4 << 20)])
def test_generator_closed_form_equals_oracle_count(name, seed, target):
    """A valid document's index holds one entry per structural character, per
    string (its opening quote, keys included) and per atom (number, true,
    false, null).  The generators count these while they emit the document,
    without the oracle; the oracle's index size must equal that count, and the
    document carries no flag."""
    from paper_1902_08318_amd import synth
    gen = {"c0": synth.gen_c0, "c1": synth.gen_c1, "c2": synth.gen_c2}[name]
    doc = gen(seed, target) if name == "c0" else gen(seed, target, pool=32)
    idx, err = oracle.index(doc.data)
    assert err == 0
    assert len(idx) == doc.expected_index
