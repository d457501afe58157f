"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
bit-exact on index positions, counts and flags."""
import itertools
import json
import os
import sys

import numpy as np
import pytest

import oracle
from gpu_common import assert_batch_matches, assert_single_matches, gpu_index_batch, gpu_index_single

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TILE = 32768


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_library_loads_and_reports_healthy():
    import paper_1902_08318_amd as jx
    _say("case: library load")
    assert os.path.exists(jx.library_path())
    assert jx.diag() == 0


def test_paper_examples():
    rows = {}
    for line in open(os.path.join(GOLDEN, "paper_fig3_5_rows.txt"), encoding="utf-8"):
        if not line.startswith("#") and line.strip():
            k, v = line.rstrip("\n").split("\t")
            rows[k] = v
    docs = [rows["INPUT"].encode(), open(os.path.join(GOLDEN, "paper_fig1_document.json"), "rb").read(),
            b'{"key1":"val1", "key2":"val2"}', b'"[1,2]"', b"[12 a]", b"123", b" 1 ", b"",
            b" \t\r\n", b"\\", b'"', b'["\\"",1]', b'["\\\\",1]', b'"\xe2\x82', b'["\xb1\x87"]']
    for i, d in enumerate(docs):
        _say(f"case: paper example {i} len {len(d)}")
        for mis in (0, 1, 7, 15):
            assert_single_matches(d, mis, f"example {i} misalign {mis}")


def test_fig5_final_row_on_gpu():
    rows = {}
    for line in open(os.path.join(GOLDEN, "paper_fig3_5_rows.txt"), encoding="utf-8"):
        if not line.startswith("#") and line.strip():
            k, v = line.rstrip("\n").split("\t")
            rows[k] = v
    idx, n, err = gpu_index_single(rows["INPUT"].encode())
    want = [i for i, c in enumerate(rows["FINAL.fig5"]) if c == "1"]
    assert list(idx) == want and err == 0


ALPHABET = [0x22, 0x5C, 0x5B, 0x3A, 0x2C, 0x61, 0x20, 0xC3, 0xA9]


def test_brute_force_all_short_strings_as_batch():
    """Every string of length 0..6 over {quote, backslash, bracket, colon,
    comma, letter, space, 0xC3, 0xA9}, one document each, in one batch."""
    alpha = np.array(ALPHABET, dtype=np.uint8)
    parts, lens = [], []
    parts.append(np.zeros(0, dtype=np.uint8))
    lens.append(np.zeros(1, dtype=np.uint64))  # the empty string
    for L in range(1, 7):
        grid = np.array(list(itertools.product(range(len(alpha)), repeat=L)), dtype=np.int64)
        X = alpha[grid]
        parts.append(X.reshape(-1))
        lens.append(np.full(X.shape[0], L, dtype=np.uint64))
    data = np.concatenate(parts)
    lens = np.concatenate(lens)
    offs = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    _say(f"case: brute force batch ndocs {lens.size} bytes {data.size}")
    assert_batch_matches(data, offs, 0, "brute force")
    assert_batch_matches(data, offs, 5, "brute force lead 5")


def _soup(rng, n, alpha=b'"\\[]{},: \tax1\xc3\xa9\xe2\x82\xac\xf0\x9f\x98\x80\n'):
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[rng.integers(0, a.size, n)].tobytes()


@pytest.mark.parametrize("seed", range(4))
def test_random_single_documents(seed):
    rng = np.random.default_rng(100 + seed)
    for k in range(12):
        n = int(rng.integers(0, 6 * TILE))
        d = _soup(rng, n)
        mis = int(rng.integers(0, 16))
        _say(f"case: random single seed {seed} k {k} len {n} misalign {mis}")
        assert_single_matches(d, mis, f"seed {seed} k {k}")


def test_backslash_runs_across_tiles():
    """Backslash runs of every length class ending at and around tile and
    segment boundaries, followed by a quote or a letter."""
    rng = np.random.default_rng(5)
    for run in [1, 2, 3, 31, 32, 33, 63, 64, 65, TILE - 1, TILE, TILE + 1, 2 * TILE + 3, 3 * TILE]:
        for start in [0, 1, 31, 32, TILE - run % TILE if run % TILE else 5, TILE - 1, TILE - 2]:
            for nxt in (b'"', b"a", b"\\"):
                d = b'["' + b"x" * start + b"\\" * run + nxt + b'",1] "' + _soup(rng, 100)
                _say(f"case: bs run {run} start {start} next {nxt!r}")
                assert_single_matches(d, 0, f"run {run} start {start}")


def test_quote_at_tile_edges_and_split_utf8():
    for off in range(-3, 4):
        base = b"a" * (TILE + off)
        for tail in (b'"x"', b'\\"x"', b"\xf0\x9f\x98\x80", b"\xe2\x82\xac", b"\xc3\xa9", b"\xf0\x9f\x98",
                     b"]", b" 1"):
            d = b'["' + base + b'", ' + tail + b' "z" ' + tail
            _say(f"case: tile edge off {off} tail {tail!r}")
            assert_single_matches(d, 0, f"edge {off} {tail!r}")
            assert_single_matches(d, 3, f"edge {off} {tail!r} mis3")


def test_dense_index_and_whitespace():
    for n in (1, 63, 64, 65, TILE - 1, TILE, TILE + 1, 3 * TILE + 7):
        _say(f"case: dense n {n}")
        assert_single_matches(b"[" * n, 0, f"dense {n}")
        assert_single_matches(b" " * n, 0, f"ws {n}")
        assert_single_matches(b"1," * n, 1, f"atoms {n}")


def test_generated_c0_and_corruptions():
    from paper_1902_08318_amd import synth
    for seed in range(5):
        doc = synth.gen_c0(seed, 1 << 20)
        _say(f"case: C0 seed {seed} len {len(doc.data)}")
        assert_single_matches(doc.data, seed, f"C0 seed {seed}")
        rng = np.random.default_rng(seed)
        for kind in (1, 2, 3):
            bad = synth.corrupt(doc.data, kind, rng)
            assert_single_matches(bad, 0, f"C0 seed {seed} corrupt {kind}")


def test_batch_mixed_sizes_including_empty():
    rng = np.random.default_rng(11)
    for trial in range(6):
        docs = []
        for _ in range(int(rng.integers(1, 400))):
            r = rng.random()
            L = 0 if r < 0.15 else (1 if r < 0.25 else int(rng.integers(2, 3000 if r < 0.95 else 3 * TILE)))
            docs.append(_soup(rng, L))
        lens = np.array([len(d) for d in docs], dtype=np.uint64)
        offs = np.zeros(len(docs) + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        lead = int(rng.integers(0, 40))
        _say(f"case: batch trial {trial} ndocs {len(docs)} bytes {int(offs[-1])} lead {lead}")
        assert_batch_matches(b"".join(docs), offs, lead, f"batch {trial}")


def test_many_empty_documents_in_one_tile():
    # more documents in one tile than the per-tile table holds
    docs = [b""] * 3000 + [b"[1]"] + [b""] * 2000 + [b'"a"'] * 1500 + [b""] * 10
    lens = np.array([len(d) for d in docs], dtype=np.uint64)
    offs = np.zeros(len(docs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    _say(f"case: many empty docs {len(docs)}")
    assert_batch_matches(b"".join(docs), offs, 3, "many empty")


def test_batch_equals_single_calls():
    from paper_1902_08318_amd import synth
    data, offs, kinds = synth.gen_c3(3, ndocs=300, pool=60)
    gi, gn, ge = gpu_index_batch(data, offs)
    for d in range(0, 300, 7):
        a, b = int(offs[d]), int(offs[d + 1])
        si, sn, se = gpu_index_single(data[a:b])
        assert sn == gn[d] and se == ge[d]
        assert np.array_equal(si, gi[a:a + sn])
        if kinds[d]:
            assert se != 0


def test_repeated_launches_reuse_workspace():
    """Many launches of varying size on one stream: the per-launch epoch and
    the descriptor scrub must keep every launch independent."""
    import paper_1902_08318_amd as jx
    rng = np.random.default_rng(21)
    for k in range(60):
        n = int(rng.integers(0, 8 * TILE)) if k % 5 else int(rng.integers(20 * TILE, 40 * TILE))
        d = _soup(rng, n)
        if k % 10 == 0:
            _say(f"case: repeated launch {k} len {n}")
        assert_single_matches(d, k % 16, f"launch {k}")
    assert jx.diag() == 0


def test_generated_c1_c2_full_size():
    """Full-size C1 and C2 against the oracle, and their index sizes against
    the generators' own count of structural characters, strings and atoms."""
    from paper_1902_08318_amd import synth
    for name, doc in (("C1", synth.gen_c1(1)), ("C2", synth.gen_c2(2))):
        _say(f"case: {name} full size {len(doc.data)}")
        assert_single_matches(doc.data, 0, name)
        _, n, err = gpu_index_single(doc.data)
        assert n == doc.expected_index and err == 0
    for seed in range(3):
        doc = synth.gen_c0(seed, 1 << 20)
        _, n, err = gpu_index_single(doc.data)
        assert n == doc.expected_index and err == 0


def test_generated_c3_full_batch():
    from paper_1902_08318_amd import synth
    data, offs, kinds = synth.gen_c3(3)
    _say(f"case: C3 full batch ndocs {offs.size - 1} bytes {len(data)}")
    assert_batch_matches(data, offs, 0, "C3")
    _, _, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert np.all((oe[kinds > 0] & 0x7) != 0)


def test_reserved_capacity_is_enforced_without_sync():
    """After jsidx_reserve, a batch larger than the reservation is flagged
    JSIDX_ERR_CAPACITY for every document (and nothing else is written)."""
    import torch
    import paper_1902_08318_amd as jx
    _say("case: reserved capacity")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        jx.reserve(1000, s)
        docs = [b'{"a":[1,2,3]}'] * 5000
        data = b"".join(docs)
        offs = np.arange(len(docs) + 1, dtype=np.int64) * len(docs[0])
        bufs = torch.frombuffer(bytearray(data), dtype=torch.uint8).to("cuda:0")
        toffs = torch.from_numpy(offs).to("cuda:0")
        out = torch.zeros(len(data), dtype=torch.int32, device="cuda:0")
        n = torch.full((len(docs),), 7, dtype=torch.int32, device="cuda:0")
        err = torch.zeros(len(docs), dtype=torch.int32, device="cuda:0")
        jx.build_batch(bufs, toffs, out, n, err, s)
        s.synchronize()
        assert torch.all(n == 0).item()
        assert torch.all((err.to(torch.int64) & 0xFFFFFFFF) == jx.ERR_CAPACITY).item()
        jx.reserve(len(data), s)
        jx.build_batch(bufs, toffs, out, n, err, s)
        s.synchronize()
        want = len(oracle.index(docs[0])[0])
        assert want == 11
        assert torch.all(n == want).item() and torch.all(err == 0).item()
        jx.release(s)


@pytest.mark.parametrize("rows", [2, 4, 8, 16])
def test_every_tile_size(rows):
    """The tile size is a tuning choice (jsidx_set_tile_rows): with every
    launch forced to `rows` rows per tile, single documents (several tiles,
    backslash runs over tile edges) and batches still match the oracle."""
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    _say(f"case: tile rows forced to {rows}")
    jx.set_tile_rows([rows] * 64)
    try:
        assert jx.tile_rows(1 << 20) == rows
        rng = np.random.default_rng(100 + rows)
        tb = 2048 * rows
        for k in range(4):
            assert_single_matches(_soup(rng, int(rng.integers(tb, 9 * tb))), k * 5, f"rows {rows} soup {k}")
        for run in (tb - 1, tb + 1, 3 * tb + 2, 4097):
            d = b'["' + b"x" * (tb - 3) + b"\\" * run + b'"' + b'",1] "z" [1]'
            assert_single_matches(d, 1, f"rows {rows} run {run}")
        doc = synth.gen_c1(50 + rows, 6 << 20, pool=64).data
        assert_single_matches(doc, 3, f"rows {rows} C1-like 6 MiB")
        data, offs, _ = synth.gen_c3(60 + rows, ndocs=3000, pool=100)
        assert_batch_matches(data, offs, 5, f"rows {rows} batch")
    finally:
        jx.set_tile_rows([])
    assert jx.diag() == 0


@pytest.mark.parametrize("variant", ["naive_classify", "xor_loop", "direct_flatten"])
def test_ablation_variants(variant):
    """Each kernel variant with one of the paper's stage-1 optimizations off
    (jsidx_set_variant) indexes exactly as the oracle: random documents over
    many tiles, backslash runs over tile edges, a dense generated document,
    the numeric pretty-printed one, and a batch."""
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    _say(f"case: kernel variant {variant}")
    jx.set_variant(jx.VARIANTS[variant])
    try:
        rng = np.random.default_rng(7 + jx.VARIANTS[variant])
        for k in range(3):
            assert_single_matches(_soup(rng, int(rng.integers(1 << 16, 1 << 20))), k * 3, f"{variant} soup {k}")
        for run in (32767, 32769, 4097):
            d = b'["' + b"x" * 32765 + b"\\" * run + b'"' + b'",1] "z" [1]'
            assert_single_matches(d, 1, f"{variant} run {run}")
        assert_single_matches(synth.gen_c1(70, 16 << 20, pool=64).data, 0, f"{variant} C1-like 16 MiB")
        assert_single_matches(synth.gen_c2(71, 8 << 20, pool=16).data, 5, f"{variant} C2-like 8 MiB")
        data, offs, _ = synth.gen_c3(72, ndocs=3000, pool=100)
        assert_batch_matches(data, offs, 5, f"{variant} batch")
    finally:
        jx.set_variant(0)
    assert jx.diag() == 0


# ---- the table of well-formed UTF-8 sequences, invalid side included -------
import utf8_cases  # noqa: E402


@pytest.mark.parametrize("length", [1, 2, 3])
def test_utf8_every_short_string(length):
    """Every 1-, 2- and 3-byte string, one document each, in one batch: the
    flags (and indices) of all of them against the oracle (Sec. 3.1.5)."""
    data, offs = utf8_cases.equal_length_batch(utf8_cases.all_strings(length), length)
    _say(f"case: every {length}-byte string, {offs.size - 1} documents")
    assert_batch_matches(data, offs, 0, f"every {length}-byte string")


def test_utf8_four_byte_boundary_alphabet():
    data, offs = utf8_cases.boundary_four_byte_batch()
    _say(f"case: four-byte boundary alphabet, {offs.size - 1} documents")
    assert_batch_matches(data, offs, 0, "four-byte boundary alphabet")


def test_utf8_lead_and_second_bytes_at_segment_and_row_edges():
    """Every lead byte C0..FF with second bytes on each range bound (80 8F 90
    9F A0 BF, a non-continuation, a lead), completed to the announced length
    or cut short at the document's end, starting across 32-byte segment edges
    and 2 KiB row (and tile) edges: invalid pairs E0 80-9F, ED A0-BF,
    F0 80-8F, F4 90-BF, leads C0, C1 and F5-FF, and their valid neighbours."""
    data, offs = utf8_cases.placed_batch(utf8_cases.lead_sequences())
    _say(f"case: placed lead sequences, {offs.size - 1} documents, {len(data)} bytes")
    _, _, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    bad = (oe & oracle.ERR_UTF8) != 0
    assert 0 < int(bad.sum()) < bad.size  # both sides of the table are present
    assert_batch_matches(data, offs, 0, "placed lead sequences")


def test_utf8_sequences_across_tile_edges_single_documents():
    """Single documents with one lead sequence each, starting 3 bytes before
    to 3 bytes after the 32 KiB and 64 KiB points, which are tile edges of the
    one-document kernel (16 KiB tiles) that jsidx_build runs."""
    seqs = utf8_cases.lead_sequences(seconds=(0x80, 0x9F, 0xA0, 0xBF, 0x8F, 0x90))
    pick = [s for s in seqs if s[0] in (0xC0, 0xC1, 0xC2, 0xE0, 0xED, 0xEF, 0xF0, 0xF4, 0xF5, 0xFF)]
    _say(f"case: lead sequences at tile edges, {len(pick)} sequences")
    for s in pick:
        for edge in (32768, 65536):
            for delta in (-3, -2, -1, 0, 1, 2, 3):
                p = edge + delta
                d = b'["' + b"x" * (p - 2) + s + b'", 1]'
                assert_single_matches(d, 0, f"seq {s.hex()} at {p}")


def test_lookback_over_more_than_64_blocks():
    """Walks over more than the 64 blocks one look-back window holds, on the
    device: full-size C1 in the one-document kernel spans 16,384 tiles in
    2,048 blocks of 8 tiles (the first tiles to finish walk back over
    hundreds of blocks), and a 90 MB batch at 2-row tiles (4 KiB) about 88
    blocks of the batch kernel."""
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    jx.set_tile_rows([2] * 64)
    try:
        doc = synth.gen_c1(1)
        _say(f"case: C1 in one launch, {len(doc.data)} bytes")
        assert len(doc.data) > 64 * 8 * 16384
        assert_single_matches(doc.data, 0, "C1")
        data, offs, _ = synth.gen_c3(3, ndocs=30000)
        _say(f"case: batch at 2-row tiles, {offs.size - 1} docs, {int(offs[-1])} bytes")
        assert int(offs[-1]) > 64 * 256 * 4096
        assert_batch_matches(data, offs, 0, "batch 2-row tiles")
    finally:
        jx.set_tile_rows([])
    assert jx.diag() == 0


@pytest.mark.parametrize("offs", [[100, 50, 60000, 70000], [0, 5000, 3000, 70000],
                                  [0, 1000, 500, 2000, 1500, 70000], [0, 70000, 0]])
def test_decreasing_offsets_flag_every_document(offs):
    """Offsets that decrease anywhere: the batch is not indexed, every
    document gets out_n = 0 and JSIDX_ERR_OFFSETS, no index entry is written;
    a good batch on the same stream afterwards is indexed normally."""
    import paper_1902_08318_amd as jx
    rng = np.random.default_rng(2)
    data = _soup(rng, 70000)
    _say(f"case: decreasing offsets {offs}")
    o = np.array(offs, dtype=np.uint64)
    gi, gn, ge = gpu_index_batch(data, o)
    assert np.all(gn == 0) and np.all(ge == jx.ERR_OFFSETS)
    assert np.all(gi == 0xFFFFFFFF)
    good = np.array([0, 1000, 5000, 70000], dtype=np.uint64)
    assert_batch_matches(data, good, 0, "good batch after a bad one")


def test_failed_workspace_growth_leaves_a_working_stream():
    """A reservation the device cannot hold fails with JSIDX_E_NOWORKSPACE and
    leaves the stream without a workspace (no stale capacity); the next calls
    on that stream allocate again and index correctly."""
    import torch
    import paper_1902_08318_amd as jx
    _say("case: failed workspace growth")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        jx.reserve(1 << 20, s)
        with pytest.raises(jx.JsidxError):
            jx.reserve(1 << 45, s)  # petabytes of workspace
        d = b'{"a":[1,2,"x\\"y"],"b":null}' * 100
        buf = torch.frombuffer(bytearray(d), dtype=torch.uint8).to("cuda:0")
        pos, n, err = jx.index(buf, s)
        oi, oe = oracle.index(d)
        assert n == len(oi) and err == oe
        assert np.array_equal(pos.cpu().numpy().view(np.uint32), oi)
        offs = torch.tensor([0, 50, len(d)], dtype=torch.int64, device="cuda:0")
        out, nn, ee = jx.index_batch(buf, offs, s)
        s.synchronize()
        on = oracle.index_batch(np.frombuffer(d, dtype=np.uint8), np.array([0, 50, len(d)], dtype=np.uint64))[1]
        assert np.array_equal(nn.cpu().numpy().view(np.uint32), on)
        jx.release(s)
    assert jx.diag() == 0
