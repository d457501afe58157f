"""The kernel body of the HIP library, run on the CPU through emulated
primitives (tests/cpu_emu), against the oracle.  Catches logic and
out-of-range accesses without a GPU; the GPU tests remain the parity proof."""
import numpy as np
import pytest

import emu
import oracle

TB = emu.tile_bytes()


def _check_single(d, nblocks, misalign, block_tiles=None, rows=None, variant=0):
    idx, n, err, viol = emu.run(d, nblocks=nblocks, misalign=misalign, block_tiles=block_tiles, rows=rows,
                                variant=variant)
    oi, oe = oracle.index(d)
    assert viol == 0
    assert n[0] == len(oi) and err[0] == oe
    assert np.array_equal(idx[:n[0]], oi)


def _check_batch(docs, nblocks, misalign, lead, block_tiles=None, rows=None, variant=0):
    data = b"\x00" * lead + b"".join(docs)
    offs = np.concatenate([[lead], lead + np.cumsum([len(x) for x in docs])]).astype(np.uint64)
    idx, n, err, viol = emu.run(data, offsets=offs, nblocks=nblocks, misalign=misalign, block_tiles=block_tiles,
                                rows=rows, variant=variant)
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert viol == 0
    assert np.array_equal(n, on) and np.array_equal(err, oe)
    for d in range(len(docs)):
        a = int(offs[d])
        assert np.array_equal(idx[a:a + n[d]], oi[a:a + on[d]]), d


def _soup(rng, n):
    a = np.frombuffer(b'"\\[]{},: \tax1\xc3\xa9\xe2\x82\xac\xf0\x9f\x98\x80', dtype=np.uint8)
    return a[rng.integers(0, a.size, n)].tobytes()


def test_small_documents():
    for d in (b"", b"1", b'{"a":1}', b"\\", b'"', b" ", b"[12 a]", b'"\xe2\x82'):
        _check_single(d, 1, 3)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_multi_tile_documents(seed):
    rng = np.random.default_rng(seed)
    for _ in range(3):
        _check_single(_soup(rng, int(rng.integers(TB, 3 * TB))), int(rng.integers(1, 4)), int(rng.integers(0, 16)))


def test_backslash_runs_spanning_tiles():
    for run, nxt in ((TB, b'"'), (TB + 1, b'"'), (2 * TB + 5, b"a"), (TB - 3, b'"')):
        for start in (0, 7, TB - 2):
            d = b'["' + b"x" * start + b"\\" * run + nxt + b'",1] "z" [1]'
            _check_single(d, 3, 0)


def test_batches_with_empty_and_tiny_documents():
    rng = np.random.default_rng(4)
    for trial in range(3):
        docs = []
        for _ in range(int(rng.integers(1, 50))):
            r = rng.random()
            L = 0 if r < 0.15 else (1 if r < 0.25 else int(rng.integers(2, 3000 if r < 0.9 else 2 * TB)))
            docs.append(_soup(rng, L))
        _check_batch(docs, int(rng.integers(1, 4)), int(rng.integers(0, 16)), int(rng.integers(0, 40)))


@pytest.mark.parametrize("block_tiles", [1, 2])
def test_many_lookback_blocks(block_tiles):
    """Builds with tiny look-back blocks, so that a few MiB span more blocks
    than one block window (64): block aggregates, block inclusive values, and
    escape-sensitive tiles inside blocks all come into play."""
    from paper_1902_08318_amd import synth
    d = synth.gen_c1(7, 3 << 20, pool=64).data
    idx, n, err, viol = emu.run(d, nblocks=64, misalign=3, block_tiles=block_tiles)
    oi, oe = oracle.index(d)
    assert viol == 0 and n[0] == len(oi) and err[0] == oe
    assert np.array_equal(idx[:n[0]], oi)
    # backslash runs long enough that the escape state entering a tile is
    # only known from the look-back
    for run, end in ((4097, 2 * TB), (TB + 1, 5 * TB + 1), (3 * TB + 2, 9 * TB)):
        s = bytearray(synth.gen_c1(9, 12 * TB, pool=16).data)
        s[end - run:end] = b"\\" * run
        _check_single(bytes(s), 40, 0, block_tiles)
    rng = np.random.default_rng(block_tiles)
    docs = [synth.gen_c0(int(rng.integers(0, 1000)), 5000).data[:int(rng.integers(0, 5000))] for _ in range(300)]
    _check_batch(docs, 48, 1, 5, block_tiles)


def test_two_tile_tickets():
    """With at least two tiles per wave, a ticket hands out two consecutive
    tiles (and a wave finishes one tile after starting the next)."""
    from paper_1902_08318_amd import synth
    d = synth.gen_c1(7, 2 << 20, pool=64).data
    for nb in (8, 16):
        _check_single(d, nb, 5)


def test_pick_rows():
    """Untuned, a launch takes the largest tile that still makes a tile for
    every eighth wave, between 2 and 16 rows of 2 KiB."""
    assert emu.pick_rows(0, 8) == 2
    assert emu.pick_rows(256 << 20, 4096) == 16
    assert emu.pick_rows(16 << 20, 4096) == 16
    assert emu.pick_rows((16 << 20) - 1, 4096) == 8
    assert emu.pick_rows(12 << 20, 4096) == 8
    assert emu.pick_rows(3 << 20, 4096) == 2
    assert emu.pick_rows(5 << 20, 4096) == 4
    assert emu.pick_rows(12871, 4096) == 2
    assert emu.pick_rows(300 << 10, 64) == 16
    assert emu.pick_rows(100 << 10, 64) == 4


@pytest.mark.parametrize("rows", [2, 4, 8, 0])
def test_smaller_tiles(rows):
    """Tiles of fewer rows (a launch over a small input uses them): documents
    over several tiles, backslash runs across tile edges, batches; rows 0 lets
    the kernel pick them for the launch's waves."""
    rng = np.random.default_rng(10 + rows)
    tb = 2048 * (rows or 2)
    for _ in range(2):
        _check_single(_soup(rng, int(rng.integers(tb, 6 * tb))), int(rng.integers(1, 12)), int(rng.integers(0, 16)),
                      rows=rows)
    for run, nxt in ((tb, b'"'), (tb + 1, b'"'), (2 * tb + 5, b"a"), (5 * 1024 + 3, b'"')):
        d = b'["' + b"x" * (tb - 2) + b"\\" * run + nxt + b'",1] "z" [1]'
        _check_single(d, 3, 0, rows=rows)
    docs = []
    for _ in range(60):
        r = rng.random()
        L = 0 if r < 0.15 else (1 if r < 0.25 else int(rng.integers(2, 3000 if r < 0.9 else 3 * tb)))
        docs.append(_soup(rng, L))
    _check_batch(docs, 20, 3, 7, rows=rows)


@pytest.mark.parametrize("variant", emu.VARIANTS)
def test_ablation_variants(variant):
    """Each variant with one of the paper's stage-1 optimizations off gives the
    same index: documents over several tiles with dense rows, backslash runs
    and quotes across edges, batches of ragged documents."""
    rng = np.random.default_rng(40 + variant)
    for _ in range(2):
        _check_single(_soup(rng, int(rng.integers(TB, 3 * TB))), int(rng.integers(1, 12)), int(rng.integers(0, 16)),
                      variant=variant)
    _check_single(b"[" + b"1," * 5000 + b"2]", 4, 1, variant=variant)  # every other byte indexed
    d = b'["' + b"x" * 2000 + b"\\" * 700 + b'\\"' + b'",1] "z" [1]'
    _check_single(d, 3, 0, variant=variant)
    docs = [_soup(rng, int(rng.integers(0, 3000))) for _ in range(40)]
    _check_batch(docs, 16, 3, 7, variant=variant)


def _check_minify_single(d, nblocks, misalign, rows=None, block_tiles=None):
    out, n, err, viol = emu.run(d, nblocks=nblocks, misalign=misalign, rows=rows, block_tiles=block_tiles,
                                minify=True)
    m, e = oracle.minify(d)
    assert viol == 0
    assert n[0] == len(m) and err[0] == e
    assert out[:n[0]].tobytes() == m


@pytest.mark.parametrize("rows", [None, 2, 0])
def test_minify(rows):
    """The minify pass (same kernel body, kept bytes as output) against the
    oracle: soups over tile edges, long backslash runs, a pretty-printed
    document, and a batch with empty and white-space-only documents."""
    from paper_1902_08318_amd import synth
    rng = np.random.default_rng(30 + (rows or 0))
    tb = 2048 * (rows or 16)
    for k in range(3):
        _check_minify_single(_soup(rng, int(rng.integers(tb, 4 * tb))), int(rng.integers(1, 12)), k * 5, rows)
    for run in (tb + 1, 5 * 1024 + 3):
        d = b'[ "' + b"x " * (tb // 4) + b"\\" * run + b'" , 1 ] "z"  [1 ]'
        _check_minify_single(d, 3, 0, rows)
    _check_minify_single(synth.gen_c0(4, 3 * tb).data, 8, 1, rows)
    docs = [b"", b"   ", b" 1 ", b'{ "a" : [ 1 , 2 ] }', b'"open ', b"\\"] + \
           [_soup(rng, int(rng.integers(0, 3 * tb))) for _ in range(20)]
    data = b"\x00" * 3 + b"".join(docs)
    offs = np.concatenate([[3], 3 + np.cumsum([len(x) for x in docs])]).astype(np.uint64)
    out, n, err, viol = emu.run(data, offsets=offs, nblocks=10, misalign=2, rows=rows, minify=True)
    om, on, oe = oracle.minify_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert viol == 0
    assert np.array_equal(n, on) and np.array_equal(err, oe)
    for d in range(len(docs)):
        a = int(offs[d])
        assert out[a:a + n[d]].tobytes() == om[a:a + on[d]].tobytes(), d


def test_utf8_invalid_side_of_the_table():
    """Lead bytes C0..FF with second bytes on each range bound, completed or
    cut short, starting across segment and row edges, as one batch; and the
    four-byte boundary alphabet."""
    import utf8_cases
    seqs = [s for s in utf8_cases.lead_sequences()
            if s[0] in (0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1, 0xED, 0xEF, 0xF0, 0xF1, 0xF4, 0xF5, 0xFF)]
    data, offs = utf8_cases.placed_batch(seqs, residues=(30, 31, 33, 2046, 2047, 0, 1))
    idx, n, err, viol = emu.run(data, offsets=offs, nblocks=16, misalign=0)
    oi, on, oe = oracle.index_batch(np.frombuffer(data, dtype=np.uint8), offs)
    assert viol == 0
    assert 0 < int(((oe & oracle.ERR_UTF8) != 0).sum()) < oe.size
    assert np.array_equal(n, on) and np.array_equal(err, oe)
    data, offs = utf8_cases.boundary_four_byte_batch()
    idx, n, err, viol = emu.run(data.tobytes(), offsets=offs, nblocks=16, misalign=0)
    oi, on, oe = oracle.index_batch(data, offs)
    assert viol == 0 and np.array_equal(n, on) and np.array_equal(err, oe)


@pytest.mark.parametrize("offs", [[100, 50, 60000, 70000], [0, 5000, 3000, 70000],
                                  [0, 1000, 500, 2000, 1500, 70000], [0, 70000, 0]])
def test_decreasing_offsets_flag_every_document(offs):
    """A batch whose offsets decrease anywhere is not indexed: no byte of it is
    read, no index entry is written, and every document gets out_n = 0 and
    JSIDX_ERR_OFFSETS."""
    rng = np.random.default_rng(1)
    data = _soup(rng, 70000)
    offs = np.array(offs, dtype=np.uint64)
    # the input may only be read inside [offsets[0], offsets[-1]): an empty
    # readable range catches any read
    idx, n, err, viol = emu.run(data, offsets=offs, nblocks=8, misalign=0)
    assert viol == 0
    assert np.all(n == 0) and np.all(err == 0x40000000)
    assert np.all(idx == 0xDEADBEEF)
