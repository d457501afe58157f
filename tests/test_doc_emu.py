"""The one-document kernel (jsidx_doc.h, behind jsidx_build) run on the CPU
through the emulated primitives (tests/cpu_emu), against the oracle: every
global access bounds-checked, every result compared element by element."""
import numpy as np
import pytest

import emu
import oracle

TB = 16384  # bytes per tile of the one-document kernel


def _check(d, nwaves=4, misalign=0, block_tiles=None, variant=0, label=""):
    idx, n, err, viol = emu.run_doc(d, nwaves=nwaves, misalign=misalign, block_tiles=block_tiles, variant=variant)
    oi, oe = oracle.index(d)
    assert viol == 0, label
    assert n[0] == len(oi) and err[0] == oe, (label, n[0], len(oi), hex(err[0]), hex(oe))
    assert np.array_equal(idx[:n[0]], oi), label


def _soup(rng, n, alpha=b'"\\[]{},: \tax1\xc3\xa9\xe2\x82\xac\xf0\x9f\x98\x80\n'):
    a = np.frombuffer(alpha, dtype=np.uint8)
    return a[rng.integers(0, a.size, n)].tobytes()


def test_tile_size():
    assert emu.doc_tile_bytes() == TB


@pytest.mark.parametrize("doc", [b"", b"1", b'{"a":1}', b"\\", b'"', b" ", b"[12 a]", b'"\xe2\x82', b" 1 ",
                                 b'["\\"",1]', b'["\\\\",1]', b"\xef\xbb\xbf[]"])
def test_small_documents(doc):
    for mis in (0, 3, 15):
        _check(doc, 4, mis, label=f"{doc!r} {mis}")


@pytest.mark.parametrize("seed", [0, 1])
def test_random_multi_tile_documents(seed):
    rng = np.random.default_rng(seed)
    for k in range(3):
        n = int(rng.integers(TB, 5 * TB))
        _check(_soup(rng, n), int(rng.integers(1, 12)), int(rng.integers(0, 16)), label=f"soup {k}")


def test_dense_rows_and_exact_tile_fits():
    """Every byte indexed, every other byte indexed, and lengths that end at,
    just before and just after a tile edge at three misalignments."""
    for n in (TB - 16, TB - 15, TB, TB + 1, 2 * TB - 3, 2 * TB):
        for mis in (0, 1, 15):
            _check(b"[" * n, 4, mis, label=f"dense {n} {mis}")
            _check(b"1," * (n // 2), 4, mis, label=f"atoms {n} {mis}")


def test_backslash_runs_before_tile_starts():
    """Runs of 1 to 3 tiles of backslashes ending around tile starts, then a
    quote, a letter or another backslash: the escape entering a tile comes
    from the bytes before it, or, after 64 or more backslashes, from the
    newest earlier tile that knows it."""
    for run in (1, 2, 63, 64, 65, TB - 1, TB + 1, 2 * TB + 3):
        for end in (TB - 1, TB, TB + 1, 2 * TB + 2):
            for nxt in (b'"', b"a", b"\\"):
                if run + 5 > end:
                    continue
                d = b'["' + b"x" * (end - run - 2) + b"\\" * run + nxt + b'",1] "z" ' + b"y" * 3000 + b'"'
                _check(d, 6, 0, label=f"run {run} end {end} next {nxt!r}")


def test_quote_before_tile_after_long_run():
    """A quote as the last byte before a tile, after 62 to 5000 backslashes:
    whether it counts as the tile's predecessor comes from the tile before."""
    for run in (62, 63, 64, 100, 5000):
        for qpos in (TB - 1, 2 * TB - 1):
            d = b'["' + b"x" * (qpos - run - 2) + b"\\" * run + b'"' + b"a,1] \"z\" [1]" + b" " * 40000
            _check(d, 5, 0, label=f"run {run} qpos {qpos}")
            d = b"[" + b"x" * (qpos - run - 1) + b"\\" * run + b'"' + b"a,1] \"z\" [1]" + b" " * 40000
            _check(d, 5, 0, label=f"outside run {run} qpos {qpos}")


def test_documents_ending_in_backslash_runs():
    for L in (TB, 2 * TB, 2 * TB + 1, 3 * TB - 1):
        for run in (1, 2, 64, 65, TB + 1, TB + 2):
            if run >= L - 2:
                continue
            d = b'"' + b"x" * (L - run - 1) + b"\\" * run
            for mis in (0, 5):
                _check(d, 4, mis, label=f"L {L} run {run} mis {mis}")
    for L in (TB, 3 * TB + 7):
        _check(b"\\" * L, 4, 0, label=f"all backslashes {L}")
        _check(b"\\" * L + b'"', 4, 0, label=f"all backslashes and a quote {L}")


def test_utf8_across_tile_edges():
    for off in range(-3, 4):
        for tail in (b'"x"', b'\\"x"', b"\xf0\x9f\x98\x80", b"\xe2\x82\xac", b"\xc3\xa9", b"\xf0\x9f\x98",
                     b"\xe0\x80\x80", b"\xed\xa0\x80", b"\xf4\x90\x80\x80", b"\xc0\x80"):
            d = b'["' + b"a" * (TB + off - 2) + tail + b'", 1, "z"]'
            _check(d, 3, 0, label=f"edge {off} {tail!r}")


@pytest.mark.parametrize("block_tiles", [1, 2])
def test_many_lookback_blocks(block_tiles):
    """Builds with blocks of 1 and 2 tiles, so that a few MiB span more than
    the 64 blocks one read holds: block aggregates, block inclusive values and
    windows of aggregates folded further back; and a backslash run over 24
    tiles ending in a quote."""
    from paper_1902_08318_amd import synth
    d = synth.gen_c1(7, 3 << 20, pool=64).data
    for nw in (16, 64):
        _check(d, nw, 3, block_tiles, label=f"C1-like {nw} waves")
    s = bytearray(synth.gen_c1(9, 40 * TB, pool=16).data)
    s[5 * TB + 7: 29 * TB + 3] = b"\\" * (24 * TB - 4)
    s[29 * TB + 3] = ord('"')
    _check(bytes(s), 24, 0, block_tiles, label="long run")


@pytest.mark.parametrize("variant", emu.VARIANTS)
def test_ablation_variants(variant):
    rng = np.random.default_rng(40 + variant)
    _check(_soup(rng, int(rng.integers(TB, 3 * TB))), 7, 5, variant=variant, label="soup")
    _check(b"[" + b"1," * 20000 + b"2]", 4, 1, variant=variant, label="dense")
    d = b'["' + b"x" * 2000 + b"\\" * 700 + b'\\"' + b'",1] "z" [1]'
    _check(d, 3, 0, variant=variant, label="run")


def test_workspace_reused_across_launches():
    """Launches of varying size on one workspace: epochs and the scrub keep
    each launch independent."""
    rng = np.random.default_rng(9)
    ws = emu.Workspace(8)
    for k in range(12):
        n = int(rng.integers(0, 6 * TB))
        d = _soup(rng, n)
        idx, cnt, err, viol = emu.run_doc(d, nwaves=5, misalign=k % 16, ws=ws)
        oi, oe = oracle.index(d)
        assert viol == 0 and cnt[0] == len(oi) and err[0] == oe and np.array_equal(idx[:cnt[0]], oi), k


@pytest.mark.parametrize("build", sorted(emu.DOC_BUILDS))
def test_other_kernel_parameters(build):
    """Builds with two mask slots per wave (tiles finished one local pass after
    they publish), 4-row tiles, and 4-wave workgroups claiming 3 tiles at a
    time: soups over many tiles, a C1-like document, long backslash runs and
    a quote right after one at a tile start."""
    from paper_1902_08318_amd import synth
    rng = np.random.default_rng(77)
    tb = int(emu.load(build).emu_doc_tile_bytes())
    for k in range(2):
        d = _soup(rng, int(rng.integers(3 * tb, 9 * tb)))
        idx, n, err, viol = emu.run_doc(d, nwaves=int(rng.integers(4, 20)), misalign=k * 7, block_tiles=build)
        oi, oe = oracle.index(d)
        assert viol == 0 and n[0] == len(oi) and err[0] == oe and np.array_equal(idx[:n[0]], oi), (build, k)
    d = synth.gen_c1(11, 40 * tb, pool=32).data
    s = bytearray(d)
    s[5 * tb + 7: 9 * tb + 3] = b"\\" * (4 * tb - 4)
    s[9 * tb + 3] = ord('"')
    s[20 * tb - 70: 20 * tb - 1] = b"\\" * 69
    s[20 * tb - 1] = ord('"')
    for doc in (d, bytes(s)):
        idx, n, err, viol = emu.run_doc(doc, nwaves=24, misalign=0, block_tiles=build)
        oi, oe = oracle.index(doc)
        assert viol == 0 and n[0] == len(oi) and err[0] == oe and np.array_equal(idx[:n[0]], oi), build
