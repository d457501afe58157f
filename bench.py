#!/usr/bin/env python3
"""Benchmark of the stage-1 structural index on one MI355X.

Workload (default): one 256 MiB minified twitter-like JSON document (seed 1),
resident in HBM.  A step is one jsidx_build call over the whole document
(every stage-1 step: UTF-8 validation, escapes, string ranges, structural and
pseudo-structural bytes, flattening to uint32 positions, flags).  Three copies
of the input and outputs are rotated so that the 256 MB Infinity Cache does
not hold the data between steps.

Prints ONE JSON line.  value = input GB/s (1e9 bytes/s) over the timed steps;
roofline = algorithmic bytes (N read + 4*S written) per launch over the launch
time against 8 TB/s HBM; cpu_baseline = the CPU oracle on the same document.
Extra workloads (numeric pretty-printed document, 100k-document batch vs one
launch per document) are reported under "extra".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "structural-index GB/s (1 doc & batched) vs HBM peak; docs/s; p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["jsidx.hip", "jsidx_doc.h", "jsidx_kernel.h", "jsidx_device.h", "jsidx_prims.h"]
PROFILE = os.path.join(ROOT, "profiles", "doc_kernel_c1_256MiB.md")


def kernel_hash() -> str:
    """sha256[:16] of the kernel sources with comments and white space removed
    (a comment edit does not change the kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1902_08318_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(variant: str = "default"):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    of the one-document kernel on C1, from the committed profile, if it was
    taken on the current kernel sources and lists this kernel variant."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    import re
    m_hash = re.search(r"sha256\[:16\]: `([0-9a-f]{16})`", text)
    if not m_hash or m_hash.group(1) != kernel_hash():
        return None
    m_bytes = re.search(r"traffic_bytes_per_launch \(variant %s\): (\d+)" % re.escape(variant), text)
    return int(m_bytes.group(1)) if m_bytes else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_single(jx, torch, host: bytes, steps: int, warmup: int, copies: int = 3):
    """Time `steps` launches over rotating copies of one document between two
    events on the launch stream (the timed region), then the same launches
    with an event after each for the per-launch distribution, then launches
    each followed by reading the count back to the host (end to end)."""
    dev = torch.device("cuda:0")
    n = len(host)
    src = torch.frombuffer(bytearray(host), dtype=torch.uint8)
    bufs = [src.to(dev) for _ in range(copies)]
    outs = [torch.empty(n, dtype=torch.int32, device=dev) for _ in range(copies)]
    cnts = [torch.empty(1, dtype=torch.int32, device=dev) for _ in range(copies)]
    errs = [torch.empty(1, dtype=torch.int32, device=dev) for _ in range(copies)]
    stream = torch.cuda.current_stream()
    jx.reserve(n, stream)
    for i in range(warmup):
        k = i % copies
        jx.build(bufs[k], outs[k], cnts[k], errs[k], stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        k = i % copies
        jx.build(bufs[k], outs[k], cnts[k], errs[k], stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    S = int(cnts[0].item())
    err = int(errs[0].item())
    # per-launch distribution: a second pass with an event after every launch
    # (each event adds a little of its own time)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        k = i % copies
        jx.build(bufs[k], outs[k], cnts[k], errs[k], stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    # end to end: launch, then read the count back to the host (synchronous)
    e2e = []
    for i in range(max(5, min(steps, 20))):
        k = i % copies
        t = time.perf_counter()
        jx.build(bufs[k], outs[k], cnts[k], errs[k], stream)
        int(cnts[k].item())
        e2e.append((time.perf_counter() - t) * 1e3)
    diag = jx.diag(stream)
    del bufs, outs
    return {"ms_total": ms, "ms_per_launch": ms / steps, "S": S, "N": n, "flags": err, "diag": diag,
            "wall_s": wall, "launch_ms": pct(per), "e2e_ms": pct(np.array(e2e))}


# The paper's ablation of stage 1 (App. B, Table of optimizations), cycles per
# input byte on one Skylake core: all optimizations, then without the carry-less
# multiplication, with the naive bit extraction, with the naive classification.
PAPER_ABLATION = {"twitter": {"default": 0.90, "xor_loop": 0.92, "direct_flatten": 1.14, "naive_classify": 1.00},
                  "canada": {"default": 0.90, "xor_loop": 0.94, "direct_flatten": 0.96, "naive_classify": 0.96}}


def ablation(jx, torch, docs: dict, steps: int, restore: int, rounds: int = 5) -> dict:
    """Each kernel variant (one of the paper's stage-1 optimizations turned
    off) timed on the same documents as the default kernel: `rounds` rounds,
    each timing `steps` launches of every variant in turn between two events
    (interleaved, so that drifts of the device hit all alike); the median per
    variant in microseconds per launch and relative to the default, beside the
    paper's relative costs (twitter for C1, canada for C2: the same kinds of
    document)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {name: {} for name in jx.VARIANTS}
    try:
        for wl, data in docs.items():
            n = len(data)
            src = torch.frombuffer(bytearray(data), dtype=torch.uint8)
            bufs = [src.to(dev) for _ in range(3)]
            idx = torch.empty(n, dtype=torch.int32, device=dev)
            cnt = torch.empty(1, dtype=torch.int32, device=dev)
            err = torch.empty(1, dtype=torch.int32, device=dev)
            jx.reserve(n, stream)
            times = {name: [] for name in jx.VARIANTS}
            counts = {}
            for _ in range(rounds):
                for name, v in jx.VARIANTS.items():
                    jx.set_variant(v)
                    for i in range(2):
                        jx.build(bufs[i % 3], idx, cnt, err, stream)
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    for i in range(steps):
                        jx.build(bufs[i % 3], idx, cnt, err, stream)
                    b.record(stream)
                    torch.cuda.synchronize()
                    times[name].append(a.elapsed_time(b) / steps * 1e3)
                    counts[name] = int(cnt.item())
            for name in jx.VARIANTS:
                us = float(np.median(times[name]))
                out[name][wl] = {"us_per_launch": round(us, 2), "input_GBps": round(n / us / 1e3, 1),
                                 "index_entries": counts[name]}
            del bufs, idx
    finally:
        jx.set_variant(restore)
    for name in out:
        for wl in docs:
            base = out["default"][wl]
            if out[name][wl]["index_entries"] != base["index_entries"]:
                raise RuntimeError(f"variant {name} gave a different index on {wl}")
            out[name][wl]["vs_default"] = round(out[name][wl]["us_per_launch"] / base["us_per_launch"], 3)
        out[name]["paper_vs_default"] = {f: round(PAPER_ABLATION[f][name] / PAPER_ABLATION[f]["default"], 3)
                                         for f in PAPER_ABLATION}
    return out


def pct(x: np.ndarray) -> dict:
    """Summary of per-launch (or per-call) times: the mean is what a timed
    region of back-to-back launches sees; the median and the tail show how
    far single slow launches pull it up."""
    return {"mean": round(float(np.mean(x)), 4), "median": round(float(np.median(x)), 4),
            "p10": round(float(np.percentile(x, 10)), 4), "p90": round(float(np.percentile(x, 90)), 4),
            "p99": round(float(np.percentile(x, 99)), 4), "max": round(float(np.max(x)), 4), "n": int(x.size)}


def time_batch(jx, torch, data: bytes, offsets: np.ndarray, steps: int, warmup: int, per_doc_docs: int = 20000):
    dev = torch.device("cuda:0")
    total = int(offsets[-1])
    nd = offsets.size - 1
    bufs = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    offs = torch.from_numpy(offsets.astype(np.int64)).to(dev)
    out = torch.empty(total, dtype=torch.int32, device=dev)
    cnt = torch.empty(nd, dtype=torch.int32, device=dev)
    err = torch.empty(nd, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    jx.reserve(total, stream)
    for _ in range(warmup):
        jx.build_batch(bufs, offs, out, cnt, err, stream)
    torch.cuda.synchronize()
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    for i in range(steps):
        jx.build_batch(bufs, offs, out, cnt, err, stream)
    a1.record(stream)
    torch.cuda.synchronize()
    ms = a0.elapsed_time(a1) / steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        jx.build_batch(bufs, offs, out, cnt, err, stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    S = int(cnt.to(torch.int64).sum().item())
    # comparator: one jsidx_build launch per document, back to back on the same
    # stream (raw pointers, so the host loop costs as little as it can)
    lib = jx.binding.lib()
    import ctypes
    sp = ctypes.c_void_p(stream.cuda_stream)
    VP = ctypes.c_void_p
    b0, o0, c0, e0 = bufs.data_ptr(), out.data_ptr(), cnt.data_ptr(), err.data_ptr()
    per_doc_docs = min(nd, per_doc_docs)
    if per_doc_docs <= 0:
        return {"ms_per_launch": ms, "S": S, "N": total, "ndocs": nd, "launch_ms": pct(per),
                "docs_per_s": nd / (ms / 1e3)}
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for d in range(per_doc_docs):
        a, b = int(offsets[d]), int(offsets[d + 1])
        rc = lib.jsidx_build(VP(b0 + a), b - a, VP(o0 + 4 * a), VP(c0 + 4 * d), VP(e0 + 4 * d), sp)
        if rc:
            raise RuntimeError(f"jsidx_build failed ({rc})")
    t1.record(stream)
    torch.cuda.synchronize()
    per_doc_ms = t0.elapsed_time(t1)
    return {"ms_per_launch": ms, "S": S, "N": total, "ndocs": nd, "launch_ms": pct(per),
            "docs_per_s": nd / (ms / 1e3), "per_doc_launch_docs_per_s": per_doc_docs / (per_doc_ms / 1e3)}


def time_minify(jx, torch, data: bytes, offsets, steps: int, warmup: int = 2) -> dict:
    """The minify pass (white space outside strings dropped) over one document
    (offsets None) or a batch, resident in HBM; two events around the launches."""
    dev = torch.device("cuda:0")
    n = len(data)
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    out = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    nd = 1 if offsets is None else offsets.size - 1
    cnt = torch.empty(nd, dtype=torch.int32, device=dev)
    err = torch.empty(nd, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    jx.reserve(n, stream)
    if offsets is None:
        call = lambda: jx.minify(buf, out, cnt, err, stream)  # noqa: E731
    else:
        offs = torch.from_numpy(offsets.astype(np.int64)).to(dev)
        call = lambda: jx.minify_batch(buf, offs, out, cnt, err, stream)  # noqa: E731
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        call()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    kept = int(cnt.to(torch.int64).sum().item())
    return {"bytes": n, "kept_bytes": kept, "ms_per_launch": round(ms, 4),
            "input_GBps": round(n / (ms / 1e3) / 1e9, 2),
            "alg_GBps": round((n + kept + (16 * nd if offsets is not None else 0)) / (ms / 1e3) / 1e9, 1)}


def time_scopes(jx, torch, data: bytes, steps: int) -> dict:
    """Scope links over the document's index (jsidx_scopes), the index already
    built and resident; two events around the launches."""
    dev = torch.device("cuda:0")
    n = len(data)
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    jx.build(buf, idx, cnt, err, stream)
    k = int(cnt.item())
    match = torch.empty(k, dtype=torch.int32, device=dev)
    serr = torch.empty(1, dtype=torch.int32, device=dev)
    call = lambda: jx.scopes(buf, idx, match, serr, stream, n=k)  # noqa: E731
    for _ in range(2):
        call()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        call()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {"entries": k, "ms_per_call": round(ms, 4), "entries_per_s": round(k / (ms / 1e3)),
            "flags": int(serr.item()) & 0xFFFFFFFF}


def time_tape(jx, torch, data: bytes, steps: int) -> dict:
    """The stage-2 tape (jsidx_tape) over the document's index and links, both
    already built and resident; two events around the launches."""
    dev = torch.device("cuda:0")
    n = len(data)
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    err = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    jx.build(buf, idx, cnt, err, stream)
    k = int(cnt.item())
    match = torch.empty(k, dtype=torch.int32, device=dev)
    serr = torch.empty(1, dtype=torch.int32, device=dev)
    jx.scopes(buf, idx, match, serr, stream, n=k)
    words = torch.empty(2 * k + 2, dtype=torch.int64, device=dev)
    sbuf = torch.empty(n + 2 * k + 4, dtype=torch.uint8, device=dev)
    tn = torch.empty(1, dtype=torch.int64, device=dev)
    sn = torch.empty(1, dtype=torch.int64, device=dev)
    terr = torch.empty(1, dtype=torch.int32, device=dev)
    call = lambda: jx.tape(buf, idx, match, words, tn, sbuf, sn, terr, stream, n=k)  # noqa: E731
    for _ in range(2):
        call()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        call()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {"entries": k, "tape_words": int(tn.item()), "string_bytes": int(sn.item()), "ms_per_call": round(ms, 4),
            "input_GBps": round(n / (ms / 1e3) / 1e9, 1), "flags": int(terr.item()) & 0xFFFFFFFF,
            "scope_flags": int(serr.item()) & 0xFFFFFFFF}


def time_stage2_batch(jx, torch, data: bytes, offsets: np.ndarray, steps: int) -> dict:
    """The batched scope links (jsidx_scopes_batch) and the batched tape
    (jsidx_tape_batch) over the batch's resident index, after reserving both
    workspaces; two events around the launches of each."""
    dev = torch.device("cuda:0")
    nd = offsets.size - 1
    total = int(offsets[-1])
    buf = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    o = torch.from_numpy(offsets.astype(np.int64)).to(dev)
    idx = torch.empty(total, dtype=torch.int32, device=dev)
    cnt = torch.empty(nd, dtype=torch.int32, device=dev)
    err = torch.empty(nd, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    jx.build_batch(buf, o, idx, cnt, err, stream)
    torch.cuda.synchronize()
    ent = int(cnt.to(torch.int64).sum().item())
    jx.scopes_reserve(ent, nd, stream)
    jx.tape_reserve(ent, nd, stream)
    match = torch.empty(total, dtype=torch.int32, device=dev)
    serr = torch.empty(nd, dtype=torch.int32, device=dev)
    words = torch.empty(2 * (ent + nd), dtype=torch.int64, device=dev)
    sbuf = torch.empty(total + 2 * ent + 4, dtype=torch.uint8, device=dev)
    pos = torch.empty(4 * nd, dtype=torch.int64, device=dev)
    terr = torch.empty(nd, dtype=torch.int32, device=dev)
    out = {"docs": nd, "entries": ent}
    for name, call in (("scopes_batch", lambda: jx.scopes_batch(buf, o, idx, cnt, match, serr, stream)),
                       ("tape_batch", lambda: jx.tape_batch(buf, o, idx, cnt, match, words, sbuf, pos, terr, stream))):
        for _ in range(2):
            call()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            call()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[name] = {"ms_per_call": round(ms, 4), "docs_per_s": round(nd / (ms / 1e3)),
                     "input_GBps": round(total / (ms / 1e3) / 1e9, 1)}
    ef = terr.cpu().numpy().view(np.uint32) | serr.cpu().numpy().view(np.uint32)
    out["documents_flagged"] = int(np.count_nonzero(ef))
    return out


def cpu_batch_baseline(data: bytes, offsets: np.ndarray, budget_s: float = 6.0) -> dict:
    """The oracle over a batch: one core, then the documents partitioned into
    contiguous byte-balanced ranges over every host core (one thread each; the
    oracle's C loop runs without the interpreter lock)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    arr = np.frombuffer(data, dtype=np.uint8)
    nd = offsets.size - 1
    t = time.perf_counter()
    oracle.index_batch(arr, offsets)
    one = time.perf_counter() - t
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(cores, 64))
    cuts = np.searchsorted(offsets, np.linspace(0, int(offsets[-1]), cores + 1)).clip(0, nd)
    parts = [(int(cuts[i]), int(cuts[i + 1])) for i in range(cores) if cuts[i + 1] > cuts[i]]

    def work(p):
        a, b = p
        return oracle.index_batch(arr, (offsets[a:b + 1]).copy())

    with ThreadPoolExecutor(len(parts)) as ex:
        reps, t = 0, time.perf_counter()
        while True:
            list(ex.map(work, parts))
            reps += 1
            el = time.perf_counter() - t
            if el >= budget_s or reps >= 20:
                break
    return {"docs_per_s_1core": round(nd / one), "GBps_1core": round(len(data) / one / 1e9, 3),
            "docs_per_s_all_cores": round(nd * reps / el), "GBps_all_cores": round(len(data) * reps / el / 1e9, 3),
            "cores": len(parts), "kind": "oracle", "sample": f"the whole {nd}-document batch"}


def host_cpu() -> dict:
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": n}


def cpu_baseline(host: bytes, budget_s: float = 10.0):
    import oracle
    oracle.index(host[: 1 << 20])  # load
    times = []
    t0 = time.perf_counter()
    while True:
        t = time.perf_counter()
        oracle.index(host)
        times.append(time.perf_counter() - t)
        el = time.perf_counter() - t0
        if el >= budget_s or len(times) >= 50:
            break
    med = float(np.median(times))
    return {"value": len(host) / med / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"whole document ({len(host)} bytes) indexed {len(times)}x by the byte-at-a-time C oracle "
                      f"on one host core ({el:.1f} s); value from the median run",
            **host_cpu()}


def copy_ceiling(torch, nbytes: int = 256 << 20, reps: int = 20) -> dict:
    """Measured HBM ceiling: a plain device-to-device copy (reads and writes
    nbytes each), rotating buffers so the last-level cache does not hold them."""
    dev = torch.device("cuda:0")
    src = [torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(7) for _ in range(2)]
    dst = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(2)]
    for i in range(3):
        dst[i % 2].copy_(src[i % 2])
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(reps):
        dst[i % 2].copy_(src[(i + 1) % 2])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"bytes_moved_per_copy": 2 * nbytes, "GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1),
            "frac_of_peak": round(2 * nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def serve_c4(jx, torch, synth, seconds: float, nstreams: int = 3, budget: int = 32 << 30,
             forced_budget: int = 256 << 20) -> dict:
    """C4: Poisson arrivals of documents of 100 B..16 MB (log-normal) served by
    the continuous-batching loop (batches on `nstreams` streams at once) at
    30/60/90% of its saturated rate, admitted by device memory (a request
    holds 5 bytes per input byte: its bytes and its index) under the 32 GB
    budget, which a 1 GiB ring never fills; then the 90% load again under a
    forced budget of `forced_budget` held bytes, which binds."""
    from paper_1902_08318_amd import serve
    log("generating C4 (request ring)")
    data, offs = synth.gen_c4(4)
    # the oracle per host core on the first ~100 MB of requests, as context
    import oracle
    k = int(np.searchsorted(offs, 100 << 20))
    t = time.perf_counter()
    oracle.index_batch(np.frombuffer(data, dtype=np.uint8)[:int(offs[k])], offs[:k + 1])
    el = time.perf_counter() - t
    cpu = {"GBps_per_core": round(int(offs[k]) / el / 1e9, 3), "docs_per_s_per_core": round(k / el),
           "kind": "oracle", "sample": f"the first {k} requests ({int(offs[k])} bytes) on one host core"}
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    ring = serve.Ring(data, offs, 256 << 20, streams)
    del data
    sat = serve.saturated_rate(ring)
    loads = []
    for i, f in enumerate((0.3, 0.6, 0.9)):
        log(f"C4 serving at {int(f * 100)}% of saturation")
        loads.append(serve.run_load(ring, sat, f, seconds, 40 + i, budget_bytes=budget).as_dict())
    log(f"C4 serving at 90% of saturation under a forced budget of {forced_budget} bytes")
    forced = serve.run_load(ring, sat, 0.9, seconds, 42, budget_bytes=forced_budget).as_dict()
    diag = any(jx.diag(st) for st in streams)
    return {"ring_bytes": ring.total, "ring_docs": ring.ndocs, "mean_doc_bytes": round(ring.total / ring.ndocs),
            "max_doc_bytes": ring.max_doc, "streams": nstreams, "saturated_GBps": round(sat / 1e9, 2),
            "held_bytes_per_request_byte": serve.REQUEST_BYTES_PER_BYTE, "budget_bytes": budget,
            "loads": loads, "forced_budget": forced, "cpu_oracle": cpu,
            "note": "request bytes resident in HBM at arrival; latency = host-observed completion - arrival",
            **({"warning": "look-back diagnostic set"} if diag else {})}


def paper_context(n: int, s: int) -> dict:
    """The paper's own single-core stage-1 figures (2019 x86, context only):
    its cost model (Sec. 5: about 1.7 cycles per index entry plus 0.62 per
    byte on a 3.4 GHz Skylake) applied to this workload's N and S, and its
    measured cycles per byte for the twitter and canada files (appendix table
    of stage-1 optimisations), converted at 3.4 GHz."""
    cycles = 1.7 * s + 0.62 * n
    return {"model_GBps_per_core_this_workload": round(n / (cycles / 3.4e9) / 1e9, 2),
            "twitter_GBps_per_core": round(3.4 / 0.90, 2), "canada_GBps_per_core": round(3.4 / 0.90, 2),
            "hardware": "one Skylake core at 3.4 GHz (derived from cycles per byte)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extra", action="store_true", help="skip the numeric and batched workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--size-mib", type=int, default=256)
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "scopes", "tape", "minify"], default="c1",
                    help="headline workload (c2/c3/scopes/tape/minify only for profiling runs; scopes: the scope "
                         "links and structure check over the C1 index; tape: the stage-2 tape of C1; minify: "
                         "the minify pass over C2)")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="C4 serving loop: seconds per offered load (0 skips it)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in tile size choice")
    ap.add_argument("--tile-rows", type=int, choices=[2, 4, 8, 16], default=None,
                    help="every launch uses tiles of this many rows (no tuning)")
    ap.add_argument("--per-doc-docs", type=int, default=20000,
                    help="C3: documents timed one launch each as the comparator (0 skips it)")
    ap.add_argument("--variant", choices=["default", "naive_classify", "xor_loop", "direct_flatten"], default=None,
                    help="use this kernel variant (the tuner then does not choose one)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 256 MiB device copies (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1902_08318_amd as jx
    from paper_1902_08318_amd import synth
    assert torch.cuda.is_available(), "needs a HIP device"

    if args.copy_calibration:
        n = args.size_mib << 20
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": args.steps}), flush=True)
        return

    tuning = None
    c3 = None
    c1 = None
    if args.workload != "c3":
        c1 = (synth.gen_c2(2, args.size_mib << 20) if args.workload in ("c2", "minify")
              else synth.gen_c1(1, args.size_mib << 20))
    if args.tile_rows:
        jx.set_tile_rows([args.tile_rows] * 64)
    elif not args.no_tune:
        from paper_1902_08318_amd import tune
        log("autotuning the batch tile size (100k-document batch) and the kernel variant")
        c3 = synth.gen_c3(3)
        tuning = tune.autotune(c3[0], c3[1], c1.data if c1 is not None else None, log=log,
                               variants=args.variant is None)
    if args.variant is not None:
        jx.set_variant(jx.VARIANTS[args.variant])
    vname = args.variant or ({v: k for k, v in jx.VARIANTS.items()}[tuning["variant"]] if tuning else "default")
    if args.workload == "tape":
        print(json.dumps({"workload": "tape of C1", **time_tape(jx, torch, c1.data, args.steps)}), flush=True)
        return
    if args.workload == "minify":
        print(json.dumps({"workload": "minify of C2", **time_minify(jx, torch, c1.data, None, args.steps)}), flush=True)
        return
    if args.workload == "scopes":
        print(json.dumps({"workload": "scopes over the C1 index",
                          **time_scopes(jx, torch, c1.data, args.steps)}), flush=True)
        return
    if args.workload == "c3":
        data, offs, _ = c3 if c3 is not None else synth.gen_c3(3)
        r3 = time_batch(jx, torch, data, offs, args.steps, args.warmup, args.per_doc_docs)
        print(json.dumps({"workload": "C3", **r3}), flush=True)
        return
    log(f"timing {args.workload}: {len(c1.data)} bytes, {args.steps} steps")
    r1 = time_single(jx, torch, c1.data, args.steps, args.warmup)
    value = r1["N"] * args.steps / (r1["ms_total"] / 1e3) / 1e9
    alg_bytes = r1["N"] + 4 * r1["S"]
    achieved = alg_bytes / (r1["ms_per_launch"] / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r1["ms_per_launch"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "C1: one minified twitter-like JSON document, seed 1" if args.workload == "c1"
                   else "C2: one pretty-printed numeric (canada-like) JSON document, seed 2",
                   "bytes": r1["N"], "index_entries": r1["S"], "bytes_per_entry": round(r1["N"] / max(1, r1["S"]), 2),
                   "flags": r1["flags"], "kernel": f"doc_kernel, variant {vname}: tiles of 8 rows of 2 KiB",
                   "launch_ms": r1["launch_ms"], "end_to_end_ms": r1["e2e_ms"],
                   "timed_vs_launch_median": round(r1["ms_per_launch"] / r1["launch_ms"]["median"], 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(vname) if args.workload == "c1" else None},
    }
    out["roofline"]["copy_ceiling"] = copy_ceiling(torch)
    extra = {}
    if not args.no_extra:
        log("C0: one 1 MiB pretty-printed document (latency-bound)")
        c0 = synth.gen_c0(0).data
        r0 = time_single(jx, torch, c0, max(20, args.steps), args.warmup)
        extra["C0"] = {"bytes": r0["N"], "index_entries": r0["S"], "ms_per_launch": round(r0["ms_per_launch"], 4),
                       "input_GBps": round(r0["N"] / (r0["ms_per_launch"] / 1e3) / 1e9, 2),
                       "launch_ms": r0["launch_ms"], "end_to_end_ms": r0["e2e_ms"]}
        if not args.no_cpu:
            extra["C0"]["cpu_oracle"] = cpu_baseline(c0, budget_s=2.0)
        log("generating C2 (numeric, pretty-printed)")
        c2 = synth.gen_c2(2, args.size_mib << 20)
        r2 = time_single(jx, torch, c2.data, args.steps, args.warmup)
        extra["C2"] = {"bytes": r2["N"], "index_entries": r2["S"], "input_GBps": round(r2["N"] / (r2["ms_per_launch"] / 1e3) / 1e9, 2),
                       "alg_GBps": round((r2["N"] + 4 * r2["S"]) / (r2["ms_per_launch"] / 1e3) / 1e9, 1),
                       "ms_per_launch": round(r2["ms_per_launch"], 4), "launch_ms": r2["launch_ms"]}
        log("scope links over the C1 index")
        extra["scopes"] = {"C1": time_scopes(jx, torch, c1.data, max(3, args.steps // 2))}
        log("tape: C1 and C2")
        extra["tape"] = {"C1": time_tape(jx, torch, c1.data, max(3, args.steps // 2)),
                         "C2": time_tape(jx, torch, c2.data, max(3, args.steps // 2))}
        log("minify: C2 and the C3 batch")
        extra["minify"] = {"C2": time_minify(jx, torch, c2.data, None, args.steps)}
        log("kernel variants (the paper's stage-1 ablation) on C1 and C2")
        extra["ablation"] = ablation(jx, torch, {"C1": c1.data, "C2": c2.data}, max(3, args.steps // 2),
                                     jx.VARIANTS[vname])
        del c2
        log("generating C3 (100k-document batch)")
        data, offs, kinds = c3 if c3 is not None else synth.gen_c3(3)
        c3 = None
        r3 = time_batch(jx, torch, data, offs, max(3, args.steps // 2), 2)
        extra["C3"] = {"bytes": r3["N"], "ndocs": r3["ndocs"], "index_entries": r3["S"],
                       "input_GBps": round(r3["N"] / (r3["ms_per_launch"] / 1e3) / 1e9, 2),
                       "alg_GBps": round((r3["N"] + 4 * r3["S"] + 16 * r3["ndocs"]) / (r3["ms_per_launch"] / 1e3) / 1e9, 1),
                       "docs_per_s": round(r3["docs_per_s"]), "per_doc_launch_docs_per_s": round(r3["per_doc_launch_docs_per_s"]),
                       "batched_vs_per_doc": round(r3["docs_per_s"] / r3["per_doc_launch_docs_per_s"], 1),
                       "ms_per_launch": round(r3["ms_per_launch"], 4), "launch_ms": r3["launch_ms"]}
        extra["minify"]["C3"] = time_minify(jx, torch, data, offs, max(3, args.steps // 2))
        log("stage 2 over the C3 batch: scope links and tape, batched")
        extra["stage2_C3_batch"] = time_stage2_batch(jx, torch, data, offs, max(3, args.steps // 4))
        if not args.no_cpu:
            log("timing the CPU oracle on C3 (1 core, then all cores)")
            extra["C3"]["cpu_oracle"] = cpu_batch_baseline(data, offs)
        del data
        if args.serve_seconds > 0:
            extra["C4"] = serve_c4(jx, torch, synth, args.serve_seconds)
    if extra:
        out["extra"] = extra
    out["paper_context"] = paper_context(r1["N"], r1["S"])
    if tuning is not None:
        out["tuning"] = {"tile_rows_by_log2_bytes": {str(b): r for b, r in enumerate(tuning["table"]) if r},
                         "variant": tuning["variant"], "variant_us": tuning["variant_us"],
                         "variant_reason": tuning["variant_reason"], "arch": tuning["arch"]}
    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(c1.data)
    else:
        out["cpu_baseline"] = None
    if r1["diag"]:
        out["warning"] = "look-back diagnostic set"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
