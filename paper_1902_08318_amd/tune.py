"""Autotuner of the batch kernel's tile size and of the kernel variant.

A batched launch (jsidx_build_batch, jsidx_minify, jsidx_minify_batch) cuts
its input into tiles; one wave indexes a tile row after row.  Small tiles
shorten the serial chain of one wave and spread a small input over more
waves; large tiles amortise the per-tile work (document table, carry
descriptors, look-back).  Where the balance lies depends on the device, so it
is measured: for every size class b (inputs of 2^b to 2^(b+1) bytes) the tuner
times a batch of documents of about 1.5 * 2^b bytes at each candidate tile
size and keeps the fastest.  The table goes to the library
(jsidx_set_tile_rows) and to a JSON cache keyed by the GPU architecture.  One
document (jsidx_build) runs a kernel with a fixed tile size and is not tuned.
The kernel variants (the default and those with one of the paper's stage-1
optimizations turned off, App. B) are alternatives too: with the table set,
each is timed on the whole batch and, if given, one large document, in
VARIANT_ROUNDS rounds over the variants in turn.  Another variant replaces the
default only if it wins on every workload by more than VARIANT_MARGIN of the
default's median time and by more than the run-to-run spread (each of its
round times below every round time of the default); the decision and its
reason are returned and logged (jsidx_set_variant).
Results never depend on the tile size or the variant; only time does.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import binding

CANDIDATES = (2, 4, 8, 16)
VARIANT_ROUNDS = 7
VARIANT_MARGIN = 0.03  # relative time a variant must save over the default


def default_cache_path(arch: str) -> str:
    root = os.environ.get("JSIDX_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "jsidx")
    return os.path.join(root, f"tile_rows_{arch}.json")


def _arch(torch) -> str:
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "unknown").split(":")[0]


def _time(torch, call, stream, reps):
    """Microseconds per launch: `reps` launches back to back between two
    events (an event between launches would add its own cost to each)."""
    for _ in range(3):
        rc = call()
        if rc:
            binding._check(rc)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        call()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e3


def choose_variant(samples: dict, margin: float = VARIANT_MARGIN) -> tuple[str, str]:
    """The variant to use from round times (samples[name][workload] = list of
    microseconds per launch): the fastest by mean relative median among those
    that beat the default on every workload by more than `margin` of its
    median and by more than the spread (every round time below every round
    time of the default); the default if none does.  Returns (name, reason)."""
    base = samples["default"]
    ok = {}
    for name, ks in samples.items():
        if name == "default":
            continue
        wins = all(np.median(t) < (1.0 - margin) * np.median(base[k]) and max(t) < min(base[k])
                   for k, t in ks.items())
        if wins:
            ok[name] = float(np.mean([np.median(t) / np.median(base[k]) for k, t in ks.items()]))
    if not ok:
        return "default", (f"no variant beat the default on every workload by more than {margin:.0%} "
                           "and beyond the spread of its round times")
    best = min(ok, key=lambda n: (ok[n], binding.VARIANTS[n]))
    return best, f"{best} beat the default on every workload (mean relative median {ok[best]:.3f})"


def autotune(data: bytes, offsets: np.ndarray, single: bytes | None = None, classes=range(12, 29),
             reps: int = 20, log=None, variants: bool = True) -> dict:
    """Measure every size class b on a prefix of the batch (whole documents,
    about 1.5 * 2^b bytes) at each candidate tile size; keep the size with
    the smallest time (ties: the larger tile).  Classes the batch does not
    reach keep the built-in choice.  Then, if `variants`, time the kernel
    variants on the whole batch and on `single` (one document) and keep one by
    choose_variant.  Sets both in the library and returns them with the
    timings (microseconds per launch) and the reason for the variant."""
    import ctypes
    import torch
    VP = ctypes.c_void_p
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    sp = VP(stream.cuda_stream)
    lib = binding.lib()
    total = int(offsets[-1])
    bufs = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    offs = torch.from_numpy(offsets.astype(np.int64)).to(dev)
    nd_all = offsets.size - 1
    cap = max(total, len(single) if single else 0)
    out = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    cnt = torch.empty(max(1, nd_all), dtype=torch.int32, device=dev)
    err = torch.empty(max(1, nd_all), dtype=torch.int32, device=dev)
    sbuf = torch.frombuffer(bytearray(single), dtype=torch.uint8).to(dev) if single else None
    binding.reserve(cap, stream, max_ndocs=nd_all)
    b0, o0, out0, c0, e0 = bufs.data_ptr(), offs.data_ptr(), out.data_ptr(), cnt.data_ptr(), err.data_ptr()

    def batch_call(nd):
        return lambda: lib.jsidx_build_batch(VP(b0), VP(o0), nd, VP(out0), VP(c0), VP(e0), sp)

    def single_call(n):
        return lambda: lib.jsidx_build(VP(sbuf.data_ptr()), n, VP(out0), VP(c0), VP(e0), sp)

    table = [0] * 64
    timings = {}
    variant, variant_us, reason = 0, {}, "variants not tuned"
    try:
        binding.set_variant(0)
        binding.set_tile_rows([])
        _time(torch, batch_call(nd_all), stream, 10)  # clocks up, memory touched
        for b in classes:
            want = int(1.5 * (1 << b))
            nd = int(np.searchsorted(offsets, offsets[0] + want, side="right")) - 1
            nd = max(1, min(nd, nd_all))
            got = int(offsets[nd] - offsets[0])
            if not (1 << b) <= got < (1 << (b + 1)) - 16:
                continue
            call = batch_call(nd)
            res = {}
            for r in CANDIDATES:
                t = [0] * 64
                t[b] = r
                binding.set_tile_rows(t)
                res[r] = _time(torch, call, stream, reps)
            best = min(CANDIDATES, key=lambda r: (res[r], -r))
            table[b] = best
            timings[b] = {"bytes": got, "docs": nd, "us": {str(r): round(v, 2) for r, v in res.items()}, "rows": best}
            if log:
                log(f"tune: class 2^{b}: batch of {nd} docs ({got} B): "
                    + " ".join(f"{r}:{res[r]:.1f}" for r in CANDIDATES) + f" us -> {best} rows")
        binding.set_tile_rows(table)
        if variants:
            work = {"batch": batch_call(nd_all)}
            if single:
                work["single"] = single_call(len(single))
            # rounds over the variants in turn (a drift of the device hits all alike)
            samples = {name: {k: [] for k in work} for name in binding.VARIANTS}
            for _ in range(VARIANT_ROUNDS):
                for name, v in binding.VARIANTS.items():
                    binding.set_variant(v)
                    for k, call in work.items():
                        samples[name][k].append(_time(torch, call, stream, max(5, reps // 2)))
            variant_us = {name: {k: {"median": round(float(np.median(t)), 2), "min": round(min(t), 2),
                                     "max": round(max(t), 2)} for k, t in ks.items()}
                          for name, ks in samples.items()}
            chosen, reason = choose_variant(samples)
            variant = binding.VARIANTS[chosen]
            if log:
                log("tune: variants " + "; ".join(
                    f"{name}: " + " ".join(f"{k} {t['median']:.1f} [{t['min']:.1f}..{t['max']:.1f}]"
                                           for k, t in us.items()) for name, us in variant_us.items())
                    + f" us -> {chosen} ({reason})")
    finally:
        binding.set_variant(0)
        binding.release(stream)
    binding.set_tile_rows(table)
    binding.set_variant(variant)
    return {"arch": _arch(torch), "table": table, "timings": timings, "variant": variant, "variant_us": variant_us,
            "variant_reason": reason, "when": time.strftime("%Y-%m-%d %H:%M:%S")}


def save(result: dict, path: str | None = None) -> str:
    path = path or default_cache_path(result["arch"])
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    return path


def load(path: str | None = None) -> dict | None:
    """Apply a cached table for this device's architecture, if there is one."""
    import torch
    arch = _arch(torch)
    path = path or default_cache_path(arch)
    try:
        with open(path) as f:
            res = json.load(f)
    except (OSError, ValueError):
        return None
    if res.get("arch") != arch or len(res.get("table", [])) != 64:
        return None
    binding.set_tile_rows(res["table"])
    binding.set_variant(int(res.get("variant", 0)))
    return res
