"""Continuous-batching serving loop over jsidx_build_batch.

Requests are documents of a ring resident in HBM (request r is ring document
r mod ndocs); each has a host arrival time.  The loop admits requests that
have arrived by device memory: a request holds its bytes and its index (one
uint32 per byte at most), REQUEST_BYTES_PER_BYTE bytes per input byte, from
admission until the host sees it completed, and the admitted requests' held
bytes never exceed the budget (a request larger than the budget by itself is
admitted alone, when nothing else is held).  The admitted requests go out as
one batch -- a contiguous run of ring documents, so one offsets slice and one
jsidx_build_batch call -- on a free stream; a batch that would pass the budget
is cut to the requests that fit, and with none fitting the loop waits for
completions (an admission wait).  Several streams,
each with its own reserved workspace, keep batches in flight at once: work
admitted while earlier batches run overlaps with them on the device.  A
request completes when the host sees the event recorded after its batch; its
latency is that time minus its arrival time.

Per request there is no host work: admission is a binary search over the
arrival times and completion a vectorised store, so the loop runs once per
batch, not once per request.  Ring slots are reused by later requests; the
outputs of slot d live at out_idx + offsets[d] and out_n/out_err[d].  The
requests in flight always span less than one turn of the ring, so no two
batches in flight share a slot.
"""
from __future__ import annotations

import ctypes
import gc
import time
from dataclasses import dataclass

import numpy as np

from . import binding

REQUEST_BYTES_PER_BYTE = 5  # input byte + its uint32 index slot


@dataclass
class ServeResult:
    offered_fraction: float
    offered_docs_per_s: float
    requests: int
    seconds: float
    served_bytes: int
    batches: int
    p50_us: float
    p90_us: float
    p99_us: float
    max_us: float
    budget_bytes: int = 0
    peak_held_bytes: int = 0
    admission_waits: int = 0
    budget_cut_batches: int = 0

    def as_dict(self):
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in self.__dict__.items()} | {
            "sustained_GBps": round(self.served_bytes / self.seconds / 1e9, 2),
            "docs_per_s": round(self.requests / self.seconds)}


class Ring:
    """Device-resident request ring: bytes, offsets (int64, ndocs+1) and the
    per-slot outputs (index positions, counts, flags), plus the streams that
    batches run on (each with a workspace reserved for max_batch_bytes)."""

    def __init__(self, data: bytes, offsets: np.ndarray, max_batch_bytes: int, streams):
        import torch
        dev = torch.device("cuda:0")
        self.ndocs = offsets.size - 1
        self.total = int(offsets[-1])
        self.offs_h = offsets.astype(np.int64)
        self.max_doc = int(np.diff(self.offs_h).max()) if self.ndocs else 0
        self.bufs = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
        self.offs = torch.from_numpy(self.offs_h).to(dev)
        self.out = torch.empty(max(1, self.total), dtype=torch.int32, device=dev)
        self.cnt = torch.zeros(self.ndocs, dtype=torch.int32, device=dev)
        self.err = torch.zeros(self.ndocs, dtype=torch.int32, device=dev)
        self.streams = list(streams) if isinstance(streams, (list, tuple)) else [streams]
        self.max_batch_bytes = int(max_batch_bytes)
        for st in self.streams:
            binding.reserve(self.max_batch_bytes, st)
        torch.cuda.synchronize()
        self._lib = binding.lib()
        self._p = (self.bufs.data_ptr(), self.offs.data_ptr(), self.out.data_ptr(), self.cnt.data_ptr(),
                   self.err.data_ptr())
        self._s = [ctypes.c_void_p(st.cuda_stream) for st in self.streams]

    def launch(self, d0: int, nd: int, k: int = 0):
        """Index ring documents [d0, d0 + nd) with one batched launch on stream k."""
        b, o, out, cnt, err = self._p
        rc = self._lib.jsidx_build_batch(ctypes.c_void_p(b), ctypes.c_void_p(o + 8 * d0), nd,
                                         ctypes.c_void_p(out), ctypes.c_void_p(cnt + 4 * d0),
                                         ctypes.c_void_p(err + 4 * d0), self._s[k])
        if rc:
            binding._check(rc)

    def batch_end(self, r0: int, r_avail: int) -> int:
        """Last request (exclusive) of a batch starting at request r0 that
        stays inside the ring (no wrap) and within the reserved byte size."""
        d0 = r0 % self.ndocs
        lim = min(r_avail - r0, self.ndocs - d0)
        cap = self.offs_h[d0] + self.max_batch_bytes
        k = int(np.searchsorted(self.offs_h, cap, side="right")) - 1 - d0  # docs that fit
        return r0 + max(1, min(lim, k))


def poisson_arrivals(rng: np.random.Generator, rate: float, n: int) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate, n))


@dataclass
class Admission:
    """What the device-memory budget did during one run of the loop."""
    budget_bytes: int
    peak_held_bytes: int = 0
    admission_waits: int = 0      # times arrived work waited for completions
    budget_cut_batches: int = 0   # batches cut short to stay within the budget


def admit(ring: Ring, nxt: int, r1: int, held: int, budget: int) -> int:
    """End (exclusive) of the requests [nxt, r1) that may be admitted with
    `held` bytes already held: the longest prefix whose held bytes fit in
    budget - held; one request alone when nothing is held; nxt when none
    fits (wait)."""
    d0 = nxt % ring.ndocs
    room = budget - held
    cap = ring.offs_h[d0] + room // REQUEST_BYTES_PER_BYTE
    k = int(np.searchsorted(ring.offs_h, cap, side="right")) - 1 - d0  # whole docs that fit
    end = nxt + max(0, min(k, r1 - nxt))
    if end == nxt and held == 0:
        end = nxt + 1
    return end


def serve(ring: Ring, arrivals: np.ndarray, budget_bytes: int = 32 << 30, stats: Admission | None = None) -> tuple:
    """Run the loop over requests with the given arrival times (seconds from
    the start), one batch in flight per stream of the ring, admitting by the
    device-memory budget (held bytes = REQUEST_BYTES_PER_BYTE * request bytes).
    Returns (latency seconds per request, elapsed seconds, served bytes,
    batches); `stats`, if given, receives the admission figures."""
    import torch
    nreq = arrivals.size
    ns = len(ring.streams)
    lat = np.empty(nreq)
    busy = [None] * ns      # per stream: (event, r0, r1, held bytes) of its batch in flight
    events = [torch.cuda.Event() for _ in range(ns)]
    nxt = 0                 # first request not launched
    done = 0                # requests completed
    held = 0                # bytes held by admitted, not completed requests
    served = 0
    batches = 0
    budget = int(budget_bytes)
    st = stats if stats is not None else Admission(budget)
    st.budget_bytes = budget
    waiting = False
    gc_was = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        while done < nreq:
            oldest = nxt
            free = -1
            for k in range(ns):
                job = busy[k]
                if job is not None and job[0].query():
                    tc = time.perf_counter() - t0
                    _, r0, r1, hb = job
                    lat[r0:r1] = tc - arrivals[r0:r1]
                    done += r1 - r0
                    held -= hb
                    d0 = r0 % ring.ndocs
                    served += int(ring.offs_h[d0 + (r1 - r0)] - ring.offs_h[d0])
                    busy[k] = job = None
                if job is None:
                    if free < 0:
                        free = k
                elif job[1] < oldest:
                    oldest = job[1]
            if free < 0 or nxt >= nreq:
                continue
            now = time.perf_counter() - t0
            avail = int(np.searchsorted(arrivals, now, side="right"))
            if avail <= nxt:
                continue
            r1 = ring.batch_end(nxt, avail)
            # in flight: requests [oldest, r1) must stay within one turn of the ring
            r1 = min(r1, oldest + ring.ndocs)
            if r1 <= nxt:
                continue
            r_fit = admit(ring, nxt, r1, held, budget)
            if r_fit == nxt:
                if not waiting:
                    st.admission_waits += 1
                    waiting = True
                continue
            waiting = False
            if r_fit < r1:
                st.budget_cut_batches += 1
                r1 = r_fit
            d0 = nxt % ring.ndocs
            hb = REQUEST_BYTES_PER_BYTE * int(ring.offs_h[d0 + (r1 - nxt)] - ring.offs_h[d0])
            ring.launch(d0, r1 - nxt, free)
            ev = events[free]
            ev.record(ring.streams[free])
            busy[free] = (ev, nxt, r1, hb)
            held += hb
            st.peak_held_bytes = max(st.peak_held_bytes, held)
            nxt = r1
            batches += 1
        elapsed = time.perf_counter() - t0
    finally:
        if gc_was:
            gc.enable()
    return lat, elapsed, served, batches


def saturated_rate(ring: Ring, seconds: float = 0.5) -> float:
    """Bytes per second with every request already waiting (max-size batches
    back to back through the same loop)."""
    n = ring.ndocs
    reps = 1
    arr = np.zeros(n * reps)
    lat, el, served, _ = serve(ring, arr)
    while el < seconds and reps < 64:
        reps *= 2
        arr = np.zeros(n * reps)
        lat, el, served, _ = serve(ring, arr)
    return served / el


def run_load(ring: Ring, sat_bytes_per_s: float, fraction: float, seconds: float, seed: int,
             min_requests: int = 100_000, budget_bytes: int = 32 << 30) -> ServeResult:
    mean = ring.total / ring.ndocs
    rate = fraction * sat_bytes_per_s / mean
    n = max(min_requests, int(rate * seconds))
    rng = np.random.default_rng(seed)
    arr = poisson_arrivals(rng, rate, n)
    st = Admission(budget_bytes)
    lat, el, served, batches = serve(ring, arr, budget_bytes, st)
    us = lat * 1e6
    return ServeResult(fraction, rate, n, el, served, batches, float(np.percentile(us, 50)),
                       float(np.percentile(us, 90)), float(np.percentile(us, 99)), float(us.max()),
                       st.budget_bytes, st.peak_held_bytes, st.admission_waits, st.budget_cut_batches)
