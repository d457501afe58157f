"""Helpers shared by the GPU tests: run the HIP library through its C ABI on
device tensors and compare with the CPU oracle element by element."""
from __future__ import annotations

import numpy as np

import oracle


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def gpu_index_single(data: bytes, misalign: int = 0):
    """jsidx_build on a device copy of `data` that starts `misalign` bytes past
    a 256-byte boundary.  Returns (positions uint32 np, n, err)."""
    import torch
    import paper_1902_08318_amd as jx
    dev = torch_dev()
    n = len(data)
    backing = torch.zeros(n + misalign + 64, dtype=torch.uint8, device=dev)
    if n:
        backing[misalign:misalign + n] = torch.frombuffer(bytearray(data), dtype=torch.uint8).to(dev)
    buf = backing[misalign:misalign + n] if n else backing[misalign:misalign]
    out = torch.full((max(1, n),), -1, dtype=torch.int32, device=dev)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=dev)
    err = torch.full((1,), -1, dtype=torch.int32, device=dev)
    jx.build(buf, out, cnt, err, length=n)
    torch.cuda.synchronize()
    k = int(cnt.item())
    return out[:max(0, k)].cpu().numpy().view(np.uint32), k, int(err.item()) & 0xFFFFFFFF


def gpu_index_batch(data: bytes | np.ndarray, offsets: np.ndarray, lead: int = 0):
    """jsidx_build_batch; returns (out_idx np uint32, out_n, out_err)."""
    import torch
    import paper_1902_08318_amd as jx
    dev = torch_dev()
    arr = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data
    total = int(offsets[-1])
    bufs = torch.zeros(arr.size + lead + 64, dtype=torch.uint8, device=dev)
    if arr.size:
        bufs[lead:lead + arr.size] = torch.from_numpy(arr.copy()).to(dev)
    offs = torch.from_numpy((offsets.astype(np.int64) + lead)).to(dev)
    out = torch.full((max(1, total + lead),), -1, dtype=torch.int32, device=dev)
    nd = offsets.size - 1
    n = torch.full((nd,), -1, dtype=torch.int32, device=dev)
    err = torch.full((nd,), -1, dtype=torch.int32, device=dev)
    jx.build_batch(bufs, offs, out, n, err)
    torch.cuda.synchronize()
    return (out.cpu().numpy().view(np.uint32)[lead:], n.cpu().numpy().view(np.uint32),
            err.cpu().numpy().view(np.uint32))


def assert_single_matches(data: bytes, misalign: int = 0, label: str = ""):
    idx, n, err = gpu_index_single(data, misalign)
    oi, oe = oracle.index(data)
    assert n == len(oi), f"{label}: count {n} != oracle {len(oi)} (len {len(data)})"
    assert err == oe, f"{label}: flags {err:#x} != oracle {oe:#x}"
    if n:
        bad = np.nonzero(idx != oi)[0]
        assert bad.size == 0, f"{label}: {bad.size} positions differ, first at {bad[0]}: {idx[bad[0]]} vs {oi[bad[0]]}"


def assert_batch_matches(data, offsets: np.ndarray, lead: int = 0, label: str = ""):
    arr = np.frombuffer(data, dtype=np.uint8) if isinstance(data, (bytes, bytearray)) else data
    gi, gn, ge = gpu_index_batch(arr, offsets, lead)
    oi, on, oe = oracle.index_batch(arr, offsets)
    bad_n = np.nonzero(gn != on)[0]
    assert bad_n.size == 0, f"{label}: {bad_n.size} counts differ, first doc {bad_n[0]}: {gn[bad_n[0]]} vs {on[bad_n[0]]}"
    bad_e = np.nonzero(ge != oe)[0]
    assert bad_e.size == 0, f"{label}: {bad_e.size} flags differ, first doc {bad_e[0]}: {ge[bad_e[0]]:#x} vs {oe[bad_e[0]]:#x}"
    # compare every document's region [offsets[d], offsets[d] + n[d])
    starts = offsets[:-1].astype(np.int64)
    total = int(offsets[-1])
    valid = np.zeros(total, dtype=bool)
    if total:
        # mark the positions that hold index entries
        cnt = on.astype(np.int64)
        nz = cnt > 0
        idx_starts = starts[nz]
        lens = cnt[nz]
        if lens.size:
            rep = np.repeat(idx_starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
            pos = rep + np.arange(int(lens.sum()))
            valid[pos] = True
        diff = np.nonzero(valid & (gi[:total] != oi[:total]))[0]
        assert diff.size == 0, f"{label}: {diff.size} index entries differ, first at {diff[0]}"
