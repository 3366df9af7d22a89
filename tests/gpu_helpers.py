"""Helpers shared by the GPU parity tests: host blobs <-> device views."""
import sys

import numpy as np

import oracle
import paper_2302_08251_amd as lm

F32x7 = ["f32"] * 7
F64x7 = ["f64"] * 7

CFG2 = {
    "aos": {"kind": "aos"},
    "soa_sb": {"kind": "soa_sb"},
    "soa_mb": {"kind": "soa_mb"},
    "aosoa32": {"kind": "aosoa", "lanes": 32},
    "aosoa64": {"kind": "aosoa", "lanes": 64},
    "bytesplit": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
}

NP = {"f32": np.float32, "f64": np.float64, "i8": np.int8, "u8": np.uint8, "i16": np.int16,
      "u16": np.uint16, "i32": np.int32, "u32": np.uint32, "i64": np.int64, "u64": np.uint64,
      "f16": np.float16, "bf16": np.uint16}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def upload(blobs):
    t = torch()
    out = []
    for b in blobs:
        d = t.empty(max(len(b), 16), dtype=t.uint8, device="cuda")
        if len(b):
            d[: len(b)].copy_(t.from_numpy(np.ascontiguousarray(b)))
        out.append(d)
    return out


def gpu_view(rec, spec, n, host_blobs=None, fill=0xA5, index="i64"):
    if host_blobs is None:
        return lm.View(rec, spec, [n], index_type=index, fill=fill)
    return lm.View(rec, spec, [n], blobs=upload(host_blobs), index_type=index)


def download(view):
    torch().cuda.synchronize()
    return [b[:s].cpu().numpy() for b, s in zip(view.blobs, view.sizes)]


def bits_planes(n, rec, seed):
    """Random bit patterns as planes of the record's types."""
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 256, n * np.dtype(NP[t]).itemsize, dtype=np.uint8).view(NP[t]) for t in rec]


def assert_blobs_equal(got, exp, what=""):
    assert len(got) == len(exp), what
    for b, (g, e) in enumerate(zip(got, exp)):
        if not np.array_equal(g, e):
            bad = np.nonzero(g != e)[0]
            raise AssertionError("%s blob %d: %d bytes differ, first at %d (got %#x, want %#x)" % (
                what, b, len(bad), bad[0], g[bad[0]], e[bad[0]]))
