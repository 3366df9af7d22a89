"""GPU parity of copies between views linearised in different orders (Sec. 2
array extents, row-major or column-major): dst(a) = src(a) for every
multi-index a, against the oracle's n-D copy, whole blobs bit for bit.  The
destination starts filled with a sentinel, so AoSoA padding lanes that a copy
must not write are checked too."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_blobs_equal, bits_planes, download, say, upload

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

LAYOUTS = {
    "aos": {"kind": "aos"},
    "soa_sb": {"kind": "soa_sb"},
    "soa_mb": {"kind": "soa_mb"},
    "aosoa32": {"kind": "aosoa", "lanes": 32},
    "aosoa3": {"kind": "aosoa", "lanes": 3},
    "bytesplit_sb": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    "bytesplit_aos": {"kind": "bytesplit", "inner": {"kind": "aos"}},
}
RECS = {"f32x7": ["f32"] * 7, "f64x3": ["f64"] * 3, "u8x5": ["u8"] * 5, "i16x3": ["i16", "u16", "i16"]}


def run(rec, sspec, dspec, ext, seed):
    n = int(np.prod(ext))
    planes = bits_planes(n, rec, seed)
    src_host = oracle.store_planes(rec, sspec, planes, fill=0x5A)
    exp = oracle.copy_nd(rec, sspec, src_host, dspec, list(ext), fill=0xA5)
    sv = lm.View(rec, sspec, list(ext), blobs=upload(src_host))
    dv = lm.View(rec, dspec, list(ext), fill=0xA5)
    lm.llama_copy(sv, dv)
    assert_blobs_equal(download(dv), exp, "%s -> %s ext=%s" % (sspec, dspec, ext))
    sv.close()
    dv.close()


@pytest.mark.parametrize("ext", [(37, 45), (5, 33, 9), (3, 4, 5, 6), (1, 70, 1, 40), (64, 64)])
@pytest.mark.parametrize("recname", sorted(RECS))
def test_row_to_column_major_all_layouts(ext, recname):
    rec = RECS[recname]
    names = sorted(LAYOUTS)
    for k, a in enumerate(names):
        b = names[(k * 3 + 1) % len(names)]
        for sc, dc in ((False, True), (True, False)):
            say("order", recname, ext, a, sc, b, dc)
            run(rec, dict(LAYOUTS[a], col_major=sc), dict(LAYOUTS[b], col_major=dc), ext, seed=k + 10 * sc)


def test_same_order_column_major_is_the_linear_copy():
    rec = RECS["f32x7"]
    for a, b in (("aos", "soa_mb"), ("aosoa32", "bytesplit_sb")):
        say("same order", a, b)
        run(rec, dict(LAYOUTS[a], col_major=True), dict(LAYOUTS[b], col_major=True), (19, 23, 3), seed=5)


def test_large_transpose_sampled_property():
    """1500 x 1501 records of 7 x f32 (63 MB per side), AoS row-major -> SoA-MB
    column-major: every record lands at its column-major position (the planes
    are numpy's C-to-F reordering of the source planes)."""
    ext = (1500, 1501)
    n = ext[0] * ext[1]
    rec = RECS["f32x7"]
    planes = bits_planes(n, rec, seed=99)
    say("large transpose", ext)
    src_host = oracle.store_planes(rec, {"kind": "aos"}, planes)
    sv = lm.View(rec, {"kind": "aos"}, list(ext), blobs=upload(src_host))
    dv = lm.View(rec, {"kind": "soa_mb", "col_major": True}, list(ext), fill=0)
    lm.llama_copy(sv, dv)
    got = download(dv)
    perm = np.arange(n).reshape(ext, order="C").ravel(order="F")
    for f in range(7):
        assert np.array_equal(got[f].view(np.uint32), planes[f].view(np.uint32)[perm]), f


def test_order_errors():
    rec = RECS["f32x7"]
    sv = lm.View(rec, {"kind": "aos"}, [4, 6], fill=0)
    with pytest.raises(lm.LlamaError) as e:
        lm.llama_copy(sv, lm.View(rec, {"kind": "aos", "col_major": True}, [6, 4], fill=0))
    assert e.value.name == "RECORD_MISMATCH"
    with pytest.raises(lm.LlamaError) as e:
        lm.Batch([sv], [lm.View(rec, {"kind": "soa_sb", "col_major": True}, [4, 6], fill=0)])
    assert e.value.name == "UNSUPPORTED"
    # one non-unit extent: both orders coincide, the copy is linear
    a = lm.View(rec, {"kind": "aos"}, [1, 50, 1], fill=0)
    lm.llama_copy(a, lm.View(rec, {"kind": "soa_sb", "col_major": True}, [1, 50, 1], fill=0))
