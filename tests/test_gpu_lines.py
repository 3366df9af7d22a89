"""GPU parity of the line-owner writes into single-blob planes off the
128-byte line grid (SoA single-blob and Bytesplit over it, with N * column
bytes not a multiple of 128), whole blobs bit for bit against the oracle.
Small explicit tiles make many tile boundaries, so every plane's boundary
lines, the halo records past each tile and the short last tile are
exercised; the destination starts filled with a sentinel."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_blobs_equal, bits_planes, download, gpu_view, say

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

RECS = {"f32x7": ["f32"] * 7, "f64x3": ["f64"] * 3, "u8x5": ["u8"] * 5, "i16x3": ["i16", "u16", "i16"]}
SRC = {
    "aos": {"kind": "aos"},
    "soa_sb": {"kind": "soa_sb"},
    "soa_mb": {"kind": "soa_mb"},
    "aosoa32": {"kind": "aosoa", "lanes": 32},
    "aosoa3": {"kind": "aosoa", "lanes": 3},
    "bs_sb": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    "bs_aosoa16": {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 16}},
}
DST = {"soa_sb": {"kind": "soa_sb"}, "bs_sb": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}}


def run(rec, a, b, n, planes, tile):
    src_host = oracle.store_planes(rec, a, planes, fill=0x5A)
    sv = gpu_view(rec, a, n, src_host)
    dv = gpu_view(rec, b, n, fill=0xA5)
    if tile:
        lm.llama_copy_ex(sv, dv, tile_records=tile)
    else:
        lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, a, src_host, b, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "%s -> %s n=%d tile=%d" % (a, b, n, tile))
    sv.close()
    dv.close()


@pytest.mark.parametrize("n", [4097, 12345, 100003, 4736])
@pytest.mark.parametrize("recname", sorted(RECS))
def test_line_owner_writes(recname, n):
    rec = RECS[recname]
    planes = bits_planes(n, rec, seed=n % 1000)
    for sname, sspec in SRC.items():
        for dname, dspec in DST.items():
            tiles = (0, 384) if sname == "aosoa3" else (0, 128, 256)
            for tile in tiles:
                say("lines", recname, sname, dname, n, tile)
                run(rec, sspec, dspec, n, planes, tile)
