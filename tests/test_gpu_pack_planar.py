"""GPU parity of the pack kernels on planes of 4-byte values (Sec. 3
BitpackIntSoA, and BitpackFloatSoA in the fixed formats e8m7, e5m10, e8m15)
against the oracle, whole streams bit for bit.  Integer codes of B <= 27 bits
(not a multiple of 8) take the planar path, the rest the tile kernels;
explicit launch parameters select the tile kernels for every width, so both
are compared.  Sizes cover a partial last chunk of the planar path (2048
values per chunk, four chunks per workgroup), one value, a chunk boundary,
and workgroups whose four chunks span two fields' planes."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_blobs_equal, bits_planes, download, gpu_view, say

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

SIZES = [1, 100, 2047, 2048, 2049, 4109]


def check(rec, sspec, dspec, n, planes, tile_too=True):
    src_host = oracle.store_planes(rec, sspec, planes, fill=0x5A)
    sv = gpu_view(rec, sspec, n, src_host)
    exp = oracle.copy(rec, sspec, src_host, dspec, n, fill=0xA5)
    dv = gpu_view(rec, dspec, n, fill=0xA5)
    lm.llama_pack(sv, dv)
    assert_blobs_equal(download(dv), exp, "planar %s -> %s n=%d" % (sspec, dspec, n))
    dv.close()
    if tile_too and n >= 128:
        dv = gpu_view(rec, dspec, n, fill=0xA5)
        lm.llama_copy_ex(sv, dv, tile_records=1024)
        assert_blobs_equal(download(dv), exp, "tile %s -> %s n=%d" % (sspec, dspec, n))
        dv.close()
    sv.close()


@pytest.mark.parametrize("n", SIZES)
def test_int_codes_every_width(n):
    for t in ("i32", "u32"):
        rec = [t]
        planes = bits_planes(n, rec, seed=n)
        for B in range(1, 33):
            say("planar int", t, B, n)
            check(rec, {"kind": "soa_mb"}, {"kind": "bitpack_int", "bits": B}, n, planes, tile_too=B in (3, 13, 32))


@pytest.mark.parametrize("n", SIZES)
def test_float_fixed_formats(n):
    """Float codes take the tile kernels (direct stores of whole code words)."""
    rec = ["f32"]
    planes = bits_planes(n, rec, seed=n + 1)
    for E, M in ((8, 7), (5, 10), (8, 15)):
        say("planar float", E, M, n)
        check(rec, {"kind": "soa_mb"}, {"kind": "bitpack_float", "exp": E, "man": M}, n, planes)


@pytest.mark.parametrize("n", [4, 2048, 6148])
def test_source_layouts_and_fields(n):
    """SoA single- and multi-blob with three fields (planes on the 16-byte grid),
    AoS and AoSoA of one field."""
    rec3 = ["i32"] * 3
    planes = bits_planes(n, rec3, seed=7)
    for s in ({"kind": "soa_sb"}, {"kind": "soa_mb"}):
        for B in (5, 17, 32):
            say("planar fields", s, B, n)
            check(rec3, s, {"kind": "bitpack_int", "bits": B}, n, planes)
    for s in ({"kind": "aos"}, {"kind": "aosoa", "lanes": 8}):
        say("planar one field", s, n)
        check(["u32"], s, {"kind": "bitpack_int", "bits": 11}, n, planes[:1])


def test_tiles_across_fields_and_many_chunks():
    """1501 chunks of 2048 values per field over three fields: workgroups of
    four chunks straddle the planes' ends (1501 is not a multiple of 4), and a
    one-field stream of 8193 chunks ends in a partial tile."""
    n = 2048 * 1500 + 1
    rec = ["i32"] * 3
    planes = bits_planes(n, rec, seed=11)
    for B in (7, 24):
        say("planar loop", B)
        check(rec, {"kind": "soa_mb"}, {"kind": "bitpack_int", "bits": B}, n, planes, tile_too=False)
    n = 2048 * 4096 * 2 + 777  # one field, every wave three chunks
    planes = bits_planes(n, ["u32"], seed=12)
    say("planar loop one field")
    check(["u32"], {"kind": "soa_mb"}, {"kind": "bitpack_int", "bits": 13}, n, planes, tile_too=False)


def test_paths_not_taken():
    """SoA single-blob planes off the 16-byte grid (n odd), rounding to nearest
    even and other float formats take the tile kernels; results still match."""
    n = 1001
    rec = ["f32"] * 2
    planes = bits_planes(n, rec, seed=3)
    check(["i32"] * 2, {"kind": "soa_sb"}, {"kind": "bitpack_int", "bits": 9}, n,
          bits_planes(n, ["i32"] * 2, seed=4), tile_too=False)
    for d in ({"kind": "bitpack_float", "exp": 8, "man": 7, "round": "rne"}, {"kind": "bitpack_float", "exp": 6, "man": 9}):
        check(rec, {"kind": "soa_mb"}, d, n, planes, tile_too=False)
