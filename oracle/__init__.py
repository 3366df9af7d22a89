"""CPU oracle for the LLAMA hot path -- TEST INFRASTRUCTURE ONLY.

Plain per-element definitions of every mapping, codec and the FP64 n-body
(oracle.c).  Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline
leg import this package; the product library never does.

Mapping specs are plain dicts shared as *data* with the tests:
    {"kind": "aos", "packed": False}       {"kind": "soa_sb"}   {"kind": "soa_mb"}
    {"kind": "aosoa", "lanes": 32}         {"kind": "bytesplit", "inner": spec}
    {"kind": "changetype", "stored": ["f32", ...], "inner": spec}
    {"kind": "bitpack_int", "bits": 12}    {"kind": "bitpack_float", "exp": 8, "man": 15}
    {"kind": "null"}    {"kind": "split", "at": k, "parts": [spec, spec]}
    {"kind": "field_access_count", "inner": spec}
    {"kind": "heatmap", "granularity": G, "inner": spec}
Records are lists of leaf type names: "f32", "f64", "i8" ... "u64", "f16", "bf16".
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_TYPES = {"f32": 0, "f64": 1, "i8": 2, "u8": 3, "i16": 4, "u16": 5, "i32": 6, "u32": 7,
          "i64": 8, "u64": 9, "f16": 10, "bf16": 11}
_KINDS = {"aos": 0, "soa_sb": 1, "soa_mb": 2, "aosoa": 3, "bytesplit": 4, "changetype": 5,
          "bitpack_int": 6, "bitpack_float": 7, "null": 8, "split": 9, "field_access_count": 10,
          "heatmap": 11}
TYPE_SIZE = {"f32": 4, "f64": 8, "i8": 1, "u8": 1, "i16": 2, "u16": 2, "i32": 4, "u32": 4,
             "i64": 8, "u64": 8, "f16": 2, "bf16": 2}


class _Rec(C.Structure):
    _fields_ = [("nf", C.c_uint32), ("types", C.POINTER(C.c_int))]


class _Map(C.Structure):
    pass


_Map._fields_ = [("kind", C.c_int), ("lanes", C.c_uint32), ("bits", C.c_uint32),
                 ("exp_bits", C.c_uint32), ("man_bits", C.c_uint32), ("aos_packed", C.c_int),
                 ("stored_types", C.POINTER(C.c_int)), ("inner", C.POINTER(_Map)), ("round_rne", C.c_int)]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        u64, u32, i32 = C.c_uint64, C.c_uint32, C.c_int
        P = C.POINTER
        L.orc_type_size.restype = u32
        L.orc_blob_count.restype = u32
        L.orc_blob_count.argtypes = [P(_Rec), P(_Map)]
        L.orc_blob_size.restype = u64
        L.orc_blob_size.argtypes = [P(_Rec), P(_Map), u64, u32]
        L.orc_locate.restype = i32
        L.orc_locate.argtypes = [P(_Rec), P(_Map), u64, u64, u32, u32, P(u32), P(u64)]
        L.orc_load.restype = u64
        L.orc_load.argtypes = [P(_Rec), P(_Map), u64, C.c_void_p, u64, u32]
        L.orc_store.restype = None
        L.orc_store.argtypes = [P(_Rec), P(_Map), u64, C.c_void_p, u64, u32, u64]
        L.orc_copy.restype = i32
        L.orc_copy.argtypes = [P(_Rec), P(_Map), C.c_void_p, P(_Map), C.c_void_p, u64, i32]
        L.orc_linearize.restype = u64
        L.orc_linearize.argtypes = [u32, C.c_void_p, C.c_void_p, i32]
        L.orc_copy_nd.restype = i32
        L.orc_copy_nd.argtypes = [P(_Rec), P(_Map), C.c_void_p, i32, P(_Map), C.c_void_p, i32, u32, C.c_void_p]
        L.orc_nbody_view.restype = None
        L.orc_nbody_view.argtypes = [P(_Rec), P(_Map), C.c_void_p, u64, u32, C.c_double, C.c_double, u32]
        L.orc_energy_view.restype = C.c_double
        L.orc_energy_view.argtypes = [P(_Rec), P(_Map), C.c_void_p, u64, C.c_double]
        L.orc_load_many.restype = None
        L.orc_load_many.argtypes = [P(_Rec), P(_Map), u64, C.c_void_p, C.c_void_p, C.c_void_p,
                                    u64, C.c_void_p]
        L.orc_locate_many.restype = None
        L.orc_locate_many.argtypes = [P(_Rec), P(_Map), u64, C.c_void_p, C.c_void_p, C.c_void_p,
                                      u64, C.c_void_p, C.c_void_p]
        L.orc_convert.restype = u64
        L.orc_convert.argtypes = [u64, i32, i32]
        L.orc_conversion_supported.restype = i32
        L.orc_conversion_supported.argtypes = [i32, i32]
        L.orc_float_encode.restype = u64
        L.orc_float_encode.argtypes = [u64, i32, u32, u32]
        L.orc_float_decode.restype = u64
        L.orc_float_decode.argtypes = [u64, i32, u32, u32]
        L.orc_convert_array.restype = None
        L.orc_convert_array.argtypes = [C.c_void_p, i32, C.c_void_p, i32, u64, i32]
        L.orc_float_encode_array.restype = None
        L.orc_float_encode_array.argtypes = [C.c_void_p, i32, u32, u32, C.c_void_p, u64, i32, i32]
        L.orc_float_decode_array.restype = None
        L.orc_float_decode_array.argtypes = [C.c_void_p, i32, u32, u32, C.c_void_p, u64, i32]
        L.orc_nbody.restype = None
        L.orc_nbody.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, u64, u32, C.c_double,
                                C.c_double, i32]
        L.orc_energy.restype = C.c_double
        L.orc_energy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, u64, C.c_double, i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


class _Keep:
    """Holds ctypes objects alive for the lifetime of a converted spec."""

    def __init__(self):
        self.objs = []


def _rec(types, keep):
    arr = (C.c_int * len(types))(*[_TYPES[t] for t in types])
    keep.objs.append(arr)
    r = _Rec(len(types), arr)
    keep.objs.append(r)
    return r


def _map(spec, keep):
    m = _Map()
    m.kind = _KINDS[spec["kind"]]
    m.lanes = spec.get("lanes", spec.get("granularity", 0))
    m.bits = spec.get("bits", 0)
    m.exp_bits = spec.get("exp", 0)
    m.man_bits = spec.get("man", 0)
    m.aos_packed = 1 if spec.get("packed", False) else 0
    m.round_rne = 1 if spec.get("round") == "rne" else 0
    if "stored" in spec:
        arr = (C.c_int * len(spec["stored"]))(*[_TYPES[t] for t in spec["stored"]])
        keep.objs.append(arr)
        m.stored_types = arr
    if "inner" in spec:
        m.inner = C.pointer(_map(spec["inner"], keep))
    if spec["kind"] == "split":  # {"kind": "split", "at": k, "parts": [first, second]}
        m.lanes = spec["at"]
        parts = (_Map * 2)(_map(spec["parts"][0], keep), _map(spec["parts"][1], keep))
        keep.objs.append(parts)
        m.inner = C.cast(parts, C.POINTER(_Map))
    keep.objs.append(m)
    return m


def _ptrs(blobs, keep):
    arr = (C.c_void_p * max(1, len(blobs)))(*[b.ctypes.data for b in blobs])
    keep.objs.append(arr)
    return arr


def blob_count(rec, spec):
    k = _Keep()
    return lib().orc_blob_count(C.byref(_rec(rec, k)), C.byref(_map(spec, k)))


def blob_size(rec, spec, n, b):
    k = _Keep()
    return lib().orc_blob_size(C.byref(_rec(rec, k)), C.byref(_map(spec, k)), n, b)


def blob_sizes(rec, spec, n):
    return [blob_size(rec, spec, n, b) for b in range(blob_count(rec, spec))]


def locate(rec, spec, n, i, f, k=0):
    kp = _Keep()
    b, o = C.c_uint32(), C.c_uint64()
    rc = lib().orc_locate(C.byref(_rec(rec, kp)), C.byref(_map(spec, kp)), n, i, f, k,
                          C.byref(b), C.byref(o))
    if rc != 0:
        raise ValueError("not a physical mapping")
    return b.value, o.value


def locate_many(rec, spec, n, idx, fields, bytes_):
    kp = _Keep()
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    fields = np.ascontiguousarray(fields, dtype=np.uint32)
    bytes_ = np.ascontiguousarray(bytes_, dtype=np.uint32)
    blob = np.zeros(len(idx), np.uint32)
    off = np.zeros(len(idx), np.uint64)
    lib().orc_locate_many(C.byref(_rec(rec, kp)), C.byref(_map(spec, kp)), n, idx.ctypes.data,
                          fields.ctypes.data, bytes_.ctypes.data, len(idx), blob.ctypes.data,
                          off.ctypes.data)
    return blob, off


def alloc_blobs(rec, spec, n, fill=0):
    return [np.full(max(s, 0), fill, dtype=np.uint8) for s in blob_sizes(rec, spec, n)]


def copy(rec, src_spec, src_blobs, dst_spec, n, dst_blobs=None, threads=0, fill=0):
    """dst(i).f = src(i).f for all i < n and all fields (element by element)."""
    kp = _Keep()
    if dst_blobs is None:
        dst_blobs = alloc_blobs(rec, dst_spec, n, fill)
    r = _rec(rec, kp)
    lib().orc_copy(C.byref(r), C.byref(_map(src_spec, kp)), _ptrs(src_blobs, kp),
                   C.byref(_map(dst_spec, kp)), _ptrs(dst_blobs, kp), n, threads)
    return dst_blobs


def linearize(extents, a, col_major=False):
    """Linear index of multi-index `a` (Sec. 2 array extents), row-major unless col_major."""
    ext = (C.c_uint64 * len(extents))(*extents)
    idx = (C.c_uint64 * len(a))(*a)
    return lib().orc_linearize(len(extents), ext, idx, 1 if col_major else 0)


def copy_nd(rec, src_spec, src_blobs, dst_spec, extents, dst_blobs=None, fill=0):
    """dst(a).f = src(a).f for every multi-index a of `extents`; a spec with
    "col_major": True linearises its view column-major (first extent fastest)."""
    kp = _Keep()
    n = int(np.prod(extents, dtype=np.uint64)) if len(extents) else 0
    if dst_blobs is None:
        dst_blobs = alloc_blobs(rec, dst_spec, n, fill)
    ext = (C.c_uint64 * len(extents))(*extents)
    rc = lib().orc_copy_nd(C.byref(_rec(rec, kp)), C.byref(_map(src_spec, kp)), _ptrs(src_blobs, kp),
                           1 if src_spec.get("col_major") else 0, C.byref(_map(dst_spec, kp)),
                           _ptrs(dst_blobs, kp), 1 if dst_spec.get("col_major") else 0, len(extents), ext)
    if rc != 0:
        raise ValueError("rank must be 1..8")
    return dst_blobs


def store_planes(rec, spec, planes, fill=0, threads=0):
    """Blobs of `spec` holding field planes[f][i] (one numpy array per field)."""
    n = len(planes[0])
    src = [np.ascontiguousarray(p).view(np.uint8).reshape(-1) for p in planes]
    return copy(rec, {"kind": "soa_mb"}, src, spec, n, fill=fill, threads=threads)


_NP = {"f32": np.float32, "f64": np.float64, "i8": np.int8, "u8": np.uint8, "i16": np.int16,
       "u16": np.uint16, "i32": np.int32, "u32": np.uint32, "i64": np.int64, "u64": np.uint64,
       "f16": np.float16, "bf16": np.uint16}


def load_planes(rec, spec, blobs, n, threads=0):
    """Field planes (numpy arrays of the user types) read back through `spec`."""
    out = [np.zeros(n, dtype=_NP[t]) for t in rec]
    dst = [o.view(np.uint8).reshape(-1) for o in out]
    copy(rec, spec, blobs, {"kind": "soa_mb"}, n, dst_blobs=dst, threads=threads)
    return out


def load_many(rec, spec, n, blobs, idx, fields):
    kp = _Keep()
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    fields = np.ascontiguousarray(fields, dtype=np.uint32)
    out = np.zeros(len(idx), np.uint64)
    lib().orc_load_many(C.byref(_rec(rec, kp)), C.byref(_map(spec, kp)), n, _ptrs(blobs, kp),
                        idx.ctypes.data, fields.ctypes.data, len(idx), out.ctypes.data)
    return out


def convert(bits, src_type, dst_type):
    return lib().orc_convert(int(bits), _TYPES[src_type], _TYPES[dst_type])


def conversion_supported(src_type, dst_type):
    return bool(lib().orc_conversion_supported(_TYPES[src_type], _TYPES[dst_type]))


def convert_array(a, src_type, dst_type, threads=0):
    a = np.ascontiguousarray(a)
    out = np.zeros(len(a), dtype=_NP[dst_type])
    lib().orc_convert_array(a.ctypes.data, _TYPES[src_type], out.ctypes.data, _TYPES[dst_type],
                            len(a), threads)
    return out


def float_encode(bits, t, E, M):
    return lib().orc_float_encode(int(bits), _TYPES[t], E, M)


def float_decode(code, t, E, M):
    return lib().orc_float_decode(int(code), _TYPES[t], E, M)


def float_encode_array(a, t, E, M, threads=0, rne=False):
    a = np.ascontiguousarray(a)
    out = np.zeros(len(a), np.uint64)
    lib().orc_float_encode_array(a.ctypes.data, _TYPES[t], E, M, out.ctypes.data, len(a), threads, int(rne))
    return out


def float_decode_array(codes, t, E, M, threads=0):
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    out = np.zeros(len(codes), dtype=_NP[t])
    lib().orc_float_decode_array(codes.ctypes.data, _TYPES[t], E, M, out.ctypes.data, len(codes),
                                 threads)
    return out


def nbody(pos, vel, mass, steps, dt, eps2, threads=0):
    """FP64 all-pairs n-body; pos, vel: (n, 3) float64, mass: (n,). Returns new (pos, vel)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).copy()
    vel = np.ascontiguousarray(vel, dtype=np.float64).copy()
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    lib().orc_nbody(pos.ctypes.data, vel.ctypes.data, mass.ctypes.data, len(mass), steps, dt,
                    eps2, threads)
    return pos, vel


def energy(pos, vel, mass, eps2, threads=0):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    return lib().orc_energy(pos.ctypes.data, vel.ctypes.data, mass.ctypes.data, len(mass), eps2,
                            threads)


def nbody_view(rec, spec, blobs, n, steps, dt, eps2, tile=256):
    """FP64 n-body reading and writing the particles through `spec` (blobs updated in
    place), one access at a time in a tiled update's access pattern, so that
    instrumented mappings count every access (Sec. 4, Sec. 5)."""
    kp = _Keep()
    lib().orc_nbody_view(C.byref(_rec(rec, kp)), C.byref(_map(spec, kp)), _ptrs(blobs, kp), n, steps, dt, eps2,
                         tile)
    return blobs


def energy_view(rec, spec, blobs, n, eps2):
    """Energy of the particles as loaded through `spec`, every leaf loaded once."""
    kp = _Keep()
    return lib().orc_energy_view(C.byref(_rec(rec, kp)), C.byref(_map(spec, kp)), _ptrs(blobs, kp), n, eps2)


def max_threads():
    return lib().orc_max_threads()
