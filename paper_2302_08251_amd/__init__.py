"""Python binding of libllama_mi.so, the gfx950 layout-copy / pack library.

Argument marshalling only: every step of a copy, pack, batch or n-body step
runs in the library's HIP kernels.  The functions keep the C ABI's names
(include/llama_mi.h); `View` and `Batch` are small conveniences that own
torch device tensors as blobs.  There is no CPU fallback: when the HIP
library is missing, loading raises `LlamaError`.

Records are lists of leaf type names ("f32", "f64", "i8" ... "u64", "f16",
"bf16"); mappings are dicts:
    {"kind": "aos"[, "packed": True]}   {"kind": "soa_sb"}   {"kind": "soa_mb"}
    {"kind": "aosoa", "lanes": L}       {"kind": "bytesplit", "inner": mapping}
    {"kind": "changetype", "stored": [types...], "inner": mapping}
    {"kind": "bitpack_int", "bits": B}  {"kind": "bitpack_float", "exp": E, "man": M}
    {"kind": "null"}    {"kind": "split", "at": k, "parts": [mapping, mapping]}
    {"kind": "field_access_count", "inner": mapping}
    {"kind": "heatmap", "granularity": G, "inner": mapping}
Any outermost mapping may add "col_major": True (extents linearised first
extent fastest).
"""
import ctypes as C
import os

__all__ = [
    "LlamaError", "lib", "View", "Batch", "LaunchParams", "BatchInfo",
    "llama_mapping_blob_count", "llama_mapping_blob_size", "llama_view_create",
    "llama_view_destroy", "llama_view_records", "llama_copy", "llama_copy_ex", "llama_pack",
    "llama_unpack", "llama_batch_create", "llama_batch_launch", "llama_batch_launch_per_view",
    "llama_batch_get_info", "llama_batch_destroy", "nbody_step", "nbody_step_noalloc", "nbody_energy",
    "llama_last_error", "llama_version", "SCALARS", "KINDS", "INDEX_TYPES",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllama_mi.so")

SCALARS = {"f32": 0, "f64": 1, "i8": 2, "u8": 3, "i16": 4, "u16": 5, "i32": 6, "u32": 7,
           "i64": 8, "u64": 9, "f16": 10, "bf16": 11}
KINDS = {"aos": 0, "soa_sb": 1, "soa_mb": 2, "aosoa": 3, "bytesplit": 4, "changetype": 5,
         "bitpack_int": 6, "bitpack_float": 7, "null": 8, "split": 9, "field_access_count": 10,
         "heatmap": 11}
INDEX_TYPES = {"i16": 0, "u16": 1, "i32": 2, "u32": 3, "i64": 4, "u64": 5}
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "INDEX_OVERFLOW",
          -4: "RECORD_MISMATCH", -5: "ALIGNMENT", -6: "HIP", -7: "NO_MEMORY"}
FLAG_AOS_PACKED = 1
FLAG_ROUND_RNE = 0x2
FLAG_COL_MAJOR = 0x4


class LlamaError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, message))


class _Record(C.Structure):
    _fields_ = [("n_fields", C.c_uint32), ("types", C.POINTER(C.c_int))]


class _Mapping(C.Structure):
    pass


_Mapping._fields_ = [("kind", C.c_int), ("lanes", C.c_uint32), ("bits", C.c_uint32),
                     ("exp_bits", C.c_uint32), ("man_bits", C.c_uint32), ("flags", C.c_uint32),
                     ("stored_types", C.POINTER(C.c_int)), ("inner", C.POINTER(_Mapping))]


class LaunchParams(C.Structure):
    _fields_ = [("tile_records", C.c_uint32), ("grid", C.c_uint32)]


class BatchInfo(C.Structure):
    _fields_ = [("n_views", C.c_uint32), ("tile_records", C.c_uint32), ("grid", C.c_uint32),
                ("total_tiles", C.c_uint64), ("algorithmic_bytes", C.c_uint64),
                ("tune_seconds", C.c_double), ("tile_map", C.c_uint32), ("reserved", C.c_uint32)]


_lib = None


def lib():
    """The loaded HIP library; raises LlamaError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LlamaError(-6, "HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    st, u32, u64, vp = C.c_int, C.c_uint32, C.c_uint64, C.c_void_p
    P = C.POINTER
    sig = {
        "llama_mapping_blob_count": [P(_Record), P(_Mapping), P(u32)],
        "llama_mapping_blob_size": [P(_Record), P(_Mapping), u32, P(u64), u32, P(u64)],
        "llama_view_create": [P(_Record), P(_Mapping), u32, P(u64), C.c_int, P(vp), P(u64), u32, P(vp)],
        "llama_view_destroy": [vp],
        "llama_view_records": [vp, P(u64)],
        "llama_copy": [vp, vp, vp],
        "llama_copy_ex": [vp, vp, P(LaunchParams), vp],
        "llama_pack": [vp, vp, vp],
        "llama_unpack": [vp, vp, vp],
        "llama_batch_create": [u32, P(vp), P(vp), C.c_char_p, P(vp)],
        "llama_batch_launch": [vp, vp],
        "llama_batch_launch_per_view": [vp, vp],
        "llama_batch_get_info": [vp, P(BatchInfo)],
        "llama_batch_destroy": [vp],
        "nbody_step": [vp, u32, C.c_float, C.c_float, vp],
        "nbody_step_noalloc": [vp, u32, C.c_float, C.c_float, vp],
        "nbody_energy": [vp, C.c_float, P(C.c_double), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = st
    L.llama_last_error.restype = C.c_char_p
    L.llama_last_error.argtypes = []
    L.llama_version.restype = C.c_char_p
    L.llama_version.argtypes = []
    _lib = L
    return L


def llama_last_error():
    return lib().llama_last_error().decode()


def llama_version():
    return lib().llama_version().decode()


def _check(status):
    if status != 0:
        raise LlamaError(status, llama_last_error())


class _Keep(list):
    pass


def _record(types, keep):
    arr = (C.c_int * len(types))(*[SCALARS[t] for t in types])
    r = _Record(len(types), arr)
    keep += [arr, r]
    return r


def _mapping(spec, keep):
    m = _Mapping()
    m.kind = KINDS[spec["kind"]]
    m.lanes = spec.get("lanes", spec.get("granularity", 0))
    m.bits = spec.get("bits", 0)
    m.exp_bits = spec.get("exp", 0)
    m.man_bits = spec.get("man", 0)
    m.flags = ((FLAG_AOS_PACKED if spec.get("packed") else 0) | (FLAG_ROUND_RNE if spec.get("round") == "rne" else 0)
               | (FLAG_COL_MAJOR if spec.get("col_major") else 0))
    if "stored" in spec:
        arr = (C.c_int * len(spec["stored"]))(*[SCALARS[t] for t in spec["stored"]])
        keep.append(arr)
        m.stored_types = arr
    if "inner" in spec:
        m.inner = C.pointer(_mapping(spec["inner"], keep))
    if spec["kind"] == "split":  # {"kind": "split", "at": k, "parts": [first, second]}
        m.lanes = spec["at"]
        parts = (_Mapping * 2)(_mapping(spec["parts"][0], keep), _mapping(spec["parts"][1], keep))
        keep.append(parts)
        m.inner = C.cast(parts, C.POINTER(_Mapping))
    keep.append(m)
    return m


def _extents(extents):
    if isinstance(extents, int):
        extents = [extents]
    return (C.c_uint64 * len(extents))(*extents), len(extents)


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return C.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(x):
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _nbytes(x):
    if hasattr(x, "data_ptr"):
        return x.numel() * x.element_size()
    raise TypeError("blob capacities are needed for raw pointers")


# ---------------------------------------------------------------- C ABI names

def llama_mapping_blob_count(record, mapping):
    k = _Keep()
    n = C.c_uint32()
    _check(lib().llama_mapping_blob_count(C.byref(_record(record, k)), C.byref(_mapping(mapping, k)),
                                          C.byref(n)))
    return n.value


def llama_mapping_blob_size(record, mapping, extents, blob):
    k = _Keep()
    ext, rank = _extents(extents)
    out = C.c_uint64()
    _check(lib().llama_mapping_blob_size(C.byref(_record(record, k)), C.byref(_mapping(mapping, k)),
                                         rank, ext, blob, C.byref(out)))
    return out.value


def blob_sizes(record, mapping, extents):
    return [llama_mapping_blob_size(record, mapping, extents, b)
            for b in range(llama_mapping_blob_count(record, mapping))]


def llama_view_create(record, mapping, extents, index_type, blobs, blob_bytes=None):
    """Returns an opaque view handle (int). `blobs` are device pointers or torch tensors."""
    k = _Keep()
    ext, rank = _extents(extents)
    ptrs = (C.c_void_p * max(1, len(blobs)))(*[_ptr(b) for b in blobs])
    if blob_bytes is None:
        blob_bytes = [_nbytes(b) for b in blobs]
    caps = (C.c_uint64 * max(1, len(blobs)))(*blob_bytes)
    out = C.c_void_p()
    _check(lib().llama_view_create(C.byref(_record(record, k)), C.byref(_mapping(mapping, k)), rank, ext,
                                   INDEX_TYPES[index_type], ptrs, caps, len(blobs), C.byref(out)))
    return out.value


def llama_view_destroy(handle):
    _check(lib().llama_view_destroy(C.c_void_p(handle)))


def llama_view_records(handle):
    n = C.c_uint64()
    _check(lib().llama_view_records(C.c_void_p(handle), C.byref(n)))
    return n.value


def _h(v):
    return C.c_void_p(v.handle if isinstance(v, View) else v)


def llama_copy(src, dst, stream=None):
    _check(lib().llama_copy(_h(src), _h(dst), _stream(stream)))


def llama_copy_ex(src, dst, tile_records=0, grid=0, stream=None):
    p = LaunchParams(tile_records, grid)
    _check(lib().llama_copy_ex(_h(src), _h(dst), C.byref(p), _stream(stream)))


def llama_pack(src, dst, stream=None):
    _check(lib().llama_pack(_h(src), _h(dst), _stream(stream)))


def llama_unpack(src, dst, stream=None):
    _check(lib().llama_unpack(_h(src), _h(dst), _stream(stream)))


def llama_batch_create(srcs, dsts, tune_cache=None):
    n = len(srcs)
    s = (C.c_void_p * n)(*[_h(v).value for v in srcs])
    d = (C.c_void_p * n)(*[_h(v).value for v in dsts])
    out = C.c_void_p()
    _check(lib().llama_batch_create(n, s, d, tune_cache.encode() if tune_cache else None, C.byref(out)))
    return out.value


def llama_batch_launch(batch, stream=None):
    _check(lib().llama_batch_launch(C.c_void_p(batch), _stream(stream)))


def llama_batch_launch_per_view(batch, stream=None):
    _check(lib().llama_batch_launch_per_view(C.c_void_p(batch), _stream(stream)))


def llama_batch_get_info(batch):
    info = BatchInfo()
    _check(lib().llama_batch_get_info(C.c_void_p(batch), C.byref(info)))
    return {f: getattr(info, f) for f, _ in BatchInfo._fields_}


def llama_batch_destroy(batch):
    _check(lib().llama_batch_destroy(C.c_void_p(batch)))


def nbody_step(view, steps, dt, eps2, stream=None):
    _check(lib().nbody_step(_h(view), steps, dt, eps2, _stream(stream)))


def nbody_step_noalloc(view, steps, dt, eps2, stream=None):
    _check(lib().nbody_step_noalloc(_h(view), steps, dt, eps2, _stream(stream)))


def nbody_energy(view, eps2, stream=None):
    e = C.c_double()
    _check(lib().nbody_energy(_h(view), eps2, C.byref(e), _stream(stream)))
    return e.value


# ---------------------------------------------------------------- conveniences

class View:
    """A view over torch uint8 device tensors (allocated here when `blobs` is None)."""

    def __init__(self, record, mapping, extents, blobs=None, index_type="i64", device="cuda",
                 fill=None):
        import torch
        self.record = list(record)
        self.mapping = mapping
        self.extents = [extents] if isinstance(extents, int) else list(extents)
        sizes = blob_sizes(self.record, mapping, self.extents)
        if blobs is None:
            blobs = []
            for s in sizes:
                t = torch.empty(max(s, 16), dtype=torch.uint8, device=device)
                if fill is not None:
                    t.fill_(fill)
                blobs.append(t)
        self.blobs = list(blobs)
        self.sizes = sizes
        self.handle = llama_view_create(self.record, mapping, self.extents, index_type, self.blobs)
        self.n = llama_view_records(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            llama_view_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, srcs, dsts, tune_cache=None):
        self.srcs, self.dsts = list(srcs), list(dsts)
        self.handle = llama_batch_create(self.srcs, self.dsts, tune_cache)

    def launch(self, stream=None):
        llama_batch_launch(self.handle, stream)

    def launch_per_view(self, stream=None):
        llama_batch_launch_per_view(self.handle, stream)

    def info(self):
        return llama_batch_get_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            llama_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
