"""ctypes wrapper of the C++ oracle (``flix_oracle.cpp``) over numpy arrays.

Test infrastructure only: the product path never imports this module.  Every
operation takes and returns host numpy arrays of the key width (uint32 or
uint64); values have the same width as keys.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u64, u32p = ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.c_int]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_bulk_load.restype = ctypes.c_int
    lib.orc_bulk_load.argtypes = [vp, vp, vp, u64]
    lib.orc_insert.restype = ctypes.c_int
    lib.orc_insert.argtypes = [vp, vp, vp, u64]
    lib.orc_delete.argtypes = [vp, vp, u64]
    lib.orc_lookup.argtypes = [vp, vp, u64, vp]
    lib.orc_successor.argtypes = [vp, vp, u64, vp, vp]
    lib.orc_predecessor.argtypes = [vp, vp, u64, vp, vp]
    lib.orc_range.argtypes = [vp, vp, vp, u64, ctypes.c_uint32, vp, vp, vp]
    lib.orc_size.restype = u64
    lib.orc_size.argtypes = [vp]
    lib.orc_dump.argtypes = [vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


class Oracle:
    """Sequential ordered map over a sorted array (see flix_oracle.cpp)."""

    def __init__(self, key_bits: int):
        assert key_bits in (32, 64)
        self.key_bits = key_bits
        self.dtype = np.uint32 if key_bits == 32 else np.uint64
        self._lib = _load()
        self._h = self._lib.orc_create(key_bits)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def _arr(self, a):
        return np.ascontiguousarray(np.asarray(a, dtype=self.dtype))

    def bulk_load(self, keys, vals) -> int:
        k, v = self._arr(keys), self._arr(vals)
        assert k.shape == v.shape
        return self._lib.orc_bulk_load(self._h, _ptr(k), _ptr(v), k.size)

    def insert(self, keys, vals) -> int:
        k, v = self._arr(keys), self._arr(vals)
        assert k.shape == v.shape
        return self._lib.orc_insert(self._h, _ptr(k), _ptr(v), k.size)

    def delete(self, keys) -> None:
        k = self._arr(keys)
        self._lib.orc_delete(self._h, _ptr(k), k.size)

    def lookup(self, q):
        q = self._arr(q)
        out = np.empty_like(q)
        self._lib.orc_lookup(self._h, _ptr(q), q.size, _ptr(out))
        return out

    def successor(self, q):
        q = self._arr(q)
        ko, vo = np.empty_like(q), np.empty_like(q)
        self._lib.orc_successor(self._h, _ptr(q), q.size, _ptr(ko), _ptr(vo))
        return ko, vo

    def predecessor(self, q):
        """Largest stored key <= q and its value; (0, NOT_FOUND) on a miss."""
        q = self._arr(q)
        ko, vo = np.empty_like(q), np.empty_like(q)
        self._lib.orc_predecessor(self._h, _ptr(q), q.size, _ptr(ko), _ptr(vo))
        return ko, vo

    def range(self, lo, hi, max_per_query: int):
        """Returns (counts[n] uint32, keys[n, max], vals[n, max]).

        Slots at or beyond min(count, max) are left as zero here; only the
        first min(count, max) slots of each row are defined by the operation.
        """
        lo, hi = self._arr(lo), self._arr(hi)
        assert lo.shape == hi.shape
        n = lo.size
        counts = np.zeros(n, dtype=np.uint32)
        ko = np.zeros((n, max(max_per_query, 0)), dtype=self.dtype)
        vo = np.zeros_like(ko)
        self._lib.orc_range(self._h, _ptr(lo), _ptr(hi), n, max_per_query,
                            _ptr(counts), _ptr(ko), _ptr(vo))
        return counts, ko, vo

    def apply_epoch(self, lookup_keys, range_lo, range_hi, range_max: int, update_keys,
                    update_vals):
        """One epoch of mixed requests, in the order the serving form defines
        (the paper itself only has single-type batches): every lookup and
        range sees the map as it was before the epoch; then the updates take
        effect one after another in array order, where a value equal to the
        all-ones pattern deletes the key and any other value sets it.

        The sequential application is folded per key (a plain dict keeps the
        last entry of each key), then applied as one delete batch and one
        insert batch, which touch disjoint keys.
        Returns (lookup values, range counts, range values [n, range_max]).
        """
        lv = self.lookup(lookup_keys)
        rc, _, rv = self.range(range_lo, range_hi, range_max)
        tomb = (1 << self.key_bits) - 1
        last = {}
        for k, v in zip(np.asarray(update_keys).tolist(), np.asarray(update_vals).tolist()):
            last[k] = v
        dels = [k for k, v in last.items() if v == tomb]
        ups = [(k, v) for k, v in last.items() if v != tomb]
        if dels:
            self.delete(np.array(dels, dtype=self.dtype))
        if ups:
            rc_ins = self.insert(np.array([k for k, _ in ups], dtype=self.dtype),
                                 np.array([v for _, v in ups], dtype=self.dtype))
            assert rc_ins == 0
        return lv, rc, rv

    def size(self) -> int:
        return int(self._lib.orc_size(self._h))

    def dump(self):
        n = self.size()
        k = np.empty(n, dtype=self.dtype)
        v = np.empty(n, dtype=self.dtype)
        if n:
            self._lib.orc_dump(self._h, _ptr(k), _ptr(v))
        return k, v
