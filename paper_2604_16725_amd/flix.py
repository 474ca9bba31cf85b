"""Thin ctypes binding of the FliX C ABI (``include/flix.h``).

Argument marshalling only: every step of every operation runs in the HIP
library ``lib/libflix.so``.  Device buffers are torch tensors on the GPU
(torch is used for device memory and streams, nothing else).  If the library
is missing, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libflix.so")

FLIX_OK, FLIX_EINVAL, FLIX_ENOMEM, FLIX_EHIP, FLIX_ESTATE = 0, -1, -2, -3, -4
_ERR_NAMES = {-1: "FLIX_EINVAL", -2: "FLIX_ENOMEM", -3: "FLIX_EHIP", -4: "FLIX_ESTATE"}


class FlixError(RuntimeError):
    def __init__(self, code: int, what: str):
        detail = ""
        if code in (FLIX_EHIP, FLIX_ENOMEM) and _lib is not None:
            detail = " (" + _lib.flix_last_error().decode(errors="replace") + ")"
        super().__init__(f"{what} failed: {_ERR_NAMES.get(code, code)}{detail}")
        self.code = code


class FlixConfig(ctypes.Structure):
    _fields_ = [
        ("key_bits", ctypes.c_uint32),
        ("bucket_capacity", ctypes.c_uint32),
        ("lanes_per_bucket", ctypes.c_uint32),
        ("radix_bits", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint64),
        ("pool_bytes", ctypes.c_uint64),
        ("fill", ctypes.c_uint32),
        ("insert_algo", ctypes.c_uint32),
        ("read_path", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


INSERT_ALGOS = {"tl_bulk": 0, "st_shift_right": 1, "st_tl_mixed": 2, "adaptive": 3}
READ_PATHS = {"sorted": 0, "groups": 1}


class FlixStats(ctypes.Structure):
    _fields_ = [
        ("buckets", ctypes.c_uint64),
        ("pool_nodes", ctypes.c_uint64),
        ("live_nodes", ctypes.c_uint64),
        ("capacity", ctypes.c_uint64),
        ("keys", ctypes.c_uint64),
    ]


class FlixBatch(ctypes.Structure):
    """One descriptor of a drained queue (layout of flix_batch in flix.h)."""
    _fields_ = [
        ("op", ctypes.c_uint32),
        ("n", ctypes.c_uint32),
        ("max_per_query", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("d_keys", ctypes.c_void_p),
        ("d_aux", ctypes.c_void_p),
        ("d_vals_out", ctypes.c_void_p),
        ("d_keys_out", ctypes.c_void_p),
        ("d_counts", ctypes.c_void_p),
        ("reserved2", ctypes.c_void_p),
    ]


class FlixEpoch(ctypes.Structure):
    """One coalesced epoch (layout of flix_epoch in flix.h)."""
    _fields_ = [
        ("n_lookup", ctypes.c_uint64),
        ("d_lookup_keys", ctypes.c_void_p),
        ("d_lookup_vals", ctypes.c_void_p),
        ("n_range", ctypes.c_uint64),
        ("range_max", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("d_range_lo", ctypes.c_void_p),
        ("d_range_hi", ctypes.c_void_p),
        ("d_range_counts", ctypes.c_void_p),
        ("d_range_keys", ctypes.c_void_p),
        ("d_range_vals", ctypes.c_void_p),
        ("n_update", ctypes.c_uint64),
        ("d_update_keys", ctypes.c_void_p),
        ("d_update_vals", ctypes.c_void_p),
    ]


EPOCH_SLOTS = 2
OP_LOOKUP, OP_SUCCESSOR, OP_RANGE, OP_INSERT, OP_DELETE, OP_PREDECESSOR = 0, 1, 2, 3, 4, 5
OPS = {"lookup": OP_LOOKUP, "successor": OP_SUCCESSOR, "range": OP_RANGE,
       "insert": OP_INSERT, "delete": OP_DELETE, "predecessor": OP_PREDECESSOR}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libflix.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"FliX HIP library not found at {path}; build it with "
            "`python -m paper_2604_16725_amd.build_lib` (no CPU fallback exists)")
    # One HIP runtime per process: torch carries its own build of it, so it is
    # loaded first and the library binds to that copy instead of a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "flix_create": (i32, [ctypes.POINTER(FlixConfig), vp, ctypes.POINTER(vp)]),
        "flix_bulk_load": (i32, [vp, vp, vp, u64, vp]),
        "flix_insert": (i32, [vp, vp, vp, u64, vp]),
        "flix_delete": (i32, [vp, vp, u64, vp]),
        "flix_lookup": (i32, [vp, vp, u64, vp, vp]),
        "flix_successor": (i32, [vp, vp, u64, vp, vp, vp]),
        "flix_predecessor": (i32, [vp, vp, u64, vp, vp, vp]),
        "flix_range": (i32, [vp, vp, vp, u64, u32, vp, vp, vp, vp]),
        "flix_destroy": (i32, [vp]),
        "flix_set_allocator": (i32, [vp, vp, vp]),
        "flix_restructure": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), vp]),
        "flix_size": (i32, [vp, ctypes.POINTER(u64), vp]),
        "flix_dump": (i32, [vp, vp, vp, u64, ctypes.POINTER(u64), vp]),
        "flix_dump_noalloc": (i32, [vp, vp, vp, u64, ctypes.POINTER(u64), vp]),
        "flix_check": (i32, [vp, vp]),
        "flix_status": (i32, [vp, vp]),
        "flix_get_stats": (i32, [vp, ctypes.POINTER(FlixStats), vp]),
        "flix_copy_layout": (i32, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(u64), vp]),
        "flix_sort_pairs": (i32, [vp, vp, u64, vp, vp, vp]),
        "flix_last_error": (ctypes.c_char_p, []),
        "flix_drain": (i32, [vp, vp, vp, u32, vp, vp]),
        "flix_drain_graph": (i32, [vp, vp, vp, u32, vp, ctypes.POINTER(vp), vp]),
        "flix_graph_launch": (i32, [vp, vp]),
        "flix_graph_destroy": (i32, [vp]),
        "flix_drain_info": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u64)]),
        "flix_set_timing": (i32, [vp, i32]),
        "flix_set_timing_only": (i32, [vp, ctypes.c_char_p]),
        "flix_epoch_prepare": (i32, [vp, u32, ctypes.POINTER(FlixEpoch), vp]),
        "flix_epoch_apply": (i32, [vp, u32, ctypes.POINTER(FlixEpoch), vp]),
        "flix_kernel_time": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(u64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_hook = None   # keeps the ctypes callbacks alive while they are installed


def use_torch_allocator(enable: bool = True):
    """Back every device buffer the library allocates afterwards with torch's
    caching allocator (flix_set_allocator), or restore hipMalloc / hipFree.
    Set it before creating stores; destroy stores created under it while it
    is still set."""
    global _hook
    import torch
    lib = load_library()
    if not enable:
        rc = lib.flix_set_allocator(None, None, None)
        if rc != FLIX_OK:
            raise FlixError(rc, "flix_set_allocator")
        _hook = None
        return

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
        except Exception:  # noqa: BLE001  (out of memory: the library reports ENOMEM)
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hook = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    rc = lib.flix_set_allocator(ctypes.cast(hook[0], ctypes.c_void_p),
                                ctypes.cast(hook[1], ctypes.c_void_p), None)
    if rc != FLIX_OK:
        raise FlixError(rc, "flix_set_allocator")
    _hook = hook


def _ptr(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Store:
    """A FliX store on the current GPU.

    Keys/values are 32- or 64-bit integer torch tensors on the GPU (signed or
    unsigned; the bits are read as unsigned keys).  Results come back in
    int32/int64 tensors carrying the unsigned bit patterns.
    """

    def __init__(self, key_bits: int = 32, capacity: int = 128, lanes: int = 16,
                 radix_bits: int = 8, max_batch: int = 1 << 20, pool_bytes: int = 0,
                 fill: int = 0, insert_algo="tl_bulk", read_path="sorted", stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.key_bits = key_bits
        self.dtype = torch.int32 if key_bits == 32 else torch.int64
        self._ok_dtypes = ((torch.int32, torch.uint32) if key_bits == 32
                           else (torch.int64, torch.uint64))
        algo = INSERT_ALGOS[insert_algo] if isinstance(insert_algo, str) else int(insert_algo)
        rp = READ_PATHS[read_path] if isinstance(read_path, str) else int(read_path)
        self.cfg = FlixConfig(key_bits, capacity, lanes, radix_bits, max_batch, pool_bytes,
                              fill, algo, rp, 0)
        h = ctypes.c_void_p()
        rc = self.lib.flix_create(ctypes.byref(self.cfg), _stream(stream), ctypes.byref(h))
        if rc != FLIX_OK:
            raise FlixError(rc, "flix_create")
        self.h = h

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.flix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc != FLIX_OK:
            raise FlixError(rc, what)

    def _dev(self, t):
        if not (t.is_cuda and t.dtype in self._ok_dtypes and t.is_contiguous()):
            raise TypeError(f"expected a contiguous {self.key_bits}-bit integer CUDA tensor, "
                            f"got {t.dtype} on {t.device}")
        return t

    def _empty(self, n, dtype=None):
        return self.torch.empty(n, dtype=dtype or self.dtype, device="cuda")

    # -- operations ----------------------------------------------------------
    def bulk_load(self, keys, vals, stream=None):
        self._chk(self.lib.flix_bulk_load(self.h, _ptr(self._dev(keys)), _ptr(self._dev(vals)),
                                          keys.numel(), _stream(stream)), "flix_bulk_load")

    def insert(self, keys, vals, stream=None, check=True):
        rc = self.lib.flix_insert(self.h, _ptr(self._dev(keys)), _ptr(self._dev(vals)),
                                  keys.numel(), _stream(stream))
        if check:
            self._chk(rc, "flix_insert")
        return rc

    def delete(self, keys, stream=None, check=True):
        rc = self.lib.flix_delete(self.h, _ptr(self._dev(keys)), keys.numel(), _stream(stream))
        if check:
            self._chk(rc, "flix_delete")
        return rc

    def lookup(self, keys, out=None, stream=None):
        out = self._empty(keys.numel()) if out is None else out
        self._chk(self.lib.flix_lookup(self.h, _ptr(self._dev(keys)), keys.numel(), _ptr(out),
                                       _stream(stream)), "flix_lookup")
        return out

    def successor(self, keys, out_k=None, out_v=None, stream=None):
        n = keys.numel()
        out_k = self._empty(n) if out_k is None else out_k
        out_v = self._empty(n) if out_v is None else out_v
        self._chk(self.lib.flix_successor(self.h, _ptr(self._dev(keys)), n, _ptr(out_k),
                                          _ptr(out_v), _stream(stream)), "flix_successor")
        return out_k, out_v

    def predecessor(self, keys, out_k=None, out_v=None, stream=None):
        n = keys.numel()
        out_k = self._empty(n) if out_k is None else out_k
        out_v = self._empty(n) if out_v is None else out_v
        self._chk(self.lib.flix_predecessor(self.h, _ptr(self._dev(keys)), n, _ptr(out_k),
                                            _ptr(out_v), _stream(stream)), "flix_predecessor")
        return out_k, out_v

    def range(self, lo, hi, max_per_query: int, counts=None, out_k=None, out_v=None,
              want_keys=True, want_vals=True, stream=None):
        n = lo.numel()
        counts = self._empty(n, self.torch.int32) if counts is None else counts
        if want_keys and out_k is None:
            out_k = self._empty(max(n * max_per_query, 1))
        if want_vals and out_v is None:
            out_v = self._empty(max(n * max_per_query, 1))
        self._chk(self.lib.flix_range(self.h, _ptr(self._dev(lo)), _ptr(self._dev(hi)), n,
                                      max_per_query, _ptr(counts),
                                      _ptr(out_k if want_keys else None),
                                      _ptr(out_v if want_vals else None), _stream(stream)),
                  "flix_range")
        return counts, out_k, out_v

    def restructure(self, stream=None):
        """Lay the store out again by the build rule; returns the nodes in use
        before and after."""
        b, a = ctypes.c_uint64(), ctypes.c_uint64()
        self._chk(self.lib.flix_restructure(self.h, ctypes.byref(b), ctypes.byref(a),
                                            _stream(stream)), "flix_restructure")
        return int(b.value), int(a.value)

    def size(self, stream=None) -> int:
        v = ctypes.c_uint64()
        self._chk(self.lib.flix_size(self.h, ctypes.byref(v), _stream(stream)), "flix_size")
        return int(v.value)

    def dump(self, stream=None):
        n = self.size(stream)
        k, v = self._empty(max(n, 1)), self._empty(max(n, 1))
        out_n = ctypes.c_uint64()
        self._chk(self.lib.flix_dump(self.h, _ptr(k), _ptr(v), max(n, 1), ctypes.byref(out_n),
                                     _stream(stream)), "flix_dump")
        m = int(out_n.value)
        return k[:m], v[:m]

    def dump_into(self, keys_out, vals_out, noalloc=False, stream=None) -> int:
        """Contents into caller-provided device buffers (flix_dump, or
        flix_dump_noalloc which allocates nothing); returns the key count."""
        fn = self.lib.flix_dump_noalloc if noalloc else self.lib.flix_dump
        out_n = ctypes.c_uint64()
        cap = min(keys_out.numel(), vals_out.numel())
        self._chk(fn(self.h, _ptr(keys_out), _ptr(vals_out), cap, ctypes.byref(out_n),
                     _stream(stream)), "flix_dump_noalloc" if noalloc else "flix_dump")
        return int(out_n.value)

    def check(self, stream=None) -> int:
        return int(self.lib.flix_check(self.h, _stream(stream)))

    def status(self, stream=None) -> int:
        return int(self.lib.flix_status(self.h, _stream(stream)))

    def stats(self, stream=None) -> dict:
        st = FlixStats()
        self._chk(self.lib.flix_get_stats(self.h, ctypes.byref(st), _stream(stream)), "flix_get_stats")
        return {f: int(getattr(st, f)) for f, _ in FlixStats._fields_}

    def copy_layout(self, stream=None):
        """Raw layout on the host as numpy arrays (tests only)."""
        import numpy as np
        st = self.stats(stream)
        nb, pool, cap = st["buckets"], st["pool_nodes"], st["capacity"]
        dt = np.uint32 if self.key_bits == 32 else np.uint64
        mkba = np.empty(nb, dtype=dt)
        hdr = np.empty(pool * 2, dtype=np.uint64)
        keys = np.empty(pool * cap, dtype=dt)
        vals = np.empty(pool * cap, dtype=dt)
        free = np.empty(pool, dtype=np.uint32)
        top = ctypes.c_uint64()
        p = lambda a: ctypes.c_void_p(a.ctypes.data)
        self._chk(self.lib.flix_copy_layout(self.h, p(mkba), p(hdr), p(keys), p(vals), p(free),
                                            ctypes.byref(top), _stream(stream)), "flix_copy_layout")
        hv = hdr.view(np.uint32).reshape(pool, 4)
        return dict(mkba=mkba, fence=hdr[0::2].copy(), size=hv[:, 2].copy(),
                    next=hv[:, 3].copy(), keys=keys.reshape(pool, cap),
                    vals=vals.reshape(pool, cap), free=free[: top.value].copy(),
                    buckets=nb, pool=pool, cap=cap)

    def sort_pairs(self, keys, stream=None):
        n = keys.numel()
        ko = self._empty(n)
        io = self._empty(n, self.torch.int32)
        self._chk(self.lib.flix_sort_pairs(self.h, _ptr(self._dev(keys)), n, _ptr(ko), _ptr(io),
                                           _stream(stream)), "flix_sort_pairs")
        return ko, io

    # -- persistent drain -----------------------------------------------------
    def make_batches(self, batches):
        """Host descriptor array from a list of dicts: op (name or code), keys,
        aux (insert values / range hi), out_v, out_k, counts, max_per_query."""
        arr = (FlixBatch * len(batches))()
        for i, b in enumerate(batches):
            op = OPS[b["op"]] if isinstance(b["op"], str) else int(b["op"])
            keys = b.get("keys")
            n = 0 if keys is None else keys.numel()
            arr[i] = FlixBatch(op, n, int(b.get("max_per_query", 0)), 0,
                               _ptr(keys).value, _ptr(b.get("aux")).value,
                               _ptr(b.get("out_v")).value, _ptr(b.get("out_k")).value,
                               _ptr(b.get("counts")).value, None)
        return arr

    def _dev_descriptors(self, arr, dev=None):
        raw = bytes(arr)
        host = self.torch.frombuffer(bytearray(raw), dtype=self.torch.uint8)
        if dev is None:
            return host.cuda()
        dev.copy_(host)
        return dev

    def drain(self, batches, timestamps=None, stream=None):
        """Run the batches in order in one persistent kernel launch."""
        arr = self.make_batches(batches)
        dev = self._dev_descriptors(arr)
        self._drain_keep = dev   # alive until the next drain
        rc = self.lib.flix_drain(self.h, ctypes.byref(arr), _ptr(dev), len(batches),
                                 _ptr(timestamps), _stream(stream))
        self._chk(rc, "flix_drain")

    def drain_graph(self, batches, timestamps=None, stream=None):
        """Capture a drain of these batches in a hipGraph; see DrainGraph."""
        return DrainGraph(self, batches, timestamps, stream)

    def drain_info(self):
        g, hz = ctypes.c_uint32(), ctypes.c_uint64()
        self._chk(self.lib.flix_drain_info(self.h, ctypes.byref(g), ctypes.byref(hz)),
                  "flix_drain_info")
        return int(g.value), int(hz.value)

    # -- epochs (serving form) -------------------------------------------------
    def make_epoch(self, lookup_keys=None, lookup_vals=None, range_lo=None, range_hi=None,
                   range_max: int = 0, range_counts=None, range_keys=None, range_vals=None,
                   update_keys=None, update_vals=None, n_lookup=None, n_range=None,
                   n_update=None):
        """An epoch descriptor over device tensors.  Counts default to the
        tensors' lengths; pass them to use a prefix of larger buffers."""
        n = lambda t, c: (0 if t is None else t.numel()) if c is None else int(c)
        return FlixEpoch(n(lookup_keys, n_lookup), _ptr(lookup_keys).value,
                         _ptr(lookup_vals).value, n(range_lo, n_range), int(range_max), 0,
                         _ptr(range_lo).value, _ptr(range_hi).value, _ptr(range_counts).value,
                         _ptr(range_keys).value, _ptr(range_vals).value, n(update_keys, n_update),
                         _ptr(update_keys).value, _ptr(update_vals).value)

    def epoch_prepare(self, slot: int, ep: FlixEpoch, stream=None):
        self._chk(self.lib.flix_epoch_prepare(self.h, slot, ctypes.byref(ep), _stream(stream)),
                  "flix_epoch_prepare")

    def epoch_apply(self, slot: int, ep: FlixEpoch, stream=None):
        self._chk(self.lib.flix_epoch_apply(self.h, slot, ctypes.byref(ep), _stream(stream)),
                  "flix_epoch_apply")

    def set_timing(self, on: bool, only: str | None = None):
        """Per-kernel HIP-event timing: every family, or only ``only``."""
        if on and only is not None:
            self._chk(self.lib.flix_set_timing_only(self.h, only.encode()), "flix_set_timing_only")
        else:
            self._chk(self.lib.flix_set_timing(self.h, 1 if on else 0), "flix_set_timing")

    def kernel_time(self, family: str):
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        self._chk(self.lib.flix_kernel_time(self.h, family.encode(), ctypes.byref(ms),
                                            ctypes.byref(n)), "flix_kernel_time")
        return ms.value, int(n.value)


class DrainGraph:
    """An instantiated hipGraph holding one drain launch.  `update(batches)`
    rewrites the device descriptors (same count) for the next replay."""

    def __init__(self, store, batches, timestamps=None, stream=None):
        self.store = store
        self.n = len(batches)
        self.stream = stream
        arr = store.make_batches(batches)
        self.dev = store._dev_descriptors(arr)
        store.torch.cuda.synchronize()
        ex = ctypes.c_void_p()
        rc = store.lib.flix_drain_graph(store.h, ctypes.byref(arr), _ptr(self.dev), self.n,
                                        _ptr(timestamps), ctypes.byref(ex), _stream(stream))
        if rc != FLIX_OK:
            raise FlixError(rc, "flix_drain_graph")
        self.ex = ex

    def update(self, batches):
        if len(batches) != self.n:
            raise ValueError("a graph replays a fixed number of batches")
        mb = self.store.cfg.max_batch
        for b in batches:
            if b.get("keys") is not None and b["keys"].numel() > mb:
                raise ValueError("batch larger than max_batch")
        arr = self.store.make_batches(batches)
        self.store._dev_descriptors(arr, self.dev)

    def launch(self, stream=None):
        rc = self.store.lib.flix_graph_launch(self.ex, _stream(stream or self.stream))
        if rc != FLIX_OK:
            raise FlixError(rc, "flix_graph_launch")

    def close(self):
        if getattr(self, "ex", None):
            self.store.lib.flix_graph_destroy(self.ex)
            self.ex = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
