"""The batching form: a stream of uneven mixed-type batches on one store,
run either as one call per batch (the plain form) or drained by the
persistent kernel captured in a hipGraph (one launch for the whole stream).

Everything here is host plumbing around the C ABI: the batches are uploaded
to HBM once, every step of every batch runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import flix

OP_CODE = {"lookup": 0, "successor": 1, "range": 2, "insert": 3, "delete": 4}


def pool_bytes_for(stream, capacity: int, max_batch: int = 1 << 20, key_bytes: int = 4,
                   limit: int | None = None) -> int:
    """Node pool for a store that bulk-loads the stream's keys and takes all of
    its inserts: twice the nodes the keys fill at the bulk-load fill (half the
    capacity), plus the per-call headroom the library reserves by default."""
    n = stream.nbatch if limit is None else min(limit, stream.nbatch)
    ins = int(stream.sizes[:n][stream.ops[:n] == 2].sum())
    f = capacity // 2
    nodes = 2 * (-(-(stream.n_keys + ins) // f)) + 2 * (-(-max_batch // f)) + 64
    return nodes * (capacity * 2 * key_bytes + 16)


class DeviceStream:
    """The first ``limit`` batches of a workload stream, resident in HBM.

    ``keys``/``vals`` hold every batch's inputs back to back (int32 carriers
    of the u32 bit patterns); ``offsets[i]`` is where batch i starts.  Output
    buffers are allocated per run with ``outputs()``.
    """

    def __init__(self, stream, limit: int | None = None, workers: int = 16):
        import torch
        self.torch = torch
        n = stream.nbatch if limit is None else min(limit, stream.nbatch)
        self.n = n
        with ThreadPoolExecutor(max_workers=workers) as ex:
            parts = list(ex.map(stream.batch, range(n)))
        self.ops = [p[0] for p in parts]
        sizes = np.array([p[1].size for p in parts], dtype=np.int64)
        self.sizes = sizes
        self.offsets = np.concatenate([[0], np.cumsum(sizes)])
        total = int(self.offsets[-1])
        self.total_ops = total
        hk = np.empty(max(total, 1), dtype=np.uint32)
        hv = np.zeros(max(total, 1), dtype=np.uint32)
        for i, (op, k, v) in enumerate(parts):
            a, b = self.offsets[i], self.offsets[i + 1]
            hk[a:b] = k
            if v is not None:
                hv[a:b] = v
        self.host_keys, self.host_vals = hk[:total], hv[:total]
        self.keys = torch.from_numpy(hk.view(np.int32)).cuda()
        self.vals = torch.from_numpy(hv.view(np.int32)).cuda()
        self.build_keys = torch.from_numpy(stream.build_keys.view(np.int32)).cuda()
        self.build_vals = torch.from_numpy(stream.build_vals.view(np.int32)).cuda()

    def outputs(self):
        t = self.torch
        n = max(self.total_ops, 1)
        return (t.full((n,), -1, dtype=t.int32, device="cuda"),
                t.full((n,), -1, dtype=t.int32, device="cuda"))

    def batch_dicts(self, out_v, out_k):
        """Descriptor dicts (``Store.make_batches`` form) over the outputs."""
        res = []
        for i, op in enumerate(self.ops):
            a, b = int(self.offsets[i]), int(self.offsets[i + 1])
            d = {"op": op, "keys": self.keys[a:b]}
            if op == "insert":
                d["aux"] = self.vals[a:b]
            if op in ("lookup", "successor"):
                d["out_v"] = out_v[a:b]
            if op == "successor":
                d["out_k"] = out_k[a:b]
            res.append(d)
        return res


def _plain_calls(st, dicts, stream_ptr):
    """(ABI function, argument tuple) of every batch, pointers resolved once."""
    lib, h = st.lib, st.h
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    calls = []
    for d in dicts:
        op, k = d["op"], d["keys"]
        n = k.numel()
        if op == "lookup":
            calls.append((lib.flix_lookup, (h, p(k), n, p(d["out_v"]), stream_ptr)))
        elif op == "successor":
            calls.append((lib.flix_successor, (h, p(k), n, p(d["out_k"]), p(d["out_v"]),
                                               stream_ptr)))
        elif op == "insert":
            calls.append((lib.flix_insert, (h, p(k), p(d["aux"]), n, stream_ptr)))
        elif op == "delete":
            calls.append((lib.flix_delete, (h, p(k), n, stream_ptr)))
        else:
            raise ValueError(op)
    return calls


def run_plain(st, ds: DeviceStream, outs, events: bool = True):
    """One ABI call per batch on the current stream.  Returns the wall time
    (s) from the first call to completion and the per-batch service times
    (s, from HIP events around each call; None without events)."""
    torch = ds.torch
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    calls = _plain_calls(st, ds.batch_dicts(*outs), sp)
    evs = ([(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in calls] if events else None)
    rcs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if events:
        for (fn, args), (e0, e1) in zip(calls, evs):
            e0.record()
            rcs.append(fn(*args))
            e1.record()
    else:
        for fn, args in calls:
            rcs.append(fn(*args))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = [i for i, rc in enumerate(rcs) if rc != flix.FLIX_OK]
    if bad:
        raise flix.FlixError(rcs[bad[0]], f"plain batch {bad[0]}")
    svc = (np.array([a.elapsed_time(b) for a, b in evs]) / 1e3) if events else None
    return wall, svc


class PersistentRun:
    """The whole stream as one persistent drain captured in a hipGraph."""

    def __init__(self, st, ds: DeviceStream, outs, stream):
        """``stream``: a torch stream other than the null stream (graph
        capture needs one); replays run on it."""
        torch = ds.torch
        self.st, self.ds, self.stream = st, ds, stream
        self.ts = torch.zeros(ds.n + 1, dtype=torch.int64, device="cuda")
        self.graph = st.drain_graph(ds.batch_dicts(*outs), timestamps=self.ts, stream=stream)

    def run(self):
        """Replay once.  Returns the wall time (s) from the replay to
        completion and the per-batch service times (s, device clock)."""
        torch = self.ds.torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.graph.launch(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        _, hz = self.st.drain_info()
        ts = self.ts.cpu().numpy().astype(np.int64)
        return wall, np.diff(ts) / float(hz)

    def close(self):
        self.graph.close()


def summarize(wall: float, svc, total_ops: int):
    out = {"Mops_s": round(total_ops / wall / 1e6, 1), "wall_ms": round(wall * 1e3, 3)}
    if svc is not None and len(svc):
        out.update(p50_us=round(float(np.percentile(svc, 50)) * 1e6, 2),
                   p99_us=round(float(np.percentile(svc, 99)) * 1e6, 2),
                   sum_service_ms=round(float(svc.sum()) * 1e3, 3))
    return out
