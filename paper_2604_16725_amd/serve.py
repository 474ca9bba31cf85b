"""The serving form: a request loop over a device-resident store.

Requests (each a mix of lookups, ranges, inserts and deletes) arrive open
loop.  The engine coalesces the requests that have arrived into epochs, in
arrival order, admits them against a device-memory budget and the epoch
capacity, and runs each epoch through the library's epoch calls: while
epoch t is applied on one stream, epoch t+1 is copied in and sorted on a
second stream (two slots).  Results go back to pinned host memory; a
request's latency runs from its arrival to the moment its results are on
the host.

Order inside an epoch (the paper has only single-type batches): reads see
the store as it was before the epoch, then the epoch's updates take effect
with the last update of a key winning.  The plain form runs every request
alone as its own epoch, one after the other.

The engine talks to a backend (``GpuBackend`` here; the tests add a CPU one
with a simulated clock), so its coalescing, admission and
accounting logic runs on any machine.
"""
from __future__ import annotations

import collections
import gc
import time

import numpy as np

LOOKUP, RANGE, INSERT, DELETE = 0, 1, 2, 3


class EpochLists:
    """The three lists of an epoch built from requests in admitted order,
    with the bookkeeping to hand results back to each request."""

    def __init__(self, wl, req_ids, tomb):
        self.req_ids = list(req_ids)
        ids = np.asarray(self.req_ids, dtype=np.int64)
        # operation indices of the requests, in admitted order, without a
        # Python loop over requests: each request's run of indices is its
        # start plus a ramp that restarts at every request
        starts = wl.offsets[ids].astype(np.int64)
        lens = wl.offsets[ids + 1].astype(np.int64) - starts
        total = int(lens.sum())
        ramp = np.arange(total, dtype=np.int64)
        idx = np.repeat(starts - (np.cumsum(lens) - lens), lens) + ramp
        ops, keys, aux = wl.ops[idx], wl.keys[idx], wl.aux[idx]
        is_l, is_r = ops == LOOKUP, ops == RANGE
        is_u = ops >= INSERT
        self.flat_lookup = idx[is_l]            # workload op index of every lookup
        self.range_ord = wl.range_ordinal[idx[is_r]]
        self.lookup_keys = keys[is_l]
        self.range_lo = keys[is_r]
        self.range_hi = aux[is_r]
        self.update_keys = keys[is_u]
        self.update_vals = np.where(ops[is_u] == INSERT, aux[is_u], tomb).astype(keys.dtype)
        self.n_ops = idx.size

    @property
    def counts(self):
        return self.lookup_keys.size, self.range_lo.size, self.update_keys.size


def request_bytes_all(wl, key_bytes, range_max):
    """request_bytes of every request at once (one pass over the operations)."""
    n = wl.n_req
    sizes = np.diff(wl.offsets).astype(np.int64)
    req = np.repeat(np.arange(n), sizes)
    nl = np.bincount(req, weights=(wl.ops == LOOKUP), minlength=n).astype(np.int64)
    nr = np.bincount(req, weights=(wl.ops == RANGE), minlength=n).astype(np.int64)
    return sizes * 2 * key_bytes + nl * key_bytes + nr * (4 + range_max * key_bytes)


def request_bytes(wl, i, key_bytes, range_max):
    """Device bytes a request occupies while in flight: its inputs (key and
    aux per operation) and its outputs (a value per lookup, a count and
    range_max values per range)."""
    a, b = int(wl.offsets[i]), int(wl.offsets[i + 1])
    ops = wl.ops[a:b]
    nl = int((ops == LOOKUP).sum())
    nr = int((ops == RANGE).sum())
    return (b - a) * 2 * key_bytes + nl * key_bytes + nr * (4 + range_max * key_bytes)


class Results:
    """Per-operation results of a whole workload run."""

    def __init__(self, wl, range_max, dtype):
        self.lookup = np.zeros(wl.total_ops, dtype=dtype)
        self.range_count = np.zeros(max(wl.n_ranges, 1), dtype=np.uint32)
        self.range_vals = np.zeros((max(wl.n_ranges, 1), range_max), dtype=dtype)

    def store(self, ep: EpochLists, lv, rc, rv, range_max):
        self.lookup[ep.flat_lookup] = lv
        if ep.range_ord.size:
            self.range_count[ep.range_ord] = rc
            self.range_vals[ep.range_ord] = rv.reshape(-1, range_max)


class Engine:
    """Coalescing, admission and epoch pipelining over a backend.

    ``max_epoch_ops``: capacity of one epoch (operations); ``budget``: bytes
    of device memory the requests in flight may occupy; ``coalesce``: False
    gives the plain form (one request per epoch, one epoch in flight)."""

    def __init__(self, backend, max_epoch_ops: int, budget: int, coalesce: bool = True):
        self.be = backend
        self.max_epoch_ops = max_epoch_ops
        self.budget = budget
        self.coalesce = coalesce
        self.slots = backend.slots if coalesce else 1

    def run(self, wl, arrivals, tomb, key_bytes, range_max):
        """Serve every request of `wl` at its arrival time.  The loop runs with
        Python's cyclic garbage collector paused (a full collection over the
        per-request objects stalls the loop for tens of milliseconds, which
        shows up as tail latency of whatever requests are waiting)."""
        was = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            return self._run(wl, arrivals, tomb, key_bytes, range_max)
        finally:
            if was:
                gc.enable()

    def _run(self, wl, arrivals, tomb, key_bytes, range_max):
        be = self.be
        n = wl.n_req
        res = Results(wl, range_max, wl.keys.dtype)
        done_at = np.full(n, np.nan)
        rbytes = request_bytes_all(wl, key_bytes, range_max)
        queue = collections.deque()
        inflight = {}              # slot -> (handle, EpochLists, bytes)
        next_slot = 0
        in_bytes = 0
        max_in_bytes = 0
        epochs = []                # admitted order: list of request id lists
        rejected = []
        nxt = 0
        finished = 0
        t0 = be.now()
        while finished + len(rejected) < n:
            now = be.now() - t0
            progressed = False
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
                progressed = True
            for slot in list(inflight):
                h, ep, b = inflight[slot]
                if be.ready(h):
                    lv, rc, rv = be.results(h)
                    res.store(ep, lv, rc, rv, range_max)
                    t_done = be.now() - t0
                    done_at[ep.req_ids] = t_done
                    finished += len(ep.req_ids)
                    in_bytes -= b
                    del inflight[slot]
                    progressed = True
            # form epochs while the next slot is free and requests wait
            while queue and next_slot not in inflight:
                take, ops, b = [], 0, 0
                while queue:
                    i = queue[0]
                    sz = int(wl.sizes[i])
                    if rbytes[i] > self.budget or sz > self.max_epoch_ops:
                        rejected.append(queue.popleft())   # can never be admitted
                        continue
                    if take and (ops + sz > self.max_epoch_ops or not self.coalesce):
                        break
                    if in_bytes + b + rbytes[i] > self.budget:
                        break
                    take.append(queue.popleft())
                    ops += sz
                    b += int(rbytes[i])
                if not take:
                    break
                ep = EpochLists(wl, take, tomb)
                h = be.submit(next_slot, ep)
                inflight[next_slot] = (h, ep, b)
                in_bytes += b
                max_in_bytes = max(max_in_bytes, in_bytes)
                epochs.append(take)
                next_slot = (next_slot + 1) % self.slots
                progressed = True
            if not progressed:
                nxt_t = arrivals[nxt] if nxt < n else None
                be.idle(t0, nxt_t, [inflight[s][0] for s in inflight])
        t_end = be.now() - t0
        lat = done_at - arrivals
        ok = ~np.isnan(lat)
        return {"results": res, "epochs": epochs, "latency": lat, "completed": int(ok.sum()),
                "rejected": rejected, "max_inflight_bytes": max_in_bytes, "span_s": t_end,
                "ops": int(wl.sizes[ok].sum())}


def summary(run, wl, rate=None):
    lat = run["latency"][~np.isnan(run["latency"])]
    out = {"requests": int(run["completed"]), "epochs": len(run["epochs"]),
           "Mops_s": round(run["ops"] / run["span_s"] / 1e6, 3),
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
           "mean_epoch_requests": round(run["completed"] / max(len(run["epochs"]), 1), 2)}
    if rate is not None:
        out["rate_req_s"] = round(rate, 1)
    return out


class GpuBackend:
    """Epochs on the GPU through the library's epoch calls.

    Per slot: pinned staging for the inputs and the results, device buffers
    for both.  Stream ``prep`` copies an epoch in and prepares it; stream
    ``apply`` applies the epochs in order and copies results back; events
    order the two (a slot's apply after its prepare; a slot is reused only
    after its previous epoch has completed, which the engine ensures)."""

    slots = 2

    def __init__(self, store, max_epoch_ops: int, range_max: int):
        import torch
        from . import flix
        self.torch, self.flix = torch, flix
        self.st = store
        self.rm = range_max
        dt = store.dtype
        E = max_epoch_ops
        pin = lambda n, d=dt: torch.empty(n, dtype=d, pin_memory=True)
        dev = lambda n, d=dt: torch.empty(n, dtype=d, device="cuda")
        self.buf = []
        for _ in range(self.slots):
            self.buf.append({
                "h_in": {k: pin(E) for k in ("lk", "rlo", "rhi", "uk", "uv")},
                "d_in": {k: dev(E) for k in ("lk", "rlo", "rhi", "uk", "uv")},
                "d_lv": dev(E), "d_rc": dev(E, torch.int32), "d_rv": dev(E * range_max),
                "h_lv": pin(E), "h_rc": pin(E, torch.int32), "h_rv": pin(E * range_max),
                "ev_prep": torch.cuda.Event(), "ev_done": torch.cuda.Event(),
            })
        self.s_prep = torch.cuda.Stream()
        self.s_apply = torch.cuda.Stream()
        self.np_dt = np.uint64 if store.key_bits == 64 else np.uint32

    def now(self):
        return time.perf_counter()

    def submit(self, slot, ep: EpochLists):
        torch = self.torch
        b = self.buf[slot]
        nl, nr, nu = ep.counts
        lists = (("lk", ep.lookup_keys), ("rlo", ep.range_lo), ("rhi", ep.range_hi),
                 ("uk", ep.update_keys), ("uv", ep.update_vals))
        with torch.cuda.stream(self.s_prep):
            for name, arr in lists:
                if arr.size:
                    b["h_in"][name].numpy().view(self.np_dt)[:arr.size] = arr
                    b["d_in"][name][:arr.size].copy_(b["h_in"][name][:arr.size], non_blocking=True)
        d = b["d_in"]
        e = self.st.make_epoch(
            lookup_keys=d["lk"], lookup_vals=b["d_lv"], n_lookup=nl,
            range_lo=d["rlo"], range_hi=d["rhi"], range_max=self.rm, range_counts=b["d_rc"],
            range_vals=b["d_rv"], n_range=nr,
            update_keys=d["uk"], update_vals=d["uv"], n_update=nu)
        self.st.epoch_prepare(slot, e, stream=self.s_prep)
        b["ev_prep"].record(self.s_prep)
        self.s_apply.wait_event(b["ev_prep"])
        self.st.epoch_apply(slot, e, stream=self.s_apply)
        with torch.cuda.stream(self.s_apply):
            if nl:
                b["h_lv"][:nl].copy_(b["d_lv"][:nl], non_blocking=True)
            if nr:
                b["h_rc"][:nr].copy_(b["d_rc"][:nr], non_blocking=True)
                b["h_rv"][:nr * self.rm].copy_(b["d_rv"][:nr * self.rm], non_blocking=True)
        b["ev_done"].record(self.s_apply)
        return (slot, nl, nr)

    def ready(self, h):
        return self.buf[h[0]]["ev_done"].query()

    def results(self, h):
        slot, nl, nr = h
        b = self.buf[slot]
        lv = b["h_lv"].numpy().view(self.np_dt)[:nl].copy()
        rc = b["h_rc"].numpy().view(np.uint32)[:nr].copy()
        rv = b["h_rv"].numpy().view(self.np_dt)[:nr * self.rm].copy()
        return lv, rc, rv

    def idle(self, t0, next_arrival, handles):
        # busy wait: the next event is an arrival or a completion
        pass
