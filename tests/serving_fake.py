"""A serving backend over the oracle with a simulated clock, so the serving
engine's coalescing, admission, ordering and latency accounting can be
tested without a GPU.  Epochs complete in submission order; each takes a
fixed cost plus a per-operation cost of simulated time."""
import numpy as np


class FakeBackend:
    slots = 2

    def __init__(self, oracle, range_max, per_epoch_s=200e-6, per_op_s=50e-9):
        self.o = oracle
        self.rm = range_max
        self.t = 0.0
        self.busy_until = 0.0
        self.per_epoch_s = per_epoch_s
        self.per_op_s = per_op_s
        self.submitted = []

    def now(self):
        return self.t

    def submit(self, slot, ep):
        lv, rc, rv = self.o.apply_epoch(ep.lookup_keys, ep.range_lo, ep.range_hi, self.rm,
                                        ep.update_keys, ep.update_vals)
        start = max(self.t, self.busy_until)
        done = start + self.per_epoch_s + self.per_op_s * ep.n_ops
        self.busy_until = done
        self.submitted.append((slot, list(ep.req_ids)))
        return {"done": done, "res": (lv, rc, rv.reshape(-1))}

    def ready(self, h):
        return self.t >= h["done"]

    def results(self, h):
        return h["res"]

    def idle(self, t0, next_arrival, handles):
        cands = [h["done"] for h in handles]
        if next_arrival is not None:
            cands.append(t0 + next_arrival)
        assert cands, "engine idle with nothing pending"
        self.t = max(self.t, min(cands))
