"""Seeded synthetic workloads for the FliX batch operations.

This module only decides WHICH keys, values and operations are requested.  It
holds none of the store's arithmetic (no bucket routing, merging or searching
of a store), and both sides of every parity check receive exactly the
arrays it returns.

The paper's workloads are all synthetic (Section 5.2.1: uniform and dense
"X/Y" key-range workloads; Section 6.1: uniform build, hit and miss probes).
Distinct keys are produced by keyed bijections applied to counters, so two
different counters can never give the same key:

* 32-bit keys: a 4-round balanced Feistel network on two 16-bit halves.
* 64-bit keys: the splitmix64 finaliser (each of its steps is invertible),
  applied to ``counter XOR key``.

Seeds follow one rule: stream s (0 keys, 1 values, 2 order, 3 arrivals/other)
of config c, round r uses ``0xF11C0000 + 100000*s + 1000*c + r``.
"""
from __future__ import annotations

import numpy as np

M32 = np.uint64(0xFFFFFFFF)
M64 = 0xFFFFFFFFFFFFFFFF

STREAM_KEYS, STREAM_VALS, STREAM_ORDER, STREAM_OTHER = 0, 1, 2, 3


def seed_for(config: int, rnd: int, stream: int) -> int:
    return 0xF11C0000 + 100000 * stream + 1000 * config + rnd


def _splitmix64_scalar(x: int) -> int:
    x = (x + 0x9E3779B97F4A7C15) & M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _fmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser on uint64 arrays (wrapping arithmetic)."""
    z = x.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def _round_fn16(r: np.ndarray, k: int) -> np.ndarray:
    """Feistel round function on uint32 arrays (arithmetic mod 2^32)."""
    t = r ^ np.uint32(k)
    t *= np.uint32(0x45D9F3B)
    t ^= t >> np.uint32(16)
    t *= np.uint32(0x45D9F3B)
    t ^= t >> np.uint32(16)
    return t & np.uint32(0xFFFF)


def perm32(counters, seed: int) -> np.ndarray:
    """Keyed bijection of [0, 2^32): counters -> distinct uint32 keys.

    Evaluated in cache-sized chunks with uint32 arithmetic."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1)
    out = np.empty(c.shape, np.uint32)
    keys = [_splitmix64_scalar(seed * 8 + i) & 0xFFFFFFFF for i in range(4)]
    chunk = 1 << 18
    for s in range(0, c.size, chunk):
        cc = (c[s:s + chunk] & M32).astype(np.uint32)
        left = cc >> np.uint32(16)
        right = cc & np.uint32(0xFFFF)
        for k in keys:
            left, right = right, left ^ _round_fn16(right, k)
        out[s:s + chunk] = (left << np.uint32(16)) | right
    return out.reshape(np.shape(counters))


def perm64(counters, seed: int) -> np.ndarray:
    """Keyed bijection of [0, 2^64): counters -> distinct uint64 keys."""
    c = np.asarray(counters, dtype=np.uint64)
    return _fmix64(c ^ np.uint64(_splitmix64_scalar(seed)))


def perm(counters, seed: int, key_bits: int) -> np.ndarray:
    return perm32(counters, seed) if key_bits == 32 else perm64(counters, seed)


def values_for(keys: np.ndarray, salt: int, key_bits: int) -> np.ndarray:
    """Deterministic values for keys; never the reserved all-ones value."""
    if key_bits == 32:
        v = perm32(np.asarray(keys, dtype=np.uint64) ^ np.uint64(salt & 0xFFFFFFFF), salt)
        v[v == np.uint32(0xFFFFFFFF)] = np.uint32(0xFFFFFFFE)
        return v
    v = perm64(np.asarray(keys, dtype=np.uint64), salt)
    v[v == np.uint64(M64)] = np.uint64(M64 - 1)
    return v


def zipf_ranks(n_items: int, count: int, s: float, rng: np.random.Generator) -> np.ndarray:
    """Zipf(s) ranks in [0, n_items): P(rank r) proportional to (r+1)^-s.

    Sampled by inversion of the exact discrete CDF (cumulative sum in fp64).
    """
    w = np.arange(1, n_items + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    u = rng.random(count) * cdf[-1]
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, n_items - 1).astype(np.int64)


# ----------------------------------------------------------------------------
# Workload recipes (one function per configuration family)
# ----------------------------------------------------------------------------

class KeySpace:
    """Tracks which counters of a keyed bijection have been handed out.

    ``build(n)`` takes counters [0, n); ``fresh(m)`` takes the next m unused
    counters; absent keys come from the top half of the counter space, which
    ``fresh`` never reaches in these workloads.
    """

    def __init__(self, key_bits: int, seed: int):
        self.key_bits = key_bits
        self.seed = seed
        self.next_counter = 0
        self.next_absent = 0

    def build(self, n: int) -> np.ndarray:
        assert self.next_counter == 0
        self.next_counter = n
        return perm(np.arange(n, dtype=np.uint64), self.seed, self.key_bits)

    def fresh(self, m: int) -> np.ndarray:
        c = np.arange(self.next_counter, self.next_counter + m, dtype=np.uint64)
        self.next_counter += m
        return perm(c, self.seed, self.key_bits)

    def absent(self, m: int) -> np.ndarray:
        top = np.uint64(1 << (self.key_bits - 1))
        c = top + np.arange(self.next_absent, self.next_absent + m, dtype=np.uint64)
        self.next_absent += m
        return perm(c, self.seed, self.key_bits)


def tiny_plain(seed_round: int = 0):
    """Small plain-method workload: u32 keys/values, node capacity 64.

    Bulk load 2^16 distinct uniform keys, then four single-type batches in
    order: 2^14 inserts of new keys, 2^14 lookups (half present with
    replacement, half absent), 2^14 deletes of distinct present keys and 2^12
    successor queries on uniform keys.
    """
    cfg = 0
    kb = 32
    ks = KeySpace(kb, seed_for(cfg, seed_round, STREAM_KEYS))
    rng = np.random.default_rng(seed_for(cfg, seed_round, STREAM_ORDER))
    build = ks.build(1 << 16)
    build_v = values_for(build, seed_for(cfg, seed_round, STREAM_VALS), kb)
    new = ks.fresh(1 << 14)
    new_v = values_for(new, seed_for(cfg, seed_round + 1, STREAM_VALS), kb)
    present = np.concatenate([build, new])
    hit = present[rng.integers(0, present.size, 1 << 13)]
    miss = ks.absent(1 << 13)
    look = np.concatenate([hit, miss])
    rng.shuffle(look)
    dele = present[rng.choice(present.size, 1 << 14, replace=False)]
    succ = rng.integers(0, 1 << 32, 1 << 12, dtype=np.uint64).astype(np.uint32)
    return dict(key_bits=kb, capacity=64, build_keys=build, build_vals=build_v,
                batches=[("insert", new, new_v), ("lookup", look),
                         ("delete", dele), ("successor", succ)])


def read_path(n_keys: int = 1 << 26, batch: int = 1 << 20, range_len: int = 16,
              zipf_s: float = 0.99, seed_round: int = 0, with_zipf: bool = True,
              with_updates: bool = False):
    """Read-path workload: u32 keys/values, node capacity 128.

    Bulk load ``n_keys`` distinct uniform keys.  Batches of ``batch`` ops:
    lookups at a 90% hit rate (present keys uniform with replacement, absent
    keys for the rest), successors on uniform keys, ranges [lo, lo+L-1] with
    uniform lo.  The Zipf variants draw present keys by Zipf(s) rank, ranks
    mapped to keys through the counter order of the keyed bijection (which
    scatters hot keys over the key space); Zipf lookups keep 10% absent keys.
    With ``with_updates`` it also returns ``batch`` new keys (never present)
    with values, for an insert batch followed by a delete of the same keys.
    """
    cfg = 1
    kb = 32
    ks = KeySpace(kb, seed_for(cfg, seed_round, STREAM_KEYS))
    rng = np.random.default_rng(seed_for(cfg, seed_round, STREAM_ORDER))
    build = ks.build(n_keys)
    build_v = values_for(build, seed_for(cfg, seed_round, STREAM_VALS), kb)
    n_hit = (batch * 9) // 10
    look = np.concatenate([build[rng.integers(0, n_keys, n_hit)], ks.absent(batch - n_hit)])
    rng.shuffle(look)
    succ = rng.integers(0, 1 << 32, batch, dtype=np.uint64).astype(np.uint32)
    lo = rng.integers(0, 1 << 32, batch, dtype=np.uint64)
    hi = np.minimum(lo + np.uint64(range_len - 1), np.uint64(0xFFFFFFFF))
    out = dict(key_bits=kb, capacity=128, build_keys=build, build_vals=build_v,
               lookup=look, successor=succ, range_lo=lo.astype(np.uint32),
               range_hi=hi.astype(np.uint32), range_len=range_len, keyspace=ks)
    if with_zipf:
        zr = zipf_ranks(n_keys, n_hit, zipf_s, rng)
        zl = np.concatenate([build[zr], ks.absent(batch - n_hit)])
        rng.shuffle(zl)
        zs = build[zipf_ranks(n_keys, batch, zipf_s, rng)]
        zlo = build[zipf_ranks(n_keys, batch, zipf_s, rng)].astype(np.uint64)
        zhi = np.minimum(zlo + np.uint64(range_len - 1), np.uint64(0xFFFFFFFF))
        out.update(zipf_lookup=zl, zipf_successor=zs, zipf_range_lo=zlo.astype(np.uint32),
                   zipf_range_hi=zhi.astype(np.uint32))
    if with_updates:
        ins = ks.fresh(batch)
        out.update(insert_keys=ins,
                   insert_vals=values_for(ins, seed_for(cfg, seed_round + 1, STREAM_VALS), kb))
    return out


def _sorted_union(present: np.ndarray, add: np.ndarray) -> np.ndarray:
    """np.union1d(present, add) for a sorted, duplicate-free ``present``, in
    O(n + m log m): the new distinct keys are inserted at their positions."""
    s = np.unique(add)
    pos = np.searchsorted(present, s)
    inb = pos < present.size
    dup = np.zeros(s.size, dtype=bool)
    dup[inb] = present[pos[inb]] == s[inb]
    return np.insert(present, pos[~dup], s[~dup])


def _sorted_difference(present: np.ndarray, drop: np.ndarray) -> np.ndarray:
    """np.setdiff1d(present, drop) for a sorted, duplicate-free ``present``."""
    d = np.sort(drop)
    pos = np.searchsorted(present, d)
    inb = pos < present.size
    hit = np.zeros(d.size, dtype=bool)
    hit[inb] = present[pos[inb]] == d[inb]
    keep = np.ones(present.size, dtype=bool)
    keep[pos[hit]] = False
    return present[keep]


class UpdateHeavy:
    """Update-heavy workload: u64 keys/values, node capacity 128.

    Bulk load ``n_keys`` distinct keys, then rounds of (insert ``batch`` new
    keys, delete ``batch`` present keys).  Even rounds are uniform.  Odd
    rounds are clustered: inserts are ``runs`` runs of consecutive integer keys
    starting at uniform positions (a run that would touch a present key is
    redrawn), deletes are ``runs`` runs of rank-contiguous present keys.

    The generator keeps a sorted array of the keys it has made present, only
    to decide what to request; the stores' contents are never read from here.
    """

    def __init__(self, n_keys: int = 1 << 24, batch: int = 1 << 20, runs: int = 64,
                 seed_round: int = 0):
        self.cfg = 2
        self.kb = 64
        self.batch = batch
        self.runs = runs
        self.ks = KeySpace(64, seed_for(self.cfg, seed_round, STREAM_KEYS))
        self.build_keys = self.ks.build(n_keys)
        self.build_vals = values_for(self.build_keys, seed_for(self.cfg, 0, STREAM_VALS), 64)
        self.present = np.sort(self.build_keys)
        self.capacity = 128

    def round(self, r: int):
        rng = np.random.default_rng(seed_for(self.cfg, r + 1, STREAM_ORDER))
        m = self.batch
        if r % 2 == 0:
            ins = self.ks.fresh(m)
        else:
            per = m // self.runs
            starts = []
            taken = []
            while len(starts) < self.runs:
                s = int(rng.integers(0, (1 << 64) - per, dtype=np.uint64))
                lo_i = np.searchsorted(self.present, np.uint64(s), side="left")
                if lo_i < self.present.size and int(self.present[lo_i]) < s + per:
                    continue
                if any(not (s + per <= t or t + per <= s) for t in taken):
                    continue
                taken.append(s)
                starts.append(s)
            ins = np.concatenate([np.arange(s, s + per, dtype=np.uint64) for s in starts])
            extra = m - ins.size
            if extra:
                ins = np.concatenate([ins, self.ks.fresh(extra)])
            rng.shuffle(ins)
        ins_v = values_for(ins, seed_for(self.cfg, r + 1, STREAM_VALS), 64)
        self.present = _sorted_union(self.present, ins)
        n = self.present.size
        if r % 2 == 0:
            dele = self.present[rng.choice(n, m, replace=False)]
        else:
            per = m // self.runs
            # non-overlapping rank windows: pick run starts among n - runs*per
            # slack positions, then space them out
            slack = n - self.runs * per
            offs = np.sort(rng.integers(0, slack + 1, self.runs))
            idx = np.concatenate([o + i * per + np.arange(per) for i, o in enumerate(offs)])
            dele = self.present[idx]
            rng.shuffle(dele)
        self.present = _sorted_difference(self.present, dele)
        return ins, ins_v, dele


class BatchStream:
    """Mixed-batch stream for the batching form: u32 keys/values.

    Bulk load ``n_keys`` distinct uniform keys, then ``nbatch`` batches whose
    sizes are floor(2^U) with U uniform on [log2_min, log2_max] and whose
    types are drawn lookup/successor/insert/delete with probabilities ``mix``.
    Keys follow the read-path recipe: lookups are 90% bulk-loaded keys
    (uniform with replacement) and 10% absent keys, successors are uniform,
    inserts are new keys, deletes are bulk-loaded keys (uniform with
    replacement; a key already deleted is a no-op).

    Sizes and types are drawn up front; batch i is generated from its own
    seed, so any batch can be regenerated alone (``batch(i)``).
    """

    OPS = ("lookup", "successor", "insert", "delete")

    def __init__(self, n_keys: int = 1 << 26, nbatch: int = 4096, log2_min: float = 8.0,
                 log2_max: float = 20.0, mix=(0.7, 0.1, 0.1, 0.1), seed_round: int = 0):
        self.cfg = 3
        self.kb = 32
        self.n_keys = n_keys
        self.nbatch = nbatch
        self.seed_round = seed_round
        self.ks = KeySpace(32, seed_for(self.cfg, seed_round, STREAM_KEYS))
        self.build_keys = self.ks.build(n_keys)
        self.build_vals = values_for(self.build_keys, seed_for(self.cfg, seed_round, STREAM_VALS), 32)
        rng = np.random.default_rng(seed_for(self.cfg, seed_round, STREAM_OTHER))
        u = rng.uniform(log2_min, log2_max, nbatch)
        self.sizes = np.floor(np.exp2(u)).astype(np.int64)
        self.ops = rng.choice(4, nbatch, p=np.asarray(mix, dtype=np.float64))
        ins = np.where(self.ops == 2, self.sizes, 0)
        self.fresh_base = n_keys + np.concatenate([[0], np.cumsum(ins)[:-1]])
        absent = np.where(self.ops == 0, self.sizes - (self.sizes * 9) // 10, 0)
        self.absent_base = np.concatenate([[0], np.cumsum(absent)[:-1]])

    @property
    def total_ops(self) -> int:
        return int(self.sizes.sum())

    def _rng(self, i: int, stream: int) -> np.random.Generator:
        return np.random.default_rng([seed_for(self.cfg, self.seed_round, stream), int(i)])

    def batch(self, i: int):
        """(op name, keys, values or None) of batch i."""
        op = self.OPS[int(self.ops[i])]
        m = int(self.sizes[i])
        rng = self._rng(i, STREAM_ORDER)
        seed = self.ks.seed
        if op == "lookup":
            n_hit = (m * 9) // 10
            top = np.uint64(1 << 31)
            c = top + np.uint64(self.absent_base[i]) + np.arange(m - n_hit, dtype=np.uint64)
            keys = np.concatenate([self.build_keys[rng.integers(0, self.n_keys, n_hit)],
                                   perm32(c, seed)])
            rng.shuffle(keys)
            return op, keys, None
        if op == "successor":
            return op, rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32), None
        if op == "insert":
            c = np.uint64(self.fresh_base[i]) + np.arange(m, dtype=np.uint64)
            keys = perm32(c, seed)
            rng.shuffle(keys)
            vals = values_for(keys, seed_for(self.cfg, self.seed_round, STREAM_VALS) ^ (int(i) + 1 << 12),
                              32)
            return op, keys, vals
        return op, self.build_keys[rng.integers(0, self.n_keys, m)], None


class ServingWorkload:
    """Open-loop serving workload: u64 keys/values.

    Bulk load ``n_keys`` distinct keys.  ``n_req`` requests, each of
    floor(4096^U) operations (U uniform on [0, 1), so 1..4096, log-uniform),
    every operation drawn lookup / range / insert / delete with ``mix``:
    lookups hit a bulk-loaded key 90% of the time (else an absent key), a
    range starts at a uniformly chosen bulk-loaded key and ends at the key
    L-1 ranks later in the bulk-loaded order (L uniform on ``range_len``),
    inserts write new keys, deletes remove bulk-loaded keys (with replacement).

    Operations are flat arrays (``ops``: 0 lookup, 1 range, 2 insert,
    3 delete; ``keys``; ``aux``: range hi or insert value) cut by
    ``offsets``.  ``gaps`` are unit-rate exponential inter-arrival gaps;
    ``arrivals(rate)`` scales them to a request rate.
    """

    LOOKUP, RANGE, INSERT, DELETE = 0, 1, 2, 3

    def __init__(self, n_keys: int = 1 << 25, n_req: int = 20000, mix=(0.8, 0.05, 0.075, 0.075),
                 range_len=(8, 64), max_ops: int = 4096, seed_round: int = 0):
        self.cfg = 4
        self.kb = 64
        self.n_keys = n_keys
        self.n_req = n_req
        self.range_max = int(range_len[1])
        ks = KeySpace(64, seed_for(self.cfg, seed_round, STREAM_KEYS))
        self.build_keys = ks.build(n_keys)
        self.build_vals = values_for(self.build_keys, seed_for(self.cfg, seed_round, STREAM_VALS), 64)
        sorted_build = np.sort(self.build_keys)
        rng = np.random.default_rng(seed_for(self.cfg, seed_round, STREAM_ORDER))
        u = rng.random(n_req)
        self.sizes = np.maximum(np.floor(np.power(float(max_ops), u)), 1).astype(np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        total = int(self.offsets[-1])
        self.ops = rng.choice(4, total, p=np.asarray(mix, dtype=np.float64)).astype(np.uint8)
        keys = np.zeros(total, dtype=np.uint64)
        aux = np.zeros(total, dtype=np.uint64)
        il = np.nonzero(self.ops == self.LOOKUP)[0]
        hit = rng.random(il.size) < 0.9
        keys[il[hit]] = self.build_keys[rng.integers(0, n_keys, int(hit.sum()))]
        keys[il[~hit]] = ks.absent(int((~hit).sum()))
        ir = np.nonzero(self.ops == self.RANGE)[0]
        rank = rng.integers(0, n_keys, ir.size)
        ln = rng.integers(int(range_len[0]), int(range_len[1]) + 1, ir.size)
        keys[ir] = sorted_build[rank]
        aux[ir] = sorted_build[np.minimum(rank + ln - 1, n_keys - 1)]
        ii = np.nonzero(self.ops == self.INSERT)[0]
        keys[ii] = ks.fresh(ii.size)
        aux[ii] = values_for(keys[ii], seed_for(self.cfg, seed_round + 1, STREAM_VALS), 64)
        idl = np.nonzero(self.ops == self.DELETE)[0]
        keys[idl] = self.build_keys[rng.integers(0, n_keys, idl.size)]
        self.keys, self.aux = keys, aux
        self.range_ordinal = np.full(total, -1, dtype=np.int64)
        self.range_ordinal[ir] = np.arange(ir.size)
        self.n_ranges = ir.size
        self.gaps = np.random.default_rng(seed_for(self.cfg, seed_round, STREAM_OTHER)).exponential(
            1.0, n_req)

    @property
    def total_ops(self) -> int:
        return int(self.offsets[-1])

    def arrivals(self, rate: float) -> np.ndarray:
        """Arrival times (s) at ``rate`` requests per second, first at 0."""
        t = np.cumsum(self.gaps) / float(rate)
        return t - t[0]
