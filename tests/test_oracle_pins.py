"""Pins for the CPU oracle (runs without a GPU).

The oracle must be tied to something other than itself:
* brute force: a Python dict replayed op by op in input order, with linear
  scans for successor and range, on tiny key universes that force duplicates,
  0 and KEY_MAX (sequential ordered-map semantics, Section 2.1);
* the paper's worked examples (Tables 2 and 3) and the build rule (Section 3.2);
* closed-form special cases and invariants at larger sizes;
* planted mistakes: mutated copies of the oracle source must fail these pins.
"""
import json
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.oracle import Oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mx(kb):
    return (1 << kb) - 1


class DictModel:
    """Ordered map by definition: a dict, sorted on demand."""

    def __init__(self, kb):
        self.kb = kb
        self.d = {}

    def bulk_load(self, ks, vs):
        if any(v == _mx(self.kb) for v in vs):
            return -1
        self.d = {}
        for k, v in zip(ks, vs):
            self.d[k] = v
        return 0

    def insert(self, ks, vs):
        if any(v == _mx(self.kb) for v in vs):
            return -1
        for k, v in zip(ks, vs):
            self.d[k] = v
        return 0

    def delete(self, ks):
        for k in ks:
            self.d.pop(k, None)

    def lookup(self, qs):
        return [self.d.get(q, _mx(self.kb)) for q in qs]

    def successor(self, qs):
        out_k, out_v = [], []
        for q in qs:
            best = None
            for k in self.d:
                if k >= q and (best is None or k < best):
                    best = k
            out_k.append(_mx(self.kb) if best is None else best)
            out_v.append(_mx(self.kb) if best is None else self.d[best])
        return out_k, out_v

    def predecessor(self, qs):
        out_k, out_v = [], []
        for q in qs:
            best = None
            for k in self.d:
                if k <= q and (best is None or k > best):
                    best = k
            out_k.append(0 if best is None else best)
            out_v.append(_mx(self.kb) if best is None else self.d[best])
        return out_k, out_v

    def range(self, los, his, maxpq):
        res = []
        for lo, hi in zip(los, his):
            ks = sorted(k for k in self.d if lo <= k <= hi)
            res.append((len(ks), ks[:maxpq], [self.d[k] for k in ks[:maxpq]]))
        return res

    def dump(self):
        ks = sorted(self.d)
        return ks, [self.d[k] for k in ks]


def _rand_keys(rnd, kb, n, universe):
    mx = _mx(kb)
    out = []
    for _ in range(n):
        r = rnd.random()
        if r < 0.1:
            out.append(0)
        elif r < 0.2:
            out.append(mx)
        elif r < 0.25:
            out.append(mx - 1)
        else:
            out.append(rnd.choice(universe))
    return out


def _rand_vals(rnd, kb, n):
    return [rnd.randrange(0, _mx(kb)) for _ in range(n)]  # never all-ones


def _check_equal(o, m, kb):
    ok, ov = o.dump()
    mk, mv = m.dump()
    assert ok.tolist() == mk and ov.tolist() == mv
    assert o.size() == len(mk)


def _run_random_session(o_cls, kb, seed):
    rnd = random.Random(seed)
    mx = _mx(kb)
    universe = sorted(set([1, 2, 3, 5, 8, 13, 21, 34, 55, mx - 2, mx // 2, mx // 2 + 1]
                          + [rnd.randrange(0, mx) for _ in range(40)]))
    o = o_cls(kb)
    m = DictModel(kb)
    n0 = rnd.randrange(0, 24)
    ks, vs = _rand_keys(rnd, kb, n0, universe), _rand_vals(rnd, kb, n0)
    assert o.bulk_load(ks, vs) == m.bulk_load(ks, vs) == 0
    _check_equal(o, m, kb)
    for _ in range(6):
        op = rnd.choice(["insert", "delete", "lookup", "successor", "predecessor", "range",
                         "bulk"])
        n = rnd.randrange(0, 20)
        ks = _rand_keys(rnd, kb, n, universe)
        if op == "insert":
            vs = _rand_vals(rnd, kb, n)
            assert o.insert(ks, vs) == m.insert(ks, vs)
        elif op == "bulk":
            vs = _rand_vals(rnd, kb, n)
            assert o.bulk_load(ks, vs) == m.bulk_load(ks, vs)
        elif op == "delete":
            o.delete(ks)
            m.delete(ks)
        elif op == "lookup":
            assert o.lookup(ks).tolist() == m.lookup(ks)
        elif op == "successor":
            gk, gv = o.successor(ks)
            mk, mv = m.successor(ks)
            assert gk.tolist() == mk and gv.tolist() == mv
        elif op == "predecessor":
            gk, gv = o.predecessor(ks)
            mk, mv = m.predecessor(ks)
            assert gk.tolist() == mk and gv.tolist() == mv
        else:
            his = _rand_keys(rnd, kb, n, universe)
            maxpq = rnd.choice([0, 1, 3, 8])
            cnt, gk, gv = o.range(ks, his, maxpq)
            for i, (c, rk, rv) in enumerate(m.range(ks, his, maxpq)):
                assert cnt[i] == c
                w = min(c, maxpq)
                assert gk[i, :w].tolist() == rk and gv[i, :w].tolist() == rv
        _check_equal(o, m, kb)


@pytest.mark.parametrize("kb", [32, 64])
def test_oracle_vs_dict_bruteforce(kb):
    for seed in range(2500):
        _run_random_session(Oracle, kb, seed * 2 + (kb == 64))


@pytest.mark.parametrize("kb", [32, 64])
def test_reserved_value_rejected_store_unchanged(kb):
    o = Oracle(kb)
    assert o.bulk_load([5, 7], [1, 2]) == 0
    assert o.insert([9, 10], [3, _mx(kb)]) == -1
    k, v = o.dump()
    assert k.tolist() == [5, 7] and v.tolist() == [1, 2]
    assert o.bulk_load([1], [_mx(kb)]) == -1
    assert o.dump()[0].tolist() == [5, 7]


def test_worked_insert_example_table2():
    g = json.load(open(os.path.join(GOLDEN, "tl_bulk_insert_example.json")))
    o = Oracle(32)
    nb = g["node_before"]
    o.bulk_load(nb, [100 + k for k in nb])
    o.insert(g["insert_first"], [100 + k for k in g["insert_first"]])
    assert o.dump()[0].tolist() == g["node_after_first"]
    o.insert(g["insert_second"], [100 + k for k in g["insert_second"]])
    k, v = o.dump()
    assert k.tolist() == g["contents_after_second"]
    assert v.tolist() == [100 + x for x in g["contents_after_second"]]


def test_worked_delete_example_table3():
    g = json.load(open(os.path.join(GOLDEN, "tl_bulk_delete_example.json")))
    o = Oracle(32)
    nb = g["node_before"]
    o.bulk_load(nb, [7 * k for k in nb])
    o.delete(g["delete"])
    k, v = o.dump()
    assert k.tolist() == g["node_after"]
    assert v.tolist() == [7 * x for x in g["node_after"]]
    # the table's mask and shift-left distances follow from the same sets
    mask = [int(x in g["delete"]) for x in nb]
    assert mask == g["deleted_mask"]
    dist = [None if mk else sum(mask[:i]) for i, mk in enumerate(mask)]
    assert dist == g["shift_left_distance"]


@pytest.mark.parametrize("kb", [32, 64])
def test_special_cases(kb):
    mx = _mx(kb)
    o = Oracle(kb)
    # empty store
    assert o.lookup([0, mx]).tolist() == [mx, mx]
    k, v = o.successor([0, 5, mx])
    assert k.tolist() == [mx] * 3 and v.tolist() == [mx] * 3
    assert o.range([0], [mx], 4)[0].tolist() == [0]
    o.bulk_load([0, mx, 10], [1, 2, 3])
    # KEY_MAX as a real key is told apart from a miss by its value
    k, v = o.successor([11, mx, 0])
    assert k.tolist() == [mx, mx, 0] and v.tolist() == [2, 2, 1]
    # successor is >= (Section 6.5), not >
    k, v = o.successor([10])
    assert k.tolist() == [10]
    # predecessor is the mirror: largest key <= q; a miss is (0, NOT_FOUND)
    k, v = o.predecessor([10, 9, mx, mx - 1, 0])
    assert k.tolist() == [10, 0, mx, 10, 0] and v.tolist() == [3, 1, 2, 3, 1]
    o2 = Oracle(kb)
    o2.bulk_load([5], [4])
    k, v = o2.predecessor([4, 5, 0])
    assert k.tolist() == [0, 5, 0] and v.tolist() == [mx, 4, mx]
    # closed range, lo > hi, saturating hi, max_per_query truncation
    c, rk, rv = o.range([0, 10, 11, 0], [10, 9, mx, mx], 2)
    assert c.tolist() == [2, 0, 1, 3]
    assert rk[0].tolist() == [0, 10] and rk[2, :1].tolist() == [mx]
    assert rk[3].tolist() == [0, 10]
    # delete of absent and duplicated keys
    o.delete([5, 10, 10, 10])
    assert o.dump()[0].tolist() == [0, mx]
    # last occurrence wins inside one insert batch
    o.insert([7, 7, 7], [1, 2, 3])
    assert o.lookup([7]).tolist() == [3]


@pytest.mark.parametrize("kb", [32, 64])
def test_invariants_medium(kb):
    rng = np.random.default_rng(1234 + kb)
    dt = np.uint32 if kb == 32 else np.uint64
    o = Oracle(kb)
    hi = (1 << kb) - 1
    keys = np.unique(rng.integers(0, hi, 50000, dtype=np.uint64).astype(dt))
    rng.shuffle(keys)
    bulk = keys[:30000]
    o.bulk_load(bulk, bulk ^ dt(5))
    new = keys[30000:40000]
    o.insert(new, new ^ dt(9))
    present = np.concatenate([bulk, new])
    dele = rng.choice(present, 8000, replace=False)
    o.delete(np.concatenate([dele, keys[45000:46000]]))  # plus absent keys
    k, v = o.dump()
    assert np.all(k[1:] > k[:-1])
    assert k.size == 30000 + 10000 - 8000
    q = rng.integers(0, hi, 20000, dtype=np.uint64).astype(dt)
    sk, sv = o.successor(q)
    idx = np.searchsorted(k, q, side="left")
    hit = idx < k.size
    assert np.all(sk[hit] >= q[hit])
    # minimal: no stored key in [q, succ)
    assert np.all(k[np.maximum(idx[hit] - 1, 0)][idx[hit] > 0] < q[hit][idx[hit] > 0])
    assert np.all(sk[~hit] == dt(hi)) and np.all(sv[~hit] == dt(hi))


# --------------------------------------------------------------------------
# Planted mistakes: each mutant of the oracle source must fail a pin above.
# --------------------------------------------------------------------------
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "flix_oracle.cpp")

MUTANTS = {
    # first occurrence wins instead of last
    "keep_first": ("bool last_of_run = (j + 1 == n) || (k[order[j + 1]] != k[i]);",
                   "bool last_of_run = (j == 0) || (k[order[j - 1]] != k[i]);"),
    # stored value kept on equal keys
    "no_overwrite": ("      } else {  // equal keys: the batch value replaces the stored one\n"
                     "        nk.push_back(bk[b]);\n        nv.push_back(bv[b]);",
                     "      } else {  // equal keys: the batch value replaces the stored one\n"
                     "        nk.push_back(keys[a]);\n        nv.push_back(vals[a]);"),
    # successor strictly greater
    "succ_gt": ("auto it = std::lower_bound(keys.begin(), keys.end(), q[i]);\n      if (it == keys.end()) {",
                "auto it = std::upper_bound(keys.begin(), keys.end(), q[i]);\n      if (it == keys.end()) {"),
    # predecessor strictly smaller
    "pred_lt": ("auto it = std::upper_bound(keys.begin(), keys.end(), q[i]);\n      if (it == keys.begin()) {",
                "auto it = std::lower_bound(keys.begin(), keys.end(), q[i]);\n      if (it == keys.begin()) {"),
    # predecessor miss reported with KEY_MAX instead of 0
    "pred_miss_key": ("        kout[i] = K(0);\n        vout[i] = kNotFound;",
                      "        kout[i] = kKeyMax;\n        vout[i] = kNotFound;"),
    # half-open range
    "range_open": ("auto last = std::upper_bound(keys.begin(), keys.end(), hi[i]);",
                   "auto last = std::lower_bound(keys.begin(), keys.end(), hi[i]);"),
    # reserved value accepted
    "reserved_ok": ("if (v[i] == kNotFound) return -1;", "if (false) return -1;"),
}


class _MutantOracle(Oracle):
    lib_path = None

    def __init__(self, kb):
        from oracle import oracle as om
        saved = om._lib
        om._lib = None
        real = om._LIB_PATH
        om._LIB_PATH = self.lib_path
        try:
            super().__init__(kb)
        finally:
            om._LIB_PATH = real
            om._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    d = tempfile.mkdtemp(prefix="orc_mut_")
    try:
        p = os.path.join(d, "m.cpp")
        open(p, "w").write(src.replace(old, new))
        lib = os.path.join(d, "libm.so")
        subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, p], check=True)
        cls = type("M_" + name, (_MutantOracle,), {"lib_path": lib})
        caught = False
        checks = [lambda: [_run_random_session(cls, kb, s) for kb in (32, 64) for s in range(300)],
                  lambda: _special(cls),
                  lambda: _reserved(cls)]
        for c in checks:
            try:
                c()
            except AssertionError:
                caught = True
                break
        assert caught, f"mutant {name} survived the pins"
    finally:
        shutil.rmtree(d, ignore_errors=True)


def _special(cls):
    mx = _mx(32)
    o = cls(32)
    o.bulk_load([0, mx, 10], [1, 2, 3])
    k, _ = o.successor([10])
    assert k.tolist() == [10]
    k, _ = o.predecessor([10])
    assert k.tolist() == [10]
    c, _, _ = o.range([0], [10], 2)
    assert c.tolist() == [2]


def _reserved(cls):
    o = cls(32)
    o.bulk_load([5], [1])
    assert o.insert([9], [_mx(32)]) == -1


@pytest.mark.parametrize("kb", [32, 64])
def test_epoch_order_vs_sequential_replay(kb):
    """An epoch's reads see the map before the epoch; its updates equal
    applying them one at a time in array order (all-ones value = delete).
    Pinned against a plain dict replayed op by op."""
    tomb = (1 << kb) - 1
    dt = np.uint32 if kb == 32 else np.uint64
    for seed in range(300):
        rng = random.Random(seed * 7 + kb)
        universe = [0, 1, 2, 5, 9, 17, 40, tomb - 1, tomb] + [rng.randrange(0, 64) for _ in range(8)]
        base = {k: rng.randrange(0, tomb) for k in rng.sample(universe, 6)}
        o = Oracle(kb)
        ks = sorted(base)
        o.bulk_load(np.array(ks, dtype=dt), np.array([base[k] for k in ks], dtype=dt))
        look = [rng.choice(universe) for _ in range(6)]
        lo = [rng.choice(universe) for _ in range(3)]
        hi = [min(x + rng.randrange(0, 20), tomb) for x in lo]
        uk = [rng.choice(universe) for _ in range(rng.randrange(0, 12))]
        uv = [tomb if rng.random() < 0.4 else rng.randrange(0, tomb) for _ in uk]
        lv, rc, rv = o.apply_epoch(np.array(look, dtype=dt), np.array(lo, dtype=dt),
                                   np.array(hi, dtype=dt), 4, np.array(uk, dtype=dt),
                                   np.array(uv, dtype=dt))
        # reads: the map before the epoch
        for q, got in zip(look, lv.tolist()):
            assert got == base.get(q, tomb)
        for i, (a, b) in enumerate(zip(lo, hi)):
            inside = sorted(k for k in base if a <= k <= b)
            assert rc[i] == len(inside)
            assert rv[i, :min(len(inside), 4)].tolist() == [base[k] for k in inside[:4]]
        # updates: sequential replay
        ref = dict(base)
        for k, v in zip(uk, uv):
            if v == tomb:
                ref.pop(k, None)
            else:
                ref[k] = v
        gk, gv = o.dump()
        assert gk.tolist() == sorted(ref) and gv.tolist() == [ref[k] for k in sorted(ref)]
