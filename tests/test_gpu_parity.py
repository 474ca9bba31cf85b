"""GPU parity: every FliX batch operation through the C ABI against the CPU
oracle, bit-exact (all of this is integer work), plus the device invariant
checker and the paper's worked examples at the node level.
"""
import json
import os

import numpy as np
import pytest

from gpu_helpers import (assert_same_contents, check_reads, ktype, log, new_pair, to_dev,
                         to_host)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_16725_amd import flix
    flix.load_library()
    yield


def _keys(rng, kb, n, hi=None):
    mx = (1 << kb) - 1 if hi is None else hi
    return rng.integers(0, mx, n, dtype=np.uint64, endpoint=True).astype(ktype(kb))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("rb", [4, 8])
@pytest.mark.parametrize("n", [1, 100, 2048, 2049, 5000, (1 << 17) + 3])
def test_sort_matches_stable_argsort(kb, rb, n):
    log(f"sort kb={kb} rb={rb} n={n}")
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=kb, capacity=64, radix_bits=rb, max_batch=1 << 18)
    rng = np.random.default_rng(n * 7 + kb + rb)
    k = _keys(rng, kb, n)
    k[rng.random(n) < 0.3] = ktype(kb)(12345)        # heavy duplicates
    k[: min(n, 3)] = [0, (1 << kb) - 1, 7][: min(n, 3)]
    ko, io = s.sort_pairs(to_dev(k))
    ko, io = to_host(ko, kb), io.cpu().numpy()
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io, ref.astype(np.int32))
    assert np.array_equal(ko, k[ref])


def test_sort_single_digit_keys_take_copy_pass():
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=64, capacity=64, radix_bits=8, max_batch=1 << 16)
    rng = np.random.default_rng(5)
    k = (np.uint64(0xABCD000000000000) + rng.integers(0, 256, 50000).astype(np.uint64))
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, 64), k[ref])


@pytest.mark.parametrize("kb", [32, 64])
def test_sort_skewed_top_digit_runs(kb):
    """Batches below 2^22 keys are split on the top 8-bit digit and every run
    is sorted by one workgroup: runs longer than the workgroup's LDS take the
    chunked global-memory path.  Here one top digit holds ~60% of the keys
    (many duplicates among them), others are uniform or empty."""
    from paper_2604_16725_amd.flix import Store
    log(f"skewed top digit kb={kb}")
    s = Store(key_bits=kb, capacity=64, radix_bits=8, max_batch=1 << 18)
    rng = np.random.default_rng(11 + kb)
    n = (1 << 17) + 3
    top = np.uint64(0x5A) << np.uint64(kb - 8)
    low = rng.integers(0, 1 << 12, int(n * 0.6), dtype=np.uint64)
    k = np.concatenate([top + low, _keys(rng, kb, n - low.size).astype(np.uint64)])
    k = rng.permutation(k).astype(ktype(kb))
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, kb), k[ref])


@pytest.mark.parametrize("n", [1 << 21, (1 << 21) + 1, 1 << 22, (1 << 22) + 1])
def test_sort_at_the_per_run_limit(n):
    """2^21 keys are the most the tile split takes (1024 tiles, one per
    thread of a run workgroup); one more key takes the top-digit onesweep
    pass and the per-run sort up to 2^22 keys (runs of ~16K items, above the
    LDS run size, take the chunked path); one more takes the onesweep
    passes."""
    from paper_2604_16725_amd.flix import Store
    log(f"sort at the per-run limit n={n}")
    s = Store(key_bits=32, capacity=64, radix_bits=8, max_batch=(1 << 22) + 1)
    rng = np.random.default_rng(n % 97)
    k = _keys(rng, 32, n)
    k[: n // 8] = k[n // 8: n // 4]   # duplicates: stability is visible
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, 32), k[ref])


@pytest.mark.parametrize("kb,nvary", [(32, 1), (32, 2), (32, 3), (64, 2), (64, 5), (64, 7)])
def test_sort_long_runs_varying_digits(kb, nvary):
    """One top digit holds 60000 keys that differ only in their lowest
    `nvary` digits (the others are equal inside the run), so the run is too
    long for LDS and too varied for the dominant-key form: its chunked global
    passes skip the digits that do not vary, with an odd or even number of
    passes left, and must still end in the output buffer, stable."""
    from paper_2604_16725_amd.flix import Store
    log(f"long runs kb={kb} nvary={nvary}")
    s = Store(key_bits=kb, capacity=64, radix_bits=8, max_batch=1 << 17)
    rng = np.random.default_rng(40 + kb + nvary)
    top = np.uint64(0xC3) << np.uint64(kb - 8)
    mid = np.uint64(0x5A5A5A5A5A5A5A5A) & np.uint64((1 << (kb - 8)) - 1)
    mid &= ~np.uint64((1 << (8 * nvary)) - 1)
    low = rng.integers(0, 1 << (8 * nvary), 60000, dtype=np.uint64)
    k = np.concatenate([top | mid | low, _keys(rng, kb, 20000).astype(np.uint64)])
    k = rng.permutation(k).astype(ktype(kb))
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, kb), k[ref])


@pytest.mark.parametrize("kb", [32, 64])
def test_sort_clustered_ranges_share_a_top_digit(kb):
    """Ranges of consecutive keys that share a top digit (a clustered batch
    where two or three runs land in one top digit): the long run is split on
    its highest varying digit, then sub-runs go to LDS in groups or, when one
    is longer than the LDS run size, through chunked passes (an even number
    of them ends with a copy into the output)."""
    from paper_2604_16725_amd.flix import Store
    log(f"clustered ranges kb={kb}")
    s = Store(key_bits=kb, capacity=64, radix_bits=8, max_batch=1 << 17)
    rng = np.random.default_rng(60 + kb)
    top = np.uint64(0x7E) << np.uint64(kb - 8)
    sh = np.uint64(kb - 16)
    starts = [top | (np.uint64(0x11) << sh), top | (np.uint64(0x93) << sh) | np.uint64(0xFF00),
              top | (np.uint64(0xC4) << sh)]
    lens = [16384, 9000, 300]
    parts = [np.arange(int(a), int(a) + n, dtype=np.uint64) for a, n in zip(starts, lens)]
    k = np.concatenate(parts + [parts[1][::7], _keys(rng, kb, 30000).astype(np.uint64)])
    k = rng.permutation(k).astype(ktype(kb))
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, kb), k[ref])


@pytest.mark.parametrize("kb", [32, 64])
def test_sort_dominant_key_run(kb):
    """A top-digit run made mostly of one repeated key (a Zipf-skewed batch):
    the repeated key's items keep their input order between the sorted
    smaller and larger keys of the run."""
    from paper_2604_16725_amd.flix import Store
    log(f"dominant key kb={kb}")
    s = Store(key_bits=kb, capacity=64, radix_bits=8, max_batch=1 << 18)
    rng = np.random.default_rng(23 + kb)
    top = np.uint64(0x3C) << np.uint64(kb - 8)
    x = top + np.uint64(777)
    near = top + rng.integers(0, 1 << (kb - 9), 3000, dtype=np.uint64)
    k = np.concatenate([np.full(60000, x, dtype=np.uint64), near, near[:500],
                        _keys(rng, kb, 60000).astype(np.uint64)])
    k = rng.permutation(k).astype(ktype(kb))
    ko, io = s.sort_pairs(to_dev(k))
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(io.cpu().numpy(), ref.astype(np.int32))
    assert np.array_equal(to_host(ko, kb), k[ref])


@pytest.mark.parametrize("kb", [32, 64])
def test_insert_repeated_key_last_wins(kb):
    """An insert batch with one key repeated 2^15 times among others: the last
    occurrence's value wins (the batch sort is stable on the long run)."""
    log(f"repeated insert key kb={kb}")
    rng = np.random.default_rng(31 + kb)
    s, o = new_pair(kb, cap=64, lanes=16, max_batch=1 << 16)
    k0 = np.unique(_keys(rng, kb, 1 << 14))
    v0 = rng.integers(0, 1 << 30, k0.size, dtype=np.uint64).astype(ktype(kb))
    s.bulk_load(to_dev(k0), to_dev(v0))
    o.bulk_load(k0, v0)
    x = k0[k0.size // 2]
    ks = np.concatenate([np.full(1 << 15, x, dtype=ktype(kb)), _keys(rng, kb, 2000)])
    ks = rng.permutation(ks)
    vs = rng.integers(0, 1 << 30, ks.size, dtype=np.uint64).astype(ktype(kb))
    s.insert(to_dev(ks), to_dev(vs))
    o.insert(ks, vs)
    assert s.status() == 0
    assert_same_contents(s, o, kb, "repeated insert")


# ---------------------------------------------------------------------------
def test_bulk_load_layout_follows_build_rule():
    g = json.load(open(os.path.join(GOLDEN, "initial_build_example.json")))
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=32, capacity=8, fill=2, max_batch=64)
    k = np.array(g["build_keys_unsorted"], dtype=np.uint32)
    s.bulk_load(to_dev(k), to_dev(k * np.uint32(3)))
    lay = s.copy_layout()
    assert lay["buckets"] == len(g["groups"])
    assert lay["mkba"].tolist() == g["mkba_u32"]
    for i, grp in enumerate(g["groups"]):
        assert lay["size"][i] == len(grp)
        assert lay["keys"][i, : len(grp)].tolist() == grp
        assert lay["vals"][i, : len(grp)].tolist() == [3 * x for x in grp]
        assert lay["next"][i] == 0xFFFFFFFF
        assert lay["fence"][i] == g["mkba_u32"][i]
    assert lay["free"].size == lay["pool"] - lay["buckets"]
    assert s.check() == 0


def test_worked_insert_example_table2():
    g = json.load(open(os.path.join(GOLDEN, "tl_bulk_insert_example.json")))
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=32, capacity=8, fill=8, max_batch=64, lanes=16)
    nb = np.array(g["node_before"], dtype=np.uint32)
    s.bulk_load(to_dev(nb), to_dev(nb + np.uint32(100)))
    ins = np.array(g["insert_first"], dtype=np.uint32)
    s.insert(to_dev(ins), to_dev(ins + np.uint32(100)))
    lay = s.copy_layout()
    assert lay["buckets"] == 1
    assert lay["size"][0] == 8 and lay["keys"][0].tolist() == g["node_after_first"]
    assert lay["next"][0] == 0xFFFFFFFF
    ins2 = np.array(g["insert_second"], dtype=np.uint32)
    s.insert(to_dev(ins2), to_dev(ins2 + np.uint32(100)))
    lay = s.copy_layout()
    left, right = g["split_halves_after_second"]
    assert lay["size"][0] == len(left) and lay["keys"][0, : len(left)].tolist() == left
    nxt = int(lay["next"][0])
    assert nxt != 0xFFFFFFFF
    assert lay["size"][nxt] == len(right) and lay["keys"][nxt, : len(right)].tolist() == right
    assert lay["fence"][0] == left[-1]
    assert lay["fence"][nxt] == 0xFFFFFFFF and lay["next"][nxt] == 0xFFFFFFFF
    assert s.check() == 0
    k, v = s.dump()
    assert to_host(k, 32).tolist() == g["contents_after_second"]
    assert to_host(v, 32).tolist() == [x + 100 for x in g["contents_after_second"]]


def test_worked_delete_example_table3():
    g = json.load(open(os.path.join(GOLDEN, "tl_bulk_delete_example.json")))
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=32, capacity=8, fill=8, max_batch=64)
    nb = np.array(g["node_before"], dtype=np.uint32)
    s.bulk_load(to_dev(nb), to_dev(nb * np.uint32(7)))
    d = np.array(g["delete"], dtype=np.uint32)
    s.delete(to_dev(d))
    lay = s.copy_layout()
    n = len(g["node_after"])
    assert lay["size"][0] == n
    assert lay["keys"][0, :n].tolist() == g["node_after"]
    assert lay["vals"][0, :n].tolist() == [7 * x for x in g["node_after"]]
    assert s.check() == 0


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("cap", [8, 64, 256])
def test_reads_small(kb, cap):
    log(f"reads kb={kb} cap={cap}")
    rng = np.random.default_rng(kb * 1000 + cap)
    s, o = new_pair(kb, cap=cap, max_batch=1 << 15)
    mx = (1 << kb) - 1
    k = np.unique(_keys(rng, kb, 20000))
    k = np.unique(np.concatenate([k, np.array([0, mx, 1, mx - 1], dtype=ktype(kb))]))
    rng.shuffle(k)
    v = (k ^ ktype(kb)(0x5A5A)) % ktype(kb)(mx)
    s.bulk_load(to_dev(k), to_dev(v))
    o.bulk_load(k, v)
    assert_same_contents(s, o, kb, "bulk")
    q = np.concatenate([k[rng.integers(0, k.size, 6000)], _keys(rng, kb, 6000),
                        np.array([0, mx, 1, mx - 1, 2], dtype=ktype(kb))])
    rng.shuffle(q)
    check_reads(s, o, kb, q, maxpq=8, where=f"cap{cap}")


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("cap,lanes", [(128, 16), (128, 32), (64, 16), (256, 64), (32, 16)])
def test_reads_at_the_half_node_boundary(kb, cap, lanes):
    """The read kernel spreads a node holding at most half of a lane group's
    slots over all of its lanes (half the comparisons per query) and uses
    every slot for a fuller node; one batch meets nodes below, at and just
    above half full, nodes close to full and chained buckets, so the lane
    groups of one wave take both forms.  Lookups of present and absent keys,
    successors, predecessors and short and long ranges, bit-exact."""
    dt = ktype(kb)
    rng = np.random.default_rng(cap * 31 + lanes + kb)
    s, o = new_pair(kb, cap=cap, lanes=lanes, max_batch=1 << 16)
    base = np.unique(_keys(rng, kb, 30000))
    s.bulk_load(to_dev(base), to_dev(base ^ dt(0x5A)))
    o.bulk_load(base, base ^ dt(0x5A))
    mk = s.copy_layout()["mkba"].astype(np.uint64)
    nb = mk.size
    half = cap // 2
    deltas = [-3, -1, 0, 1, 2, half // 2, half - 1, half + 3]
    present = set(int(x) for x in base)
    ins, dele = [], []
    for b in rng.choice(np.arange(1, nb - 1), size=min(240, nb - 2), replace=False):
        lo_b, hi_b = int(mk[b - 1]) + 1, int(mk[b])
        d = deltas[int(rng.integers(0, len(deltas)))]
        if d > 0:
            got = 0
            while got < d:
                x = int(rng.integers(lo_b, hi_b, endpoint=True, dtype=np.uint64))
                if x not in present:
                    present.add(x)
                    ins.append(x)
                    got += 1
        elif d < 0:
            own = base[(base >= lo_b) & (base <= hi_b)]
            dele.extend(int(x) for x in own[: -d])
    ins = np.array(ins, dtype=np.uint64).astype(dt)
    dele = np.array(dele, dtype=np.uint64).astype(dt)
    s.insert(to_dev(ins), to_dev(ins ^ dt(0x33)))
    o.insert(ins, ins ^ dt(0x33))
    s.delete(to_dev(dele))
    o.delete(dele)
    assert s.status() == 0
    assert_same_contents(s, o, kb, "half-node boundary store")
    sizes = s.copy_layout()["size"][:nb]
    log(f"half-node boundary cap={cap} lanes={lanes}: node sizes {np.bincount(np.minimum(sizes, cap))[half - 3: half + 4]} around half, max {sizes.max()}")
    cur, _ = o.dump()
    q = np.concatenate([cur[rng.integers(0, cur.size, 6000)], _keys(rng, kb, 3000),
                        mk.astype(dt), (mk[:-1] + 1).astype(dt), ins[:2000], dele[:500]])
    rng.shuffle(q)
    check_reads(s, o, kb, q, maxpq=8, where="half-node boundary")
    hi = np.minimum(q.astype(np.uint64) + np.uint64(40), np.uint64((1 << kb) - 1)).astype(dt)
    check_reads(s, o, kb, q, maxpq=4, lo=q, hi=hi, where="half-node boundary, short ranges")


@pytest.mark.parametrize("kb", [32, 64])
def test_reads_on_empty_and_single(kb):
    s, o = new_pair(kb, cap=64, max_batch=1024)
    mx = (1 << kb) - 1
    q = np.array([0, 5, mx], dtype=ktype(kb))
    check_reads(s, o, kb, q, maxpq=4, where="empty")
    s.bulk_load(to_dev(np.array([mx], dtype=ktype(kb))), to_dev(np.array([9], dtype=ktype(kb))))
    o.bulk_load(np.array([mx], dtype=ktype(kb)), np.array([9], dtype=ktype(kb)))
    check_reads(s, o, kb, q, maxpq=4, where="single")
    # n == 0 calls are no-ops
    import torch
    e = torch.empty(0, dtype=torch.int32 if kb == 32 else torch.int64, device="cuda")
    s.lookup(e)
    s.insert(e, e)
    s.delete(e)
    assert_same_contents(s, o, kb, "after empty calls")


# ---------------------------------------------------------------------------
def test_tiny_plain_workload_full_sequence():
    """u32, capacity 64: bulk 2^16, then insert, lookup, delete, successor."""
    from paper_2604_16725_amd import workloads as w
    t = w.tiny_plain()
    kb = 32
    s, o = new_pair(kb, cap=t["capacity"], max_batch=1 << 16)
    s.bulk_load(to_dev(t["build_keys"]), to_dev(t["build_vals"]))
    o.bulk_load(t["build_keys"], t["build_vals"])
    assert_same_contents(s, o, kb, "bulk")
    for b in t["batches"]:
        log("tiny_plain", b[0])
        if b[0] == "insert":
            s.insert(to_dev(b[1]), to_dev(b[2]))
            assert o.insert(b[1], b[2]) == 0
            assert s.status() == 0
            assert_same_contents(s, o, kb, "insert")
        elif b[0] == "delete":
            s.delete(to_dev(b[1]))
            o.delete(b[1])
            assert_same_contents(s, o, kb, "delete")
        elif b[0] == "lookup":
            g = to_host(s.lookup(to_dev(b[1])), kb)
            assert np.array_equal(g, o.lookup(b[1]))
        else:
            gk, gv = s.successor(to_dev(b[1]))
            ok, ov = o.successor(b[1])
            assert np.array_equal(to_host(gk, kb), ok) and np.array_equal(to_host(gv, kb), ov)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("cap,lanes", [(8, 16), (16, 32), (64, 64), (32, 16)])
def test_random_sessions(kb, cap, lanes):
    """Tiny key universes force duplicates, overwrites, absent deletes, empty
    buckets, splits, merges and chains; contents are compared after every op."""
    log(f"sessions kb={kb} cap={cap} lanes={lanes}")
    mx = (1 << kb) - 1
    for seed in range(6):
        rng = np.random.default_rng(seed * 31 + cap + kb)
        universe = np.unique(np.concatenate([
            _keys(rng, kb, 3000), np.array([0, 1, 2, mx, mx - 1], dtype=ktype(kb))]))
        s, o = new_pair(kb, cap=cap, lanes=lanes, max_batch=8192)
        n0 = int(rng.integers(0, 1500))
        k0 = rng.choice(universe, n0)
        v0 = rng.integers(0, mx, n0, dtype=np.uint64).astype(ktype(kb))
        s.bulk_load(to_dev(k0), to_dev(v0)) if n0 else None
        o.bulk_load(k0, v0)
        assert_same_contents(s, o, kb, f"s{seed} bulk")
        for step in range(10):
            op = rng.choice(["insert", "insert", "delete", "read"])
            n = int(rng.integers(1, 4096))
            ks = rng.choice(universe, n)
            if op == "insert":
                vs = rng.integers(0, mx, n, dtype=np.uint64).astype(ktype(kb))
                s.insert(to_dev(ks), to_dev(vs))
                o.insert(ks, vs)
                assert s.status() == 0
                assert_same_contents(s, o, kb, f"s{seed} step{step} insert")
            elif op == "delete":
                s.delete(to_dev(ks))
                o.delete(ks)
                assert_same_contents(s, o, kb, f"s{seed} step{step} delete")
            else:
                q = np.concatenate([ks, _keys(rng, kb, 200)])
                check_reads(s, o, kb, q, maxpq=5, where=f"s{seed} step{step}")


@pytest.mark.parametrize("kb", [32, 64])
def test_clustered_runs_long_chains(kb):
    """Dense runs of consecutive keys land in few buckets: long chains, chunked
    merges, many splits; then rank-contiguous deletes merge and free nodes."""
    rng = np.random.default_rng(77 + kb)
    s, o = new_pair(kb, cap=16, lanes=16, max_batch=1 << 15)
    base = np.unique(_keys(rng, kb, 4000))
    s.bulk_load(to_dev(base), to_dev(base))
    o.bulk_load(base, base)
    for r in range(4):
        starts = rng.integers(0, (1 << kb) - 5000, 6, dtype=np.uint64)
        ins = np.unique(np.concatenate([np.arange(st, st + 3000, dtype=np.uint64) for st in starts]))
        ins = ins.astype(ktype(kb))
        rng.shuffle(ins)
        vals = (ins * ktype(kb)(3)) % ktype(kb)((1 << kb) - 1)
        s.insert(to_dev(ins), to_dev(vals))
        o.insert(ins, vals)
        assert s.status() == 0
        assert_same_contents(s, o, kb, f"round{r} insert")
        check_reads(s, o, kb, np.concatenate([ins[:2000], _keys(rng, kb, 2000)]), maxpq=16,
                    where=f"round{r}")
        cur, _ = o.dump()
        st = int(rng.integers(0, max(1, cur.size - 5000)))
        dele = cur[st: st + 5000].copy()
        rng.shuffle(dele)
        s.delete(to_dev(dele))
        o.delete(dele)
        assert_same_contents(s, o, kb, f"round{r} delete")
    st = s.stats()
    assert st["live_nodes"] <= st["pool_nodes"]


def test_insert_into_empty_store_grows_one_bucket():
    kb = 32
    s, o = new_pair(kb, cap=32, max_batch=1 << 14)
    rng = np.random.default_rng(3)
    k = _keys(rng, kb, 10000)
    s.insert(to_dev(k), to_dev(k))
    o.insert(k, k)
    assert s.status() == 0
    assert_same_contents(s, o, kb, "grow")
    assert s.stats()["buckets"] == 1


# ---------------------------------------------------------------------------
def test_error_paths_leave_store_unchanged():
    from paper_2604_16725_amd.flix import FLIX_EINVAL, FLIX_ENOMEM, Store
    kb = 32
    s, o = new_pair(kb, cap=16, max_batch=4096)
    rng = np.random.default_rng(9)
    k = np.unique(_keys(rng, kb, 2000))
    s.bulk_load(to_dev(k), to_dev(k))
    o.bulk_load(k, k)
    # n > max_batch: rejected on the host
    big = _keys(rng, kb, 5000)
    assert s.insert(to_dev(big), to_dev(big), check=False) == FLIX_EINVAL
    # reserved value: rejected on the device, whole batch cancelled
    ins = _keys(rng, kb, 100)
    vals = ins.copy()
    vals[50] = np.uint32(0xFFFFFFFF)
    assert s.insert(to_dev(ins), to_dev(vals), check=False) == 0
    assert s.status() == FLIX_EINVAL
    assert s.status() == 0   # cleared
    assert_same_contents(s, o, kb, "after reserved value")
    # pool exhaustion: tiny fixed pool
    node_bytes = 16 * 2 * 4 + 16
    t = Store(key_bits=32, capacity=16, max_batch=4096, pool_bytes=node_bytes * 300)
    kk = np.unique(_keys(rng, kb, 1000))
    t.bulk_load(to_dev(kk), to_dev(kk))
    o2 = __import__("oracle.oracle", fromlist=["Oracle"]).Oracle(32)
    o2.bulk_load(kk, kk)
    flood = _keys(rng, kb, 4000)
    assert t.insert(to_dev(flood), to_dev(flood), check=False) == 0
    assert t.status() == FLIX_ENOMEM
    assert_same_contents(t, o2, kb, "after ENOMEM")
    # the store keeps working
    small = _keys(rng, kb, 50)
    t.insert(to_dev(small), to_dev(small))
    o2.insert(small, small)
    assert t.status() == 0
    assert_same_contents(t, o2, kb, "after ENOMEM then insert")


@pytest.mark.parametrize("kb", [32, 64])
def test_work_list_region_overflow(kb):
    """Small max_batch (region capacity 64 work items) on a store of 65536
    buckets: uniform batches fill some regions past capacity after their first
    share, and a batch over consecutive buckets overflows every region, so the
    work items of the overflow region and the valid prefix of each region are
    both exercised; contents and reads match the oracle after every batch."""
    log(f"work-list overflow kb={kb}")
    rng = np.random.default_rng(77 + kb)
    s, o = new_pair(kb, cap=16, lanes=16, max_batch=4096)
    k0 = np.unique(_keys(rng, kb, 1 << 19))
    v0 = rng.integers(0, 1 << 30, k0.size, dtype=np.uint64).astype(ktype(kb))
    s.bulk_load(to_dev(k0), to_dev(v0))
    o.bulk_load(k0, v0)
    srt = np.sort(k0)
    dense = srt[1000:1000 + 8 * 4096:8] + ktype(kb)(1)   # one key per bucket, consecutive buckets
    for name, ks in [("uniform", _keys(rng, kb, 4096)), ("dense", dense)]:
        vs = rng.integers(0, 1 << 30, ks.size, dtype=np.uint64).astype(ktype(kb))
        s.insert(to_dev(ks), to_dev(vs))
        o.insert(ks, vs)
        assert s.status() == 0
        assert_same_contents(s, o, kb, f"{name} insert")
        check_reads(s, o, kb, ks[:2000], maxpq=4, where=f"{name} reads")
        s.delete(to_dev(ks))
        o.delete(ks)
        assert s.status() == 0
        assert_same_contents(s, o, kb, f"{name} delete")


@pytest.mark.parametrize("kb", [32, 64])
def test_range_edge_cases(kb):
    """Ranges with lo > hi (also repeated), max_per_query = 0, null key or
    value outputs, hi = KEY_MAX, one lo with several different hi in one
    slice, and dense ranges spanning many nodes and buckets; slots beyond
    min(count, max_per_query) keep the caller's contents."""
    import torch
    log(f"range edge cases kb={kb}")
    mx = (1 << kb) - 1
    dt = ktype(kb)
    s, o = new_pair(kb, cap=16, max_batch=1 << 14)
    rng = np.random.default_rng(77 + kb)
    keys = np.unique(_keys(rng, kb, 6000, hi=200000)).astype(dt)
    keys = np.concatenate([keys, np.array([0, mx - 1, mx], dtype=dt)])
    vals = (keys.astype(np.uint64) * np.uint64(3) + np.uint64(1)).astype(dt)
    vals[vals == dt(mx)] = dt(5)
    s.bulk_load(to_dev(keys), to_dev(vals))
    o.bulk_load(keys, vals)
    # grow chains so that dense ranges cross chained nodes and buckets
    extra = np.arange(1000, 3000, dtype=np.uint64).astype(dt)
    s.insert(to_dev(extra), to_dev(extra))
    o.insert(extra, extra)
    n = 4096
    lo = _keys(rng, kb, n, hi=210000)
    hi = (lo.astype(np.uint64) + rng.integers(0, 3000, n).astype(np.uint64)).astype(dt)
    sw = rng.random(n) < 0.15                       # lo > hi
    lo[sw], hi[sw] = hi[sw] + dt(1), lo[sw]
    lo[:64] = dt(1500)                              # one lo, many different hi
    hi[:64] = (np.arange(64, dtype=np.uint64) * np.uint64(40) + np.uint64(1400)).astype(dt)
    lo[64:96] = dt(2500)                            # repeated lo > hi
    hi[64:96] = dt(2499)
    hi[96:128] = dt(mx)                             # saturating upper end
    lo[128:136] = dt(mx)
    lo[136:144] = dt(0)
    perm = rng.permutation(n)
    lo, hi = lo[perm], hi[perm]
    oc, ok2, ov2 = o.range(lo, hi, 8)
    for maxpq in (0, 1, 8):
        for want_k, want_v in ((True, True), (False, True), (True, False)):
            sent = -7
            ck = torch.full((max(n * maxpq, 1),), sent, dtype=s.dtype, device="cuda")
            cv = torch.full((max(n * maxpq, 1),), sent, dtype=s.dtype, device="cuda")
            c, rk, rv = s.range(to_dev(lo), to_dev(hi), maxpq, out_k=ck if want_k else None,
                                out_v=cv if want_v else None, want_keys=want_k,
                                want_vals=want_v)
            c = c.cpu().numpy().view(np.uint32)
            assert np.array_equal(c, oc), f"counts maxpq={maxpq}"
            if maxpq == 0:
                assert (ck.cpu().numpy() == sent).all() and (cv.cpu().numpy() == sent).all()
                continue
            oc_m, ok_m, ov_m = o.range(lo, hi, maxpq)
            w = np.minimum(oc_m, maxpq)
            mask = np.arange(maxpq)[None, :] < w[:, None]
            sent_u = dt(sent & mx)
            for want, buf, ref in ((want_k, ck, ok_m), (want_v, cv, ov_m)):
                if not want:
                    continue   # passed as NULL
                got = to_host(buf, kb)[: n * maxpq].reshape(n, maxpq)
                assert np.array_equal(got[mask], ref[mask]), f"maxpq={maxpq} results"
                assert (got[~mask] == sent_u).all(), f"maxpq={maxpq}: slot beyond count written"
    assert s.status() == 0


@pytest.mark.parametrize("kb", [32, 64])
def test_reads_across_long_runs_of_empty_buckets(kb):
    """Successor, predecessor and range across more than 10^4 consecutive
    empty buckets (a contiguous key range deleted), and at both ends of the
    key space; the occupancy summary is part of the device invariant check."""
    log(f"empty-bucket gaps kb={kb}")
    dt = ktype(kb)
    s, o = new_pair(kb, cap=16, max_batch=1 << 19)
    n = 1 << 19
    keys = (np.arange(n, dtype=np.uint64) * np.uint64(7) + np.uint64(100)).astype(dt)
    vals = (keys.astype(np.uint64) ^ np.uint64(0x5A5A)).astype(dt)
    s.bulk_load(to_dev(keys), to_dev(vals))
    o.bulk_load(keys, vals)
    # 8 keys per bucket: deleting 160000 consecutive keys empties 20000 buckets;
    # also empty the first and the last 2000 buckets
    gone = np.concatenate([keys[100000:260000], keys[:16000], keys[-16000:]])
    rng = np.random.default_rng(3 + kb)
    rng.shuffle(gone)
    s.delete(to_dev(gone))
    o.delete(gone)
    assert_same_contents(s, o, kb, "after the gap deletes")
    lo_gap, hi_gap = int(keys[100000]), int(keys[259999])
    q = np.concatenate([
        rng.integers(lo_gap - 50, hi_gap + 50, 3000, dtype=np.uint64).astype(dt),
        rng.integers(0, int(keys[16000]) + 10, 500, dtype=np.uint64).astype(dt),
        rng.integers(int(keys[-16000]) - 10, int(keys[-1]) + 10, 500, dtype=np.uint64).astype(dt),
        np.array([0, (1 << kb) - 1], dtype=dt)])
    lo = q.copy()
    hi = np.minimum(q.astype(np.uint64) + np.uint64(hi_gap - lo_gap + 40),
                    np.uint64((1 << kb) - 1)).astype(dt)
    check_reads(s, o, kb, q, maxpq=4, lo=lo, hi=hi, where="gap")
    # refill part of the gap: buckets become non-empty again
    back = keys[150000:150100]
    s.insert(to_dev(back), to_dev(vals[150000:150100]))
    o.insert(back, vals[150000:150100])
    assert_same_contents(s, o, kb, "after refilling")
    check_reads(s, o, kb, q, maxpq=4, lo=lo, hi=hi, where="gap refilled")


def test_torch_allocator_hook_backs_a_store():
    """With the allocator hook set to torch's caching allocator, a store's
    directory, pool and scratch come from torch (its allocated bytes grow by
    at least the pool) and every operation still matches the oracle; after
    destroy and reset, hipMalloc serves again."""
    import torch
    from paper_2604_16725_amd import flix
    kb = 32
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    flix.use_torch_allocator(True)
    try:
        s, o = new_pair(kb, cap=32, max_batch=1 << 14)
        rng = np.random.default_rng(12)
        k = np.unique(_keys(rng, kb, 50000))
        s.bulk_load(to_dev(k), to_dev(k))
        o.bulk_load(k, k)
        grown = torch.cuda.memory_allocated() - before
        st = s.stats()
        assert grown >= st["pool_nodes"] * (16 + 2 * 32 * 4), grown
        ins = _keys(rng, kb, 10000)
        s.insert(to_dev(ins), to_dev(ins))
        o.insert(ins, ins)
        s.delete(to_dev(k[:5000]))
        o.delete(k[:5000])
        assert_same_contents(s, o, kb, "torch-allocated store")
        check_reads(s, o, kb, np.concatenate([ins[:3000], _keys(rng, kb, 3000)]), maxpq=4,
                    where="torch-allocated store")
        s.restructure()
        assert_same_contents(s, o, kb, "torch-allocated store, restructured")
        s.close()
    finally:
        flix.use_torch_allocator(False)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + (1 << 20)
    s2, o2 = new_pair(kb, cap=32, max_batch=1 << 10)
    s2.bulk_load(to_dev(k[:100]), to_dev(k[:100]))
    o2.bulk_load(k[:100], k[:100])
    assert_same_contents(s2, o2, kb, "after resetting the hook")
    s2.close()


@pytest.mark.parametrize("kb", [32, 64])
def test_dense_ranges_every_result(kb):
    """Ranges that hold hundreds of keys each, across many nodes and buckets
    (after growth, so chains too), with room for every result: counts, keys
    and values all bit-exact."""
    rng = np.random.default_rng(900 + kb)
    dt = ktype(kb)
    s, o = new_pair(kb, cap=64, max_batch=1 << 16)
    k = np.unique(_keys(rng, kb, 1 << 18))
    s.bulk_load(to_dev(k), to_dev(k ^ dt(3)))
    o.bulk_load(k, k ^ dt(3))
    ins = _keys(rng, kb, 1 << 16)
    s.insert(to_dev(ins), to_dev(ins))
    o.insert(ins, ins)
    width = np.uint64(((1 << kb) // (1 << 18)) * 300)
    lo = _keys(rng, kb, 4000)
    hi = np.minimum(lo.astype(np.uint64) + width, np.uint64((1 << kb) - 1)).astype(dt)
    check_reads(s, o, kb, lo, maxpq=512, lo=lo, hi=hi, where="dense ranges")
