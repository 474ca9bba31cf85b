"""GPU parity of the workgroup-wide insert (a long slice into a single-node
bucket is merged by a whole workgroup, Section 3.4 elastic compute), against
the oracle: dense runs of new keys with repeated keys inside the run (the
last pair wins), present keys inside the run's range (upserts), runs into
empty buckets, runs into the last bucket (maxBucket = KEY_MAX), slices just
below and at the length threshold, and a mix with ordinary slices in the same
batch.  Reads and the device invariant check follow every batch.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same_contents, check_reads, ktype, log, new_pair, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _keys(rng, kb, n):
    return rng.integers(0, (1 << kb) - 1, n, dtype=np.uint64, endpoint=True).astype(ktype(kb))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("cap", [16, 128])
def test_wide_insert_dense_runs(kb, cap):
    rng = np.random.default_rng(5100 + kb + cap)
    dt = ktype(kb)
    mx = (1 << kb) - 1
    wmin = max(4 * cap, 256)
    s, o = new_pair(kb, cap=cap, max_batch=1 << 17)
    base = np.unique(_keys(rng, kb, 30000))
    s.bulk_load(to_dev(base), to_dev(base ^ dt(9)))
    o.bulk_load(base, base ^ dt(9))
    for r in range(4):
        runs = []
        # a run well past the threshold, one just below, one exactly at it,
        # one into the last bucket, one that covers present keys (upserts)
        for length in (5 * wmin + 7, wmin - 1, wmin, 3 * wmin):
            st = int(rng.integers(0, mx - 4 * length, dtype=np.uint64))
            runs.append(np.arange(st, st + length, dtype=np.uint64))
        runs.append(np.append(np.arange(mx - 2 * wmin, mx, dtype=np.uint64), np.uint64(mx)))
        cur, _ = o.dump()
        mid = int(cur[cur.size // 2])
        runs.append(np.arange(mid - wmin, mid + wmin, dtype=np.uint64))
        ins = np.concatenate(runs).astype(dt)
        # repeats inside the runs, with their own values (last pair wins)
        rep = ins[rng.integers(0, ins.size, ins.size // 8)]
        ins = np.concatenate([ins, rep, _keys(rng, kb, 3000)])
        rng.shuffle(ins)
        vals = (ins * dt(5) + np.arange(ins.size, dtype=dt) + dt(r + 1)) % dt(mx)
        s.insert(to_dev(ins), to_dev(vals))
        o.insert(ins, vals)
        assert s.status() == 0, f"round {r}: device error"
        assert_same_contents(s, o, kb, f"wide kb={kb} cap={cap} round {r}")
        q = np.concatenate([ins[rng.integers(0, ins.size, 4000)], _keys(rng, kb, 2000),
                            np.array([0, mx, mx - 1], dtype=dt)])
        check_reads(s, o, kb, q, maxpq=8, where=f"wide round {r}")
        # delete part of what was inserted, so later runs land in chains and
        # in emptied buckets too
        dele = ins[rng.integers(0, ins.size, ins.size // 2)]
        s.delete(to_dev(dele))
        o.delete(dele)
        assert_same_contents(s, o, kb, f"wide kb={kb} cap={cap} round {r} delete")
    st = s.stats()
    log(f"wide kb={kb} cap={cap}: keys={st['keys']} buckets={st['buckets']} nodes={st['live_nodes']}")


def test_wide_insert_into_empty_store():
    """One bucket, no keys: a run of 2^16 keys becomes a chain of half-full
    pieces in one workgroup merge."""
    kb = 32
    s, o = new_pair(kb, cap=64, max_batch=1 << 17)
    k = np.arange(1000, 1000 + (1 << 16), dtype=np.uint32)
    rng = np.random.default_rng(8)
    rng.shuffle(k)
    s.insert(to_dev(k), to_dev(k + np.uint32(1)))
    o.insert(k, k + np.uint32(1))
    assert_same_contents(s, o, kb, "wide into an empty store")
    st = s.stats()
    assert st["buckets"] == 1 and st["live_nodes"] == (1 << 16) // 32
    check_reads(s, o, kb, np.concatenate([k[:3000], np.array([0, 999, 1 << 20], dtype=np.uint32)]),
                maxpq=4, where="wide empty store")


@pytest.mark.parametrize("kb", [32, 64])
def test_wide_insert_into_chains(kb):
    """Long slices into chained buckets: a dense run first becomes a chain of
    pieces; then runs that interleave with it (every node of the chain gets
    keys), runs that upsert part of it, and runs past its end are merged node
    by node by the workgroup-wide kernel; contents and reads match the
    oracle after every batch."""
    rng = np.random.default_rng(6200 + kb)
    dt = ktype(kb)
    s, o = new_pair(kb, cap=32, max_batch=1 << 16)
    base = np.unique(_keys(rng, kb, 4000))
    s.bulk_load(to_dev(base), to_dev(base))
    o.bulk_load(base, base)
    mx = (1 << kb) - 1
    st = int(rng.integers(1 << 20, mx - (1 << 20), dtype=np.uint64))
    # between two stored keys: find a gap wide enough for the runs
    lo = int(base[np.searchsorted(base, np.uint64(st).astype(dt))])
    start = lo + 1
    evens = np.arange(start, start + 2 * 6000, 2, dtype=np.uint64).astype(dt)
    odds = evens + dt(1)
    batches = [
        ("evens", evens),                                        # one long slice -> a chain
        ("odds", odds),                                          # interleaves with every node
        ("upserts", np.concatenate([evens[::3], odds[1000:3000]])),
        ("past the end", np.arange(start + 20000, start + 23000, dtype=np.uint64).astype(dt)),
        ("mixed", np.concatenate([evens[:700] + dt(0), _keys(rng, kb, 2000)])),
    ]
    for r, (name, ins) in enumerate(batches):
        ins = ins.copy()
        rng.shuffle(ins)
        vals = (ins ^ dt(0x1234)) + dt(r)
        vals[vals == dt(mx)] = 0
        s.insert(to_dev(ins), to_dev(vals))
        o.insert(ins, vals)
        assert s.status() == 0, f"{name}: device error"
        assert_same_contents(s, o, kb, f"wide into chains: {name}")
        q = np.concatenate([ins[:2000], evens[::7], _keys(rng, kb, 500)])
        check_reads(s, o, kb, q, maxpq=8, where=f"wide into chains: {name}")
    log(f"wide into chains kb={kb}: {s.stats()}")
