"""GPU parity of restructuring (Section 3.5, Section 6.6): after growth into
long chains and deletes that leave underfull nodes, flix_restructure lays the
store out again by the initial-build rule of Section 3.2.  Contents and every
read stay bit-exact against the oracle (restructuring changes no pair), the
directory equals the build rule applied to the live keys, every bucket is one
node at the bulk-load fill, and later updates and reads still match.
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


def _expect_build_rule(lay, keys, vals, fill, kb):
    """The Section 3.2 layout of the sorted live pairs: groups of `fill`
    consecutive keys, one node per bucket, maxBucket = the group's last key and
    KEY_MAX for the last bucket."""
    n = keys.size
    nb = max(1, -(-n // fill))
    assert lay["buckets"] == nb, f"{lay['buckets']} buckets, expected {nb}"
    mk = np.empty(nb, dtype=ktype(kb))
    for b in range(nb):
        lo, hi = b * fill, min((b + 1) * fill, n)
        mk[b] = keys[hi - 1] if hi > lo else 0
        assert lay["size"][b] == hi - lo
        assert np.array_equal(lay["keys"][b, : hi - lo], keys[lo:hi])
        assert np.array_equal(lay["vals"][b, : hi - lo], vals[lo:hi])
        assert lay["next"][b] == 0xFFFFFFFF
    mk[-1] = (1 << kb) - 1
    assert np.array_equal(lay["mkba"], mk)


@pytest.mark.parametrize("kb", [32, 64])
def test_restructure_after_clustered_growth_and_deletes(kb):
    rng = np.random.default_rng(4100 + kb)
    cap, fill = 32, 16
    s, o = new_pair(kb, cap=cap, lanes=16, max_batch=1 << 15)
    base = np.unique(_keys(rng, kb, 6000))
    s.bulk_load(to_dev(base), to_dev(base ^ ktype(kb)(5)))
    o.bulk_load(base, base ^ ktype(kb)(5))
    # growth: dense runs (long chains in few buckets) and uniform keys
    for r in range(3):
        starts = rng.integers(0, (1 << kb) - 8000, 4, dtype=np.uint64)
        ins = np.concatenate([np.arange(st, st + 2500, dtype=np.uint64) for st in starts])
        ins = np.concatenate([ins.astype(ktype(kb)), _keys(rng, kb, 3000)])
        rng.shuffle(ins)
        vals = (ins * ktype(kb)(7) + ktype(kb)(r)) % ktype(kb)((1 << kb) - 1)
        s.insert(to_dev(ins), to_dev(vals))
        o.insert(ins, vals)
    # deletes: two rank-contiguous stretches and scattered keys leave underfull nodes
    cur, _ = o.dump()
    dele = np.concatenate([cur[100:4100], cur[9000:12000], cur[rng.integers(0, cur.size, 3000)]])
    rng.shuffle(dele)
    s.delete(to_dev(dele))
    o.delete(dele)
    assert s.status() == 0
    assert_same_contents(s, o, kb, "before restructuring")
    st0 = s.stats()
    assert st0["live_nodes"] > st0["buckets"], "the workload should have built chains"
    before, after = s.restructure()
    st1 = s.stats()
    log(f"kb={kb}: nodes {before} -> {after} ({100.0 * (before - after) / before:.1f}% recovered), "
        f"buckets {st0['buckets']} -> {st1['buckets']}")
    assert before == st0["live_nodes"]
    assert after == st1["live_nodes"] == st1["buckets"]
    assert st1["pool_nodes"] == st0["pool_nodes"]
    assert_same_contents(s, o, kb, "after restructuring")
    ok, ov = o.dump()
    _expect_build_rule(s.copy_layout(), ok, ov, fill, kb)
    q = np.concatenate([ok[rng.integers(0, ok.size, 3000)], _keys(rng, kb, 3000)])
    check_reads(s, o, kb, q, maxpq=8, where="after restructuring")
    # the restructured store keeps working: more updates, then reads
    ins = _keys(rng, kb, 5000)
    vals = ins // ktype(kb)(3)
    s.insert(to_dev(ins), to_dev(vals))
    o.insert(ins, vals)
    dele = ok[rng.integers(0, ok.size, 4000)]
    s.delete(to_dev(dele))
    o.delete(dele)
    assert s.status() == 0
    assert_same_contents(s, o, kb, "updates after restructuring")
    check_reads(s, o, kb, np.concatenate([ins[:2000], _keys(rng, kb, 2000)]), maxpq=8,
                where="reads after restructuring and updates")


def test_restructure_empty_and_tiny_stores():
    kb = 32
    s, o = new_pair(kb, cap=16, max_batch=1 << 10)
    before, after = s.restructure()
    assert after == 1 and s.stats()["buckets"] == 1
    assert_same_contents(s, o, kb, "empty")
    k = np.array([0, 1, 7, (1 << 32) - 1], dtype=np.uint32)
    s.insert(to_dev(k), to_dev(k + np.uint32(1)))
    o.insert(k, k + np.uint32(1))
    s.restructure()
    assert_same_contents(s, o, kb, "four keys")
    _expect_build_rule(s.copy_layout(), *o.dump(), 8, kb)
    check_reads(s, o, kb, np.array([0, 2, 8, (1 << 32) - 1, (1 << 32) - 2], dtype=np.uint32))
    s.delete(to_dev(k))
    o.delete(k)
    s.restructure()
    assert_same_contents(s, o, kb, "emptied")
    assert s.stats()["buckets"] == 1


def test_restructure_at_full_fill():
    """A store built at fill = capacity restructures to full nodes again."""
    kb = 32
    cap = 16
    s, o = new_pair(kb, cap=cap, fill=cap, max_batch=1 << 12)
    k = np.arange(1, 1 + 64 * cap, dtype=np.uint32) * np.uint32(3)
    s.bulk_load(to_dev(k), to_dev(k))
    o.bulk_load(k, k)
    ins = k[:200] + np.uint32(1)
    s.insert(to_dev(ins), to_dev(ins))
    o.insert(ins, ins)
    before, after = s.restructure()
    assert before > 64 and after == -(-(k.size + ins.size) // cap)
    assert_same_contents(s, o, kb, "full-fill store")
    _expect_build_rule(s.copy_layout(), *o.dump(), cap, kb)
