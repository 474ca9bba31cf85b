"""GPU parity of the bucket-group read pipeline (FLIX_READ_GROUPS: one
partition pass by groups of consecutive buckets, then each group's items
sorted in LDS and resolved by the same workgroup), bit-exact against the
oracle: uniform and skewed query batches (groups larger than one chunk),
chained buckets after growth, empty-bucket gaps, every read operation.
"""
import numpy as np
import pytest

from gpu_helpers import assert_same_contents, check_reads, ktype, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _pair(kb, cap, max_batch):
    from oracle.oracle import Oracle
    from paper_2604_16725_amd.flix import Store
    return (Store(key_bits=kb, capacity=cap, lanes=16, max_batch=max_batch, read_path="groups"),
            Oracle(kb))


def _keys(rng, kb, n):
    return rng.integers(0, (1 << kb) - 1, n, dtype=np.uint64, endpoint=True).astype(ktype(kb))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("cap", [16, 128])
def test_group_reads_uniform_skewed_and_grown(kb, cap):
    rng = np.random.default_rng(700 + kb + cap)
    s, o = _pair(kb, cap, 1 << 18)
    k = np.unique(_keys(rng, kb, 1 << 18))
    v = k ^ ktype(kb)(0x77)
    s.bulk_load(to_dev(k), to_dev(v))
    o.bulk_load(k, v)
    mx = (1 << kb) - 1
    # uniform, then a hot slice (many repeats of few keys: groups of several
    # chunks), then queries at the ends of the key space
    q = np.concatenate([k[rng.integers(0, k.size, 60000)], _keys(rng, kb, 40000)])
    hot = np.repeat(k[rng.integers(0, k.size, 8)], 9000)
    edge = np.array([0, 1, mx, mx - 1] * 50, dtype=ktype(kb))
    for name, qq in (("uniform", q), ("hot", hot), ("edge", edge)):
        qq = qq.copy()
        rng.shuffle(qq)
        check_reads(s, o, kb, qq, maxpq=8, where=f"groups {name}")
    # growth chains the buckets; reads again
    for r in range(2):
        ins = _keys(rng, kb, 1 << 17)
        s.insert(to_dev(ins), to_dev(ins))
        o.insert(ins, ins)
    assert_same_contents(s, o, kb, "groups after growth")
    q2 = np.concatenate([ins[rng.integers(0, ins.size, 30000)], _keys(rng, kb, 30000)])
    check_reads(s, o, kb, q2, maxpq=8, where="groups grown")
    # a deleted stretch leaves empty buckets in the middle of groups
    cur, _ = o.dump()
    gone = cur[10000:60000]
    s.delete(to_dev(gone))
    o.delete(gone)
    lo = np.concatenate([gone[rng.integers(0, gone.size, 5000)], _keys(rng, kb, 5000)])
    hi = np.minimum(lo.astype(np.uint64) + np.uint64(1 << (kb - 6)), np.uint64(mx)).astype(ktype(kb))
    check_reads(s, o, kb, lo, maxpq=4, lo=lo, hi=hi, where="groups gaps")
    log(f"group reads kb={kb} cap={cap}: ok")
