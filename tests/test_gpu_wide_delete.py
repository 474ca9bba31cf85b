"""GPU parity of the workgroup-wide delete (a delete slice into a long chain,
or a long slice, is taken by a whole workgroup: Section 3.4 elastic
compute), against the oracle's contents and, node for node, against a host
replay of the delete structure rule (Section 4.4: compaction, a node joins
its predecessor when their sizes sum to at most cap/2, when it is empty, or
when the predecessor is the emptied head; the head is never freed) run over
the layout copied before the batch.  Cases: deletes spread over every node
of chains of hundreds of nodes, every other key (joins down the chain), a
whole chain (the emptied head), a chain longer than one window of the
kernel, deletes only in the tail nodes, and a batch that mixes wide and
lane-group items.
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


NIL = 0xFFFFFFFF


def _chain(lay, b):
    out = []
    x = b
    while x != NIL:
        out.append(int(x))
        x = int(lay["next"][x])
    return out


def _replay_delete(lay, b, dkeys):
    """The delete structure rule over bucket b's chain: returns the chain
    after the batch as (node id, sorted keys, fence) in chain order."""
    cap = lay["cap"]
    f = cap // 2
    nodes = _chain(lay, b)
    ks = [list(lay["keys"][x][: lay["size"][x]]) for x in nodes]
    fence = [int(lay["fence"][x]) for x in nodes]
    dset = set(int(k) for k in dkeys)
    d_sorted = sorted(dset)
    # part of the slice of every node: keys in (previous fence, fence]; the
    # last node takes the rest
    parts = []
    lo = -1
    for i, x in enumerate(nodes):
        hi = fence[i] if i + 1 < len(nodes) else 1 << 64
        parts.append([k for k in d_sorted if lo < k <= hi])
        lo = hi
    j_end = len(d_sorted)
    consumed = 0
    P = None   # [id, keys, fence, dirty, is_head]
    result = []
    for i, x in enumerate(nodes):
        if P is not None:
            more = consumed < j_end or (P[4] and len(P[1]) == 0) or (P[3] and len(P[1]) <= f)
            if not more:
                result.append(P)
                result.extend([[y, ks[r], fence[r], False, False]
                               for r, y in enumerate(nodes) if r >= i])
                P = None
                break
        part = set(parts[i])
        consumed += len(parts[i])
        surv = [k for k in ks[i] if int(k) not in part]
        touched = len(parts[i]) > 0
        if P is not None and (len(P[1]) + len(surv) <= f or len(surv) == 0
                              or (P[4] and len(P[1]) == 0)):
            P[1] = P[1] + surv
            P[2] = fence[i]
            P[3] = True
        else:
            if P is not None:
                result.append(P)
            P = [x, surv, fence[i], touched, x == b]
    if P is not None:
        result.append(P)
    return [(r[0], [int(k) for k in r[1]], r[2]) for r in result]


def _device_chain(lay, b):
    return [(x, [int(k) for k in lay["keys"][x][: lay["size"][x]]], int(lay["fence"][x]))
            for x in _chain(lay, b)]


def _run_case(s, o, kb, dele, where, watch):
    """Delete `dele`; every bucket in `watch` must match the replay."""
    lay0 = s.copy_layout()
    mk = lay0["mkba"]
    expect = {}
    for b in watch:
        lo = mk[b - 1] if b > 0 else None
        sel = dele[(dele <= mk[b]) & ((dele > lo) if lo is not None else True)]
        expect[b] = _replay_delete(lay0, b, sel)
    s.delete(to_dev(dele))
    o.delete(dele)
    assert s.status() == 0, f"{where}: device error"
    assert_same_contents(s, o, kb, where)
    lay1 = s.copy_layout()
    for b, exp in expect.items():
        got = _device_chain(lay1, b)
        assert [g[0] for g in got] == [e[0] for e in exp], f"{where}: bucket {b} node ids differ"
        for g, e in zip(got, exp):
            assert g[1] == e[1], f"{where}: bucket {b} node {g[0]} keys differ"
            assert g[2] == e[2], f"{where}: bucket {b} node {g[0]} fence {g[2]} != {e[2]}"


def _chained_store(kb, runs, run_len, seed):
    """A store whose buckets hold long chains: dense runs of new keys (the
    workgroup-wide insert cuts each into half-full pieces)."""
    rng = np.random.default_rng(seed)
    dt = ktype(kb)
    s, o = new_pair(kb, cap=128, max_batch=1 << 18)
    base = np.unique(rng.integers(0, (1 << kb) - 1, 20000, dtype=np.uint64).astype(dt))
    s.bulk_load(to_dev(base), to_dev(base ^ dt(3)))
    o.bulk_load(base, base ^ dt(3))
    starts = []
    used = set()
    while len(starts) < runs:
        # a gap between two stored keys, wide enough for the run
        i = int(rng.integers(1, base.size - 1))
        st = int(base[i]) + 1
        if i in used or int(base[i + 1]) - st < run_len:
            continue
        used.add(i)
        starts.append(st)
    ins = np.concatenate([np.arange(x, x + run_len, dtype=np.uint64) for x in starts]).astype(dt)
    rng.shuffle(ins)
    s.insert(to_dev(ins), to_dev(ins ^ dt(0x55)))
    o.insert(ins, ins ^ dt(0x55))
    assert_same_contents(s, o, kb, "chained store")
    mk = s.copy_layout()["mkba"]
    buckets = sorted(set(int(np.searchsorted(mk, np.array([x], dtype=dt))[0]) for x in starts))
    return s, o, rng, starts, buckets


@pytest.mark.parametrize("kb", [32, 64])
def test_wide_delete_spread_every_other_and_whole_chain(kb):
    dt = ktype(kb)
    s, o, rng, starts, watch = _chained_store(kb, 12, 16384, 300 + kb)
    cur, _ = o.dump()
    lay = s.copy_layout()
    log(f"wide delete kb={kb}: chains {[len(_chain(lay, b)) for b in watch]}")
    # 1. uniform over everything (every chain node touched, ~6%)
    d1 = cur[rng.random(cur.size) < 0.06]
    _run_case(s, o, kb, d1, "spread", watch)
    # 2. every other key of the first runs: every node halves, joins follow
    runs = [np.arange(x, x + 16384, dtype=np.uint64).astype(dt) for x in starts]
    d2 = np.concatenate([r[::2] for r in runs[:4]])
    rng.shuffle(d2)
    _run_case(s, o, kb, d2, "every other", watch)
    # 3. the whole bucket of one run (the head ends empty), tail of another
    cur, _ = o.dump()
    mk = s.copy_layout()["mkba"]
    b = watch[0]
    lo = mk[b - 1] if b > 0 else dt(0)
    whole = cur[(cur <= mk[b]) & (cur > lo)] if b > 0 else cur[cur <= mk[b]]
    tail = runs[5][-3000:]
    d3 = np.concatenate([whole, tail])
    rng.shuffle(d3)
    _run_case(s, o, kb, d3, "whole chain and a tail", watch)
    q = np.concatenate([runs[0][::97], runs[5][-4000::13], cur[rng.integers(0, cur.size, 3000)],
                        np.array([lo, mk[b]], dtype=dt)])
    check_reads(s, o, kb, q, maxpq=8, where="after wide deletes")


def test_wide_delete_chain_longer_than_a_window():
    """One run of 40,000 keys: a chain of ~625 nodes, more than the kernel's
    512-node window; deletes spread over it, then every third key."""
    kb = 32
    dt = ktype(kb)
    s, o, rng, starts, watch = _chained_store(kb, 1, 40000, 77)
    lay = s.copy_layout()
    n0 = len(_chain(lay, watch[0]))
    log(f"long chain: {n0} nodes")
    assert n0 > 512
    run = np.arange(starts[0], starts[0] + 40000, dtype=np.uint64).astype(dt)
    d1 = run[rng.random(run.size) < 0.05]
    _run_case(s, o, kb, d1, "window spread", watch)
    d2 = run[::3]
    _run_case(s, o, kb, d2, "window every third", watch)
    check_reads(s, o, kb, np.concatenate([run[::11], run[1::17]]), maxpq=8, where="long chain")
