"""Shared helpers of the GPU parity tests (host <-> device conversion, store
builders, full-contents comparison against the oracle)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        t = torch.from_numpy(a.view(np.int32))
    elif a.dtype == np.uint64:
        t = torch.from_numpy(a.view(np.int64))
    else:
        t = torch.from_numpy(a)
    return t.cuda()


def to_host(t, kb: int) -> np.ndarray:
    a = t.detach().cpu().numpy()
    if kb == 32:
        return a.view(np.uint32)
    return a.view(np.uint64)


def ktype(kb):
    return np.uint32 if kb == 32 else np.uint64


def new_pair(kb, cap=64, lanes=16, rb=8, max_batch=1 << 16, pool_bytes=0, fill=0):
    from oracle.oracle import Oracle
    from paper_2604_16725_amd.flix import Store
    s = Store(key_bits=kb, capacity=cap, lanes=lanes, radix_bits=rb, max_batch=max_batch,
              pool_bytes=pool_bytes, fill=fill)
    return s, Oracle(kb)


def assert_same_contents(store, orc, kb, where=""):
    gk, gv = store.dump()
    gk, gv = to_host(gk, kb), to_host(gv, kb)
    ok, ov = orc.dump()
    assert gk.size == ok.size, f"{where}: size {gk.size} != {ok.size}"
    if gk.size:
        bad = np.nonzero((gk != ok) | (gv != ov))[0]
        assert bad.size == 0, f"{where}: first mismatch at {bad[:5]}: " \
                              f"{gk[bad[:3]]}/{gv[bad[:3]]} vs {ok[bad[:3]]}/{ov[bad[:3]]}"
    assert store.size() == orc.size()
    rc = store.check()
    assert rc == 0, f"{where}: device invariant check failed with code {rc}"


def check_reads(store, orc, kb, q, maxpq=8, lo=None, hi=None, where=""):
    """Lookup, successor, predecessor and range on the same keys, bit-exact."""
    dq = to_dev(q)
    g = to_host(store.lookup(dq), kb)
    o = orc.lookup(q)
    bad = np.nonzero(g != o)[0]
    assert bad.size == 0, f"{where} lookup mismatch at {bad[:5]}: q={q[bad[:3]]} {g[bad[:3]]} vs {o[bad[:3]]}"
    gk, gv = store.successor(dq)
    gk, gv = to_host(gk, kb), to_host(gv, kb)
    ok, ov = orc.successor(q)
    bad = np.nonzero((gk != ok) | (gv != ov))[0]
    assert bad.size == 0, f"{where} successor mismatch at {bad[:5]}: q={q[bad[:3]]} {gk[bad[:3]]} vs {ok[bad[:3]]}"
    gk, gv = store.predecessor(dq)
    gk, gv = to_host(gk, kb), to_host(gv, kb)
    ok, ov = orc.predecessor(q)
    bad = np.nonzero((gk != ok) | (gv != ov))[0]
    assert bad.size == 0, f"{where} predecessor mismatch at {bad[:5]}: q={q[bad[:3]]} {gk[bad[:3]]} vs {ok[bad[:3]]}"
    if lo is None:
        lo = q
        mx = (1 << kb) - 1
        hi = np.minimum(q.astype(np.uint64) + np.uint64(1 << (kb - 8)), np.uint64(mx)).astype(ktype(kb))
    c, rk, rv = store.range(to_dev(lo), to_dev(hi), maxpq)
    c = c.cpu().numpy().view(np.uint32)
    rk = to_host(rk, kb)[: lo.size * maxpq].reshape(lo.size, maxpq) if maxpq else None
    rv = to_host(rv, kb)[: lo.size * maxpq].reshape(lo.size, maxpq) if maxpq else None
    oc, ok2, ov2 = orc.range(lo, hi, maxpq)
    bad = np.nonzero(c != oc)[0]
    assert bad.size == 0, f"{where} range count mismatch at {bad[:5]}: {c[bad[:3]]} vs {oc[bad[:3]]}"
    if maxpq:
        w = np.minimum(oc, maxpq)
        mask = np.arange(maxpq)[None, :] < w[:, None]
        assert np.array_equal(rk[mask], ok2[mask]), f"{where} range keys mismatch"
        assert np.array_equal(rv[mask], ov2[mask]), f"{where} range values mismatch"
