"""Full-size parity: the read-path store (2^26 u32 keys, capacity 128, 2^20-op
batches, the launch configuration bench.py times) and the update-heavy u64
store (2^24 keys, 2^20-op insert and delete rounds, uniform and clustered),
compared with the oracle on every output element and on the full contents.

FLIX_FULL_ROUNDS (default 4) sets the number of update-heavy rounds; the
workload defines 100.
"""
import os

import numpy as np
import pytest

from gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _cmp(name, g, o):
    bad = np.nonzero(g != o)[0]
    assert bad.size == 0, f"{name}: {bad.size} mismatches, first at {bad[:5]}: {g[bad[:3]]} vs {o[bad[:3]]}"


def test_read_path_full_size_bit_exact():
    from oracle.oracle import Oracle
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    log("read path: generating 2^26 keys")
    wl = w.read_path(n_keys=1 << 26, batch=1 << 20, with_zipf=True, with_updates=True)
    st = flix.Store(key_bits=32, capacity=128, lanes=16, radix_bits=8, max_batch=1 << 20)
    st.bulk_load(to_dev(wl["build_keys"]), to_dev(wl["build_vals"]))
    o = Oracle(32)
    o.bulk_load(wl["build_keys"], wl["build_vals"])
    assert st.size() == o.size() == 1 << 26
    L = wl["range_len"]
    for tag in ["", "zipf_"]:
        log(f"read path: {tag}lookup/successor/range")
        q = wl[tag + "lookup"]
        _cmp(tag + "lookup", to_host(st.lookup(to_dev(q)), 32), o.lookup(q))
        q = wl[tag + "successor"]
        gk, gv = st.successor(to_dev(q))
        ok, ov = o.successor(q)
        _cmp(tag + "successor keys", to_host(gk, 32), ok)
        _cmp(tag + "successor vals", to_host(gv, 32), ov)
        lo, hi = wl[tag + "range_lo"], wl[tag + "range_hi"]
        c, rk, rv = st.range(to_dev(lo), to_dev(hi), L)
        oc, ork, orv = o.range(lo, hi, L)
        c = c.cpu().numpy().view(np.uint32)
        _cmp(tag + "range counts", c, oc)
        m = np.arange(L)[None, :] < np.minimum(oc, L)[:, None]
        _cmp(tag + "range keys", to_host(rk, 32).reshape(-1, L)[m], ork[m])
        _cmp(tag + "range vals", to_host(rv, 32).reshape(-1, L)[m], orv[m])
    log("read path: insert + delete of 2^20 new keys, full contents")
    ik, iv = wl["insert_keys"], wl["insert_vals"]
    st.insert(to_dev(ik), to_dev(iv))
    o.insert(ik, iv)
    assert st.status() == 0
    gk, gv = st.dump()
    ok, ov = o.dump()
    _cmp("contents keys after insert", to_host(gk, 32), ok)
    _cmp("contents vals after insert", to_host(gv, 32), ov)
    del gk, gv
    assert st.check() == 0
    st.delete(to_dev(ik))
    o.delete(ik)
    gk, gv = st.dump()
    ok, ov = o.dump()
    _cmp("contents keys after delete", to_host(gk, 32), ok)
    _cmp("contents vals after delete", to_host(gv, 32), ov)
    assert st.check() == 0
    st.close()


def test_update_heavy_full_size_rounds():
    from oracle.oracle import Oracle
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    rounds = int(os.environ.get("FLIX_FULL_ROUNDS", "4"))
    log(f"update heavy: 2^24 u64 keys, {rounds} rounds")
    u = w.UpdateHeavy(n_keys=1 << 24, batch=1 << 20, runs=64)
    st = flix.Store(key_bits=64, capacity=128, lanes=16, radix_bits=8, max_batch=1 << 20)
    st.bulk_load(to_dev(u.build_keys), to_dev(u.build_vals))
    o = Oracle(64)
    o.bulk_load(u.build_keys, u.build_vals)
    for r in range(rounds):
        ins, iv, dele = u.round(r)
        log(f"round {r} ({'uniform' if r % 2 == 0 else 'clustered'}): insert")
        st.insert(to_dev(ins), to_dev(iv))
        assert o.insert(ins, iv) == 0
        assert st.status() == 0
        log(f"round {r}: delete")
        st.delete(to_dev(dele))
        o.delete(dele)
        assert st.status() == 0
        gk, gv = st.dump()
        ok, ov = o.dump()
        _cmp(f"round {r} keys", to_host(gk, 64), ok)
        _cmp(f"round {r} vals", to_host(gv, 64), ov)
        del gk, gv
        rc = st.check()
        assert rc == 0, f"round {r}: invariant check code {rc}"
        stats = st.stats()
        log(f"round {r}: keys={stats['keys']} live_nodes={stats['live_nodes']}")
    st.close()
