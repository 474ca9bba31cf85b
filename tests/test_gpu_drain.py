"""Persistent fused drain: a queue of mixed batches in one launch (and in a
hipGraph replay) gives exactly the results of the per-batch calls and of the
oracle applying the same batches in order."""
import numpy as np
import pytest

from gpu_helpers import assert_same_contents, ktype, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _queue(rng, kb, universe, nbatch, max_n, mix=(0.55, 0.1, 0.1, 0.15, 0.1)):
    import torch
    mx = (1 << kb) - 1
    dt = torch.int32 if kb == 32 else torch.int64
    ops = ["lookup", "successor", "range", "insert", "delete"]
    q = []
    for i in range(nbatch):
        op = ops[int(rng.choice(5, p=mix))]
        n = int(rng.integers(0, max_n + 1)) if rng.random() > 0.05 else 0
        keys = rng.choice(universe, n) if n else np.zeros(0, dtype=ktype(kb))
        b = {"op": op, "np_keys": keys, "keys": to_dev(keys) if n else None}
        if op == "insert":
            v = rng.integers(0, mx, n, dtype=np.uint64).astype(ktype(kb))
            b["np_aux"] = v
            b["aux"] = to_dev(v) if n else None
        if op == "range":
            hi = np.minimum(keys.astype(np.uint64) + np.uint64(1 << (kb - 12)),
                            np.uint64(mx)).astype(ktype(kb))
            b["np_aux"] = hi
            b["aux"] = to_dev(hi) if n else None
            b["max_per_query"] = 4
            b["counts"] = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
            b["out_k"] = torch.zeros(max(n * 4, 1), dtype=dt, device="cuda")
            b["out_v"] = torch.zeros(max(n * 4, 1), dtype=dt, device="cuda")
        if op in ("lookup", "successor"):
            b["out_v"] = torch.zeros(max(n, 1), dtype=dt, device="cuda")
        if op == "successor":
            b["out_k"] = torch.zeros(max(n, 1), dtype=dt, device="cuda")
        q.append(b)
    return q


def _oracle_apply_and_check(o, q, kb, where):
    """Apply the queue to the oracle in order; compare every read batch."""
    for i, b in enumerate(q):
        n = b["np_keys"].size
        if n == 0:
            continue
        k = b["np_keys"]
        if b["op"] == "insert":
            assert o.insert(k, b["np_aux"]) == 0
        elif b["op"] == "delete":
            o.delete(k)
        elif b["op"] == "lookup":
            g = to_host(b["out_v"], kb)[:n]
            assert np.array_equal(g, o.lookup(k)), f"{where} batch {i} lookup"
        elif b["op"] == "successor":
            ok, ov = o.successor(k)
            assert np.array_equal(to_host(b["out_k"], kb)[:n], ok), f"{where} batch {i} succ keys"
            assert np.array_equal(to_host(b["out_v"], kb)[:n], ov), f"{where} batch {i} succ vals"
        else:
            oc, ork, orv = o.range(k, b["np_aux"], 4)
            c = b["counts"].cpu().numpy().view(np.uint32)[:n]
            assert np.array_equal(c, oc), f"{where} batch {i} range counts"
            m = np.arange(4)[None, :] < np.minimum(oc, 4)[:, None]
            assert np.array_equal(to_host(b["out_k"], kb)[: n * 4].reshape(n, 4)[m], ork[m])
            assert np.array_equal(to_host(b["out_v"], kb)[: n * 4].reshape(n, 4)[m], orv[m])


def _plain(store, q):
    for b in q:
        if b["keys"] is None:
            continue
        if b["op"] == "lookup":
            store.lookup(b["keys"], out=b["out_v"])
        elif b["op"] == "successor":
            store.successor(b["keys"], out_k=b["out_k"], out_v=b["out_v"])
        elif b["op"] == "range":
            store.range(b["keys"], b["aux"], 4, counts=b["counts"], out_k=b["out_k"],
                        out_v=b["out_v"])
        elif b["op"] == "insert":
            store.insert(b["keys"], b["aux"])
        else:
            store.delete(b["keys"])


@pytest.mark.parametrize("kb,cap,lanes,rb", [(32, 64, 16, 8), (64, 128, 32, 8), (32, 32, 64, 4)])
def test_drain_matches_oracle_and_plain(kb, cap, lanes, rb):
    import torch
    from oracle.oracle import Oracle
    from paper_2604_16725_amd.flix import Store
    rng = np.random.default_rng(kb + cap + lanes)
    mx = (1 << kb) - 1
    universe = np.unique(rng.integers(0, mx, 60000, dtype=np.uint64).astype(ktype(kb)))
    build = rng.choice(universe, 20000, replace=False)
    sd = Store(key_bits=kb, capacity=cap, lanes=lanes, radix_bits=rb, max_batch=8192)
    sp = Store(key_bits=kb, capacity=cap, lanes=lanes, radix_bits=rb, max_batch=8192)
    o = Oracle(kb)
    for st in (sd, sp):
        st.bulk_load(to_dev(build), to_dev(build))
    o.bulk_load(build, build)
    q = _queue(rng, kb, universe, 40, 8192)
    log(f"drain kb={kb} cap={cap}: {sum(b['np_keys'].size for b in q)} ops in 40 batches")
    sd.drain(q)
    torch.cuda.synchronize()
    assert sd.status() == 0, "drain reported a device error"
    _oracle_apply_and_check(o, q, kb, "drain")
    assert_same_contents(sd, o, kb, "after drain")
    drained = [{k: (v.clone() if hasattr(v, "clone") else v) for k, v in b.items()} for b in q]
    _plain(sp, q)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(drained, q)):
        for key in ("out_v", "out_k", "counts"):
            if key in a and a["keys"] is not None:
                assert torch.equal(a[key], b[key]), f"batch {i} {key}: drain != plain"
    assert_same_contents(sp, o, kb, "plain after the same queue")
    g, hz = sd.drain_info()
    assert g > 0 and hz > 0


def test_drain_graph_replays_with_eager_work_between():
    import torch
    from oracle.oracle import Oracle
    from paper_2604_16725_amd.flix import Store
    kb = 32
    rng = np.random.default_rng(11)
    universe = np.unique(rng.integers(0, 1 << 32, 40000, dtype=np.uint64).astype(np.uint32))
    build = rng.choice(universe, 10000, replace=False)
    s = Store(key_bits=kb, capacity=64, lanes=16, max_batch=4096)
    o = Oracle(kb)
    s.bulk_load(to_dev(build), to_dev(build))
    o.bulk_load(build, build)
    stream = torch.cuda.Stream()
    ts = torch.zeros(11, dtype=torch.int64, device="cuda")
    q = _queue(rng, kb, universe, 10, 4096)
    with torch.cuda.stream(stream):
        graph = s.drain_graph(q, timestamps=ts, stream=stream)
    for rep in range(3):
        if rep:
            q = _queue(rng, kb, universe, 10, 4096)
            graph.update(q)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert s.status() == 0
        _oracle_apply_and_check(o, q, kb, f"replay {rep}")
        t = ts.cpu().numpy()
        assert np.all(np.diff(t) >= 0) and t[-1] > t[0]
        # eager work between replays
        extra = rng.choice(universe, 500)
        s.insert(to_dev(extra), to_dev(extra))
        o.insert(extra, extra)
        torch.cuda.synchronize()
        assert_same_contents(s, o, kb, f"after replay {rep}")
    graph.close()


def test_drain_graph_captured_before_bulk_loads_that_grow_the_store():
    """A graph captured on a freshly created (empty) store keeps working after
    bulk loads that reallocate the directory and the pool: replays read the
    store's current layout, not the one seen at capture."""
    import torch
    from oracle.oracle import Oracle
    from paper_2604_16725_amd.flix import Store
    kb = 32
    rng = np.random.default_rng(17)
    universe = np.unique(rng.integers(0, 1 << 32, 60000, dtype=np.uint64).astype(np.uint32))
    s = Store(key_bits=kb, capacity=32, lanes=16, radix_bits=4, max_batch=4096)
    stream = torch.cuda.Stream()
    q = _queue(rng, kb, universe, 8, 4096)
    with torch.cuda.stream(stream):
        graph = s.drain_graph(q, stream=stream)   # captured on the empty store
    for rep, nbuild in enumerate((20000, 4000, 30000)):
        build = rng.choice(universe, nbuild, replace=False)
        s.bulk_load(to_dev(build), to_dev(build))
        o = Oracle(kb)
        o.bulk_load(build, build)
        if rep:
            q = _queue(rng, kb, universe, 8, 4096)
            graph.update(q)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert s.status() == 0
        _oracle_apply_and_check(o, q, kb, f"replay {rep} after a bulk load of {nbuild}")
        assert_same_contents(s, o, kb, f"replay {rep}")
    graph.close()
    s.close()
