"""Serving engine logic on the CPU: coalescing in arrival order, admission
against the epoch capacity and the memory budget, result hand-back and
latency accounting, against an oracle-backed fake backend with a simulated
clock.  The results of every request are checked against a replay of the
admitted epochs on a second oracle."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2604_16725_amd import serve
from paper_2604_16725_amd.workloads import ServingWorkload
from serving_fake import FakeBackend

TOMB = (1 << 64) - 1
RM = 64


def _wl(n_req=240, n_keys=1 << 12, seed=0):
    return ServingWorkload(n_keys=n_keys, n_req=n_req, max_ops=512, seed_round=seed)


def _oracle(wl):
    o = Oracle(64)
    o.bulk_load(wl.build_keys, wl.build_vals)
    return o


def _replay_and_compare(wl, run):
    """Replay the admitted epochs on a fresh oracle; every completed
    request's results must match."""
    o = _oracle(wl)
    res = run["results"]
    for ids in run["epochs"]:
        ep = serve.EpochLists(wl, ids, TOMB)
        lv, rc, rv = o.apply_epoch(ep.lookup_keys, ep.range_lo, ep.range_hi, RM,
                                   ep.update_keys, ep.update_vals)
        assert np.array_equal(res.lookup[ep.flat_lookup], lv)
        if ep.range_ord.size:
            assert np.array_equal(res.range_count[ep.range_ord], rc)
            got = res.range_vals[ep.range_ord]
            m = np.arange(RM)[None, :] < np.minimum(rc, RM)[:, None]
            assert np.array_equal(got[m], rv[m])
    return o


@pytest.mark.parametrize("rate", [2e3, 2e4])
def test_engine_coalesces_in_order_and_matches_replay(rate):
    wl = _wl()
    be = FakeBackend(_oracle(wl), RM)
    eng = serve.Engine(be, max_epoch_ops=4096, budget=64 << 30)
    run = eng.run(wl, wl.arrivals(rate), TOMB, 8, RM)
    assert run["completed"] == wl.n_req and not run["rejected"]
    flat = [i for ids in run["epochs"] for i in ids]
    assert flat == list(range(wl.n_req))            # admitted order = arrival order
    for ids in run["epochs"]:
        assert sum(int(wl.sizes[i]) for i in ids) <= 4096 or len(ids) == 1
    lat = run["latency"]
    assert np.all(lat >= 200e-6 - 1e-12)             # at least one epoch's service time
    slots = [s for s, _ in be.submitted]
    assert slots == [i % 2 for i in range(len(slots))]   # the two slots alternate
    _replay_and_compare(wl, run)
    s = serve.summary(run, wl, rate)
    assert s["requests"] == wl.n_req and s["p99_ms"] >= s["p50_ms"] > 0


def test_high_rate_coalesces_more():
    wl = _wl()
    runs = {}
    for rate in (1e3, 1e5):
        be = FakeBackend(_oracle(wl), RM)
        runs[rate] = serve.Engine(be, 4096, 64 << 30).run(wl, wl.arrivals(rate), TOMB, 8, RM)
    assert len(runs[1e5]["epochs"]) < len(runs[1e3]["epochs"])


def test_budget_and_capacity_admission():
    wl = _wl(n_req=160)
    rb = np.array([serve.request_bytes(wl, i, 8, RM) for i in range(wl.n_req)])
    assert np.array_equal(serve.request_bytes_all(wl, 8, RM), rb)
    budget = int(np.sort(rb)[-3])                    # the 2 largest requests never fit
    be = FakeBackend(_oracle(wl), RM)
    run = serve.Engine(be, max_epoch_ops=600, budget=budget).run(wl, wl.arrivals(1e5), TOMB, 8,
                                                                  RM)
    too_big = set(np.nonzero(rb > budget)[0].tolist())
    assert set(run["rejected"]) == too_big and len(too_big) >= 1
    assert run["max_inflight_bytes"] <= budget
    assert run["completed"] == wl.n_req - len(too_big)
    for ids in run["epochs"]:
        assert sum(int(wl.sizes[i]) for i in ids) <= 600
    _replay_and_compare(wl, run)


def test_plain_form_runs_requests_alone():
    wl = _wl(n_req=60)
    be = FakeBackend(_oracle(wl), RM)
    run = serve.Engine(be, 4096, 64 << 30, coalesce=False).run(wl, wl.arrivals(1e5), TOMB, 8, RM)
    assert all(len(ids) == 1 for ids in run["epochs"]) and len(run["epochs"]) == wl.n_req
    assert all(s == 0 for s, _ in be.submitted)
    _replay_and_compare(wl, run)


def test_probe_results_same_alone_and_in_mix():
    """Requests whose keys no other request writes give the same results in
    the mix as alone (each probe run as the only request on a fresh store)."""
    wl = _wl(n_req=200)
    upd = np.isin(wl.ops, (serve.INSERT, serve.DELETE))
    written = np.sort(wl.keys[upd])
    probes = []
    for i in range(wl.n_req):
        a, b = int(wl.offsets[i]), int(wl.offsets[i + 1])
        ops = wl.ops[a:b]
        if np.any(ops >= serve.INSERT):
            continue
        lo, hi = wl.keys[a:b], np.where(ops == serve.RANGE, wl.aux[a:b], wl.keys[a:b])
        # no written key inside any [lo, hi] of the request
        if np.all(np.searchsorted(written, lo, "left") == np.searchsorted(written, hi, "right")):
            probes.append(i)
    assert len(probes) >= 20
    be = FakeBackend(_oracle(wl), RM)
    mix = serve.Engine(be, 4096, 64 << 30).run(wl, wl.arrivals(3e4), TOMB, 8, RM)["results"]
    for i in probes[:20]:
        alone = _oracle(wl)
        ep = serve.EpochLists(wl, [i], TOMB)
        lv, rc, rv = alone.apply_epoch(ep.lookup_keys, ep.range_lo, ep.range_hi, RM,
                                       ep.update_keys, ep.update_vals)
        assert np.array_equal(mix.lookup[ep.flat_lookup], lv)
        if ep.range_ord.size:
            assert np.array_equal(mix.range_count[ep.range_ord], rc)


def test_epoch_lists_match_per_request_slices():
    """The vectorised index construction equals concatenating each request's
    own slice of operations, in admitted order (empty lists included)."""
    wl = _wl(n_req=300)
    rng = np.random.default_rng(5)
    for ids in ([], [7], [3, 1, 2], list(rng.permutation(wl.n_req)[:120])):
        ep = serve.EpochLists(wl, ids, TOMB)
        ref = (np.concatenate([np.arange(wl.offsets[i], wl.offsets[i + 1]) for i in ids])
               if ids else np.zeros(0, dtype=np.int64))
        is_l = wl.ops[ref] == serve.LOOKUP
        assert np.array_equal(ep.flat_lookup, ref[is_l])
        assert ep.n_ops == ref.size
        assert np.array_equal(ep.lookup_keys, wl.keys[ref][is_l])
