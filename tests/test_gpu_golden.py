"""Long parity runs against stored oracle digests (``tests/golden/*.json``,
written by ``tests/golden/make_golden.py`` from the oracle alone).

* update-heavy: u64 store, 2^24-key bulk load, all 100 rounds of 2^20 inserts
  then 2^20 deletes (uniform and clustered rounds alternating); after every
  round the full contents must hash to the oracle's digest and the device
  invariant checker must pass;
* mixed-batch stream: all 4096 batches on the 2^26-key u32 store, once as one
  call per batch and once drained by the persistent kernel from a hipGraph;
  every read batch's outputs and the final contents must hash to the
  oracle's digests.

On the first mismatch the oracle is replayed up to that point and the first
differing elements are printed.
"""
import json
import os

import numpy as np
import pytest

from golden_digest import digest
from gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _first_diff(name, g, o):
    if g.size != o.size:
        return f"{name}: {g.size} elements vs the oracle's {o.size}"
    bad = np.nonzero(g != o)[0]
    return f"{name}: {bad.size} mismatches, first at {bad[:5]}: {g[bad[:5]]} vs {o[bad[:5]]}"


def test_update_heavy_all_rounds_vs_golden():
    from oracle.oracle import Oracle
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    gold = json.load(open(os.path.join(GOLDEN, "update_heavy_rounds.json")))
    rounds = gold["rounds"]
    log(f"update heavy: 2^24 u64 keys, {len(rounds)} rounds against stored digests")
    u = w.UpdateHeavy(n_keys=1 << 24, batch=1 << 20, runs=64)
    st = flix.Store(key_bits=64, capacity=128, lanes=16, radix_bits=8, max_batch=1 << 20)
    st.bulk_load(to_dev(u.build_keys), to_dev(u.build_vals))
    history = []
    for rec in rounds:
        r = rec["round"]
        ins, iv, dele = u.round(r)
        history.append((ins, iv, dele))
        st.insert(to_dev(ins), to_dev(iv))
        st.delete(to_dev(dele))
        assert st.status() == 0, f"round {r}: device error"
        gk, gv = st.dump()
        hk, hv = to_host(gk, 64), to_host(gv, 64)
        del gk, gv
        stats = st.stats()
        log(f"round {r} ({rec['kind']}): keys={stats['keys']} live_nodes={stats['live_nodes']} "
            f"free={stats['pool_nodes'] - stats['live_nodes']}")
        if hk.size != rec["keys"] or digest(hk, hv) != rec["digest"]:
            o = Oracle(64)
            o.bulk_load(u.build_keys, u.build_vals)
            for a, b, c in history:
                o.insert(a, b)
                o.delete(c)
            ok, ov = o.dump()
            pytest.fail(f"round {r}: contents differ from the stored digest; "
                        + _first_diff("keys", hk, ok) + "; " + _first_diff("vals", hv, ov))
        rc = st.check()
        assert rc == 0, f"round {r}: invariant check code {rc}"
    st.close()


def _run_stream_form(form, cfg, ds, stream, outs):
    import torch
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd.batching import PersistentRun, pool_bytes_for, run_plain
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        st = flix.Store(key_bits=32, capacity=cfg["capacity"], lanes=cfg["lanes"],
                        radix_bits=cfg["radix_bits"], max_batch=1 << 20,
                        pool_bytes=pool_bytes_for(stream, cfg["capacity"]))
        st.bulk_load(ds.build_keys, ds.build_vals)
        if form == "plain":
            run_plain(st, ds, outs, events=False)
        else:
            run = PersistentRun(st, ds, outs, cs)
            run.run()
            run.close()
        torch.cuda.synchronize()
        assert st.status() == 0, f"{form}: device error"
        gk, gv = st.dump()
        final = (to_host(gk, 32), to_host(gv, 32))
        st.close()
    return final


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_mixed_stream_all_batches_vs_golden(form):
    from paper_2604_16725_amd import autotune
    from paper_2604_16725_amd.batching import DeviceStream
    from paper_2604_16725_amd.workloads import BatchStream
    gold = json.load(open(os.path.join(GOLDEN, "mixed_stream_4096.json")))
    nb = len(gold["batches"])
    stream = BatchStream(n_keys=1 << 26, nbatch=nb)
    ds = DeviceStream(stream)
    log(f"mixed stream ({form}): {ds.n} batches, {ds.total_ops} ops resident")
    cfg = autotune.tuned_config(form=form)
    outs = ds.outputs()
    fk, fv = _run_stream_form(form, cfg, ds, stream, outs)
    ov_all = to_host(outs[0], 32)
    ok_all = to_host(outs[1], 32)
    del outs
    bad = None
    for rec in gold["batches"]:
        i, op = rec["i"], rec["op"]
        assert op == ds.ops[i] and rec["n"] == int(ds.sizes[i])
        a, b = int(ds.offsets[i]), int(ds.offsets[i + 1])
        if op == "lookup":
            got = digest(ov_all[a:b])
        elif op == "successor":
            got = digest(ok_all[a:b], ov_all[a:b])
        else:
            continue
        if got != rec["digest"]:
            bad = i
            break
    if bad is not None:
        from oracle.oracle import Oracle
        o = Oracle(32)
        o.bulk_load(stream.build_keys, stream.build_vals)
        for i in range(bad):
            op, k, v = stream.batch(i)
            if op == "insert":
                o.insert(k, v)
            elif op == "delete":
                o.delete(k)
        op, k, _ = stream.batch(bad)
        a, b = int(ds.offsets[bad]), int(ds.offsets[bad + 1])
        if op == "lookup":
            msg = _first_diff("values", ov_all[a:b], o.lookup(k))
        else:
            ek, ev = o.successor(k)
            msg = _first_diff("keys", ok_all[a:b], ek) + "; " + _first_diff("vals", ov_all[a:b], ev)
        pytest.fail(f"{form}: batch {bad} ({op}, {b - a} ops) differs from the stored digest; {msg}")
    assert fk.size == gold["final"]["keys"], f"{form}: final size {fk.size}"
    assert digest(fk, fv) == gold["final"]["digest"], f"{form}: final contents differ"
