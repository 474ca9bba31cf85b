"""The batching form on the mixed-batch stream (uneven lookup / successor /
insert / delete batches): the persistent drain replayed from a hipGraph and
the plain per-batch calls both match the oracle applying the same batches in
order, batch by batch, and end with the oracle's contents.  One case runs a
reduced store; one runs the 2^26-key store with 2^8..2^20-op batches (a
prefix of the stream).  The tuner's sweep is checked on a small grid.
"""
import os

import numpy as np
import pytest

from gpu_helpers import assert_same_contents, log, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _check_stream(ds, outs, o, where):
    """Replay the resident stream on the oracle; compare every read batch."""
    ov_all = to_host(outs[0], 32)
    ok_all = to_host(outs[1], 32)
    for i, op in enumerate(ds.ops):
        a, b = int(ds.offsets[i]), int(ds.offsets[i + 1])
        k = ds.host_keys[a:b]
        if op == "insert":
            assert o.insert(k, ds.host_vals[a:b]) == 0
        elif op == "delete":
            o.delete(k)
        elif op == "lookup":
            g = ov_all[a:b]
            e = o.lookup(k)
            bad = np.nonzero(g != e)[0]
            assert bad.size == 0, f"{where} batch {i} lookup: {bad.size} mismatches"
        else:
            ek, ev = o.successor(k)
            assert np.array_equal(ok_all[a:b], ek), f"{where} batch {i} successor keys"
            assert np.array_equal(ov_all[a:b], ev), f"{where} batch {i} successor vals"


def _run(n_keys, nbatch, prefix, log2_max, cap, lanes, rb):
    import torch
    from oracle.oracle import Oracle
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd.batching import DeviceStream, PersistentRun, run_plain
    from paper_2604_16725_amd.workloads import BatchStream

    stream = BatchStream(n_keys=n_keys, nbatch=nbatch, log2_max=log2_max)
    ds = DeviceStream(stream, limit=prefix)
    log(f"stream: {ds.n} batches, {ds.total_ops} ops, store {n_keys} keys, cap {cap} "
        f"lanes {lanes} radix {rb}")
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        st = flix.Store(key_bits=32, capacity=cap, lanes=lanes, radix_bits=rb,
                        max_batch=1 << int(np.ceil(log2_max)))
        outs_p, outs_g = ds.outputs(), ds.outputs()
        st.bulk_load(ds.build_keys, ds.build_vals)
        log("plain form")
        run_plain(st, ds, outs_p, events=False)
        assert st.status() == 0
        o = Oracle(32)
        o.bulk_load(stream.build_keys, stream.build_vals)
        _check_stream(ds, outs_p, o, "plain")
        assert_same_contents(st, o, 32, "plain end")
        log("persistent form (graph), two replays from the same bulk load")
        run = PersistentRun(st, ds, outs_g, cs)
        for rep in range(2):
            outs_g[0].fill_(-1)
            outs_g[1].fill_(-1)
            st.bulk_load(ds.build_keys, ds.build_vals)
            wall, svc = run.run()
            assert st.status() == 0
            assert svc.shape == (ds.n,) and np.all(svc >= 0)
            assert torch.equal(outs_p[0], outs_g[0]) and torch.equal(outs_p[1], outs_g[1]), \
                f"replay {rep}: persistent outputs differ from the plain form"
            assert_same_contents(st, o, 32, f"persistent replay {rep} end")
        run.close()
        st.close()


def test_stream_reduced_vs_oracle():
    _run(n_keys=1 << 18, nbatch=96, prefix=None, log2_max=14.0, cap=64, lanes=16, rb=8)


def test_stream_reduced_radix4_lanes64():
    _run(n_keys=1 << 17, nbatch=64, prefix=None, log2_max=13.0, cap=32, lanes=64, rb=4)


@pytest.mark.parametrize("cap,lanes,rb", [(c, g, r) for c in (32, 128) for g in (16, 64)
                                           for r in (4, 8)])
def test_stream_small_store_grid_vs_oracle(cap, lanes, rb):
    _run(n_keys=1 << 16, nbatch=24, prefix=None, log2_max=14.0, cap=cap, lanes=lanes, rb=rb)


@pytest.mark.parametrize("cap,lanes,rb", [(32, 16, 4), (128, 16, 4), (256, 32, 8)])
def test_stream_batches_larger_than_store_vs_oracle(cap, lanes, rb):
    """Batches of up to 2^20 operations on a 2^16-key store: long chains,
    multi-piece splits, chunked merges and emptied buckets."""
    _run(n_keys=1 << 16, nbatch=24, prefix=None, log2_max=20.0, cap=cap, lanes=lanes, rb=rb)


def test_stream_full_size_prefix_vs_oracle():
    n = int(os.environ.get("FLIX_STREAM_PREFIX", "64"))
    _run(n_keys=1 << 26, nbatch=4096, prefix=n, log2_max=20.0, cap=128, lanes=16, rb=8)


def test_autotune_small_grid(tmp_path):
    from paper_2604_16725_amd import autotune
    res = autotune.sweep(n_keys=1 << 16, nbatch=24, prefix=24, reps=1, log2_max=14.0,
                         grid={"capacity": (32, 128), "lanes": (16, 64), "radix_bits": (4, 8)},
                         with_plain=True, log=log)
    assert len(res["points"]) == 8
    for p in res["points"]:
        assert p["persistent"]["Mops_s"] > 0 and p["plain"]["Mops_s"] > 0
    path = tmp_path / "t.json"
    import json
    path.write_text(json.dumps(res))
    cfg = autotune.tuned_config(str(path))
    assert cfg == {k: res["best"][k] for k in ("capacity", "lanes", "radix_bits")}
