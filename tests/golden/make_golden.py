#!/usr/bin/env python3
"""Write the stored expected results of the long parity runs.

Only the oracle (``oracle/``) and the seeded input generators
(``paper_2604_16725_amd/workloads.py``) are called here; nothing comes from
the HIP path.

  update_heavy_rounds.json  the update-heavy workload (u64 keys and values,
      bulk load of 2^24 keys, then 100 rounds of 2^20 inserts followed by
      2^20 deletes; even rounds uniform, odd rounds clustered into 64 runs):
      after every round, the number of stored keys and the digest of the full
      contents (keys, then values, ascending).
  mixed_stream_4096.json    the mixed-batch stream (u32, 2^26-key bulk load,
      4096 batches of floor(2^U) operations, U ~ U[8, 20], 70/10/10/10
      lookup/successor/insert/delete): the digest of every read batch's
      outputs (lookup: values; successor: keys, then values) and the final
      contents.

    python tests/golden/make_golden.py [update_heavy] [mixed_stream]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from golden_digest import digest  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from paper_2604_16725_amd import workloads as w  # noqa: E402


def update_heavy(rounds=100, n_keys=1 << 24, batch=1 << 20, runs=64):
    u = w.UpdateHeavy(n_keys=n_keys, batch=batch, runs=runs)
    o = Oracle(64)
    assert o.bulk_load(u.build_keys, u.build_vals) == 0
    out = []
    t0 = time.time()
    for r in range(rounds):
        ins, iv, dele = u.round(r)
        assert o.insert(ins, iv) == 0
        o.delete(dele)
        k, v = o.dump()
        out.append({"round": r, "kind": "uniform" if r % 2 == 0 else "clustered",
                    "keys": int(k.size), "digest": digest(k, v)})
        print(f"update_heavy round {r}: {k.size} keys ({time.time() - t0:.0f}s)", flush=True)
    return {"workload": f"update-heavy: u64 keys/values, bulk load 2^{n_keys.bit_length() - 1} keys, "
                        f"{rounds} rounds of 2^{batch.bit_length() - 1} inserts then "
                        f"2^{batch.bit_length() - 1} deletes, even rounds uniform, odd rounds "
                        f"clustered into {runs} runs",
            "digest": "blake2b-128 of the ascending keys' bytes, then the values' bytes",
            "written_by": "tests/golden/make_golden.py (oracle only)",
            "rounds": out}


def mixed_stream(nbatch=4096, n_keys=1 << 26):
    s = w.BatchStream(n_keys=n_keys, nbatch=nbatch)
    o = Oracle(32)
    assert o.bulk_load(s.build_keys, s.build_vals) == 0
    out = []
    t0 = time.time()
    for i in range(nbatch):
        op, k, v = s.batch(i)
        rec = {"i": i, "op": op, "n": int(k.size)}
        if op == "lookup":
            rec["digest"] = digest(o.lookup(k))
        elif op == "successor":
            rec["digest"] = digest(*o.successor(k))
        elif op == "insert":
            assert o.insert(k, v) == 0
        else:
            o.delete(k)
        out.append(rec)
        if i % 64 == 0:
            print(f"mixed_stream batch {i} ({time.time() - t0:.0f}s)", flush=True)
    k, v = o.dump()
    return {"workload": f"mixed-batch stream: u32, bulk load 2^{n_keys.bit_length() - 1} keys, "
                        f"{nbatch} batches of floor(2^U) ops, U ~ U[8, 20], 70/10/10/10 "
                        f"lookup/successor/insert/delete",
            "digest": "blake2b-128; lookup: values; successor: keys then values; final: "
                      "ascending keys then values",
            "written_by": "tests/golden/make_golden.py (oracle only)",
            "batches": out, "final": {"keys": int(k.size), "digest": digest(k, v)}}


def main():
    which = sys.argv[1:] or ["update_heavy", "mixed_stream"]
    if "update_heavy" in which:
        res = update_heavy()
        with open(os.path.join(HERE, "update_heavy_rounds.json"), "w") as f:
            json.dump(res, f, indent=0)
    if "mixed_stream" in which:
        res = mixed_stream()
        with open(os.path.join(HERE, "mixed_stream_4096.json"), "w") as f:
            json.dump(res, f, indent=0)


if __name__ == "__main__":
    main()
