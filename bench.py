#!/usr/bin/env python3
"""FliX batch-operation benchmark on one MI355X.

Workload: the read-path store of the paper's method at full size: 2^26
distinct uniform uint32 keys with uint32 values, node capacity 128 (bulk fill
64), batches of 2^20 operations.  One step is one pass of the whole hot path:
  lookup    2^20 keys, 90% present (uniform with replacement), 10% absent
  successor 2^20 uniform keys
  range     2^20 ranges [lo, lo+15], uniform lo, up to 16 results each
  insert    2^20 new keys
  delete    the same 2^20 keys (the store returns to its bulk-loaded contents)
Every call sorts its batch on the device (onesweep), finds every bucket's slice
and applies it; inputs are resident in HBM before the timed region starts.

Prints ONE JSON line (rank 0) with the throughput of the step in Mops/s, the
HBM roofline of the dominant kernel (algorithmic bytes / its average duration
from HIP events), and the CPU oracle timed on a bounded sample as a baseline.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mops/s lookup/insert/delete at 2^26 keys; p99 batch latency vs plain launch"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--keys-log2", type=int, default=26)
    ap.add_argument("--batch-log2", type=int, default=20)
    ap.add_argument("--capacity", type=int, default=128)
    ap.add_argument("--lanes", type=int, default=16)
    ap.add_argument("--radix-bits", type=int, default=8)
    ap.add_argument("--read-path", choices=["sorted", "groups"], default="sorted",
                    help="read-batch pipeline of the store (device-wide sort, or bucket groups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the mixed-batch stream (persistent drain vs plain launches)")
    ap.add_argument("--nbatch", type=int, default=4096, help="batches in the mixed stream")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving comparison (request loop vs plain per-request form)")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per arrival rate")
    ap.add_argument("--serve-keys-log2", type=int, default=25)
    ap.add_argument("--no-grown", action="store_true",
                    help="skip the reads on a store grown by +100% and restructured")
    ap.add_argument("--update-rounds", type=int, default=20,
                    help="rounds of the update-heavy workload (0 skips it)")
    ap.add_argument("--no-insert-kernels", action="store_true",
                    help="skip the insert-kernel comparison")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="first copy a MiB-sized device buffer 4 times (a plain copy kernel of "
                         "known size, to scale hardware byte counters)")
    return ap.parse_args()


def ensure_built():
    from paper_2604_16725_amd import build_lib
    if not os.path.exists(build_lib.LIB):
        build_lib.build()


# ----------------------------------------------------------------------------
# Algorithmic byte model (what the method must move: directory entries, the
# sorted batch, headers and live node lines of touched buckets, values, outputs)
# ----------------------------------------------------------------------------
def byte_model(wl, mkba, sizes_cap, kbytes=4, vbytes=4, rb=8, read_path="sorted"):
    """Bytes per step for every kernel family, from the actual batches."""
    m = wl["lookup"].size
    nb = mkba.size
    P = (8 * kbytes + rb - 1) // rb
    live_line = lambda size: np.ceil(size * kbytes / 128.0) * 128.0

    def touched(keys):
        b = np.searchsorted(mkba, keys, side="left")
        return np.unique(b)

    build_sorted = wl["_build_sorted"]
    size_of = sizes_cap  # keys per bucket after bulk load (array over buckets)
    groups = read_path == "groups"

    fam = {}
    # sorts per step: insert (key + value) and delete (key only), plus the
    # three read batches (key + input position) on the sorted read path
    pay = [vbytes, 0] if groups else [4, 4, 4, vbytes, 0]
    # input payload read by the first launch: the read batches' input
    # positions are generated, not read
    pay_in = [vbytes, 0] if groups else [0, 0, 0, vbytes, 0]
    split = rb == 8 and m <= (1 << 21)
    if split:
        # batches of up to 2^21 keys with 8-bit digits: the tile split reads
        # the pairs and writes them back split, with one 256-entry row of
        # digit starts per 2048-key tile; the per-run sort reads its column
        # of the rows (two entries per tile), the split pairs and writes the
        # sorted ones
        ntiles = -(-m // 2048)
        fam["sort_pass"] = sum(m * (kbytes + pi) + m * (kbytes + p) + ntiles * 1024
                               for p, pi in zip(pay, pay_in))
        fam["sort_local"] = sum(m * 2 * (kbytes + p) + 256 * ntiles * 8 for p in pay)
    else:
        fam["sort_hist"] = len(pay) * m * kbytes
        # up to 2^22 keys: one device-wide pass on the top digit, then the
        # per-run sort; otherwise P device-wide passes
        local = rb == 8 and m <= (1 << 22)
        fam["sort_pass"] = sum((1 if local else P) * m * 2 * (kbytes + p) for p in pay)
        if local:
            fam["sort_local"] = sum(m * 2 * (kbytes + p) for p in pay)

    def read_bytes(keys, extra_out, val_reads, hi_bytes=0, head_bytes=16):
        # every maxBucket entry, the sorted (or grouped) batch (key +
        # position), the header of each touched bucket, the live prefix of
        # each touched node in whole 128-byte lines, values read, outputs
        t = touched(keys)
        return (nb * kbytes + m * (kbytes + 4) + hi_bytes + t.size * head_bytes
                + float(live_line(size_of[t]).sum()) + val_reads * vbytes + extra_out)

    hits = np.isin(wl["lookup"], build_sorted).sum()
    lo, hi = wl["range_lo"], wl["range_hi"]
    cnt = (np.searchsorted(build_sorted, hi, side="right")
           - np.searchsorted(build_sorted, lo, side="left")).sum()
    if groups:
        # bucket groups: at most 1024 groups of equal bucket counts; k_part
        # reads the keys, writes keys + input positions grouped per tile, the
        # tile group-start rows and the group totals
        bpg = -(-nb // 1024)
        ngroups = -(-nb // bpg)
        ntiles = -(-m // 4096)
        fam["part"] = 3 * (m * kbytes + m * (kbytes + 4) + ntiles * (ngroups + 1) * 4
                           + ngroups * 4)
        look = read_bytes(wl["lookup"], m * vbytes, hits, head_bytes=8)
        succ = read_bytes(wl["successor"], m * (kbytes + vbytes), m, head_bytes=8)
        rng = read_bytes(lo, m * 4 + cnt * (kbytes + vbytes), cnt, hi_bytes=m * kbytes,
                         head_bytes=8)
        fam["group_read"] = look + succ + rng
    else:
        look = read_bytes(wl["lookup"], m * vbytes, hits)
        succ = read_bytes(wl["successor"], m * (kbytes + vbytes), m)
        rng = read_bytes(lo, m * (4 + kbytes) + cnt * (kbytes + vbytes), cnt)
        fam["read_apply"] = look + succ + rng
        # cut list of each read call: one u32 per share boundary, found by a
        # 33-ary search (32 probes per round, half a wave per cut) whose
        # probes read one batch key and one maxBucket entry each
        ncuts = -(-(m + nb) // 512) + 1
        rounds = int(np.ceil(np.log(max(m + nb, 2)) / np.log(33)))
        fam["read_cuts"] = 3 * ncuts * (4 + rounds * 32 * (kbytes + kbytes))

    ins = wl["insert_keys"]
    bi = np.searchsorted(mkba, ins, side="left")
    ti = touched(ins)
    per_bucket = np.bincount(bi, minlength=nb)[ti]
    node = size_of[ti] * (kbytes + vbytes)
    # slot of the smallest new key in its node: items before it keep their
    # slots, so only the suffix from there on is written (insert), and the
    # same suffix moves back when those keys are deleted again
    mins = np.full(nb, np.iinfo(np.uint64).max, dtype=np.uint64)
    np.minimum.at(mins, bi, ins.astype(np.uint64))
    fill = int(size_of[0])
    first = np.searchsorted(build_sorted, mins[ti].astype(build_sorted.dtype)) - ti * fill
    first = np.clip(first, 0, size_of[ti])
    fam["slices"] = 2 * (nb * kbytes + m * kbytes + ti.size * (16 + 4 + 16)) + m * vbytes
    fam["insert_apply"] = float(ti.size * 16 + m * (kbytes + vbytes) + node.sum()
                                + ((size_of[ti] + per_bucket - first) * (kbytes + vbytes)).sum()
                                + ti.size * 16)
    node_after = (size_of[ti] + per_bucket) * (kbytes + vbytes)
    fam["delete_apply"] = float(ti.size * 16 + m * kbytes + node_after.sum()
                                + ((size_of[ti] - first) * (kbytes + vbytes)).sum() + ti.size * 16)
    return fam


def counter_traffic(kernel):
    """HBM bytes per launch of kernel family `kernel` from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by what it reads for
    a plain copy), or None when the kernel sources no longer hash to what was
    measured or the family was not measured."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "read_path_step_hbm_counters.md")
    try:
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        rec = json.loads(m.group(1))
        fam = rec["families"][kernel]
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    h = hashlib.sha256()
    for fn in rec["sources"]:
        try:
            with open(os.path.join(ROOT, "paper_2604_16725_amd", "csrc", fn), "rb") as fh:
                h.update(fh.read())
        except OSError:
            return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return fam["traffic_bytes_per_launch"]


def timed_calls(fn, reps):
    """Median and p99 of `reps` calls of fn, each bracketed by events on the
    current stream (one untimed call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    gc.disable()
    try:
        for a, b in evs:
            a.record()
            fn()
            b.record()
    finally:
        gc.enable()
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.median(ms)), float(np.percentile(ms, 99))


def grown_store_reads(args, wl, dev, bufs):
    """Reads after growth and restructuring after deletes (the paper's queries
    after update rounds, and its restructuring experiment): the 2^keys_log2
    store grows by +100% through 2^batch_log2-key insert batches of new uniform
    keys (about half the buckets become chains); the step's read batches are
    timed there.  Then half of all keys, drawn uniformly, are deleted, which
    leaves underfull nodes; restructuring lays the store out again at the
    bulk-load fill (nodes before and after), and the reads are timed again."""
    import torch
    from paper_2604_16725_amd import flix
    n_keys, m = 1 << args.keys_log2, 1 << args.batch_log2
    ks = wl["keyspace"]
    node_bytes = 16 + 2 * args.capacity * 4
    st = flix.Store(key_bits=32, capacity=args.capacity, lanes=args.lanes,
                    radix_bits=args.radix_bits, max_batch=m,
                    pool_bytes=node_bytes * (4 * n_keys // args.capacity + 4096))
    st.bulk_load(dev(wl["build_keys"]), dev(wl["build_vals"]))
    t0 = time.time()
    nbatches = n_keys // m
    grown_keys = []
    for i in range(nbatches):
        k = ks.fresh(m)
        v = k ^ np.uint32(0x2545F491)
        v[v == np.uint32(0xFFFFFFFF)] = 0
        st.insert(dev(k), dev(v))
        grown_keys.append(k)
    torch.cuda.synchronize()
    if st.status() != 0:
        raise RuntimeError("device error while growing the store")
    log(f"[bench] grown store: +{nbatches * m} keys in {time.time() - t0:.1f}s")
    dl, ds, dlo, dhi = bufs["lookup"], bufs["successor"], bufs["range_lo"], bufs["range_hi"]
    ol, sk, sv, rc, rk, rv, L = (bufs[x] for x in ("ol", "sk", "sv", "rc", "rk", "rv", "L"))
    reps = max(5, args.steps)
    calls = {"lookup": lambda: st.lookup(dl, out=ol),
             "successor": lambda: st.successor(ds, out_k=sk, out_v=sv),
             "range16": lambda: st.range(dlo, dhi, L, counts=rc, out_k=rk, out_v=rv)}

    def measure(tag):
        stt = st.stats()
        nb, keys, live = stt["buckets"], stt["keys"], stt["live_nodes"]
        # algorithmic bytes of the bucket kernel per read batch: every
        # maxBucket entry, the sorted batch, the header of every node of a
        # touched bucket and its live keys in whole lines, values, outputs
        touched = nb * (1.0 - np.exp(-m / nb))
        per_bucket = keys / nb
        chain = live / nb
        lines = np.ceil(per_bucket * 4 / 128.0) * 128.0 + (chain - 1) * 64.0
        base = nb * 4 + m * 8 + touched * (16 * chain + lines)
        outb = {"lookup": m * 4 + 0.9 * m * 4, "successor": m * 8 + m * 4,
                "range16": m * 4 + m * 4 + m * 8}
        rows = {}
        for name, fn in calls.items():
            st.set_timing(True, only="read_apply")
            p50, p99 = timed_calls(fn, reps)
            kms, kn = st.kernel_time("read_apply")
            st.set_timing(False)
            kus = 1000.0 * kms / kn if kn else None
            ab = base + outb[name]
            rows[name] = {"Mops_s": round(m / (p50 / 1000) / 1e6, 1), "p50_ms": round(p50, 4),
                          "p99_ms": round(p99, 4),
                          "bucket_kernel_us": round(kus, 2) if kus else None,
                          "bucket_kernel_alg_MB": round(ab / 1e6, 1),
                          "bucket_kernel_frac": (round(ab / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                                 if kus else None)}
        log(f"[bench] {tag}: buckets {nb}, keys {keys}, nodes {live}: {rows}")
        return {"buckets": nb, "keys": keys, "live_nodes": live, "reads": rows}

    grown = measure("grown")
    # delete half of all keys, uniformly
    t0 = time.time()
    present = np.concatenate([wl["build_keys"]] + grown_keys)
    del grown_keys
    rng = np.random.default_rng(0xF11C0D)
    gone = present[rng.permutation(present.size)[: present.size // 2]]
    del present
    for i in range(0, gone.size, m):
        st.delete(dev(gone[i:i + m]))
    torch.cuda.synchronize()
    if st.status() != 0:
        raise RuntimeError("device error while deleting")
    log(f"[bench] deleted {gone.size} keys in {time.time() - t0:.1f}s")
    del gone
    after_deletes = st.stats()
    t0 = time.perf_counter()
    before, after = st.restructure()
    rs_ms = (time.perf_counter() - t0) * 1000.0
    restructured = measure("restructured")
    if st.status() != 0 or st.check() != 0:
        raise RuntimeError("device error or invariant violation in the grown-store runs")
    st.close()
    return {"workload": f"2^{args.keys_log2} u32 keys grown by +100% ({nbatches} insert batches of "
                        f"2^{args.batch_log2} new uniform keys), reads; then half of all keys "
                        f"deleted, restructured, reads",
            "grown": grown,
            "after_deletes": {"keys": after_deletes["keys"],
                              "live_nodes": after_deletes["live_nodes"],
                              "buckets": after_deletes["buckets"]},
            "restructure": {"ms": round(rs_ms, 2), "nodes_before": before, "nodes_after": after,
                            "recovered_frac": round((before - after) / before, 4)},
            "restructured": restructured}


def successor_across_gap(args):
    """Successor and range queries that must cross a long run of empty
    buckets: a 2^24-key u32 store (capacity 128, 2^18 buckets) loses a
    rank-contiguous quarter of its keys (65,536 consecutive buckets emptied);
    2^20 successors and 16-key ranges start uniformly inside that gap, so
    every answer lies past it.  The same queries on the intact store are the
    reference.  The occupancy summary makes each crossing a few word reads
    instead of a walk over the empty buckets' headers."""
    import torch
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    m = 1 << 20
    ks = w.KeySpace(32, 0xF11C6000)
    keys = np.sort(ks.build(1 << 24))
    st = flix.Store(key_bits=32, capacity=128, lanes=16, max_batch=m)
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    st.bulk_load(dk, dk)
    lo_i, hi_i = (1 << 23), (1 << 23) + (1 << 22)
    rng = np.random.default_rng(0xF11C6001)
    q = rng.integers(int(keys[lo_i]), int(keys[hi_i - 1]), m, dtype=np.uint64).astype(np.uint32)
    dq = torch.from_numpy(q.view(np.int32)).cuda()
    dhi = torch.from_numpy(np.minimum(q.astype(np.uint64) + 15, 0xFFFFFFFF).astype(np.uint32)
                           .view(np.int32)).cuda()
    ok = torch.empty(m, dtype=torch.int32, device="cuda")
    ov = torch.empty(m, dtype=torch.int32, device="cuda")
    rc = torch.empty(m, dtype=torch.int32, device="cuda")
    rv = torch.empty(m * 16, dtype=torch.int32, device="cuda")
    reps = max(5, args.steps)
    out = {}
    for tag in ("intact", "gap"):
        if tag == "gap":
            gone = keys[lo_i:hi_i].copy()
            rng.shuffle(gone)
            for i in range(0, gone.size, m):
                st.delete(torch.from_numpy(gone[i:i + m].view(np.int32)).cuda())
            torch.cuda.synchronize()
        p50s, _ = timed_calls(lambda: st.successor(dq, out_k=ok, out_v=ov), reps)
        p50r, _ = timed_calls(lambda: st.range(dq, dhi, 16, counts=rc, out_v=rv, want_keys=False),
                              reps)
        out[tag] = {"successor_ms": round(p50s, 4), "range16_ms": round(p50r, 4)}
    if st.status() != 0:
        raise RuntimeError("device error in the gap queries")
    # every successor of the gap queries is the first key after the gap
    got = ok.cpu().numpy().view(np.uint32)
    out["answers_past_gap"] = bool((got == keys[hi_i]).all())
    st.close()
    out["workload"] = ("2^24 u32 keys, 2^22 rank-contiguous keys deleted (65,536 empty buckets), "
                       "2^20 successors and 16-key ranges starting inside the gap")
    log(f"[bench] successor across a gap: {out}")
    return out


def update_heavy_rounds(args):
    """The update-heavy workload: u64 keys and values, bulk load 2^24 keys,
    rounds of 2^20 inserts of new keys then 2^20 deletes of present keys,
    uniform (even rounds) and clustered into 64 runs (odd rounds); every call
    timed with events.  The rounds run twice on fresh stores: as they come,
    and with a restructuring after every clustered insert batch (the paper's
    knob against the long chains the dense runs leave), timed on its own.
    Algorithmic bytes per op follow the byte model of the update kernels."""
    import torch
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    t0 = time.time()
    u = w.UpdateHeavy(n_keys=1 << 24, batch=1 << 20, runs=64)
    build_k = torch.from_numpy(u.build_keys.view(np.int64)).cuda()
    build_v = torch.from_numpy(u.build_vals.view(np.int64)).cuda()
    rounds = []
    for r in range(args.update_rounds):
        ins, iv, dele = u.round(r)
        rounds.append((torch.from_numpy(ins.view(np.int64)).cuda(),
                       torch.from_numpy(iv.view(np.int64)).cuda(),
                       torch.from_numpy(dele.view(np.int64)).cuda()))
    log(f"[bench] update heavy: {len(rounds)} rounds generated ({time.time() - t0:.0f}s)")
    m = 1 << 20

    def run(restructure):
        st = flix.Store(key_bits=64, capacity=128, lanes=16, radix_bits=8, max_batch=m)
        st.bulk_load(build_k, build_v)
        rows = {"uniform": {"insert": [], "delete": []},
                "clustered": {"insert": [], "delete": []}}
        kern = {"uniform": {"insert": [], "delete": []},
                "clustered": {"insert": [], "delete": []}}
        fams_ms = {"uniform": {"insert": [], "delete": []},
                   "clustered": {"insert": [], "delete": []}}
        rs = []
        for r, (di, dv, dd) in enumerate(rounds):
            kind = "uniform" if r % 2 == 0 else "clustered"
            steps = [("insert", lambda: st.insert(di, dv), ("insert_apply", "insert_wide")),
                     ("delete", lambda: st.delete(dd), ("delete_apply", "delete_wide"))]
            fam_all = ("sort_hist", "sort_pass", "sort_local", "slices", "insert_apply",
                       "insert_wide", "delete_apply", "delete_wide")
            for name, fn, fams in steps:
                st.set_timing(True)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record()
                fn()
                b.record()
                torch.cuda.synchronize()
                kms = sum(st.kernel_time(f)[0] for f in fams)
                per_fam = {f: st.kernel_time(f)[0] for f in fam_all}
                st.set_timing(False)
                rows[kind][name].append(a.elapsed_time(b))
                kern[kind][name].append(kms)
                fams_ms[kind][name].append(per_fam)
                if restructure and kind == "clustered" and name == "insert":
                    # the dense runs became long chains: flatten them before
                    # the deletes and the next rounds walk them
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    before, after = st.restructure()
                    rs.append(((time.perf_counter() - t1) * 1e3, before, after))
            if st.status() != 0:
                raise RuntimeError(f"device error in update round {r}")
        stt = st.stats()
        st.close()
        res = {"final": stt}
        for kind in rows:
            d = {}
            for name in ("insert", "delete"):
                ms = np.array(rows[kind][name])
                if ms.size == 0:
                    continue
                d[name] = {"Mops_s_median": round(m / (np.median(ms) / 1000) / 1e6, 1),
                           "ms_median": round(float(np.median(ms)), 4),
                           "ms_max": round(float(ms.max()), 4), "rounds": int(ms.size),
                           "ms_per_round": [round(float(x), 3) for x in ms],
                           "apply_kernels_ms_median": round(float(np.median(kern[kind][name])), 4),
                           "kernel_ms_median": {f: round(float(np.median([p[f] for p in fams_ms[kind][name]])), 4)
                                                for f in fams_ms[kind][name][0]
                                                if any(p[f] for p in fams_ms[kind][name])}}
            if d:
                res[kind] = d
        if rs:
            a = np.array(rs)
            res["restructure"] = {"count": len(rs), "ms_median": round(float(np.median(a[:, 0])), 2),
                                  "nodes_recovered_frac_median":
                                      round(float(np.median((a[:, 1] - a[:, 2]) / a[:, 1])), 4)}
        return res

    plain = run(False)
    with_rs = run(True)
    # algorithmic bytes per op (u64 keys and values, capacity 128, bulk fill 64)
    sort_b = 8 + (8 + 16) + 7 * 2 * 16      # histogram read, top-digit pass, local passes
    ins_b = sort_b + 8 + 12 + 3 + 0.98 * (64 + 68) * 16 / 4
    del_b = sort_b - 7 * 2 * 8 + 8 + 3 + 0.98 * (64 + 68) * 16 / 4
    for res in (plain, with_rs):
        if "uniform" in res and "insert" in res["uniform"]:
            for name, b_ in (("insert", ins_b), ("delete", del_b)):
                res["uniform"][name]["frac_whole_call"] = round(
                    b_ * m / (res["uniform"][name]["ms_median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    out = {"workload": f"u64 store, bulk load 2^24 keys, {args.update_rounds} rounds of 2^20 "
                       f"inserts then 2^20 deletes, even rounds uniform, odd rounds clustered "
                       f"into 64 runs",
           "alg_bytes_per_op_model_uniform": {"insert": ins_b, "delete": del_b},
           "rounds_as_they_come": plain,
           "restructure_after_clustered_inserts": with_rs}
    log(f"[bench] update heavy ({time.time() - t0:.0f}s): {out}")
    return out


def insert_kernel_choice(args):
    """Insert throughput of each insert kernel (TL-Bulk, ST-Shift-Right,
    ST-TL-Mixed, adaptive) at light and heavy loads per bucket: one 2^20-key
    batch of new uniform u32 keys into stores of 2^22 keys at capacity 8
    (about one key per touched bucket) and 2^24 keys at capacity 128 (about
    four keys per bucket).  Each batch is deleted again between samples."""
    import torch
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w
    m = 1 << 20
    res = {}
    for keys_log2, cap in ((22, 8), (24, 128)):
        ks = w.KeySpace(32, 0xF11C7000 + cap)
        bk = ks.build(1 << keys_log2)
        ins = ks.fresh(m)
        dbk = torch.from_numpy(bk.view(np.int32)).cuda()
        di = torch.from_numpy(ins.view(np.int32)).cuda()
        row = {}
        for algo in ("tl_bulk", "st_shift_right", "st_tl_mixed", "adaptive"):
            st = flix.Store(key_bits=32, capacity=cap, lanes=16 if cap >= 16 else 16,
                            max_batch=m, insert_algo=algo)
            st.bulk_load(dbk, dbk)

            def one():
                st.insert(di, di)
                st.delete(di)
            times = []
            for _ in range(max(5, args.steps // 2)):
                st.delete(di)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                st.insert(di, di)
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b))
            if st.status() != 0:
                raise RuntimeError(f"device error in the {algo} insert runs")
            ms = float(np.median(times[1:]))
            row[algo] = {"Mops_s": round(m / (ms / 1000) / 1e6, 1), "ms": round(ms, 4)}
            st.close()
        res[f"2^{keys_log2} keys, capacity {cap}"] = row
        log(f"[bench] insert kernels at 2^{keys_log2} keys, capacity {cap}: {row}")
    return res


def batching_compare(args):
    """The mixed-batch stream on a 2^keys_log2 u32 store: one ABI call per
    batch versus the persistent drain replayed from a hipGraph.  Both start
    from the same bulk load; their outputs and final contents must agree."""
    import torch
    from paper_2604_16725_amd import autotune, flix
    from paper_2604_16725_amd.batching import (DeviceStream, PersistentRun, pool_bytes_for,
                                               run_plain, summarize)
    from paper_2604_16725_amd.workloads import BatchStream

    cfg = autotune.tuned_config(form="persistent")
    cfg_plain = autotune.tuned_config(form="plain")
    t0 = time.time()
    stream = BatchStream(n_keys=1 << args.keys_log2, nbatch=args.nbatch)
    ds = DeviceStream(stream)
    log(f"[bench] mixed stream: {ds.n} batches, {ds.total_ops} ops resident "
        f"({time.time() - t0:.1f}s)")
    cs = torch.cuda.Stream()
    res = {}
    with torch.cuda.stream(cs):
        # each form runs on the layout its own sweep picked
        st = flix.Store(key_bits=32, capacity=cfg_plain["capacity"], lanes=cfg_plain["lanes"],
                        radix_bits=cfg_plain["radix_bits"], max_batch=1 << 20,
                        pool_bytes=pool_bytes_for(stream, cfg_plain["capacity"]))
        outs_p, outs_g = ds.outputs(), ds.outputs()
        plain = None
        for rep in range(2):
            st.bulk_load(ds.build_keys, ds.build_vals)
            wall, svc = run_plain(st, ds, outs_p, events=(rep == 0))
            if rep == 0:
                plain = summarize(wall, svc, ds.total_ops)
                svc_plain = svc
            else:
                plain["Mops_s"] = round(ds.total_ops / wall / 1e6, 1)
                plain["wall_ms"] = round(wall * 1e3, 3)
        if st.status() != 0:
            raise RuntimeError("device error in the plain stream")
        dump_p = st.dump()
        log(f"[bench] plain: {plain}")
        st.close()
        st = flix.Store(key_bits=32, capacity=cfg["capacity"], lanes=cfg["lanes"],
                        radix_bits=cfg["radix_bits"], max_batch=1 << 20,
                        pool_bytes=pool_bytes_for(stream, cfg["capacity"]))
        run = PersistentRun(st, ds, outs_g, cs)
        pers = None
        for rep in range(2):
            st.bulk_load(ds.build_keys, ds.build_vals)
            wall, svc = run.run()
            cur = summarize(wall, svc, ds.total_ops)
            if pers is None or cur["Mops_s"] > pers["Mops_s"]:
                pers = cur
                svc_pers = svc
        if st.status() != 0:
            raise RuntimeError("device error in the persistent stream")
        dump_g = st.dump()
        log(f"[bench] persistent: {pers}")
        same = (torch.equal(outs_p[0], outs_g[0]) and torch.equal(outs_p[1], outs_g[1])
                and torch.equal(dump_p[0], dump_g[0]) and torch.equal(dump_p[1], dump_g[1]))
        # mean service time per batch-size band (both forms, same batches)
        bands = {}
        lg = np.log2(ds.sizes)
        for lo_, hi_ in ((8, 11), (11, 14), (14, 17), (17, 20.01)):
            m_ = (lg >= lo_) & (lg < hi_)
            if m_.any():
                bands[f"2^{lo_}..2^{int(hi_)}"] = {
                    "batches": int(m_.sum()),
                    "plain_mean_us": round(float(svc_plain[m_].mean()) * 1e6, 1),
                    "persistent_mean_us": round(float(svc_pers[m_].mean()) * 1e6, 1)}
        res = {"workload": f"{ds.n} mixed batches, sizes floor(2^U) U~U[8,20], 70/10/10/10 "
                           f"lookup/successor/insert/delete, 2^{args.keys_log2} u32 keys",
               "ops": ds.total_ops, "store_plain": cfg_plain, "store_persistent": cfg,
               "drain_workgroups": st.drain_info()[0],
               "plain": plain, "persistent_graph": pers,
               "speedup_Mops": round(pers["Mops_s"] / plain["Mops_s"], 3),
               "p99_ratio_plain_over_persistent": round(plain["p99_us"] / pers["p99_us"], 3),
               "service_by_size": bands,
               "results_identical": bool(same)}
        run.close()
        st.close()
    if not res["results_identical"]:
        raise RuntimeError("persistent and plain results differ")
    return res


def serving_compare(args):
    """Open-loop Poisson arrivals on a 2^serve_keys_log2 u64 store: the
    coalescing request loop (two pipelined epoch slots) against the plain
    form (every request its own epoch, one at a time), at 0.2..0.95 of the
    plain form's saturation rate (measured first with all requests queued
    at time 0), and at 1.5 and 3 times it, beyond what the plain form can
    serve.  The serving form's own saturation is measured the same way.
    Each run starts from the same bulk load."""
    import torch
    from paper_2604_16725_amd import flix, serve
    from paper_2604_16725_amd.workloads import ServingWorkload

    t0 = time.time()
    wl = ServingWorkload(n_keys=1 << args.serve_keys_log2, n_req=args.serve_requests)
    log(f"[bench] serving workload: {wl.n_req} requests, {wl.total_ops} ops "
        f"({time.time() - t0:.1f}s)")
    E = 1 << 16
    budget = 64 << 30
    tomb = (1 << 64) - 1
    st = flix.Store(key_bits=64, capacity=128, lanes=16, radix_bits=8, max_batch=E)
    bk = torch.from_numpy(wl.build_keys.view(np.int64)).cuda()
    bv = torch.from_numpy(wl.build_vals.view(np.int64)).cuda()
    be = serve.GpuBackend(st, E, wl.range_max)

    def one(rate, coalesce):
        st.bulk_load(bk, bv)
        torch.cuda.synchronize()
        arr = np.zeros(wl.n_req) if rate is None else wl.arrivals(rate)
        run = serve.Engine(be, E, budget, coalesce=coalesce).run(wl, arr, tomb, 8, wl.range_max)
        if st.status() != 0:
            raise RuntimeError("device error in the serving runs")
        return run

    one(None, False)                               # warm-up (slot scratch, kernels)
    sat = one(None, False)
    sat_rate = sat["completed"] / sat["span_s"]
    log(f"[bench] plain form saturation: {sat_rate:.0f} requests/s")
    sat_s = one(None, True)
    sat_rate_s = sat_s["completed"] / sat_s["span_s"]
    log(f"[bench] serving form saturation: {sat_rate_s:.0f} requests/s")
    rows = []
    for frac in (0.2, 0.4, 0.6, 0.8, 0.95, 1.5, 3.0):
        rate = frac * sat_rate
        row = {"load": frac, "rate_req_s": round(rate, 1)}
        for name, coalesce in (("plain", False), ("serving", True)):
            row[name] = serve.summary(one(rate, coalesce), wl)
        log(f"[bench] load {frac}: plain {row['plain']}, serving {row['serving']}")
        rows.append(row)
    st.close()
    return {"workload": f"{wl.n_req} requests per rate, 1..4096 ops each (log-uniform), "
                        f"80/5/7.5/7.5 lookup/range/insert/delete, ranges of 8..64 keys, "
                        f"2^{args.serve_keys_log2} u64 keys, Poisson arrivals",
            "epoch_capacity_ops": E, "budget_bytes": budget,
            "plain_saturation_req_s": round(sat_rate, 1),
            "plain_saturation_Mops_s": round(sat["ops"] / sat["span_s"] / 1e6, 3),
            "serving_saturation_req_s": round(sat_rate_s, 1),
            "serving_saturation_Mops_s": round(sat_s["ops"] / sat_s["span_s"] / 1e6, 3),
            "rates": rows}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the store would shard by key range). Run with --gpus 1.",
              file=sys.stderr, flush=True)
        sys.exit(2)
    ensure_built()
    import torch
    from paper_2604_16725_amd import flix
    from paper_2604_16725_amd import workloads as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration: 4 device copies of {args.calibrate_copy} MiB")
        del src, dst
    n_keys, m = 1 << args.keys_log2, 1 << args.batch_log2
    t0 = time.time()
    wl = w.read_path(n_keys=n_keys, batch=m, with_zipf=not args.no_breakdown, with_updates=True)
    log(f"[bench] workload generated in {time.time() - t0:.1f}s")

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()

    st = flix.Store(key_bits=32, capacity=args.capacity, lanes=args.lanes,
                    radix_bits=args.radix_bits, max_batch=m, read_path=args.read_path)
    bk, bv = dev(wl["build_keys"]), dev(wl["build_vals"])
    t0 = time.time()
    st.bulk_load(bk, bv)
    log(f"[bench] bulk load of {n_keys} keys in {time.time() - t0:.2f}s")
    del bk, bv
    stats = st.stats()
    dl, ds = dev(wl["lookup"]), dev(wl["successor"])
    dlo, dhi = dev(wl["range_lo"]), dev(wl["range_hi"])
    di, dv = dev(wl["insert_keys"]), dev(wl["insert_vals"])
    ol = torch.empty(m, dtype=torch.int32, device="cuda")
    sk = torch.empty(m, dtype=torch.int32, device="cuda")
    sv = torch.empty(m, dtype=torch.int32, device="cuda")
    L = wl["range_len"]
    rc = torch.empty(m, dtype=torch.int32, device="cuda")
    rk = torch.empty(m * L, dtype=torch.int32, device="cuda")
    rv = torch.empty(m * L, dtype=torch.int32, device="cuda")

    def step():
        st.lookup(dl, out=ol)
        st.successor(ds, out_k=sk, out_v=sv)
        st.range(dlo, dhi, L, counts=rc, out_k=rk, out_v=rv)
        st.insert(di, dv)
        st.delete(di)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if st.status() != 0:
        raise RuntimeError("device error during warmup")
    log("[bench] warmup done")

    fams = ["sort_hist", "sort_pass", "sort_local", "read_cuts", "read_apply", "part",
            "group_read", "slices", "insert_apply", "delete_apply", "insert_st", "insert_wide",
            "delete_wide"]

    def run_steps(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1000.0 / k

    # -- per-family breakdown (untimed for `value`): every family's launches
    #    carry HIP events; picks the dominant family
    st.set_timing(True)
    ms_step_all = run_steps(args.steps)
    fam_all = {f: st.kernel_time(f) for f in fams}
    st.set_timing(False)
    dom_fam = max((f for f in fams if fam_all[f][1]), key=lambda f: fam_all[f][0])

    # -- timed region: exactly K steps; only the dominant family's launches
    #    carry HIP events (stamped by the dispatches on the library's stream)
    st.set_timing(True, only=dom_fam)
    ms_step = run_steps(args.steps)
    dom_t = st.kernel_time(dom_fam)
    st.set_timing(False)
    ops_step = 5 * m
    value = ops_step / (ms_step / 1000.0) / 1e6
    log(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step, {value:.1f} Mops/s "
        f"(events on {dom_fam}; {ms_step_all:.3f} ms/step with events on every family)")
    if st.status() != 0:
        raise RuntimeError("device error during timed steps")

    # same K steps without any events (overhead check)
    ms_step_noev = run_steps(args.steps)

    # -- roofline of the dominant kernel ------------------------------------
    build_sorted = np.sort(wl["build_keys"])
    wl["_build_sorted"] = build_sorted
    f = st.cfg.fill or args.capacity // 2
    nb = stats["buckets"]
    mkba = build_sorted[f - 1::f].copy()
    if mkba.size < nb:
        mkba = np.append(mkba, np.uint32(0xFFFFFFFF))
    mkba[-1] = np.uint32(0xFFFFFFFF)
    assert mkba.size == nb, (mkba.size, nb)
    sizes = np.full(nb, f, dtype=np.int64)
    sizes[-1] = n_keys - f * (nb - 1)
    model = byte_model(wl, mkba, sizes, rb=args.radix_bits, read_path=args.read_path)
    per_fam = {}
    for fam, (ms, n) in fam_all.items():
        if n == 0:
            continue
        bytes_step = model.get(fam, 0.0)
        per_fam[fam] = {
            "ms_per_step": ms / args.steps,
            "launches_per_step": n / args.steps,
            "avg_launch_us": 1000.0 * ms / n,
            "alg_GBps": bytes_step / (ms / args.steps / 1000.0) / 1e9,
        }
    dom = dom_fam
    dom_ms, dom_n = dom_t
    dom_us = 1000.0 * dom_ms / dom_n
    ach = model.get(dom, 0.0) / per_fam[dom]["launches_per_step"] / (dom_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dom),
                "alg_bytes_per_launch": model[dom] / per_fam[dom]["launches_per_step"],
                "traffic_unit": "HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE)",
                "avg_launch_us": round(dom_us, 2)}

    # -- per-operation breakdown (each call timed alone with events) --------
    breakdown = {}
    if not args.no_breakdown:
        reps = max(5, args.steps)

        def timeit(name, fn, nops):
            fn()   # one untimed call: first-use costs stay out of the samples
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(reps)]
            # no collector pause between an event and the launches it brackets
            gc.disable()
            try:
                for a, b in evs:
                    a.record()
                    fn()
                    b.record()
            finally:
                gc.enable()
            torch.cuda.synchronize()
            ms = np.array([a.elapsed_time(b) for a, b in evs])
            breakdown[name] = {"Mops_s": round(nops / (np.median(ms) / 1000) / 1e6, 1),
                               "p50_ms": round(float(np.percentile(ms, 50)), 4),
                               "p99_ms": round(float(np.percentile(ms, 99)), 4)}

        timeit("lookup", lambda: st.lookup(dl, out=ol), m)
        timeit("successor", lambda: st.successor(ds, out_k=sk, out_v=sv), m)
        timeit("range16", lambda: st.range(dlo, dhi, L, counts=rc, out_k=rk, out_v=rv), m)

        def ins_then_del():
            st.insert(di, dv)
            st.delete(di)
        timeit("insert+delete", ins_then_del, 2 * m)
        zl, zs = dev(wl["zipf_lookup"]), dev(wl["zipf_successor"])
        zlo, zhi = dev(wl["zipf_range_lo"]), dev(wl["zipf_range_hi"])
        timeit("zipf_lookup", lambda: st.lookup(zl, out=ol), m)
        timeit("zipf_successor", lambda: st.successor(zs, out_k=sk, out_v=sv), m)
        timeit("zipf_range16", lambda: st.range(zlo, zhi, L, counts=rc, out_k=rk, out_v=rv), m)
        # dense ranges (an extra beside the workload's 16-key intervals, which
        # hold 0.25 keys on average): 2^16 ranges of 2^16 consecutive key
        # values, about 1024 stored keys each, all returned
        nd, Ld = 1 << 16, 1024
        dlo_np = np.random.default_rng(0xF11CD).integers(0, (1 << 32) - (1 << 16), nd,
                                                           dtype=np.uint64)
        ddlo = dev(dlo_np.astype(np.uint32))
        ddhi = dev((dlo_np + (1 << 16) - 1).astype(np.uint32))
        drc = torch.empty(nd, dtype=torch.int32, device="cuda")
        drk = torch.empty(nd * Ld, dtype=torch.int32, device="cuda")
        drv = torch.empty(nd * Ld, dtype=torch.int32, device="cuda")
        timeit("range_dense_1024", lambda: st.range(ddlo, ddhi, Ld, counts=drc, out_k=drk,
                                                    out_v=drv), nd)
        res_n = int(drc.to(torch.int64).sum().item())
        breakdown["range_dense_1024"]["results_per_range"] = round(res_n / nd, 1)
        breakdown["range_dense_1024"]["Mresults_s"] = round(
            res_n / (breakdown["range_dense_1024"]["p50_ms"] / 1000) / 1e6, 1)
        del drk, drv
        if st.status() != 0:
            raise RuntimeError("device error during breakdown")

    st.close()
    del st
    def leg(name, fn, *a):
        # a secondary measurement that fails is reported in the JSON line
        # instead of taking the headline number with it
        try:
            return fn(*a)
        except Exception as e:  # noqa: BLE001
            import traceback
            traceback.print_exc()
            log(f"[bench] {name} failed: {e!r}")
            return {"error": repr(e)}

    grown = None
    if not args.no_grown:
        bufs = {"lookup": dl, "successor": ds, "range_lo": dlo, "range_hi": dhi, "ol": ol,
                "sk": sk, "sv": sv, "rc": rc, "rk": rk, "rv": rv, "L": L}
        grown = leg("grown_store", grown_store_reads, args, wl, dev, bufs)
    gap = None if args.no_breakdown else leg("successor_gap", successor_across_gap, args)
    update_heavy = leg("update_heavy", update_heavy_rounds, args) if args.update_rounds > 0 else None
    insert_kernels = None if args.no_insert_kernels else leg("insert_kernels", insert_kernel_choice,
                                                               args)
    batching = None if args.no_batching else leg("batching", batching_compare, args)
    serving = None if args.no_serving else leg("serving", serving_compare, args)

    # -- CPU baseline: the oracle on a bounded sample -----------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle
        # the oracle is single-threaded; pin this process to one core for it
        nproc = os.cpu_count()
        model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        saved_aff = os.sched_getaffinity(0)
        core = min(saved_aff)
        os.sched_setaffinity(0, {core})
        o = Oracle(32)
        t0 = time.time()
        o.bulk_load(wl["build_keys"], wl["build_vals"])
        log(f"[bench] oracle bulk load {time.time() - t0:.1f}s (untimed)")
        t0 = time.perf_counter()
        o.lookup(wl["lookup"])
        o.successor(wl["successor"])
        o.range(wl["range_lo"], wl["range_hi"], L)
        o.insert(wl["insert_keys"], wl["insert_vals"])
        o.delete(wl["insert_keys"])
        cpu_s = time.perf_counter() - t0
        os.sched_setaffinity(0, saved_aff)
        cpu = {"value": round(ops_step / cpu_s / 1e6, 3), "unit": "Mops/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one step (lookup, successor, range16, insert, delete of {m} ops each) "
                         f"on the bulk-loaded {n_keys}-key store, single thread pinned to core "
                         f"{core}, {cpu_s:.2f}s",
               "host_nproc": nproc, "host_cpu": model}
        log(f"[bench] oracle step {cpu_s:.2f}s")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "flix read-path store, 2^26 uniform u32 keys, capacity 128, "
                               "step = lookup+successor+range16+insert+delete of 2^20 ops each",
                   "keys": n_keys, "batch": m, "capacity": args.capacity, "lanes": args.lanes,
                   "radix_bits": args.radix_bits, "read_path": args.read_path,
                   "ops_per_step": ops_step,
                   "global_batch": m, "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ms_per_step_without_kernel_events": round(ms_step_noev, 4),
        "ms_per_step_events_on_every_family": round(ms_step_all, 4),
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in per_fam.items()},
        "breakdown": breakdown,
        "grown_store": grown,
        "successor_across_gap": gap,
        "update_heavy": update_heavy,
        "insert_kernels": insert_kernels,
        "batching": batching,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
