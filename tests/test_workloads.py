"""Host-side checks of the seeded workload generators (no GPU)."""
import numpy as np

from paper_2604_16725_amd import workloads as w


def test_perm32_is_bijective_on_a_block():
    c = np.arange(0, 1 << 20, dtype=np.uint64)
    k = w.perm32(c, 7)
    assert np.unique(k).size == k.size
    # disjoint counter ranges give disjoint keys
    k2 = w.perm32(c + np.uint64(1 << 31), 7)
    assert np.intersect1d(k, k2).size == 0


def test_perm32_full_domain_small_seed_is_permutation_of_high_half_sample():
    # A Feistel network is a bijection on the whole 32-bit domain; check the
    # 2^24 smallest counters map to distinct keys.
    c = np.arange(0, 1 << 24, dtype=np.uint64)
    assert np.unique(w.perm32(c, 3)).size == c.size


def test_perm64_distinct_and_deterministic():
    c = np.arange(0, 1 << 20, dtype=np.uint64)
    a = w.perm64(c, 11)
    assert np.unique(a).size == a.size
    assert np.array_equal(a, w.perm64(c, 11))
    assert not np.array_equal(a, w.perm64(c, 12))


def test_values_never_reserved():
    k = np.arange(0, 1 << 16, dtype=np.uint64)
    assert not np.any(w.values_for(k.astype(np.uint32), 5, 32) == np.uint32(0xFFFFFFFF))
    assert not np.any(w.values_for(k, 5, 64) == np.uint64(0xFFFFFFFFFFFFFFFF))


def test_tiny_plain_shapes_and_semantics():
    t = w.tiny_plain()
    assert t["build_keys"].size == 1 << 16
    assert np.unique(t["build_keys"]).size == 1 << 16
    kinds = [b[0] for b in t["batches"]]
    assert kinds == ["insert", "lookup", "delete", "successor"]
    ins = t["batches"][0][1]
    assert np.intersect1d(ins, t["build_keys"]).size == 0
    look = t["batches"][1][1]
    present = np.concatenate([t["build_keys"], ins])
    assert np.isin(look, present).sum() == 1 << 13
    dele = t["batches"][2][1]
    assert np.unique(dele).size == dele.size and np.all(np.isin(dele, present))


def test_read_path_small():
    r = w.read_path(n_keys=1 << 14, batch=1 << 12)
    hit = np.isin(r["lookup"], r["build_keys"]).sum()
    assert hit == (9 * (1 << 12)) // 10
    assert np.all(r["range_hi"].astype(np.int64) - r["range_lo"].astype(np.int64) <= 15)
    assert np.all(np.isin(r["zipf_successor"], r["build_keys"]))


def test_zipf_rank_frequencies():
    rng = np.random.default_rng(0)
    r = w.zipf_ranks(1 << 16, 1 << 18, 0.99, rng)
    h = np.bincount(r, minlength=4)
    # P(1)/P(2) = 2^0.99
    assert abs(h[0] / h[1] - 2 ** 0.99) < 0.1


def test_update_heavy_rounds_small():
    u = w.UpdateHeavy(n_keys=1 << 14, batch=1 << 12, runs=8)
    before = set(u.present.tolist())
    ins, v, dele = u.round(1)
    assert np.unique(ins).size == ins.size
    assert not (set(ins.tolist()) & before)
    s = np.sort(ins)
    assert np.sum(np.diff(s) == 1) >= ins.size - 8  # 8 runs of consecutive keys
    assert np.unique(dele).size == dele.size


def test_batch_stream_small():
    s = w.BatchStream(n_keys=1 << 14, nbatch=400, log2_max=12.0)
    assert s.sizes.min() >= 256 and s.sizes.max() <= 1 << 12
    frac = np.bincount(s.ops, minlength=4) / s.nbatch
    assert abs(frac[0] - 0.7) < 0.08 and all(abs(f - 0.1) < 0.05 for f in frac[1:])
    build = set(s.build_keys.tolist())
    seen_new = set()
    for i in range(s.nbatch):
        op, k, v = s.batch(i)
        assert k.dtype == np.uint32 and k.size == s.sizes[i]
        op2, k2, v2 = s.batch(i)          # each batch regenerates alone, identically
        assert op2 == op and np.array_equal(k, k2)
        if op == "insert":
            ks = set(k.tolist())
            assert len(ks) == k.size and not (ks & build) and not (ks & seen_new)
            seen_new |= ks
            assert np.all(v != np.uint32(0xFFFFFFFF))
        elif op == "lookup":
            hits = np.isin(k, s.build_keys).sum()
            assert hits == (k.size * 9) // 10
        elif op == "delete":
            assert np.all(np.isin(k, s.build_keys))


def test_tuned_config_fallback(tmp_path):
    from paper_2604_16725_amd import autotune
    assert autotune.tuned_config(str(tmp_path / "missing.json")) == autotune.FALLBACK
    p = tmp_path / "t.json"
    p.write_text('{"best": {"capacity": 64, "lanes": 32, "radix_bits": 4, "Mops_s": 1.0}}')
    assert autotune.tuned_config(str(p)) == {"capacity": 64, "lanes": 32, "radix_bits": 4}
