"""The allocation-free dump (flix_dump_noalloc) through the C ABI against
flix_dump, bit-exact, on two calls in a row: a large store, then a smaller
one (the shared scratch keeps the first call's contents), plus the bucket
limit and the capacity error."""
import numpy as np
import pytest

from gpu_helpers import ktype, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _store_with(kb, n, seed, cap=32):
    from paper_2604_16725_amd.flix import Store
    rng = np.random.default_rng(seed)
    k = rng.integers(0, (1 << kb) - 1, n, dtype=np.uint64, endpoint=True).astype(ktype(kb))
    s = Store(key_bits=kb, capacity=cap, max_batch=1 << 16)
    s.bulk_load(to_dev(k), to_dev(k ^ ktype(kb)(0x33)))
    # grow a few chains so the dump walks more than one node per bucket
    ins = rng.integers(0, (1 << kb) - 1, 1 << 15, dtype=np.uint64).astype(ktype(kb))
    s.insert(to_dev(ins), to_dev(ins))
    return s


def _both(s, kb):
    import torch
    n = s.size()
    dt = torch.int32 if kb == 32 else torch.int64
    a_k = torch.empty(n, dtype=dt, device="cuda")
    a_v = torch.empty(n, dtype=dt, device="cuda")
    b_k = torch.full((n,), -1, dtype=dt, device="cuda")
    b_v = torch.full((n,), -1, dtype=dt, device="cuda")
    na = s.dump_into(a_k, a_v)
    nb = s.dump_into(b_k, b_v, noalloc=True)
    assert na == nb == n
    for x, y, what in ((a_k, b_k, "keys"), (a_v, b_v, "values")):
        x, y = to_host(x, kb), to_host(y, kb)
        bad = np.nonzero(x != y)[0]
        assert bad.size == 0, f"{what} differ at {bad[:5]}"
    return n


@pytest.mark.parametrize("kb", [32, 64])
def test_noalloc_dump_matches_dump_twice(kb):
    big = _store_with(kb, 1 << 21, 1 + kb)
    n1 = _both(big, kb)
    small = _store_with(kb, 5000, 2 + kb, cap=8)
    n2 = _both(small, kb)
    log(f"kb={kb}: {n1} then {n2} pairs, identical")
    assert n2 < n1
    # capacity too small: error, like flix_dump
    import torch
    from paper_2604_16725_amd.flix import FlixError
    dt = torch.int32 if kb == 32 else torch.int64
    with pytest.raises(FlixError):
        small.dump_into(torch.empty(10, dtype=dt, device="cuda"),
                        torch.empty(10, dtype=dt, device="cuda"), noalloc=True)
    big.close()
    small.close()


def test_noalloc_dump_rejects_stores_beyond_its_scratch():
    import torch
    from paper_2604_16725_amd.flix import FLIX_EINVAL, FlixError, Store
    n = (1 << 21) * 4 + 4
    k = torch.arange(n, dtype=torch.int64, device="cuda").to(torch.int32)
    s = Store(key_bits=32, capacity=8, max_batch=1 << 10)
    s.bulk_load(k, k)
    assert s.stats()["buckets"] > (1 << 21)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    out2 = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(FlixError) as e:
        s.dump_into(out, out2, noalloc=True)
    assert e.value.code == FLIX_EINVAL
    assert s.dump_into(out, out2) == n
    s.close()
