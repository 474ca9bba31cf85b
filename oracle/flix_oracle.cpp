// FliX batch-semantics oracle: a plain, slow, single-threaded CPU reference.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
// call this file: only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code, header, table or helper
// with the HIP library.
//
// What it computes.  FliX (arXiv 2604.16725) is a GPU-resident ordered map
// (Section 2.1 lists the ordered-map operations: search, insert, delete,
// range, successor/predecessor).  Every FliX batch operation reaches exactly
// the result of applying the batch to a sequential ordered map; the buckets,
// node chains and the sorted batch are only how the GPU gets there.  So the
// oracle is that definition written out over the simplest ordered map there
// is: two parallel arrays (keys strictly increasing, values beside them).
//
// Readings of the paper that this file fixes (the paper is silent on them):
//  * NOT_FOUND is the all-ones value of the value width (Section 3.3 names a
//    miss result but gives it no encoding).  Inserting it is rejected
//    (return -1) and the store is left unchanged.  KEY_MAX is the all-ones key; every key, 0 and KEY_MAX
//    included, is a legal key.
//  * Duplicate keys inside one insert batch: the last occurrence in input order
//    wins (sequential semantics).  Duplicates in a delete batch are harmless.
//    Read batches answer every occurrence.
//  * Successor is the smallest stored key that is >= q (Section 6.5).  A miss
//    returns (KEY_MAX, NOT_FOUND).
//  * Predecessor, the mirror operation that Section 2.1 lists beside it, is the
//    largest stored key that is <= q.  A miss returns (0, NOT_FOUND): 0 is the
//    smallest key, and the reserved value tells the miss apart from a stored 0.
//  * Range [lo, hi] is closed; lo > hi yields count 0.  The first
//    min(count, max_per_query) pairs are written in ascending key order.
//
// Parity pins for every function live in tests/test_oracle_pins.py (brute
// force against a Python dict replayed op by op, the paper's worked examples
// in Tables 2 and 3, closed-form special cases, planted mistakes).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

template <typename K>
struct Store {
  // S: keys strictly increasing; vals[i] belongs to keys[i].
  std::vector<K> keys;
  std::vector<K> vals;

  static constexpr K kNotFound = ~K(0);
  static constexpr K kKeyMax = ~K(0);

  // Batch insert (Section 3.2: an absent key is added to its node; an
  // existing key takes the new value).  Sequential meaning: for
  // i = 0..n-1 in input order, S[k_i] <- v_i.  Written as: stable sort of the
  // batch by key, keep the last pair of each equal-key run, then one linear
  // merge with S in which the batch pair wins on equal keys.
  int insert(const K* k, const K* v, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i)
      if (v[i] == kNotFound) return -1;  // reserved value: reject whole batch
    std::vector<uint64_t> order(n);
    for (uint64_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint64_t a, uint64_t b) { return k[a] < k[b]; });
    std::vector<K> bk, bv;  // deduplicated batch, last occurrence wins
    for (uint64_t j = 0; j < n; ++j) {
      uint64_t i = order[j];
      bool last_of_run = (j + 1 == n) || (k[order[j + 1]] != k[i]);
      if (last_of_run) {
        bk.push_back(k[i]);
        bv.push_back(v[i]);
      }
    }
    std::vector<K> nk, nv;
    nk.reserve(keys.size() + bk.size());
    nv.reserve(keys.size() + bk.size());
    size_t a = 0, b = 0;
    while (a < keys.size() || b < bk.size()) {
      if (b == bk.size() || (a < keys.size() && keys[a] < bk[b])) {
        nk.push_back(keys[a]);
        nv.push_back(vals[a]);
        ++a;
      } else if (a == keys.size() || bk[b] < keys[a]) {
        nk.push_back(bk[b]);
        nv.push_back(bv[b]);
        ++b;
      } else {  // equal keys: the batch value replaces the stored one
        nk.push_back(bk[b]);
        nv.push_back(bv[b]);
        ++a;
        ++b;
      }
    }
    keys.swap(nk);
    vals.swap(nv);
    return 0;
  }

  // Initial build (Section 3.2): the store is made from the given pairs only.
  // Its contents equal an empty store followed by one insert batch.
  int bulk_load(const K* k, const K* v, uint64_t n) {
    Store<K> fresh;
    if (fresh.insert(k, v, n) != 0) return -1;
    keys.swap(fresh.keys);
    vals.swap(fresh.vals);
    return 0;
  }

  // Batch delete (Section 3.2 and 4.4): keys are physically removed; a key
  // that is not present is a no-op.  Written as a set difference S \ K.
  void erase(const K* k, uint64_t n) {
    std::vector<K> del(k, k + n);
    std::sort(del.begin(), del.end());
    del.erase(std::unique(del.begin(), del.end()), del.end());
    std::vector<K> nk, nv;
    nk.reserve(keys.size());
    nv.reserve(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
      if (!std::binary_search(del.begin(), del.end(), keys[i])) {
        nk.push_back(keys[i]);
        nv.push_back(vals[i]);
      }
    }
    keys.swap(nk);
    vals.swap(nv);
  }

  // Point query (Section 3.3): the stored value, or NOT_FOUND on a miss.
  void lookup(const K* q, uint64_t n, K* out) const {
    for (uint64_t i = 0; i < n; ++i) {
      auto it = std::lower_bound(keys.begin(), keys.end(), q[i]);
      out[i] = (it != keys.end() && *it == q[i]) ? vals[it - keys.begin()]
                                                  : kNotFound;
    }
  }

  // Successor (Section 6.5): smallest stored key k' >= q.
  void successor(const K* q, uint64_t n, K* kout, K* vout) const {
    for (uint64_t i = 0; i < n; ++i) {
      auto it = std::lower_bound(keys.begin(), keys.end(), q[i]);
      if (it == keys.end()) {
        kout[i] = kKeyMax;
        vout[i] = kNotFound;
      } else {
        kout[i] = *it;
        vout[i] = vals[it - keys.begin()];
      }
    }
  }

  // Predecessor (Section 2.1): largest stored key k' <= q.  upper_bound gives
  // the first key > q; the entry before it, if any, is the answer.
  void predecessor(const K* q, uint64_t n, K* kout, K* vout) const {
    for (uint64_t i = 0; i < n; ++i) {
      auto it = std::upper_bound(keys.begin(), keys.end(), q[i]);
      if (it == keys.begin()) {
        kout[i] = K(0);
        vout[i] = kNotFound;
      } else {
        --it;
        kout[i] = *it;
        vout[i] = vals[it - keys.begin()];
      }
    }
  }

  // Range (Section 2.1): all pairs with lo <= k <= hi, ascending.
  void range(const K* lo, const K* hi, uint64_t n, uint32_t maxpq,
             uint32_t* counts, K* kout, K* vout) const {
    for (uint64_t i = 0; i < n; ++i) {
      if (lo[i] > hi[i]) {
        counts[i] = 0;
        continue;
      }
      auto first = std::lower_bound(keys.begin(), keys.end(), lo[i]);
      auto last = std::upper_bound(keys.begin(), keys.end(), hi[i]);
      uint64_t cnt = uint64_t(last - first);
      counts[i] = uint32_t(cnt);
      uint64_t w = std::min<uint64_t>(cnt, maxpq);
      for (uint64_t r = 0; r < w; ++r) {
        size_t pos = size_t(first - keys.begin()) + r;
        if (kout) kout[i * maxpq + r] = keys[pos];
        if (vout) vout[i * maxpq + r] = vals[pos];
      }
    }
  }
};

struct Handle {
  int key_bits;
  Store<uint32_t> s32;
  Store<uint64_t> s64;
};

}  // namespace

extern "C" {

void* orc_create(int key_bits) {
  if (key_bits != 32 && key_bits != 64) return nullptr;
  Handle* h = new Handle;
  h->key_bits = key_bits;
  return h;
}

void orc_destroy(void* hp) { delete static_cast<Handle*>(hp); }

#define ORC_DISPATCH(h, call32, call64) \
  ((h)->key_bits == 32 ? (call32) : (call64))

int orc_bulk_load(void* hp, const void* k, const void* v, uint64_t n) {
  Handle* h = static_cast<Handle*>(hp);
  return ORC_DISPATCH(
      h, h->s32.bulk_load((const uint32_t*)k, (const uint32_t*)v, n),
      h->s64.bulk_load((const uint64_t*)k, (const uint64_t*)v, n));
}

int orc_insert(void* hp, const void* k, const void* v, uint64_t n) {
  Handle* h = static_cast<Handle*>(hp);
  return ORC_DISPATCH(
      h, h->s32.insert((const uint32_t*)k, (const uint32_t*)v, n),
      h->s64.insert((const uint64_t*)k, (const uint64_t*)v, n));
}

void orc_delete(void* hp, const void* k, uint64_t n) {
  Handle* h = static_cast<Handle*>(hp);
  if (h->key_bits == 32)
    h->s32.erase((const uint32_t*)k, n);
  else
    h->s64.erase((const uint64_t*)k, n);
}

void orc_lookup(void* hp, const void* q, uint64_t n, void* out) {
  Handle* h = static_cast<Handle*>(hp);
  if (h->key_bits == 32)
    h->s32.lookup((const uint32_t*)q, n, (uint32_t*)out);
  else
    h->s64.lookup((const uint64_t*)q, n, (uint64_t*)out);
}

void orc_successor(void* hp, const void* q, uint64_t n, void* kout,
                   void* vout) {
  Handle* h = static_cast<Handle*>(hp);
  if (h->key_bits == 32)
    h->s32.successor((const uint32_t*)q, n, (uint32_t*)kout, (uint32_t*)vout);
  else
    h->s64.successor((const uint64_t*)q, n, (uint64_t*)kout, (uint64_t*)vout);
}

void orc_predecessor(void* hp, const void* q, uint64_t n, void* kout,
                     void* vout) {
  Handle* h = static_cast<Handle*>(hp);
  if (h->key_bits == 32)
    h->s32.predecessor((const uint32_t*)q, n, (uint32_t*)kout, (uint32_t*)vout);
  else
    h->s64.predecessor((const uint64_t*)q, n, (uint64_t*)kout, (uint64_t*)vout);
}

void orc_range(void* hp, const void* lo, const void* hi, uint64_t n,
               uint32_t maxpq, uint32_t* counts, void* kout, void* vout) {
  Handle* h = static_cast<Handle*>(hp);
  if (h->key_bits == 32)
    h->s32.range((const uint32_t*)lo, (const uint32_t*)hi, n, maxpq, counts,
                 (uint32_t*)kout, (uint32_t*)vout);
  else
    h->s64.range((const uint64_t*)lo, (const uint64_t*)hi, n, maxpq, counts,
                 (uint64_t*)kout, (uint64_t*)vout);
}

uint64_t orc_size(void* hp) {
  Handle* h = static_cast<Handle*>(hp);
  return h->key_bits == 32 ? h->s32.keys.size() : h->s64.keys.size();
}

void orc_dump(void* hp, void* kout, void* vout) {
  Handle* h = static_cast<Handle*>(hp);
  size_t es = h->key_bits / 8;
  size_t n = h->key_bits == 32 ? h->s32.keys.size() : h->s64.keys.size();
  if (h->key_bits == 32) {
    std::memcpy(kout, h->s32.keys.data(), n * es);
    std::memcpy(vout, h->s32.vals.data(), n * es);
  } else {
    std::memcpy(kout, h->s64.keys.data(), n * es);
    std::memcpy(vout, h->s64.vals.data(), n * es);
  }
}

}  // extern "C"
