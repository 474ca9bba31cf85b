// Initial build (bulk load), contents dump and the device invariant checker.
#pragma once

#include "flix_device.hpp"
#include "flix_occ.hpp"

namespace flix {

// ---------------------------------------------------------------------------
// Stream compaction of a sorted run: keep the LAST item of every equal-key
// run (upsert semantics: the stable sort keeps input order among equal keys).
// Three kernels: per-block counts, one-block scan of the counts, scatter.
// ---------------------------------------------------------------------------
constexpr int kCompactNT = 256;
constexpr int kCompactIPT = 8;
constexpr int kCompactTile = kCompactNT * kCompactIPT;

template <typename K>
__device__ __forceinline__ bool keep_last(const K* k, u64 i, u64 n) {
  return (i + 1 == n) || (k[i] != k[i + 1]);
}

template <typename K>
__global__ __launch_bounds__(kCompactNT) void k_compact_count(const K* __restrict__ k, u64 n,
                                                             u32* __restrict__ bsum) {
  __shared__ u32 s_tmp[kCompactNT / 64 + 1];
  u64 base = (u64)blockIdx.x * kCompactTile + (u64)threadIdx.x * kCompactIPT;
  u32 c = 0;
  for (int j = 0; j < kCompactIPT; ++j) {
    u64 i = base + j;
    if (i < n && keep_last(k, i, n)) ++c;
  }
  u32 tot;
  block_exclusive_scan<kCompactNT>(c, s_tmp, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block: exclusive scan of nb block counts in place; total -> *total.
__global__ __launch_bounds__(1024) void k_scan_small(u32* __restrict__ a, u32 nb,
                                                    u32* __restrict__ total) {
  __shared__ u32 s_tmp[1024 / 64 + 1];
  u32 per = (nb + 1023) / 1024;
  u32 beg = threadIdx.x * per;
  u32 sum = 0;
  for (u32 i = beg; i < beg + per && i < nb; ++i) sum += a[i];
  u32 tot;
  u32 ex = block_exclusive_scan<1024>(sum, s_tmp, &tot);
  for (u32 i = beg; i < beg + per && i < nb; ++i) {
    u32 t = a[i];
    a[i] = ex;
    ex += t;
  }
  if (threadIdx.x == 0) *total = tot;
}

template <typename K>
__global__ __launch_bounds__(kCompactNT) void k_compact_scatter(const K* __restrict__ k,
                                                               const K* __restrict__ v, u64 n,
                                                               const u32* __restrict__ boff,
                                                               K* __restrict__ ko,
                                                               K* __restrict__ vo) {
  __shared__ u32 s_tmp[kCompactNT / 64 + 1];
  u64 base = (u64)blockIdx.x * kCompactTile + (u64)threadIdx.x * kCompactIPT;
  u32 c = 0;
  for (int j = 0; j < kCompactIPT; ++j) {
    u64 i = base + j;
    if (i < n && keep_last(k, i, n)) ++c;
  }
  u32 tot;
  u32 pos = block_exclusive_scan<kCompactNT>(c, s_tmp, &tot) + boff[blockIdx.x];
  for (int j = 0; j < kCompactIPT; ++j) {
    u64 i = base + j;
    if (i < n && keep_last(k, i, n)) {
      ko[pos] = k[i];
      vo[pos] = v[i];
      ++pos;
    }
  }
}

// Any value equal to the reserved NOT_FOUND pattern -> *err = -1.
template <typename K>
__global__ void k_check_reserved(const K* __restrict__ v, u64 n, u32* __restrict__ err) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (u64)gridDim.x * blockDim.x)
    if (v[i] == key_max<K>()) atomicExch(err, 0xFFFFFFFFu);
}

// ---------------------------------------------------------------------------
// Initial build (Section 3.2): the n distinct sorted pairs are cut into
// groups of `fill` keys; group i becomes the single node of bucket i and its
// last key becomes maxBucket (MKBA[i]).  The last bucket's bound is KEY_MAX so
// that every key maps to a bucket.  Node i is the head of bucket i.
// ---------------------------------------------------------------------------
template <typename K>
__global__ void k_build_nodes(const K* __restrict__ sk, const K* __restrict__ sv, u64 n,
                              u32 fill, u32 cap, K* __restrict__ nkeys, K* __restrict__ nvals) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (u64)gridDim.x * blockDim.x) {
    u64 b = i / fill, s = i % fill;
    nkeys[b * cap + s] = sk[i];
    nvals[b * cap + s] = sv[i];
  }
}

template <typename K>
__global__ void k_build_dir(const K* __restrict__ sk, u64 n, u32 fill, u32 nb,
                            K* __restrict__ mkba, NodeHdr* __restrict__ hdr,
                            u32* __restrict__ bnodes) {
  for (u32 b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    u64 lo = (u64)b * fill;
    u64 hi = lo + fill < n ? lo + fill : n;
    K fence = (b + 1 == nb) ? key_max<K>() : sk[hi - 1];
    mkba[b] = fence;
    NodeHdr h;
    h.fence = (u64)fence;
    h.size = (u32)(hi > lo ? hi - lo : 0);
    h.next = kNil;
    hdr[b] = h;
    bnodes[b] = 1;
  }
}

// Free stack holds every node id >= nb; Ctl counters reset.
__global__ void k_build_free(u32 nb, u32 pool, u64 nkeys, u32* __restrict__ free_ids,
                             Ctl* __restrict__ ctl) {
  u32 nfree = pool - nb;
  for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < nfree; j += gridDim.x * blockDim.x)
    free_ids[j] = pool - 1 - j;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->free_top = nfree;
    ctl->nkeys = nkeys;
    ctl->need = 0;
    ctl->call_err = 0;
    ctl->call_abort = 0;
    ctl->work_ovf = 0;
  }
}

// ---------------------------------------------------------------------------
// Dump: per-bucket totals (walking each chain), scan, then copy in key order.
// ---------------------------------------------------------------------------
__global__ void k_bucket_totals(const NodeHdr* __restrict__ hdr, u32 nb, u32 pool,
                                u32* __restrict__ tot) {
  for (u32 b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    u32 t = 0;
    u32 node = b;
    u32 steps = 0;
    while (node < pool && steps++ < pool) {
      NodeHdr h = hdr[node];
      t += h.size;
      node = h.next;
    }
    tot[b] = t;
  }
}

// Exclusive scan of per-bucket totals: per-block partials, block-sum scan,
// add-back.  Used on the (non-hot) dump path.
__global__ __launch_bounds__(256) void k_scan_blocks_u32(const u32* __restrict__ in, u32 n,
                                                        u32* __restrict__ out,
                                                        u32* __restrict__ bsum) {
  __shared__ u32 s_tmp[256 / 64 + 1];
  u32 i = blockIdx.x * 256 + threadIdx.x;
  u32 v = i < n ? in[i] : 0u;
  u32 tot;
  u32 ex = block_exclusive_scan<256>(v, s_tmp, &tot);
  if (i < n) out[i] = ex;
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_addback(u32* __restrict__ out, u32 n, const u32* __restrict__ bsum) {
  u32 i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] += bsum[blockIdx.x];
}

template <typename K>
__global__ void k_dump_copy(const NodeHdr* __restrict__ hdr, const K* __restrict__ nkeys,
                            const K* __restrict__ nvals, u32 nb, u32 cap, u32 pool,
                            const u32* __restrict__ off, K* __restrict__ ko,
                            K* __restrict__ vo, u64 out_cap) {
  // one wave per bucket
  u32 wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  u32 lane = threadIdx.x & 63;
  u32 nw = (gridDim.x * blockDim.x) >> 6;
  for (u32 b = wave; b < nb; b += nw) {
    u64 o = off[b];
    u32 node = b;
    u32 steps = 0;
    while (node < pool && steps++ < pool) {
      NodeHdr h = hdr[node];
      u32 sz = h.size < cap ? h.size : cap;
      for (u32 s = lane; s < sz; s += 64) {
        if (o + s < out_cap) {
          ko[o + s] = nkeys[(u64)node * cap + s];
          vo[o + s] = nvals[(u64)node * cap + s];
        }
      }
      o += sz;
      node = h.next;
    }
  }
}

// ---------------------------------------------------------------------------
// Device invariant checker.  err codes (first failure recorded):
//  1 key order inside a node      2 key outside its node's range
//  3 fence order along a chain    4 last fence != maxBucket
//  5 size > capacity              6 empty non-head node / empty head with next
//  7 chain length != bnodes       8 node id out of range / revisited
//  9 total keys != nkeys          10 live + free != pool
//  11 free id invalid or duplicated
// ---------------------------------------------------------------------------
template <typename K>
__global__ void k_check_buckets(const K* __restrict__ mkba, const NodeHdr* __restrict__ hdr,
                                const K* __restrict__ nkeys, const u32* __restrict__ bnodes,
                                u32 nb, u32 cap, u32 pool, u32* __restrict__ mark,
                                unsigned long long* __restrict__ counters,
                                u32* __restrict__ err) {
  for (u32 b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    bool has_lo = b > 0;
    K lo = has_lo ? mkba[b - 1] : K(0);  // keys must be > lo (if has_lo)
    if (has_lo && !(mkba[b - 1] < mkba[b])) atomicCAS(err, 0u, 3u);
    u32 node = b;
    u32 len = 0;
    u64 keys = 0;
    bool first = true;
    K prev_fence = lo;
    bool have_prev = has_lo;
    while (node != kNil) {
      if (node >= pool) { atomicCAS(err, 0u, 8u); break; }
      if (atomicAdd(&mark[node], 1u) != 0u) { atomicCAS(err, 0u, 8u); break; }
      NodeHdr h = hdr[node];
      K fence = (K)h.fence;
      if (have_prev && !(prev_fence < fence)) atomicCAS(err, 0u, 3u);
      if (h.size > cap) { atomicCAS(err, 0u, 5u); break; }
      if (h.size == 0 && (!first || h.next != kNil)) atomicCAS(err, 0u, 6u);
      for (u32 s = 0; s < h.size; ++s) {
        K k = nkeys[(u64)node * cap + s];
        if (s > 0 && !(nkeys[(u64)node * cap + s - 1] < k)) atomicCAS(err, 0u, 1u);
        if ((have_prev && !(k > prev_fence)) || k > fence) atomicCAS(err, 0u, 2u);
      }
      keys += h.size;
      ++len;
      prev_fence = fence;
      have_prev = true;
      first = false;
      if (h.next == kNil && fence != mkba[b]) atomicCAS(err, 0u, 4u);
      node = h.next;
      if (len > pool) { atomicCAS(err, 0u, 8u); break; }
    }
    if (len != bnodes[b]) atomicCAS(err, 0u, 7u);
    atomicAdd(&counters[0], (unsigned long long)keys);
    atomicAdd(&counters[1], (unsigned long long)len);
  }
}

__global__ void k_check_free(const u32* __restrict__ free_ids, const Ctl* __restrict__ ctl,
                             u32 pool, u32* __restrict__ mark, u32* __restrict__ err) {
  u32 top = ctl->free_top;
  if (top > pool) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(err, 0u, 11u);
    return;
  }
  for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < top; j += gridDim.x * blockDim.x) {
    u32 id = free_ids[j];
    if (id >= pool || atomicAdd(&mark[id], 1u) != 0u) atomicCAS(err, 0u, 11u);
  }
}

// ---------------------------------------------------------------------------
// Occupancy summary (flix_occ.hpp): build at bulk load, invariant check.
// ---------------------------------------------------------------------------
// Level 0 from the head sizes (a bucket is empty exactly when its head node is
// empty: an empty head never has a successor node).
__global__ void k_occ_build0(const NodeHdr* __restrict__ hdr, u32 nb, u64* __restrict__ w0) {
  const u64 w = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= occ_words0(nb)) return;
  u64 bits = 0;
  for (u32 i = 0; i < 64; ++i) {
    const u64 b = w * 64 + i;
    if (b < nb && hdr[b].size > 0) bits |= 1ull << i;
  }
  w0[w] = bits;
}

// Level l+1 from level l (`n_hi` words above `n_lo` words below).
__global__ void k_occ_build_up(const u64* __restrict__ lo, u64 n_lo, u64* __restrict__ hi,
                               u64 n_hi) {
  const u64 w = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_hi) return;
  u64 bits = 0;
  for (u32 i = 0; i < 64; ++i) {
    const u64 j = w * 64 + i;
    if (j < n_lo && lo[j] != 0) bits |= 1ull << i;
  }
  hi[w] = bits;
}

// Invariant check: level 0 equals the head sizes, upper levels summarise the
// lower ones.  Records error 12 in *err.
__global__ void k_occ_check(const NodeHdr* __restrict__ hdr, u32 nb, OccLevels o,
                            u32* __restrict__ err) {
  const u64 n0 = occ_words0(nb), n1 = occ_words1(nb), n2 = occ_words2(nb);
  for (u64 w = (u64)blockIdx.x * blockDim.x + threadIdx.x; w < n0 + n1 + n2;
       w += (u64)gridDim.x * blockDim.x) {
    u64 want = 0, got;
    if (w < n0) {
      for (u32 i = 0; i < 64; ++i) {
        const u64 b = w * 64 + i;
        if (b < nb && hdr[b].size > 0) want |= 1ull << i;
      }
      got = o.w0[w];
    } else if (w < n0 + n1) {
      const u64 v = w - n0;
      for (u32 i = 0; i < 64; ++i)
        if (v * 64 + i < n0 && o.w0[v * 64 + i] != 0) want |= 1ull << i;
      got = o.w1[v];
    } else {
      const u64 v = w - n0 - n1;
      for (u32 i = 0; i < 64; ++i)
        if (v * 64 + i < n1 && o.w1[v * 64 + i] != 0) want |= 1ull << i;
      got = o.w2[v];
    }
    if (want != got) atomicCAS(err, 0u, 12u);
  }
}

}  // namespace flix
