// Read batches (point lookup, successor, range) in the flipped, compute-to-
// bucket form (Section 3.3; Section 4.1 common steps): shared definitions and
// the global-memory helpers of the read kernel in flix_read2.hpp.
//
// Every bucket finds the slice of the sorted batch it owns by a bound search
// against its maxBucket value: bucket i owns the keys in (MKBA[i-1], MKBA[i]].
// Keys of buckets that are chains of several nodes resolve by walking the node
// links in global memory (Section 4.1: the first node whose maxKey is >= k).
// Every link is checked against the pool size before it is followed: a link
// outside the pool is reported as an internal error instead of being used.
#pragma once

#include "flix_device.hpp"

namespace flix {

constexpr int kOpLookup = 0;
constexpr int kOpSuccessor = 1;
constexpr int kOpRange = 2;

template <typename K>
struct ReadArgs {
  const K* skeys;      // sorted batch keys [m]
  const u32* sidx;     // input position of each sorted key [m]
  u32 m;
  const K* mkba;       // [nb]
  u32 nb;
  const NodeHdr* hdr;  // [pool]
  const K* nkeys;      // [pool * cap]
  const K* nvals;      // [pool * cap]
  u32 cap;
  u32 share;           // merged items (buckets + keys) per workgroup
  K* out_v;            // lookup, successor, range values
  K* out_k;            // successor, range keys (range: may be null)
  const K* hi;         // range upper bounds in input order
  u32* counts;         // range counts in input order
  u32 maxpq;           // range output stride
  u32 pool;            // nodes in the pool (bound of every link)
  u32* err;            // sticky status word for internal errors
};

// Number of batch keys among the first d items of merge(keys, mkba), ties to
// the keys: a key equal to MKBA[i] belongs to bucket i.
template <typename K>
__device__ u32 merge_path_keys(const K* a, u32 na, const K* mk, u32 nm, u64 d) {
  u32 lo = d > nm ? (u32)(d - nm) : 0u;
  u32 hi = d < na ? (u32)d : na;
  while (lo < hi) {
    u32 mid = (lo + hi) >> 1;
    if (a[mid] <= mk[(u32)(d - mid - 1)]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

constexpr u32 kBadLink = 0xFFFFFFFEu;   // a link outside the pool

// Node of bucket b whose range holds x (first node with x <= maxKey), or
// kBadLink when a link on the way points outside the pool.
__device__ __forceinline__ u32 locate_node(const NodeHdr* hdr, u32 pool, u32 b, u64 x,
                                           NodeHdr* out) {
  u32 node = b;
  NodeHdr h = hdr[node];
  while (x > h.fence && h.next != kNil) {
    node = h.next;
    if (node >= pool) return kBadLink;
    h = hdr[node];
  }
  *out = h;
  return node;
}

// First node after (bucket b, node with header h) that holds a key: the next
// node of the chain (non-head nodes are never empty), else the head of the
// next non-empty bucket.  Returns kNil when none exists, kBadLink for a link
// outside the pool.
__device__ __forceinline__ u32 next_nonempty(const NodeHdr* hdr, u32 nb, u32 pool, u32* b,
                                             const NodeHdr& h, NodeHdr* out) {
  if (h.next != kNil) {
    if (h.next >= pool) return kBadLink;
    *out = hdr[h.next];
    return h.next;
  }
  for (u32 bb = *b + 1; bb < nb; ++bb) {
    NodeHdr g = hdr[bb];
    if (g.size > 0) {
      *b = bb;
      *out = g;
      return bb;
    }
  }
  return kNil;
}

}  // namespace flix
