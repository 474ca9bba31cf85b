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
#include "flix_occ.hpp"

namespace flix {

constexpr int kOpLookup = 0;
constexpr int kOpSuccessor = 1;
constexpr int kOpRange = 2;
constexpr int kOpPredecessor = 5;   // 3 and 4 are the update operations

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
  u64* occ;            // occupancy summary of the nb buckets, its three levels
                       // laid out from here (flix_occ.hpp: occ_levels)
  const u32* cuts;     // merge-path cut of every share boundary [nshares + 1], or
                       // nullptr: each workgroup searches its own two cuts
};

// Cooperative merge-path cut for the two diagonals d[0], d[1] of one
// workgroup (NT == 256: threads 0..127 search d[0], 128..255 search d[1]).
// Returns, for both diagonals, the number of batch keys among the first d
// items of merge(keys, mkba) with ties to the keys (a key equal to MKBA[i]
// belongs to bucket i).
template <typename K>
__device__ void coop_merge_path(const K* a, u32 na, const K* mk, u32 nm, const u64 d[2],
                                u32* s_lo, u32* s_hi, u32* s_wc, u32* out) {
  const u32 tid = threadIdx.x;
  const u32 half = tid >> 7;
  const u32 t = tid & 127;
  if (t == 0) {
    u64 dd = d[half];
    s_lo[half] = dd > nm ? (u32)(dd - nm) : 0u;
    s_hi[half] = dd < na ? (u32)dd : na;
  }
  __syncthreads();
  for (int round = 0; round < 8; ++round) {
    const u32 lo = s_lo[half], hi = s_hi[half];
    const bool any = (s_lo[0] < s_hi[0]) || (s_lo[1] < s_hi[1]);
    if (!any) break;
    const u64 dd = d[half];
    const u32 span = hi - lo;
    u32 p = 0;
    bool pred = false;
    if (span > 0) {
      p = span <= 128 ? lo + t : lo + (u32)(((u64)span * t) / 128u);
      if (span > 128 || t < span) pred = a[p] <= mk[(u32)(dd - p - 1)];
    }
    u64 bal = wave_ballot(pred);
    if ((tid & 63) == 0) s_wc[tid >> 6] = (u32)__popcll(bal);
    __syncthreads();
    if (t == 0 && span > 0) {
      u32 c = s_wc[2 * half] + s_wc[2 * half + 1];
      if (span <= 128) {
        s_lo[half] = lo + c;
        s_hi[half] = lo + c;
      } else if (c == 0) {
        s_hi[half] = lo;
      } else {
        u32 pl = lo + (u32)(((u64)span * (c - 1)) / 128u);
        s_lo[half] = pl + 1;
        if (c < 128) s_hi[half] = lo + (u32)(((u64)span * c) / 128u);
      }
    }
    __syncthreads();
  }
  if (tid < 2) out[tid] = s_lo[tid];
  __syncthreads();
}

// Merge-path cuts of "MKBA (+) sorted batch" at every share boundary, for
// the read kernel: cut c is the number of batch keys among the first
// min(c * share, m + nb) items of the merge, ties to the keys (a key equal to
// MKBA[i] belongs to bucket i).  Half a wave per cut, 32-ary search: 32
// probes split the candidate range into 33 parts and one ballot keeps the
// part that holds the cut (four dependent rounds for 2^21 items, each probe a
// cache line), so the read kernel's workgroups start from one load instead
// of a search of their own.
template <typename K>
__global__ __launch_bounds__(256) void k_merge_cuts(const K* __restrict__ a, u32 na,
                                                    const K* __restrict__ mk, u32 nm, u32 share,
                                                    u32 ncuts, u32* __restrict__ cuts) {
  const u32 c = blockIdx.x * 8u + (threadIdx.x >> 5);
  const u32 lane = threadIdx.x & 31u;
  const u64 half = 0xFFFFFFFFull << (32u * ((threadIdx.x >> 5) & 1u));
  if (c >= ncuts) return;   // whole half-waves
  const u64 total = (u64)na + nm;
  const u64 d = (u64)c * share < total ? (u64)c * share : total;
  // the predicate a[p] <= mk[d - p - 1] holds exactly for p < cut, cut in [lo, hi]
  u32 lo = d > nm ? (u32)(d - nm) : 0u;
  u32 hi = d < na ? (u32)d : na;
  while (lo < hi) {
    const u32 span = hi - lo;
    if (span <= 32u) {
      bool pr = false;
      if (lane < span) {
        const u32 p = lo + lane;
        pr = a[p] <= mk[(u32)(d - p - 1)];
      }
      lo += (u32)__popcll(wave_ballot(pr) & half);
      break;
    }
    // probes x_l = lo + floor(span * (l + 1) / 33): strictly increasing, all < hi
    const u32 p = lo + (u32)(((u64)span * (lane + 1u)) / 33u);
    const bool pr = a[p] <= mk[(u32)(d - p - 1)];
    const u32 t = (u32)__popcll(wave_ballot(pr) & half);   // probes below the cut
    const u32 nlo = t ? lo + (u32)(((u64)span * t) / 33u) + 1u : lo;
    const u32 nhi = t < 32u ? lo + (u32)(((u64)span * (t + 1u)) / 33u) : hi;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) cuts[c] = lo;
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
// next bucket that holds a key (occupancy summary).  Returns kNil when none
// exists, kBadLink for a link outside the pool.
__device__ __forceinline__ u32 next_nonempty(const NodeHdr* hdr, const OccLevels& occ, u32 nb,
                                             u32 pool, u32* b, const NodeHdr& h, NodeHdr* out) {
  if (h.next != kNil) {
    if (h.next >= pool) return kBadLink;
    *out = hdr[h.next];
    return h.next;
  }
  const u32 bb = occ_next(occ, nb, *b);
  if (bb >= nb) return kNil;
  *b = bb;
  *out = hdr[bb];
  return bb;
}

// Predecessor of x in the store, x owned by bucket b (Section 2.1): the
// largest stored key <= x.  Walks b's chain to the node whose range holds x,
// remembering the node before it; if that node has no key <= x the answer is
// the last key of the previous node, else of the last node of the previous
// bucket that holds keys.  Returns the slot (node * cap + position) or
// ~0ull when there is none; kBadLink in *bad for a link outside the pool.
template <typename K>
__device__ inline u64 predecessor_slot(const NodeHdr* hdr, const K* nkeys, const OccLevels& occ,
                                       u32 pool, u32 cap, u32 b, K x, bool* bad) {
  u32 node = b, prevn = kNil;
  NodeHdr h = hdr[node], hp;
  hp.size = 0;
  while ((u64)x > h.fence && h.next != kNil) {
    prevn = node;
    hp = h;
    node = h.next;
    if (node >= pool) { *bad = true; return ~0ull; }
    h = hdr[node];
  }
  if (h.size > cap || hp.size > cap) { *bad = true; return ~0ull; }   // never expected
  const u32 p = upper_bound_idx<K>(nkeys + (u64)node * cap, 0u, h.size, x);
  if (p > 0) return (u64)node * cap + (p - 1);
  if (prevn != kNil && hp.size > 0) return (u64)prevn * cap + (hp.size - 1);
  const u32 pb = occ_prev(occ, b);
  if (pb == kNil) return ~0ull;
  node = pb;
  h = hdr[node];
  u32 steps = 0;
  while (h.next != kNil) {
    node = h.next;
    if (node >= pool || ++steps > pool) { *bad = true; return ~0ull; }
    h = hdr[node];
  }
  if (h.size == 0 || h.size > cap) { *bad = true; return ~0ull; }   // summary or node corrupt
  return (u64)node * cap + (h.size - 1);
}

}  // namespace flix
