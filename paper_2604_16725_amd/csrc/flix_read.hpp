// Read batches (point lookup, successor, range) in the flipped, compute-to-
// bucket form (Section 3.3; Section 4.1 common steps).
//
// Every bucket finds the slice of the sorted batch it owns by a bound search
// against its maxBucket value: bucket i owns the keys in (MKBA[i-1], MKBA[i]].
// On gfx950 that search is done cooperatively: the merged sequence
// "MKBA (+) sorted batch" is cut by merge-path into equal shares, one share
// per workgroup, so a workgroup owns a contiguous run of buckets together with
// exactly the batch keys that fall into them.  Inside the share each bucket
// takes its slice with one upper_bound of its maxBucket over the share's keys
// (in LDS).  Buckets with a non-empty slice have their live keys staged into
// LDS with coalesced 16-byte loads (the node is read once per bucket, however
// many keys its slice holds); then every key of the share is resolved by one
// lane against the staged node.  A hot bucket whose slice spans several shares
// is staged once per share, which splits skewed slices across workgroups.
//
// Buckets that are chains of several nodes, or that do not fit the staging
// area, resolve their keys by walking the node links in global memory
// (Section 4.1: the first node whose maxKey is >= k).
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

// Node of bucket b whose range holds x (first node with x <= maxKey).
__device__ __forceinline__ u32 locate_node(const NodeHdr* hdr, u32 b, u64 x, NodeHdr* out) {
  u32 node = b;
  NodeHdr h = hdr[node];
  while (x > h.fence && h.next != kNil) {
    node = h.next;
    h = hdr[node];
  }
  *out = h;
  return node;
}

// First node after (bucket b, node with header h) that holds a key: the next
// node of the chain (non-head nodes are never empty), else the head of the
// next non-empty bucket.  Returns kNil when none exists.
__device__ __forceinline__ u32 next_nonempty(const NodeHdr* hdr, u32 nb, u32* b,
                                             const NodeHdr& h, NodeHdr* out) {
  if (h.next != kNil) {
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

template <typename K, int NT, int S, int STAGE_CH, int OP>
__global__ __launch_bounds__(NT) void k_read_apply(ReadArgs<K> a) {
  constexpr u32 KPC = 16 / sizeof(K);  // keys per 16-byte chunk
  __shared__ K s_q[S];
  __shared__ K s_mk[S];
  __shared__ u32 s_e[S + 1];      // end of each local bucket's slice
  __shared__ u32 s_size[S + 1];   // head size of touched buckets
  __shared__ u32 s_next[S + 1];   // head next link of touched buckets
  __shared__ u32 s_off[S + 2];    // staging offsets (16-byte chunks)
  __shared__ uint4 s_stage[STAGE_CH];
  __shared__ u32 s_tmp[NT / 64 + 1];
  __shared__ u32 s_part[4];

  const u32 tid = threadIdx.x;
  const u64 total = (u64)a.m + a.nb;
  const u64 d0 = (u64)blockIdx.x * a.share;
  const u64 d1 = d0 + a.share < total ? d0 + a.share : total;
  if (tid == 0) {
    u32 q0 = merge_path_keys(a.skeys, a.m, a.mkba, a.nb, d0);
    s_part[0] = q0;
    s_part[2] = (u32)(d0 - q0);
  } else if (tid == 64 % NT) {
    u32 q1 = merge_path_keys(a.skeys, a.m, a.mkba, a.nb, d1);
    s_part[1] = q1;
    s_part[3] = (u32)(d1 - q1);
  }
  __syncthreads();
  const u32 q0 = s_part[0], q1 = s_part[1];
  const u32 b0 = s_part[2], b1 = s_part[3];
  const u32 nq = q1 - q0;
  if (nq == 0) return;  // no batch key falls into this share's buckets
  const u32 nbl = b1 - b0;  // maxBucket entries in the share
  // local buckets 0..nbl; local bucket nbl is bucket b1 (its maxBucket lies in
  // the next share) and exists only if b1 < nb.
  for (u32 j = tid; j < nq; j += NT) s_q[j] = a.skeys[q0 + j];
  for (u32 i = tid; i < nbl; i += NT) s_mk[i] = a.mkba[b0 + i];
  __syncthreads();

  // Bound search: each bucket pulls its slice of the share's keys.
  for (u32 lb = tid; lb <= nbl; lb += NT)
    s_e[lb] = (lb < nbl) ? upper_bound_idx<K>(s_q, 0u, nq, s_mk[lb]) : nq;
  __syncthreads();

  // Heads of touched buckets; staging size in 16-byte chunks (single-node
  // buckets only).
  constexpr u32 PER = (S + 1 + NT - 1) / NT;
  u32 chunks[PER];
  u32 mysum = 0;
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    u32 lb = tid * PER + r;
    u32 c = 0;
    if (lb <= nbl) {
      u32 s = lb ? s_e[lb - 1] : 0u;
      bool touched = s_e[lb] > s && (b0 + lb) < a.nb;
      u32 size = 0, next = kNil;
      if (touched) {
        NodeHdr h = a.hdr[b0 + lb];
        size = h.size;
        next = h.next;
        if (next == kNil) c = (size + KPC - 1) / KPC;
      }
      s_size[lb] = size;
      s_next[lb] = next;
    }
    chunks[r] = c;
    mysum += c;
  }
  u32 tot_chunks;
  u32 ex = block_exclusive_scan<NT>(mysum, s_tmp, &tot_chunks);
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    u32 lb = tid * PER + r;
    if (lb <= nbl) s_off[lb] = ex;
    ex += chunks[r];
  }
  if (tid == 0) s_off[nbl + 1] = tot_chunks;
  __syncthreads();

  // Stage live keys: flattened (bucket, chunk) copy, 16 bytes per lane.
  const u32 ncopy = tot_chunks < (u32)STAGE_CH ? tot_chunks : (u32)STAGE_CH;
  for (u32 c0 = tid; c0 < ncopy; c0 += 4 * NT) {
    uint4 v[4];
    u32 cc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      u32 c = c0 + u * NT;
      cc[u] = c;
      if (c < ncopy) {
        u32 lb = upper_bound_idx<u32>(s_off, 0u, nbl + 1, c) - 1;
        const uint4* src = reinterpret_cast<const uint4*>(a.nkeys + (u64)(b0 + lb) * a.cap);
        v[u] = src[c - s_off[lb]];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (cc[u] < ncopy) s_stage[cc[u]] = v[u];
  }
  __syncthreads();

  const K* stage = reinterpret_cast<const K*>(s_stage);
  const K NF = key_max<K>();

  // Resolve every key of the share, one lane per key.
  for (u32 j = tid; j < nq; j += NT) {
    const K x = s_q[j];
    const u32 lb = upper_bound_idx<u32>(s_e, 0u, nbl + 1, j);
    u32 b = b0 + lb;
    const u32 orig = a.sidx[q0 + j];
    const u32 size = s_size[lb];
    const bool single = s_next[lb] == kNil;
    const bool fits = single && s_off[lb + 1] <= (u32)STAGE_CH;
    // Current node: staged copy (fits) or global memory.
    u32 node = b;
    NodeHdr h;
    const K* keys;
    u32 pos;
    if (fits) {
      h.fence = 0;  // unused for staged single nodes
      h.size = size;
      h.next = kNil;
      keys = stage + (u64)s_off[lb] * KPC;
    } else {
      node = locate_node(a.hdr, b, (u64)x, &h);
      keys = a.nkeys + (u64)node * a.cap;
    }
    pos = lower_bound_idx<K>(keys, 0u, h.size, x);

    if (OP == kOpLookup) {
      K val = NF;
      if (pos < h.size && keys[pos] == x) val = a.nvals[(u64)node * a.cap + pos];
      a.out_v[orig] = val;
    } else if (OP == kOpSuccessor) {
      K rk = NF, rv = NF;
      if (pos < h.size) {
        rk = keys[pos];
        rv = a.nvals[(u64)node * a.cap + pos];
      } else {
        NodeHdr g;
        u32 nn = next_nonempty(a.hdr, a.nb, &b, h, &g);
        if (nn != kNil) {
          rk = a.nkeys[(u64)nn * a.cap];
          rv = a.nvals[(u64)nn * a.cap];
        }
      }
      a.out_k[orig] = rk;
      a.out_v[orig] = rv;
    } else {  // range [x, hi]
      const K hi = a.hi[orig];
      u32 cnt = 0;
      if (x <= hi) {
        const u64 ob = (u64)orig * a.maxpq;
        while (true) {
          u32 ub = upper_bound_idx<K>(keys, pos, h.size, hi);
          for (u32 r = pos; r < ub; ++r, ++cnt) {
            if (cnt < a.maxpq) {
              if (a.out_k) a.out_k[ob + cnt] = keys[r];
              if (a.out_v) a.out_v[ob + cnt] = a.nvals[(u64)node * a.cap + r];
            }
          }
          if (ub < h.size) break;
          NodeHdr g;
          u32 nn = next_nonempty(a.hdr, a.nb, &b, h, &g);
          if (nn == kNil) break;
          node = nn;
          h = g;
          keys = a.nkeys + (u64)node * a.cap;
          pos = 0;
        }
      }
      a.counts[orig] = cnt;
    }
  }
}

}  // namespace flix
