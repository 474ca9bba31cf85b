// Read batches, register-resident form (the default read kernel).
//
// Same flipped structure as flix_read.hpp (Section 3.3: every bucket pulls the
// slice of the sorted batch that falls into (MKBA[i-1], MKBA[i]]), organised
// for wave64 latency hiding:
//   1. merge-path cut of "MKBA (+) sorted batch" into equal shares: loaded
//      from the cut list (written by the run sort, else by k_merge_cuts), or
//      (persistent drain) found by a cooperative 128-ary search (three
//      dependent rounds instead of ~21);
//   2. one coalesced round of loads: the share's keys, their input positions,
//      MKBA entries and node headers (and range upper bounds);
//   3. every bucket takes its slice by upper_bound of its maxBucket in LDS;
//      the touched buckets are listed by slice length;
//   4. phase A: groups of GL lanes hold the live keys of U buckets at a time in
//      registers (KPL keys per lane, or KPL/2 spread over all lanes for a node
//      at most half full; 16-byte loads) and resolve each key of the slice
//      with ballots: lookup match, successor / range lower and upper bounds
//      inside the node (and a successor's key); the result goes to LDS;
//   5. phase B: one lane per key loads the value(s) and writes the outputs,
//      all keys of the share in flight at once.
// Keys whose answer lies outside the single staged node take the global-memory
// path of flix_read.hpp: chained buckets from their head, a successor or range
// running past its node's end from where phase A left it.
#pragma once

#include "flix_device.hpp"
#include "flix_read.hpp"

namespace flix {

constexpr u32 kPosMiss = 0xFFFFu;   // lookup miss inside a single-node bucket
constexpr u32 kPosSlow = 0xFFFEu;   // resolve on the global-memory path
// The answer continues past the end of a single-node bucket's node: a
// successor goes straight to the next bucket that holds a key, a range copies
// from position lt of the node (lt | size << 16 in the count slot) onwards,
// without locating the node or searching it again.
constexpr u32 kPosNext = 0xFFFDu;
constexpr u32 kChainBit = 0x80000000u;   // head-word flag: the bucket is a chain

// LDS arrays of one set of slices being resolved: the sorted keys of the
// slices, their input positions, range upper bounds, result codes, the end
// of every local bucket's slice, its head word and the touched-bucket list.
template <typename K>
struct SliceView {
  const K* q;
  const K* hi;
  const u32* idx;
  u32* pos;
  u32* cnt;
  const u32* e;
  const u32* hw;
  const unsigned short* tl;
  u32* list;        // LDS room for the ranges handed to the wave-wide copy
  u32 list_cap;     // (0: none; every range then stays on the one-lane path)
  u32* nlist;       // LDS counter of that list
  u32* lnode;       // per list entry: node and bucket where the copy resumes
  u32* lbk;         // (the position goes to pos[j], the results so far to cnt[j])
};

// A range on the one-lane path hands its copy to a whole wave when one node
// holds more than this many of its results.
constexpr u32 kLaneRangeMax = 16;

template <typename K, int KPL>
struct alignas(sizeof(K) * KPL >= 16 ? 16 : sizeof(K) * KPL) KeyVec {
  K k[KPL];
};

template <typename K, int S, int NT>
struct ReadSmem {
  K q[S];
  K hi[S];
  u32 idx[S];
  u32 pos[S];       // (local bucket << 16) | position / code
  u32 cnt[S];       // range: results inside the node
  K mk[S];
  u32 e[S + 1];
  u32 hw[S + 1];    // head node: size | kChainBit when the bucket has more nodes
  unsigned short tl[S + 1];
  u32 tmp[NT / 64 + 1];
  u32 lo[2], hiw[2], wc[4], cut[2], ntouch;
  u32 nslow;        // ranges listed for the wave-wide copy
};

// Ranges handed over by the one-lane path (a node holds more than
// kLaneRangeMax of their results): one wave per range resumes at the node and
// position the lane reached, 64 keys per step with coalesced loads, and
// writes the results it keeps with coalesced stores; the keys of a node are
// sorted, so the in-range lanes of a step form a prefix.  All threads call.
template <typename K, int NT>
__device__ __forceinline__ void range_waves(const ReadArgs<K>& a, const SliceView<K>& v) {
  __syncthreads();
  const u32 n = *v.nlist < v.list_cap ? *v.nlist : v.list_cap;
  const u32 lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  constexpr u32 NW = NT / 64;
  const OccLevels occ = occ_levels(a.occ, a.nb);
  for (u32 li = wv; li < n; li += NW) {
    const u32 j = v.list[li];
    u32 node = v.lnode[li];
    u32 b = v.lbk[li];
    u32 p = v.pos[j];
    u32 cnt = v.cnt[j];
    const K hi = v.hi[j];
    const u32 orig = v.idx[j];
    const u64 ob = (u64)orig * a.maxpq;
    u32 size = 0, next = 0;
    if (lane == 0) {
      const NodeHdr h = a.hdr[node];
      size = h.size;
      next = h.next;
    }
    size = __shfl(size, 0, 64);
    next = __shfl(next, 0, 64);
    bool bad = size > a.cap;
    bool done = bad;
    while (!done) {
      const K* keys = a.nkeys + (u64)node * a.cap;
      const K* vals = a.nvals + (u64)node * a.cap;
      for (u32 i0 = p; i0 < size; i0 += 64) {
        const u32 i = i0 + lane;
        const bool valid = i < size;
        const K k = valid ? keys[i] : K(0);
        const bool in = valid && k <= hi;
        const u32 nin = (u32)__popcll(wave_ballot(in));
        if (in) {
          const u32 r = cnt + lane;
          if (r < a.maxpq) {
            if (a.out_k) a.out_k[ob + r] = k;
            if (a.out_v) a.out_v[ob + r] = vals[i];
          }
        }
        cnt += nin;
        const u32 avail = size - i0 < 64u ? size - i0 : 64u;
        if (nin < avail) {   // a key above hi: the range ends in this node
          done = true;
          break;
        }
      }
      if (done) break;
      // next node of the chain, else the next bucket that holds a key
      u32 nn = 0, nsize = 0, nnext = 0;
      if (lane == 0) {
        NodeHdr h, g;
        h.next = next;
        h.size = size;
        nn = next_nonempty(a.hdr, occ, a.nb, a.pool, &b, h, &g);
        nsize = g.size;
        nnext = g.next;
      }
      nn = __shfl(nn, 0, 64);
      nsize = __shfl(nsize, 0, 64);
      nnext = __shfl(nnext, 0, 64);
      b = __shfl(b, 0, 64);
      if (nn == kNil) break;
      if (nn == kBadLink || nsize > a.cap) {
        bad = true;
        break;
      }
      node = nn;
      size = nsize;
      next = nnext;
      p = 0;
    }
    if (bad && lane == 0) atomicCAS(a.err, 0u, kErrInternal);
    if (bad) cnt = 0;
    if (lane == 0) a.counts[orig] = cnt;
  }
}

template <typename K>
__device__ __forceinline__ K shfl_key(K v, u32 src) {
  if constexpr (sizeof(K) == 4) {
    return (K)__shfl((int)v, (int)src, 64);
  } else {
    const u32 lo = (u32)__shfl((int)(u32)v, (int)src, 64);
    const u32 hi = (u32)__shfl((int)(u32)((u64)v >> 32), (int)src, 64);
    return (K)(((u64)hi << 32) | lo);
  }
}

// n consecutive (key, value) results of a node, from slot `at` of the pool,
// to outputs from position `o`: loads of four results are issued before
// their stores.
template <typename K>
__device__ __forceinline__ void copy_results(const ReadArgs<K>& a, u64 at, u32 n, u64 o) {
  for (u32 r0 = 0; r0 < n; r0 += 4) {
    K kk[4], vv[4];
#pragma unroll
    for (u32 q = 0; q < 4; ++q) {
      if (r0 + q < n) {
        if (a.out_k) kk[q] = a.nkeys[at + r0 + q];
        if (a.out_v) vv[q] = a.nvals[at + r0 + q];
      }
    }
#pragma unroll
    for (u32 q = 0; q < 4; ++q) {
      if (r0 + q < n) {
        if (a.out_k) a.out_k[o + r0 + q] = kk[q];
        if (a.out_v) a.out_v[o + r0 + q] = vv[q];
      }
    }
  }
}

// Phases A and B over the touched buckets of one set of slices (all threads
// of the workgroup call; `ntouch` buckets listed in v.tl, local bucket lb is
// global bucket b0 + lb, at most RQ * NT keys).
template <typename K, int NT, int GL, int KPL, int U, int RQ>
__device__ __forceinline__ void resolve_slices(const ReadArgs<K>& a, int op, const SliceView<K>& v, u32 b0,
                               u32 nq, u32 ntouch) {
  constexpr int NG = NT / GL;
  const u32 tid = threadIdx.x;
  const K* s_q = v.q;
  K* s_kq = const_cast<K*>(v.q);   // successor: answer keys of resolved queries
  const K* s_hi = v.hi;
  const u32* s_idx = v.idx;
  u32* s_pos = v.pos;
  u32* s_cnt = v.cnt;
  const u32* s_e = v.e;
  const u32* s_hw = v.hw;
  const unsigned short* s_tl = v.tl;
  // Phase A: groups resolve positions inside single-node buckets.
  {
    const u32 gid = tid / GL;
    const u32 gl = tid % GL;
    const u32 gbase = (tid & 63) - gl;
    const u64 gmask = (GL == 64) ? ~0ull : (((1ull << GL) - 1ull) << gbase);
    // A node holding at most half the group's slots (a bulk-loaded node at
    // fill cap/2) is spread over all GL lanes, KH keys each, and the
    // comparisons of the upper KPL - KH slots are skipped while no group of
    // the wave holds a fuller node: half the comparisons per key.
    constexpr bool kHalf = KPL >= 2;
    constexpr int KH = kHalf ? KPL / 2 : KPL;
    for (u32 i0 = gid * U; i0 < ntouch; i0 += NG * U) {
      KeyVec<K, KPL> kv[U];
      u32 lbs[U], sizes[U], kpls[U];
      bool single[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        u32 i = i0 + u;
        lbs[u] = i < ntouch ? s_tl[i] : 0u;
        const u32 hw = (i < ntouch) ? s_hw[lbs[u]] : 0u;
        sizes[u] = hw & ~kChainBit;
        single[u] = (i < ntouch) && !(hw & kChainBit);
        kpls[u] = (kHalf && sizes[u] <= (u32)(GL * KH)) ? (u32)KH : (u32)KPL;
        if (single[u] && gl * kpls[u] < sizes[u]) {
          const K* src = a.nkeys + (u64)(b0 + lbs[u]) * a.cap + (u64)gl * kpls[u];
          if (kHalf && kpls[u] == (u32)KH) {
            const KeyVec<K, KH> h = *reinterpret_cast<const KeyVec<K, KH>*>(src);
#pragma unroll
            for (int k = 0; k < KH; ++k) kv[u].k[k] = h.k[k];
          } else {
            kv[u] = *reinterpret_cast<const KeyVec<K, KPL>*>(src);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (i0 + u >= ntouch) break;
        const u32 lb = lbs[u];
        const u32 s = lb ? s_e[lb - 1] : 0u;
        const u32 e = s_e[lb];
        const u32 size = sizes[u];
        const u32 kpl = kpls[u];
        const bool full = kpl == (u32)KPL;
        if (!single[u]) {
          for (u32 j = s + gl; j < e; j += GL) s_pos[j] = (lb << 16) | kPosSlow;
          continue;
        }
        K prev = K(0), prev_hi = K(0);
        for (u32 j = s; j < e; ++j) {
          const K x = s_q[j];
          const K hi = (op == kOpRange) ? s_hi[j] : K(0);
          // a repeated query (skewed batches) takes the previous query's
          // answer; that answer was written to LDS earlier by a lane of this
          // wave (a range also needs the same upper bound)
          if (j > s && x == prev && hi == prev_hi) {
            wave_lds_sync();
            if (gl == 0) {
              s_pos[j] = s_pos[j - 1];
              if (op == kOpRange) s_cnt[j] = s_cnt[j - 1];
              if (op == kOpSuccessor) s_kq[j] = s_kq[j - 1];
            }
            continue;
          }
          prev = x;
          prev_hi = hi;
          if (op == kOpLookup) {
            int hit = -1;
#pragma unroll
            for (int k = 0; k < KH; ++k)
              if (gl * kpl + k < size && kv[u].k[k] == x) hit = k;
            if (kHalf && full) {
#pragma unroll
              for (int k = KH; k < KPL; ++k)
                if (gl * kpl + k < size && kv[u].k[k] == x) hit = k;
            }
            u64 bal = wave_ballot(hit >= 0) & gmask;
            if (bal == 0) {
              if (gl == 0) s_pos[j] = (lb << 16) | kPosMiss;
            } else if (hit >= 0) {
              s_pos[j] = (lb << 16) | (gl * kpl + (u32)hit);
            }
          } else {
            // Lower bound of x (and upper bound of hi for ranges).  The
            // node is sorted and lane l holds positions [l*kpl, l*kpl+kpl),
            // so the lanes whose first key is below x form a prefix of L
            // lanes and the bound lies in lane L-1: one ballot over first
            // keys plus that lane's own count.
            // A predecessor needs the upper bound of x itself.
            const bool v0 = gl * kpl < size;
            const K ub = (op == kOpRange) ? hi : x;
            const bool need_ub = op == kOpRange || op == kOpPredecessor;
            u32 c_lt = 0, c_le = 0;
#pragma unroll
            for (int k = 0; k < KH; ++k) {
              const bool v = gl * kpl + k < size;
              c_lt += (v && kv[u].k[k] < x) ? 1u : 0u;
              if (need_ub) c_le += (v && kv[u].k[k] <= ub) ? 1u : 0u;
            }
            if (kHalf && full) {
#pragma unroll
              for (int k = KH; k < KPL; ++k) {
                const bool v = gl * kpl + k < size;
                c_lt += (v && kv[u].k[k] < x) ? 1u : 0u;
                if (need_ub) c_le += (v && kv[u].k[k] <= ub) ? 1u : 0u;
              }
            }
            u32 lt = 0;
            K skey = K(0);
            if (op != kOpPredecessor) {
              const u32 L1 = (u32)__popcll(wave_ballot(v0 && kv[u].k[0] < x) & gmask);
              const u32 s_lt = (u32)__shfl((int)c_lt, (int)(gbase + (L1 ? L1 - 1 : 0)), 64);
              lt = L1 ? (L1 - 1) * kpl + s_lt : 0u;
              if (op == kOpSuccessor) {
                // the key at lt: this lane's first slot >= x, taken from lane
                // L1-1, or from lane L1's first slot when lane L1-1 holds
                // nothing >= x
                K cand = kv[u].k[0];
#pragma unroll
                for (int k = 1; k < KH; ++k)
                  if (c_lt == (u32)k) cand = kv[u].k[k];
                if (kHalf && full) {
#pragma unroll
                  for (int k = KH; k < KPL; ++k)
                    if (c_lt == (u32)k) cand = kv[u].k[k];
                }
                const u32 src = L1 == 0 ? 0u : (s_lt < kpl ? L1 - 1 : L1);
                skey = shfl_key(cand, gbase + src);
              }
            }
            u32 le = 0;
            if (need_ub) {
              const u32 L2 = (u32)__popcll(wave_ballot(v0 && kv[u].k[0] <= ub) & gmask);
              const u32 s_le = (u32)__shfl((int)c_le, (int)(gbase + (L2 ? L2 - 1 : 0)), 64);
              le = L2 ? (L2 - 1) * kpl + s_le : 0u;
            }
            if (gl == 0) {
              u32 code;
              if (op == kOpSuccessor) {
                code = lt < size ? lt : kPosNext;   // past the node: next bucket
                if (lt < size) s_kq[j] = skey;   // the answer's key replaces the query
              } else if (op == kOpPredecessor) {
                code = le > 0 ? le - 1 : kPosSlow;   // none in this node: look before it
              } else {
                if (x > hi) {
                  code = 0;
                  s_cnt[j] = 0;
                } else if (le < size) {
                  code = lt;
                  s_cnt[j] = le > lt ? le - lt : 0u;
                } else {
                  code = kPosNext;   // every key from lt on is in the range
                  s_cnt[j] = lt | (size << 16);
                }
              }
              s_pos[j] = (lb << 16) | code;
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // Phase B: one lane per key.  Lookups, successors and predecessors resolved
  // in phase A issue all of a thread's value (and key) loads before its
  // output writes.
  const K NF = key_max<K>();
  const bool with_key = op == kOpSuccessor || op == kOpPredecessor;
  if (op != kOpRange) {
    K rv[RQ], rk[RQ];
    u32 pc[RQ];
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      pc[r] = j < nq ? s_pos[j] : kPosSlow;
      u32 pos = pc[r] & 0xFFFFu;
      rv[r] = NF;
      rk[r] = NF;
      if (pos < kPosNext) {
        const u64 at = (u64)(b0 + (pc[r] >> 16)) * a.cap + pos;
        // a value is read once, from a random line: a non-temporal load
        // leaves the cache to the lines that are reused (read kernel in the
        // store step 86 -> 83 us; non-temporal output stores were slower)
        rv[r] = __builtin_nontemporal_load(&a.nvals[at]);
        if (op == kOpSuccessor) rk[r] = s_q[j];
        else if (with_key) rk[r] = a.nkeys[at];
      }
    }
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      const u32 pos = pc[r] & 0xFFFFu;
      if (pos != kPosSlow && pos != kPosNext) {
        const u32 orig = s_idx[j];
        a.out_v[orig] = rv[r];
        if (with_key) a.out_k[orig] = rk[r];
      }
    }
  }
  for (u32 j = tid; j < nq; j += NT) {
    const u32 code = s_pos[j];
    const u32 lb = code >> 16;
    const u32 pos = code & 0xFFFFu;
    u32 b = b0 + lb;
    const u32 orig = s_idx[j];
    const K x = s_q[j];
    if (pos != kPosSlow && pos != kPosNext) {
      if (op != kOpRange) continue;   // written above
      const u32 cnt = s_cnt[j];
      const u32 wn = cnt < a.maxpq ? cnt : a.maxpq;
      copy_results<K>(a, (u64)b * a.cap + pos, wn, (u64)orig * a.maxpq);
      a.counts[orig] = cnt;
      continue;
    }
    if (op == kOpPredecessor) {
      bool bad = false;
      const u64 at = predecessor_slot<K>(a.hdr, a.nkeys, occ_levels(a.occ, a.nb), a.pool, a.cap, b, x, &bad);
      if (bad) atomicCAS(a.err, 0u, kErrInternal);
      a.out_k[orig] = at == ~0ull ? K(0) : a.nkeys[at];
      a.out_v[orig] = at == ~0ull ? NF : a.nvals[at];
      continue;
    }
    NodeHdr h;
    u32 node, p;
    bool all_in = false;   // range: every key from p to the node's end is in it
    if (pos == kPosNext) {
      // single-node bucket, resolved up to its node's end in phase A
      node = b;
      h.fence = 0;
      h.next = kNil;
      if (op == kOpRange) {
        const u32 c = s_cnt[j];
        p = c & 0xFFFFu;
        h.size = c >> 16;
        all_in = true;
      } else {
        p = 0;
        h.size = 0;   // successor: nothing left in this node
      }
    } else {
      // Global-memory path: walk the chain to the node holding x.
      node = locate_node(a.hdr, a.pool, b, (u64)x, &h);
      if (node == kBadLink) {
        atomicCAS(a.err, 0u, kErrInternal);
        if (op == kOpRange) a.counts[orig] = 0;
        else a.out_v[orig] = NF;
        if (op == kOpSuccessor) a.out_k[orig] = NF;
        continue;
      }
      p = lower_bound_idx<K>(a.nkeys + (u64)node * a.cap, 0u, h.size, x);
    }
    const K* keys = a.nkeys + (u64)node * a.cap;
    if (op == kOpLookup) {
      a.out_v[orig] = (p < h.size && keys[p] == x) ? a.nvals[(u64)node * a.cap + p] : NF;
    } else if (op == kOpSuccessor) {
      K rk = NF, rv = NF;
      if (p < h.size) {
        rk = keys[p];
        rv = a.nvals[(u64)node * a.cap + p];
      } else {
        NodeHdr g;
        u32 nn = next_nonempty(a.hdr, occ_levels(a.occ, a.nb), a.nb, a.pool, &b, h, &g);
        if (nn == kBadLink) {
          atomicCAS(a.err, 0u, kErrInternal);
        } else if (nn != kNil) {
          rk = a.nkeys[(u64)nn * a.cap];
          rv = a.nvals[(u64)nn * a.cap];
        }
      }
      a.out_k[orig] = rk;
      a.out_v[orig] = rv;
    } else {
      const K hi = s_hi[j];
      u32 cnt = 0;
      bool handed = false;
      if (x <= hi) {
        const u64 ob = (u64)orig * a.maxpq;
        while (true) {
          // more than kLaneRangeMax results in this node: a wave copies them
          u32 lim = h.size;
          if (v.list_cap && p + kLaneRangeMax < h.size) {
            if (all_in || keys[p + kLaneRangeMax] <= hi) {
              const u32 li = atomicAdd(v.nlist, 1u);
              if (li < v.list_cap) {
                v.list[li] = j;
                v.lnode[li] = node;
                v.lbk[li] = b;
                s_pos[j] = p;
                s_cnt[j] = cnt;
                handed = true;
                break;
              }
            } else {
              lim = p + kLaneRangeMax;   // keys[lim] > hi: the range ends before lim
            }
          }
          const u32 ub = all_in ? h.size : upper_bound_idx<K>(keys, p, lim, hi);
          all_in = false;
          if (cnt < a.maxpq) {
            const u32 room = a.maxpq - cnt;
            copy_results<K>(a, (u64)node * a.cap + p, ub - p < room ? ub - p : room, ob + cnt);
          }
          cnt += ub - p;
          if (ub < h.size) break;
          NodeHdr g;
          u32 nn = next_nonempty(a.hdr, occ_levels(a.occ, a.nb), a.nb, a.pool, &b, h, &g);
          if (nn == kBadLink) {
            atomicCAS(a.err, 0u, kErrInternal);
            break;
          }
          if (nn == kNil) break;
          node = nn;
          h = g;
          keys = a.nkeys + (u64)node * a.cap;
          p = 0;
        }
      }
      if (!handed) a.counts[orig] = cnt;
    }
  }
  if (op == kOpRange && v.list_cap) range_waves<K, NT>(a, v);
}

// One share (workgroup-sized unit) of a read batch; `vb` is the share index.
template <typename K, int NT, int S, int GL, int KPL, int U>
__device__ __forceinline__ void read_share(const ReadArgs<K>& a, int op, u32 vb,
                                           ReadSmem<K, S, NT>& sm) {
  static_assert(NT == 256, "merge-path search assumes 256 threads");
  constexpr int NG = NT / GL;
  K* s_q = sm.q;
  K* s_hi = sm.hi;
  u32* s_idx = sm.idx;
  u32* s_pos = sm.pos;
  u32* s_cnt = sm.cnt;
  K* s_mk = sm.mk;
  u32* s_e = sm.e;
  u32* s_hw = sm.hw;
  unsigned short* s_tl = sm.tl;
  u32* s_tmp = sm.tmp;
  u32* s_lo = sm.lo;
  u32* s_hiw = sm.hiw;
  u32* s_wc = sm.wc;
  u32* s_cut = sm.cut;
  u32& s_ntouch = sm.ntouch;

  const u32 tid = threadIdx.x;
  const u64 total = (u64)a.m + a.nb;
  u64 d[2];
  d[0] = (u64)vb * a.share;
  d[1] = d[0] + a.share < total ? d[0] + a.share : total;
  if (a.cuts) {
    if (tid < 2) s_cut[tid] = a.cuts[vb + tid];
    __syncthreads();
  } else {
    coop_merge_path<K>(a.skeys, a.m, a.mkba, a.nb, d, s_lo, s_hiw, s_wc, s_cut);
  }
  const u32 q0 = s_cut[0], q1 = s_cut[1];
  // Cuts of a sorted batch are ordered; anything else (an unsorted batch)
  // is reported instead of indexing past the share.
  if (q1 < q0 || q1 > a.m || d[0] < q0 || d[1] < q1 || d[0] - q0 > d[1] - q1 ||
      d[1] - q1 > a.nb) {
    if (tid == 0) atomicCAS(a.err, 0u, kErrInternal);
    return;
  }
  const u32 b0 = (u32)(d[0] - q0), b1 = (u32)(d[1] - q1);
  const u32 nq = q1 - q0;
  if (nq == 0) return;
  const u32 nbl = b1 - b0;

  // One round of coalesced loads: a share holds at most S keys and S + 1
  // bucket entries, and every load of a thread is issued before its first
  // LDS store (range upper bounds follow, indexed by the input positions).
  constexpr u32 RQ = (S + NT - 1) / NT;
  constexpr u32 RBK = (S + 1 + NT - 1) / NT;
  {
    K qk[RQ];
    u32 qi[RQ];
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      if (j < nq) {
        qk[r] = a.skeys[q0 + j];
        qi[r] = a.sidx[q0 + j];
      }
    }
    K mk[RBK];
    u64 hw[RBK];   // size | next << 32 of the bucket's head node
#pragma unroll
    for (u32 r = 0; r < RBK; ++r) {
      const u32 i = tid + r * NT;
      hw[r] = (u64)kNil << 32;
      if (i < nbl) mk[r] = a.mkba[b0 + i];
      if (i <= nbl && b0 + i < a.nb)
        hw[r] = *reinterpret_cast<const u64*>(&a.hdr[b0 + i].size);
    }
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      if (j < nq) {
        s_q[j] = qk[r];
        s_idx[j] = qi[r];
        if (op == kOpRange) s_hi[j] = a.hi[qi[r]];
      }
    }
#pragma unroll
    for (u32 r = 0; r < RBK; ++r) {
      const u32 i = tid + r * NT;
      if (i <= nbl) {
        if (i < nbl) s_mk[i] = mk[r];
        s_hw[i] = (u32)hw[r] | ((u32)(hw[r] >> 32) != kNil ? kChainBit : 0u);
      }
    }
  }
  __syncthreads();

  // Bound search: every bucket pulls its slice; compact the touched buckets.
  constexpr u32 PER = (S + 1 + NT - 1) / NT;
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    u32 lb = tid * PER + r;
    if (lb <= nbl) {
      u32 e = (lb < nbl) ? upper_bound_idx<K>(s_q, 0u, nq, s_mk[lb]) : nq;
      s_e[lb] = e;
    }
  }
  __syncthreads();
  // The touched buckets are listed by slice length (one key, two keys,
  // more), so the lane groups of a wave, which step through their buckets'
  // slices together, mostly hold slices of one length.
  static_assert(S + 1 < 1024, "class counts are packed in 10 bits");
  u32 flags = 0, packed = 0;
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    u32 lb = tid * PER + r;
    if (lb <= nbl) {
      const u32 s = lb ? s_e[lb - 1] : 0u;
      const u32 len = s_e[lb] - s;
      if (len > 0) {
        const u32 c = len < 3u ? len - 1u : 2u;
        flags |= (c + 1u) << (2u * r);
        packed += 1u << (10u * c);
      }
    }
  }
  u32 tot;
  const u32 ex = block_exclusive_scan<NT>(packed, s_tmp, &tot);
  const u32 t0 = tot & 1023u, t1 = (tot >> 10) & 1023u, t2 = tot >> 20;
  u32 w0 = ex & 1023u, w1 = t0 + ((ex >> 10) & 1023u), w2 = t0 + t1 + (ex >> 20);
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    const u32 c = (flags >> (2u * r)) & 3u;
    const unsigned short lb = (unsigned short)(tid * PER + r);
    if (c == 1u) s_tl[w0++] = lb;
    else if (c == 2u) s_tl[w1++] = lb;
    else if (c == 3u) s_tl[w2++] = lb;
  }
  const u32 ntot = t0 + t1 + t2;
  if (tid == 0) s_ntouch = ntot;
  __syncthreads();
  const u32 ntouch = s_ntouch;

  SliceView<K> v;
  v.q = s_q;
  v.hi = s_hi;
  v.idx = s_idx;
  v.pos = s_pos;
  v.cnt = s_cnt;
  v.e = s_e;
  v.hw = s_hw;
  v.tl = s_tl;
  // the maxBucket entries are no longer needed: their room lists the ranges
  // that continue past their node
  v.list = reinterpret_cast<u32*>(s_mk);
  v.list_cap = S;
  v.nlist = &sm.nslow;
  v.lnode = s_e;    // phase A is done with the slice ends and head words
  v.lbk = s_hw;     // when phase B hands ranges over
  if (tid == 0) sm.nslow = 0;
  resolve_slices<K, NT, GL, KPL, U, RQ>(a, op, v, b0, nq, ntouch);
}

// Eight waves per SIMD (64 VGPRs): the kernel is latency-bound, and the
// register budget, not LDS, otherwise caps it at six workgroups per CU.  One
// instantiation per operation: the paths of the other operations are compiled
// out, which keeps the register and scalar-register budget for the one that
// runs.
template <typename K, int NT, int S, int GL, int KPL, int U, int OP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_read_apply2(
    ReadArgs<K> a) {
  __shared__ ReadSmem<K, S, NT> sm;
  read_share<K, NT, S, GL, KPL, U>(a, OP, blockIdx.x, sm);
}

}  // namespace flix
