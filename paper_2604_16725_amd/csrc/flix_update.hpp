// Update batches: insert (merge + split) and delete (compaction + node
// reclamation), in the flipped form of Section 4.1: each bucket pulls its
// slice of the sorted update list and applies it to its node chain.
//
// Pipeline per update batch (all on the caller's stream):
//   sort (stable, key+value for inserts, keys only for deletes)
//   k_slices   merge-path shares over MKBA (+) batch; every bucket with a
//              non-empty slice is appended to the work list.  For inserts it
//              also counts live keys (last of each equal-key run), rejects the
//              reserved value and sums an upper bound of the nodes the batch
//              may take from the free list.
//   k_insert_apply / k_delete_apply
//              a group of GL lanes per work item (bucket).  Inserts first check
//              the node budget against the free-list height captured before
//              the kernel, so a batch that could run out of nodes is rejected
//              as a whole before any node is touched.
#pragma once

#include "flix_device.hpp"
#include "flix_occ.hpp"
#include "flix_read.hpp"

namespace flix {

// Work item: bucket and its slice [s, e) of the sorted batch, plus the head
// node's size with kSingleNode set when the bucket is that one node.
struct alignas(16) WorkItem {
  u32 b, s, e, head;
};
constexpr u32 kSingleNode = 0x80000000u;

// Delete items for the workgroup-wide delete (k_delete_wide): a slice of at
// least `wide_min` keys, or at least kWideDelKeys keys into a chain of at
// least kWideDelChain nodes.  The slice kernel sets kWideItem in their head
// word and lists them; the lane-group delete skips them.
constexpr u32 kWideDelChain = 8;
constexpr u32 kWideDelKeys = 16;
constexpr u32 kWideItem = 0x40000000u;

__device__ __forceinline__ bool wide_delete_item(u32 len, u32 chain_nodes, u32 wide_min) {
  return wide_min != 0 &&
         (len >= wide_min || (chain_nodes >= kWideDelChain && len >= kWideDelKeys));
}

template <typename K>
struct SliceArgs {
  const K* skeys;
  const K* svals;   // inserts only
  u32 m;
  const K* mkba;
  u32 nb;
  const NodeHdr* hdr;
  const u32* bnodes;
  u32 cap;
  u32 share;
  WorkItem* work;   // [work_slots(max_batch)]
  u32 rcap;         // work_region_cap(max_batch)
  Ctl* ctl;
  u32 wide_min = 0; // > 0: items with at least this many keys are also
                    // listed for the workgroup-wide insert kernel
  u32 wide_cap = 0;
  WorkItem* wide = nullptr;   // [wide_cap]
};

template <typename K, int S, int NT>
struct SliceSmem {
  K q[S + 1];
  K mk[S];
  u32 e[S + 1];
  u32 live[S + 1];   // exclusive prefix of live flags
  u32 tmp[NT / 64 + 1];
  u32 part[4];
  u32 lo[2], hiw[2], wc[4];
  u32 wbase;
  unsigned long long need;
  u32 bad;
  u32 gstart;
};

template <typename K, int NT, int S, bool INSERT>
__device__ void slices_share(const SliceArgs<K>& a, u32 vb, SliceSmem<K, S, NT>& sm) {
  K* s_q = sm.q;
  K* s_mk = sm.mk;
  u32* s_e = sm.e;
  u32* s_live = sm.live;
  u32* s_tmp = sm.tmp;
  u32* s_part = sm.part;
  u32& s_wbase = sm.wbase;
  unsigned long long& s_need = sm.need;
  u32& s_bad = sm.bad;
  u32& s_gstart = sm.gstart;

  static_assert(NT == 256, "the cooperative cut uses 256 threads");
  const u32 tid = threadIdx.x;
  const u64 total = (u64)a.m + a.nb;
  const u64 d0 = (u64)vb * a.share;
  const u64 d1 = d0 + a.share < total ? d0 + a.share : total;
  if (vb == 0 && tid == 0) a.ctl->free_snapshot = a.ctl->free_top;
  if (tid == 0) {
    s_need = 0;
    s_bad = 0;
  }
  {
    const u64 dd[2] = {d0, d1};
    u32* cut = s_part;   // cut[0] = q0, cut[1] = q1
    coop_merge_path<K>(a.skeys, a.m, a.mkba, a.nb, dd, sm.lo, sm.hiw, sm.wc, cut);
  }
  if (tid == 0) {
    s_part[2] = (u32)(d0 - s_part[0]);
    s_part[3] = (u32)(d1 - s_part[1]);
  }
  __syncthreads();
  // cuts of a sorted batch are ordered; report anything else instead of
  // indexing past the share
  if (s_part[1] < s_part[0] || s_part[3] < s_part[2] || s_part[3] > a.nb) {
    if (tid == 0) atomicCAS(&a.ctl->status, 0u, kErrInternal);
    __syncthreads();
    return;
  }
  const u32 q0 = s_part[0], q1 = s_part[1];
  const u32 b0 = s_part[2], b1 = s_part[3];
  const u32 nq = q1 - q0;
  const u32 nbl = b1 - b0;
  // A bucket is emitted by the share that holds its maxBucket entry, with its
  // whole slice; only local bucket 0 can have keys in earlier shares.
  if (nbl == 0) {
    __syncthreads();
    return;
  }
  // Slice start of local bucket 0: the keys of skeys[0, q0) above
  // MKBA[b0 - 1] form a suffix.  The first wave probes the 64 keys below q0
  // (lane l takes q0 - 1 - l) in the same round as the loads below; a longer
  // suffix falls back to a binary search under the probed window.
  if (tid < 64) {
    u32 g = 0;
    if (b0 != 0) {
      const K x = a.mkba[b0 - 1];
      const bool in = tid < q0;
      const K kk = in ? a.skeys[q0 - 1 - tid] : K(0);
      const u32 n_gt = (u32)__popcll(wave_ballot(in && kk > x));
      g = q0 - n_gt;
      if (n_gt == 64 && q0 > 64 && tid == 0) g = upper_bound_idx<K>(a.skeys, 0u, q0 - 64, x);
    }
    if (tid == 0) s_gstart = g;
  }
  {
    // every load of a thread is issued before its first LDS store (the
    // share holds at most S keys plus the one after it, and S buckets)
    constexpr u32 RQ = (S + 1 + NT - 1) / NT;
    constexpr u32 RM = (S + NT - 1) / NT;
    K qk[RQ], mk[RM];
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      if (j <= nq && (j < nq || q0 + j < a.m)) qk[r] = a.skeys[q0 + j];
    }
#pragma unroll
    for (u32 r = 0; r < RM; ++r) {
      const u32 i = tid + r * NT;
      if (i < nbl) mk[r] = a.mkba[b0 + i];
    }
#pragma unroll
    for (u32 r = 0; r < RQ; ++r) {
      const u32 j = tid + r * NT;
      if (j <= nq && (j < nq || q0 + j < a.m)) s_q[j] = qk[r];
    }
#pragma unroll
    for (u32 r = 0; r < RM; ++r) {
      const u32 i = tid + r * NT;
      if (i < nbl) s_mk[i] = mk[r];
    }
  }
  __syncthreads();
  for (u32 lb = tid; lb <= nbl; lb += NT)
    s_e[lb] = (lb < nbl) ? upper_bound_idx<K>(s_q, 0u, nq, s_mk[lb]) : nq;

  if (INSERT) {
    // live flags (last of each equal-key run in the whole batch) -> prefix
    constexpr u32 PER = (S + NT - 1) / NT;
    u32 f[PER];
    u32 sum = 0;
    bool bad = false;
#pragma unroll
    for (u32 r = 0; r < PER; ++r) {
      u32 j = tid * PER + r;
      u32 live = 0;
      if (j < nq) {
        bool last = (q0 + j + 1 == a.m) || (s_q[j] != s_q[j + 1]);
        live = last ? 1u : 0u;
        if (a.svals[q0 + j] == key_max<K>()) bad = true;
      }
      f[r] = live;
      sum += live;
    }
    if (bad) s_bad = 1;
    u32 tot;
    u32 ex = block_exclusive_scan<NT>(sum, s_tmp, &tot);
#pragma unroll
    for (u32 r = 0; r < PER; ++r) {
      u32 j = tid * PER + r;
      if (j < nq) s_live[j] = ex;
      ex += f[r];
    }
    if (tid == 0) s_live[nq] = tot;
  }
  __syncthreads();

  // Append touched buckets to the work list (one atomic per workgroup, on
  // the counter of this share's region).
  // Local bucket lb < nbl has the global slice [q0 + s, q0 + e), except that
  // bucket 0 starts at gstart (<= q0).  Local bucket nbl is left to the next
  // share.
  const u32 gstart = s_gstart;
  constexpr u32 PERB = (S + NT - 1) / NT;
  u32 cnt = 0;
  unsigned long long need = 0;
  u32 info[PERB];   // head size | kSingleNode, passed to the apply kernel
#pragma unroll
  for (u32 r = 0; r < PERB; ++r) {
    u32 lb = tid * PERB + r;
    info[r] = 0;
    if (lb < nbl) {
      u32 s = lb ? q0 + s_e[lb - 1] : gstart;
      u32 e = q0 + s_e[lb];
      if (e > s) {
        ++cnt;
        const u32 b = b0 + lb;
        const NodeHdr h = a.hdr[b];
        const bool single = h.next == kNil;
        info[r] = h.size | (single ? kSingleNode : 0u);
        // a long slice or a long chain goes to the workgroup-wide delete
        if (!INSERT && a.wide_min &&
            wide_delete_item(e - s, single ? 1u : a.bnodes[b], a.wide_min))
          info[r] |= kWideItem;
        if (INSERT) {
          // live keys inside this share, plus (bucket 0 only) every key before
          // q0 counted as live: an upper bound is all the budget needs
          u32 sl = lb ? s_e[lb - 1] : 0u;
          u32 t = s_live[e - q0] - s_live[sl] + (lb ? 0u : q0 - gstart);
          u32 f = a.cap / 2;
          if (single) {
            u64 c = (u64)h.size + t;
            if (c > a.cap) need += c / f - 1;
          } else {
            u32 bn = a.bnodes[b];
            need += (u64)(bn < t ? bn : t) + t / f;
          }
        }
      }
    }
  }
  u32 tot_items;
  u32 ex = block_exclusive_scan<NT>(cnt, s_tmp, &tot_items);
  if (INSERT && need) atomicAdd(&s_need, need);
  if (tid == 0 && tot_items) {
    // claim slots in this share's region (consecutive shares share a region,
    // so the list stays in bucket order); a claim that does not fit records
    // where the region's valid items end and goes to the overflow region
    const u32 nsh = (u32)((total + a.share - 1) / a.share);
    const u32 spr = (nsh + kWorkRegions - 1) / kWorkRegions;
    const u32 r = vb / spr;
    const u32 old = atomicAdd(&a.ctl->wreg[r][0], tot_items);
    if ((u64)old + tot_items <= a.rcap) {
      s_wbase = r * a.rcap + old;
    } else {
      atomicMin(&a.ctl->wreg[r][1], old);
      s_wbase = kWorkRegions * a.rcap + atomicAdd(&a.ctl->work_ovf, tot_items);
    }
  }
  __syncthreads();
  u32 w = s_wbase + ex;
#pragma unroll
  for (u32 r = 0; r < PERB; ++r) {
    u32 lb = tid * PERB + r;
    if (lb < nbl) {
      u32 s = lb ? q0 + s_e[lb - 1] : gstart;
      u32 e = q0 + s_e[lb];
      if (e > s) {
        WorkItem it;
        it.b = b0 + lb;
        it.s = s;
        it.e = e;
        it.head = info[r];
        a.work[w++] = it;
        if (INSERT ? (a.wide_min && e - s >= a.wide_min) : (it.head & kWideItem) != 0) {
          const u32 k = atomicAdd(&a.ctl->wide_n, 1u);
          if (k < a.wide_cap) a.wide[k] = it;
          else atomicCAS(&a.ctl->status, 0u, kErrInternal);   // bound violated: never expected
        }
      }
    }
  }
  if (INSERT && tid == 0) {
    if (s_need) atomicAdd((unsigned long long*)&a.ctl->need, s_need);
    if (s_bad) atomicExch(&a.ctl->call_err, kErrInval);
  }
  __syncthreads();
}

template <typename K, int NT, int S, bool INSERT>
__global__ __launch_bounds__(NT) void k_slices(SliceArgs<K> a) {
  __shared__ SliceSmem<K, S, NT> sm;
  slices_share<K, NT, S, INSERT>(a, blockIdx.x, sm);
}

// ---------------------------------------------------------------------------
// Lane groups: GL consecutive lanes of a wave cooperate on one bucket.  All
// lanes of a group follow the same control flow; groups of one wave may
// diverge, so group code never uses workgroup barriers.
// ---------------------------------------------------------------------------
template <int GL>
struct Group {
  u32 lane;   // lane index inside the group
  u32 gbase;  // wave lane of the group's lane 0
  u64 gmask;  // wave-positioned mask of the group's lanes
  __device__ __forceinline__ Group() {
    u32 wl = lane_id();
    lane = wl % GL;
    gbase = wl - lane;
    gmask = (GL == 64) ? ~0ull : (((1ull << GL) - 1ull) << gbase);
  }
  __device__ __forceinline__ u64 ballot(bool p) const { return wave_ballot(p) & gmask; }
  __device__ __forceinline__ u32 count(bool p) const { return (u32)__popcll(ballot(p)); }
  __device__ __forceinline__ u32 rank(bool p) const { return rank_below(ballot(p)); }
  template <typename T>
  __device__ __forceinline__ T bcast(T v, u32 src) const {
    return __shfl(v, (int)(gbase + src), 64);
  }
};

// Re-reads of node data that the same wave wrote earlier in this kernel.  The
// writer and the reader are lanes of one wave, so a workgroup-scope fence
// between them is enough; these loads are workgroup-scope atomics so the
// compiler can neither cache nor reorder them across that fence.
template <typename K>
__device__ __forceinline__ K ld_fresh(const K* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ NodeHdr ld_hdr(const NodeHdr* p, bool fresh) {
  if (!fresh) return *p;
  NodeHdr h;
  const u64* q = reinterpret_cast<const u64*>(p);
  h.fence = ld_fresh(q);
  u64 w = ld_fresh(q + 1);
  h.size = (u32)w;
  h.next = (u32)(w >> 32);
  return h;
}

// Copy n consecutive items (keys and values) into LDS: every lane issues up
// to four loads before the first LDS store, so one round trip covers 4*GL
// items.  `fresh` marks data this wave wrote earlier in the kernel.
template <typename K, int GL>
__device__ __forceinline__ void stage_items(K* dk, K* dv, const K* sk, const K* sv, u32 n,
                                            u32 lane, bool fresh) {
  for (u32 i0 = 0; i0 < n; i0 += 4 * GL) {
    K kk[4], vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const u32 i = i0 + r * GL + lane;
      if (i < n) {
        kk[r] = fresh ? ld_fresh(sk + i) : sk[i];
        vv[r] = fresh ? ld_fresh(sv + i) : sv[i];
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const u32 i = i0 + r * GL + lane;
      if (i < n) {
        dk[i] = kk[r];
        dv[i] = vv[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Insert kernel choice.  The work list of an insert call can be split between
// the single-lane kernel (k_insert_st) and the lane-group kernel
// (k_insert_apply):
//   kSelAll     every item
//   kSelShort   items whose slice holds at most `st_max` batch keys
//   kSelLong    the other items
//   kSelRound   every item when the call averages at most `st_max` batch keys
//               per touched bucket, else none
//   kSelRoundL  the complement of kSelRound
// ---------------------------------------------------------------------------
constexpr u32 kSelAll = 0, kSelShort = 1, kSelLong = 2, kSelRound = 3, kSelRoundL = 4;

__device__ __forceinline__ bool sel_takes(u32 sel, u32 st_max, u32 len, u32 m, u32 nitems) {
  switch (sel) {
    case kSelShort: return len <= st_max;
    case kSelLong: return len > st_max;
    case kSelRound: return (u64)m <= (u64)st_max * nitems;
    case kSelRoundL: return (u64)m > (u64)st_max * nitems;
    default: return true;
  }
}

template <typename K>
struct UpdArgs {
  const K* mkba;
  const K* skeys;
  const K* svals;
  u32 m;
  NodeHdr* hdr;
  K* nkeys;
  K* nvals;
  u32* bnodes;
  u32* free_ids;
  u32 cap;
  u32 chunk;          // batch items staged per merge step (<= per-group LDS room)
  u32 pool;           // node pool size
  const WorkItem* work;
  u32 rcap;           // work_region_cap(max_batch)
  Ctl* ctl;
  u32* status;        // sticky status word (== &ctl->status)
  OccLevels occ;      // bucket occupancy summary, kept current here
  u32 sel = 0;        // insert kernels: which work items this launch takes (kSel*)
  u32 st_max = 0;     // slice-length threshold of the kernel choice
  u32 wide_min = 0;   // > 0: buckets with at least this many batch keys in
                      // their slice belong to the workgroup-wide insert kernel
  u32 wide_cap = 0;
  const WorkItem* wide = nullptr;   // those items, listed by the slice kernel
};

// Work items of the workgroup-wide insert kernel (k_insert_wide).
__device__ __forceinline__ bool is_wide(u32 wide_min, const WorkItem& w) {
  return wide_min != 0 && w.e - w.s >= wide_min;
}

// Workgroup-shared state of the apply kernels: a key counter and the map of
// the work list's regions.
struct UpdShared {
  unsigned long long counter;
  u32 pre[kWorkRegions + 1];
};

// Header write that leaves the fence alone when the caller never loaded it.
__device__ __forceinline__ void write_hdr(NodeHdr* p, const NodeHdr& h, bool with_fence) {
  if (with_fence) {
    *p = h;
  } else {
    p->size = h.size;
    p->next = h.next;
  }
}

// Position of merged item `pos` among k pieces of c items: piece p covers
// [floor(p*c/k), floor((p+1)*c/k)).
__device__ __forceinline__ u32 piece_start(u32 p, u32 c, u32 k) {
  return (u32)(((u64)p * c) / k);
}
__device__ __forceinline__ u32 piece_of(u32 pos, u32 c, u32 k) {
  u32 p = (u32)(((u64)pos * k) / c);
  if (p + 1 < k && piece_start(p + 1, c, k) <= pos) ++p;
  return p;
}

// ---------------------------------------------------------------------------
// Insert (Section 4.3.2 TL-Bulk, re-expressed for wave64 + LDS): for the node
// X whose range holds the next batch keys, the group stages X's keys and a
// chunk of at most `chunk` batch items (deduplicated: last of each equal-key
// run), computes every item's merged position by binary search in LDS (equal
// keys: the batch pair replaces the stored one), and writes the result back.
// If the merged count c exceeds the capacity, X splits (Section 5.3.1) into
// k = floor(c / (cap/2)) pieces of near-equal size; pieces 1..k-1 come from
// the free list and are linked after X; every piece but the last is fenced by
// its last key and the last one keeps X's fence and link.
// ---------------------------------------------------------------------------
// Insert work of workgroup `blk` of `nblk` (groups stride over the work list).
// `s_dyn`: per-group LDS regions; `sh`: workgroup-shared counter and work map.
template <typename K, int GL, int NT>
__device__ void insert_items(const UpdArgs<K>& a, u32 lds_items, u32 blk, u32 nblk,
                             unsigned char* s_dyn, UpdShared& sh) {
  unsigned long long& s_added = sh.counter;
  constexpr int GPB = NT / GL;
  Group<GL> g;
  const u32 gid = threadIdx.x / GL;
  K* gk = reinterpret_cast<K*>(s_dyn) + (size_t)gid * 2 * lds_items;  // keys region
  K* gv = gk + lds_items;                                               // values region
  K* ak = gk;                  // node keys   [cap]
  K* av = gv;
  K* bk = gk + a.cap;          // batch chunk [chunk]
  K* bv = gv + a.cap;
  if (threadIdx.x == 0) s_added = 0;
  __syncthreads();
  const Ctl* ctl = a.ctl;
  bool abort_all = ctl->call_err != 0 || ctl->need > ctl->free_snapshot || ctl->call_abort != 0;
  if (abort_all) {
    if (blk == 0 && threadIdx.x == 0 && ctl->call_err == 0)
      atomicCAS(a.status, 0u, kErrNomem);
    if (blk == 0 && threadIdx.x == 0 && ctl->call_err != 0)
      atomicCAS(a.status, 0u, ctl->call_err);
    __syncthreads();
    return;
  }
  const u32 nitems = load_work_map(ctl, sh.pre);
  // a call-level choice that gives this kernel nothing ends it here (uniform)
  if ((a.sel == kSelRound || a.sel == kSelRoundL) && !sel_takes(a.sel, a.st_max, 0u, a.m, nitems))
    return;
  const u32 f = a.cap / 2;
  u64 added = 0;
  const u32 stride = nblk * GPB;
  u32 it = blk * GPB + gid;
  WorkItem wnext;
  WorkCursor cur;
  cur.seek(sh.pre, it);
  if (it < nitems) wnext = a.work[cur.slot(it, a.rcap)];
  for (; it < nitems; it += stride) {
    const WorkItem w = wnext;
    if (it + stride < nitems) {   // prefetch
      cur.move(sh.pre, it + stride);
      wnext = a.work[cur.slot(it + stride, a.rcap)];
    }
    if (!sel_takes(a.sel, a.st_max, w.e - w.s, a.m, nitems) || is_wide(a.wide_min, w)) continue;
    u32 X = w.b;
    NodeHdr hX;
    bool fence_known = true;
    if (w.head & kSingleNode) {   // single-node bucket: header from the work item
      hX.size = w.head & ~kSingleNode;
      hX.next = kNil;
      hX.fence = 0;
      fence_known = false;
    } else {
      hX = a.hdr[X];
    }
    bool fresh = false;   // this group has written nodes of this bucket: read coherently
    u32 j = w.s;
    u32 nodes_added = 0;
    const u64 added_before = added;
    const bool was_empty = (w.head & kSingleNode) && (w.head & ~kSingleNode) == 0;
    while (j < w.e) {
      bool broken = false;
      if (hX.next != kNil) {   // chain: walk to the node holding skeys[j]
        const K first = a.skeys[j];
        while ((u64)first > hX.fence) {
          if (hX.next >= a.pool) { broken = true; break; }   // end of chain, or a bad link
          X = hX.next;
          hX = ld_hdr(a.hdr + X, fresh);
        }
      }
      if (broken || hX.size > a.cap) {   // never on a consistent store
        if (g.lane == 0) atomicCAS(a.status, 0u, kErrInternal);
        break;
      }
      // the last node of a chain holds every remaining key of the slice
      u32 j2 = (hX.next == kNil) ? w.e : upper_bound_idx<K>(a.skeys, j, w.e, (K)hX.fence);
      if (j2 - j > a.chunk) j2 = j + a.chunk;
      const u32 sa = hX.size;
      // One round trip for the node and the chunk: the node's first 4*GL
      // items are loaded into registers before the chunk is staged (keeping
      // the last item of each equal-key run), then written to LDS.
      const K* nsk = a.nkeys + (u64)X * a.cap;
      const K* nsv = a.nvals + (u64)X * a.cap;
      const u32 first = sa < 4u * GL ? sa : 4u * GL;
      K nk[4], nv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const u32 i = r * GL + g.lane;
        if (i < first) {
          nk[r] = fresh ? ld_fresh(nsk + i) : nsk[i];
          nv[r] = fresh ? ld_fresh(nsv + i) : nsv[i];
        }
      }
      u32 tb = 0;
      for (u32 base = j; base < j2; base += GL) {
        u32 idx = base + g.lane;
        bool in = idx < j2;
        K kk = K(0), kn = K(0), vv = K(0);
        if (in) {
          kk = a.skeys[idx];
          vv = a.svals[idx];
          if (idx + 1 < a.m) kn = a.skeys[idx + 1];
        }
        bool live = in && (idx + 1 == a.m || kn != kk);
        u32 r = g.rank(live);
        if (live) {
          bk[tb + r] = kk;
          bv[tb + r] = vv;
        }
        tb += g.count(live);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const u32 i = r * GL + g.lane;
        if (i < first) {
          ak[i] = nk[r];
          av[i] = nv[r];
        }
      }
      if (sa > first)
        stage_items<K, GL>(ak + first, av + first, nsk + first, nsv + first, sa - first, g.lane,
                           fresh);
      wave_lds_sync();
      if (tb == 0) {   // only shadowed duplicates in this chunk
        j = j2;
        continue;
      }
      // Node items below the chunk's smallest key neither move nor meet a
      // chunk key: the duplicate scan starts at the group-aligned run that
      // holds the first node key >= bk[0].  When the whole node is in the
      // registers and node plus chunk fit it, the merge cannot split it: the
      // first key >= bk[0] is counted by ballots, the duplicate scan is
      // skipped (the merged count follows from the move below) and the node
      // items move from the registers.
      const bool fast = first == sa && sa + tb <= a.cap;
      u32 f0 = 0;
      if (fast) {
        const K c0 = bk[0];
#pragma unroll
        for (int r = 0; r < 4; ++r) f0 += g.count((u32)r * GL + g.lane < sa && nk[r] < c0);
      } else {
        f0 = lower_bound_idx<K>(ak, 0u, sa, bk[0]);
      }
      const u32 i_lo = f0 - f0 % GL;
      // duplicates between node and chunk
      u32 dd = 0;
      if (!fast) {
        for (u32 i0 = i_lo; i0 < sa; i0 += GL) {
          u32 i = i0 + g.lane;
          bool drop = false;
          if (i < sa) {
            u32 p = lower_bound_idx<K>(bk, 0u, tb, ak[i]);
            drop = p < tb && bk[p] == ak[i];
          }
          dd += g.count(drop);
        }
      }
      u32 c = sa + tb - dd;   // fast: an upper bound until the move has counted duplicates
      u32 k = 1;
      u32 base_id = 0;
      if (c > a.cap) {
        if (!fence_known) {   // a single node's fence is its bucket's maxBucket
          hX.fence = (u64)a.mkba[w.b];
          fence_known = true;
        }
        k = c / f;
        if (g.lane == 0) base_id = atomicSub(&a.ctl->free_top, k - 1);
        base_id = g.bcast(base_id, 0);
        if (base_id < k - 1 || base_id > a.pool) {   // budget bound violated: never expected
          if (g.lane == 0) atomicCAS(a.status, 0u, kErrInternal);
          break;
        }
        nodes_added += k - 1;
      }
      if (k == 1) {
        // No split: the merge stays in X.  Node items from the first moving
        // one are shifted right by the chunk keys below them (less the
        // duplicates before them); chunk items land at their merged rank.
        K* const xk = a.nkeys + (u64)X * a.cap;
        K* const xv = a.nvals + (u64)X * a.cap;
        u32 drop_before = 0;
        if (fast) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if ((u32)r * GL < i_lo || (u32)r * GL >= sa) continue;   // uniform in the group
            const u32 i = (u32)r * GL + g.lane;
            bool drop = false;
            u32 pos = 0;
            if (i < sa) {
              const u32 p = lower_bound_idx<K>(bk, 0u, tb, nk[r]);
              drop = p < tb && bk[p] == nk[r];
              pos = i - (drop_before + g.rank(drop)) + p;
            }
            drop_before += g.count(drop);
            if (i < sa && !drop && pos != i) {
              xk[pos] = nk[r];
              xv[pos] = nv[r];
            }
          }
          c = sa + tb - drop_before;
        } else {
          for (u32 i0 = i_lo; i0 < sa; i0 += GL) {
            const u32 i = i0 + g.lane;
            bool drop = false;
            u32 pos = 0;
            K kk = K(0), vv = K(0);
            if (i < sa) {
              kk = ak[i];
              vv = av[i];
              const u32 p = lower_bound_idx<K>(bk, 0u, tb, kk);
              drop = p < tb && bk[p] == kk;
              pos = i - (drop_before + g.rank(drop)) + p;
            }
            drop_before += g.count(drop);
            if (i < sa && !drop && pos != i) {
              xk[pos] = kk;
              xv[pos] = vv;
            }
          }
        }
        u32 match_before = 0;
        for (u32 j0 = 0; j0 < tb; j0 += GL) {
          const u32 jj = j0 + g.lane;
          bool match = false;
          u32 pos = 0;
          K kk = K(0), vv = K(0);
          if (jj < tb) {
            kk = bk[jj];
            vv = bv[jj];
            const u32 p = lower_bound_idx<K>(ak, 0u, sa, kk);
            match = p < sa && ak[p] == kk;
            pos = jj + p - (match_before + g.rank(match));
          }
          match_before += g.count(match);
          if (jj < tb) {
            xk[pos] = kk;
            xv[pos] = vv;
          }
        }
        added += c - sa;
        if (g.lane == 0) a.hdr[X].size = c;
        hX.size = c;
        j = j2;
        if (j < w.e) {
          fresh = true;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        }
        wave_lds_sync();
        continue;
      }
      // node id of piece p: X for p == 0, free_ids[base_id - p] otherwise
      // write node items
      u32 drop_before = 0;
      for (u32 i0 = 0; i0 < sa; i0 += GL) {
        u32 i = i0 + g.lane;
        bool drop = false;
        u32 pos = 0;
        K kk = K(0), vv = K(0);
        if (i < sa) {
          kk = ak[i];
          vv = av[i];
          u32 p = lower_bound_idx<K>(bk, 0u, tb, kk);
          drop = p < tb && bk[p] == kk;
          pos = i - (drop_before + g.rank(drop)) + p;
        }
        drop_before += g.count(drop);
        if (i < sa && !drop && !(k == 1 && pos == i)) {   // an item that keeps its slot stays
          u32 pc = (k == 1) ? 0u : piece_of(pos, c, k);
          u32 node = pc == 0 ? X : a.free_ids[base_id - pc];
          if (node >= a.pool) {   // a free-stack entry outside the pool: never expected
            atomicCAS(a.status, 0u, kErrInternal);
            continue;
          }
          u32 slot = (k == 1) ? pos : pos - piece_start(pc, c, k);
          a.nkeys[(u64)node * a.cap + slot] = kk;
          a.nvals[(u64)node * a.cap + slot] = vv;
          if (k > 1 && pc + 1 < k && slot + 1 == piece_start(pc + 1, c, k) - piece_start(pc, c, k))
            a.hdr[node].fence = (u64)kk;
        }
      }
      // write chunk items
      u32 match_before = 0;
      for (u32 j0 = 0; j0 < tb; j0 += GL) {
        u32 jj = j0 + g.lane;
        bool match = false;
        u32 pos = 0;
        K kk = K(0), vv = K(0);
        if (jj < tb) {
          kk = bk[jj];
          vv = bv[jj];
          u32 p = lower_bound_idx<K>(ak, 0u, sa, kk);
          match = p < sa && ak[p] == kk;
          pos = jj + p - (match_before + g.rank(match));
        }
        match_before += g.count(match);
        if (jj < tb) {
          u32 pc = (k == 1) ? 0u : piece_of(pos, c, k);
          u32 node = pc == 0 ? X : a.free_ids[base_id - pc];
          if (node >= a.pool) {
            atomicCAS(a.status, 0u, kErrInternal);
            continue;
          }
          u32 slot = (k == 1) ? pos : pos - piece_start(pc, c, k);
          a.nkeys[(u64)node * a.cap + slot] = kk;
          a.nvals[(u64)node * a.cap + slot] = vv;
          if (k > 1 && pc + 1 < k && slot + 1 == piece_start(pc + 1, c, k) - piece_start(pc, c, k))
            a.hdr[node].fence = (u64)kk;
        }
      }
      added += c - sa;
      // headers: size and link of every piece; the last keeps X's fence/link
      if (k == 1) {
        if (g.lane == 0) a.hdr[X].size = c;
        hX.size = c;
      } else {
        for (u32 p = g.lane; p < k; p += GL) {
          u32 node = p == 0 ? X : a.free_ids[base_id - p];
          if (node >= a.pool) {
            atomicCAS(a.status, 0u, kErrInternal);
            continue;
          }
          u32 sz = piece_start(p + 1, c, k) - piece_start(p, c, k);
          a.hdr[node].size = sz;
          a.hdr[node].next = (p + 1 < k) ? a.free_ids[base_id - (p + 1)] : hX.next;
          if (p + 1 == k) a.hdr[node].fence = hX.fence;
        }
      }
      j = j2;
      if (j < w.e) {
        // More keys for this bucket: they may fall into any piece, so the walk
        // continues from piece 0 (X), reading what this wave just wrote.
        fresh = true;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (k > 1) {
          hX = ld_hdr(a.hdr + X, true);
          fence_known = true;
        }
      }
      wave_lds_sync();
    }
    if (nodes_added && g.lane == 0) a.bnodes[w.b] += nodes_added;
    if (was_empty && added > added_before && g.lane == 0) occ_set(a.occ, w.b);
  }
  // per-lane `added` is identical across a group's lanes: count once per group
  if (g.lane == 0 && added) atomicAdd(&s_added, added);
  __syncthreads();
  if (threadIdx.x == 0 && s_added) atomicAdd((unsigned long long*)&a.ctl->nkeys, s_added);
  __syncthreads();
}

// Five waves per SIMD for 32-bit keys (85 VGPRs, no spills): the register
// path of a node that fits the registers needs more than the 80 registers of
// six waves, which spilled and was 6% slower; 64-bit keys take what they need.
template <typename K, int GL, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(sizeof(K) == 4 ? 5 : 1))) void k_insert_apply(
    UpdArgs<K> a, u32 lds_items) {
  extern __shared__ unsigned char s_dyn[];
  __shared__ UpdShared sh;
  insert_items<K, GL, NT>(a, lds_items, blockIdx.x, gridDim.x, s_dyn, sh);
}

// ---------------------------------------------------------------------------
// ST-Shift-Right insert (Section 4.2.1): one lane owns one bucket.  For every
// live batch key of its slice (last of each equal-key run), in ascending
// order, the lane walks the chain to the node whose fence covers the key,
// binary-searches the node: an equal key takes the new value; otherwise the
// keys from the insertion point on shift right by one slot and the pair is
// written.  A full node first splits into two halves (left half floor(c/2),
// Section 5.3.1): the right half goes to a node popped from the free list and
// linked after it, the left node is fenced by its last key, the right one
// inherits the old fence and link.  The lane's own writes are re-read only by
// the same lane, so program order keeps them visible.
// ---------------------------------------------------------------------------
template <typename K>
__device__ void st_insert_bucket(const UpdArgs<K>& a, const WorkItem& w, u64& added) {
  u32 X = w.b;
  NodeHdr hX;
  if (w.head & kSingleNode) {
    hX.size = w.head & ~kSingleNode;
    hX.next = kNil;
    hX.fence = (u64)a.mkba[w.b];
  } else {
    hX = a.hdr[X];
  }
  const bool was_empty = (w.head & kSingleNode) && (w.head & ~kSingleNode) == 0;
  const u64 added_before = added;
  u32 nodes_added = 0;
  for (u32 j = w.s; j < w.e; ++j) {
    const K k = a.skeys[j];
    if (j + 1 < a.m && a.skeys[j + 1] == k) continue;   // a later pair of the key wins
    const K v = a.svals[j];
    // the slice is ascending, so the walk only moves forward
    bool broken = false;
    while ((u64)k > hX.fence) {
      if (hX.next >= a.pool) { broken = true; break; }
      X = hX.next;
      hX = a.hdr[X];
    }
    if (broken || hX.size > a.cap) {
      atomicCAS(a.status, 0u, kErrInternal);
      break;
    }
    K* xk = a.nkeys + (u64)X * a.cap;
    K* xv = a.nvals + (u64)X * a.cap;
    u32 p = lower_bound_idx<K>(xk, 0u, hX.size, k);
    if (p < hX.size && xk[p] == k) {   // upsert in place
      xv[p] = v;
      continue;
    }
    if (hX.size == a.cap) {
      // split into halves; the new node takes the right one
      const u32 top = atomicSub(&a.ctl->free_top, 1u);
      if (top == 0 || top > a.pool) {   // budget bound violated: never expected
        atomicCAS(a.status, 0u, kErrInternal);
        break;
      }
      const u32 Y = a.free_ids[top - 1];
      if (Y >= a.pool) {
        atomicCAS(a.status, 0u, kErrInternal);
        break;
      }
      const u32 h = a.cap / 2;
      K* yk = a.nkeys + (u64)Y * a.cap;
      K* yv = a.nvals + (u64)Y * a.cap;
      for (u32 i = h; i < a.cap; ++i) {
        yk[i - h] = xk[i];
        yv[i - h] = xv[i];
      }
      NodeHdr hY;
      hY.fence = hX.fence;
      hY.size = a.cap - h;
      hY.next = hX.next;
      a.hdr[Y] = hY;
      hX.fence = (u64)xk[h - 1];
      hX.size = h;
      hX.next = Y;
      a.hdr[X] = hX;
      ++nodes_added;
      if ((u64)k > hX.fence) {   // the key belongs to the right half
        X = Y;
        hX = hY;
        xk = yk;
        xv = yv;
        p -= h;
      }
    }
    for (u32 i = hX.size; i > p; --i) {
      xk[i] = xk[i - 1];
      xv[i] = xv[i - 1];
    }
    xk[p] = k;
    xv[p] = v;
    ++hX.size;
    a.hdr[X].size = hX.size;
    ++added;
  }
  if (nodes_added) a.bnodes[w.b] += nodes_added;
  if (was_empty && added > added_before) occ_set(a.occ, w.b);
}

// One lane per work item taken by `sel`; the node budget was checked by the
// slice kernel's bound exactly as for the lane-group kernel (a split-produced
// node holds at least cap/2 keys, so the same per-bucket bound holds).
template <typename K, int NT>
__global__ __launch_bounds__(NT) void k_insert_st(UpdArgs<K> a) {
  __shared__ UpdShared sh;
  if (threadIdx.x == 0) sh.counter = 0;
  __syncthreads();
  const Ctl* ctl = a.ctl;
  if (ctl->call_err != 0 || ctl->need > ctl->free_snapshot || ctl->call_abort != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      atomicCAS(a.status, 0u, ctl->call_err != 0 ? ctl->call_err : kErrNomem);
    return;
  }
  const u32 nitems = load_work_map(ctl, sh.pre);
  if ((a.sel == kSelRound || a.sel == kSelRoundL) && !sel_takes(a.sel, a.st_max, 0u, a.m, nitems))
    return;
  u64 added = 0;
  const u32 stride = gridDim.x * NT;
  u32 it = blockIdx.x * NT + threadIdx.x;
  WorkCursor cur;
  cur.seek(sh.pre, it);
  for (; it < nitems; it += stride) {
    cur.move(sh.pre, it);
    const WorkItem w = a.work[cur.slot(it, a.rcap)];
    if (!sel_takes(a.sel, a.st_max, w.e - w.s, a.m, nitems)) continue;
    st_insert_bucket<K>(a, w, added);
  }
  for (int off = 32; off > 0; off >>= 1) added += __shfl_xor(added, off, 64);
  if ((threadIdx.x & 63u) == 0 && added) atomicAdd(&sh.counter, added);
  __syncthreads();
  if (threadIdx.x == 0 && sh.counter) atomicAdd((unsigned long long*)&a.ctl->nkeys, sh.counter);
}

// ---------------------------------------------------------------------------
// Workgroup-wide insert (elastic compute for a hot bucket, Section 3.4): a
// bucket whose slice holds at least `wide_min` batch keys (a dense run of new
// keys) is merged by a whole workgroup instead of one lane group walking the
// slice in node-sized chunks.  Node by node along the chain, the node X whose
// range holds the next slice keys is staged in LDS (keys A[0, S)); every live
// slice key of its part (last of its equal-key run) and every kept node key
// gets its merged position from counts, so all of them are written in
// parallel:
//   pos(live slice key k) = rank of k among live slice keys
//                           + #{node keys < k} - #{dropped node keys < k}
//   pos(node key i)       = i - #{dropped node keys before i}
//                           + #{live slice keys < A[i]}
// where a node key is dropped when a live slice key equals it (the batch pair
// replaces it).  The c merged pairs form k = max(1, floor(c / (cap/2))) pieces
// of near-equal size (the split rule of the lane-group kernel); pieces 1..k-1
// come from the free list and are chained after X, the last piece keeps X's
// fence and link.  The node budget bound of the slice kernel covers the new
// nodes: floor((S + t) / (cap/2)) - 1 for a single-node bucket, and for a
// chain at most one more than t_X / (cap/2) per touched node X, which sums to
// within min(chain length, t) + t / (cap/2).
// ---------------------------------------------------------------------------
template <typename K>
struct WideLds {
  K ak[256], av[256];       // staged node
  u32 cnt[257];             // live slice keys by lower bound in the node
  u32 eq[257];              // node key i is replaced by a slice key
  u32 qinc[257];            // inclusive prefix of cnt
  u32 dropx[257];           // exclusive prefix of eq
  u32 tmp[8];
  u32 live_total, match_total;
  u32 base_id;
  u32 bad;
};

// Merge node X (header hX) with the slice part [s0, s0 + t) of the sorted
// batch, all of whose keys lie in X's range.  Returns the pieces made.
template <typename K, int NT>
__device__ u32 wide_merge_node(const UpdArgs<K>& a, const WorkItem& w, u32 X, const NodeHdr& hX,
                               u32 s0, u32 t, WideLds<K>& L, unsigned long long& added_total) {
  const u32 tid = threadIdx.x, lane = tid & 63u;
  const u32 f = a.cap / 2;
  const u32 S = hX.size;
  K* const xk = a.nkeys + (u64)X * a.cap;
  K* const xv = a.nvals + (u64)X * a.cap;
  for (u32 i = tid; i < S; i += NT) {
    L.ak[i] = xk[i];
    L.av[i] = xv[i];
  }
  for (u32 i = tid; i <= S; i += NT) {
    L.cnt[i] = 0;
    L.eq[i] = 0;
  }
  if (tid == 0) {
    L.live_total = 0;
    L.match_total = 0;
    L.bad = 0;
  }
  __syncthreads();
  // 1. counts: live keys by lower bound in the node (wave-aggregated: the
  //    slice is sorted, so a wave's lower bounds form runs), matches
  u32 my_live = 0, my_match = 0;
  for (u32 j0 = 0; j0 < t; j0 += NT) {
    const u32 j = j0 + tid;
    const bool valid = j < t;
    K k = K(0);
    bool live = false;
    u32 lb = 0;
    if (valid) {
      const u32 g = s0 + j;
      k = a.skeys[g];
      live = (g + 1 == a.m) || a.skeys[g + 1] != k;
      lb = lower_bound_idx<K>(L.ak, 0u, S, k);
      if (live && lb < S && L.ak[lb] == k) {
        L.eq[lb] = 1;
        ++my_match;
      }
    }
    my_live += live ? 1u : 0u;
    const u64 live_m = wave_ballot(live);
    const u32 lb_next = (u32)__shfl_down((int)lb, 1, 64);
    const bool valid_next = lane < 63 && j + 1 < t;
    const bool seg_end = valid && (!valid_next || lb_next != lb);
    const u64 end_m = wave_ballot(seg_end);
    if (seg_end) {
      const u64 below = end_m & ((1ull << lane) - 1ull);
      const u32 first = below ? 64u - (u32)__clzll(below) : 0u;   // one past the previous end
      const u64 span = (lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull)) & ~((1ull << first) - 1ull);
      const u32 c = (u32)__popcll(live_m & span);
      if (c) atomicAdd(&L.cnt[lb], c);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    my_live += __shfl_xor(my_live, off, 64);
    my_match += __shfl_xor(my_match, off, 64);
  }
  if (lane == 0) {
    if (my_live) atomicAdd(&L.live_total, my_live);
    if (my_match) atomicAdd(&L.match_total, my_match);
  }
  __syncthreads();
  // prefixes over the node positions (at most 257 entries, one thread)
  if (tid == 0) {
    u32 q = 0, d = 0;
    for (u32 i = 0; i <= S; ++i) {
      q += L.cnt[i];
      L.qinc[i] = q;
      L.dropx[i] = d;
      d += L.eq[i];
    }
  }
  __syncthreads();
  const u32 c = S + L.live_total - L.match_total;
  const u32 k = c > a.cap ? c / f : 1u;
  if (k > 1) {
    if (tid == 0) {
      const u32 top = atomicSub(&a.ctl->free_top, k - 1);
      L.base_id = top;
      if (top < k - 1 || top > a.pool) {   // budget bound violated: never expected
        atomicCAS(a.status, 0u, kErrInternal);
        L.bad = 1;
      }
    }
    __syncthreads();
    if (L.bad) return 0;
  }
  const u32 base_id = k > 1 ? L.base_id : 0u;
  const u64 fence_last = hX.fence;
  auto node_of = [&](u32 p) -> u32 { return p == 0 ? X : a.free_ids[base_id - p]; };
  auto put = [&](u32 pos, K kk, K vv) {
    const u32 pc = (k == 1) ? 0u : piece_of(pos, c, k);
    const u32 node = node_of(pc);
    if (node >= a.pool) {
      atomicCAS(a.status, 0u, kErrInternal);
      return;
    }
    const u32 slot = (k == 1) ? pos : pos - piece_start(pc, c, k);
    a.nkeys[(u64)node * a.cap + slot] = kk;
    a.nvals[(u64)node * a.cap + slot] = vv;
    if (k > 1 && pc + 1 < k && slot + 1 == piece_start(pc + 1, c, k) - piece_start(pc, c, k))
      a.hdr[node].fence = (u64)kk;
  };
  // 2. kept node keys
  for (u32 i = tid; i < S; i += NT) {
    if (L.eq[i]) continue;
    const u32 q = L.qinc[i];   // live keys with lower bound <= i; none equals A[i]
    put(i - L.dropx[i] + q, L.ak[i], L.av[i]);
  }
  // 3. live slice keys, ranked by a running block scan
  u32 run = 0;
  for (u32 j0 = 0; j0 < t; j0 += NT) {
    const u32 j = j0 + tid;
    bool live = false;
    K kk = K(0);
    if (j < t) {
      const u32 g = s0 + j;
      kk = a.skeys[g];
      live = (g + 1 == a.m) || a.skeys[g + 1] != kk;
    }
    u32 tot;
    const u32 r = block_exclusive_scan<NT>(live ? 1u : 0u, L.tmp, &tot);
    if (live) {
      const u32 lb = lower_bound_idx<K>(L.ak, 0u, S, kk);
      put(run + r + lb - L.dropx[lb], kk, a.svals[s0 + j]);
    }
    run += tot;
  }
  // 4. headers: sizes and links of the pieces; the last keeps the fence
  for (u32 p = tid; p < k; p += NT) {
    const u32 node = node_of(p);
    if (node >= a.pool) {
      atomicCAS(a.status, 0u, kErrInternal);
      continue;
    }
    a.hdr[node].size = piece_start(p + 1, c, k) - piece_start(p, c, k);
    a.hdr[node].next = (p + 1 < k) ? node_of(p + 1) : hX.next;
    if (p + 1 == k) a.hdr[node].fence = fence_last;
  }
  if (tid == 0) {
    if (k > 1) a.bnodes[w.b] += k - 1;
    if (S == 0 && c > 0 && X == w.b && hX.next == kNil) occ_set(a.occ, w.b);
    added_total += c - S;
  }
  __syncthreads();   // LDS is reused by the next node or item
  return k;
}

// A bucket's slice, node by node along its chain: every node whose range holds
// keys of the slice is merged with them by the whole workgroup.  A dense run
// of new keys lies between two stored keys, so it usually meets one node.
template <typename K, int NT>
__device__ void wide_insert_bucket(const UpdArgs<K>& a, const WorkItem& w, WideLds<K>& L,
                                   unsigned long long& added_total) {
  __shared__ u32 s_node, s_j2;
  __shared__ NodeHdr s_h;
  u32 j = w.s;
  if (threadIdx.x == 0) {
    s_node = w.b;
    s_h = a.hdr[w.b];
  }
  __syncthreads();
  while (j < w.e) {
    if (threadIdx.x == 0) {
      // walk to the node whose range holds skeys[j]; its part of the slice
      // ends after its fence (the last node takes the rest)
      u32 X = s_node;
      NodeHdr h = s_h;
      const K first = a.skeys[j];
      u32 steps = 0;
      while ((u64)first > h.fence && h.next != kNil) {
        if (h.next >= a.pool || ++steps > a.pool) {   // never on a consistent store
          atomicCAS(a.status, 0u, kErrInternal);
          X = kNil;
          break;
        }
        X = h.next;
        h = a.hdr[X];
      }
      s_node = X;
      s_h = h;
      s_j2 = (X == kNil) ? w.e
             : (h.next == kNil) ? w.e : upper_bound_idx<K>(a.skeys, j, w.e, (K)h.fence);
      if (X != kNil && h.size > a.cap) {
        atomicCAS(a.status, 0u, kErrInternal);
        s_node = kNil;
      }
    }
    __syncthreads();
    const u32 X = s_node;
    const NodeHdr h = s_h;
    const u32 j2 = s_j2;
    __syncthreads();
    if (X == kNil) return;
    if (j2 > j) wide_merge_node<K, NT>(a, w, X, h, j, j2 - j, L, added_total);
    j = j2;
    if (j < w.e && threadIdx.x == 0) {
      // continue after the pieces, at the node that followed X
      if (h.next == kNil || h.next >= a.pool) {
        atomicCAS(a.status, 0u, kErrInternal);
        s_node = kNil;
      } else {
        s_node = h.next;
        s_h = a.hdr[h.next];
      }
    }
    __syncthreads();
    if (s_node == kNil) return;
  }
}

// The slice kernel lists the wide items; workgroup g merges items g, g + G, ...
template <typename K, int NT>
__global__ __launch_bounds__(NT) void k_insert_wide(UpdArgs<K> a) {
  __shared__ WideLds<K> L;
  const Ctl* ctl = a.ctl;
  if (ctl->call_err != 0 || ctl->need > ctl->free_snapshot || ctl->call_abort != 0)
    return;   // the other kernels report it
  const u32 n = ctl->wide_n < a.wide_cap ? ctl->wide_n : a.wide_cap;
  unsigned long long added = 0;
  for (u32 i = blockIdx.x; i < n; i += gridDim.x) {
    const WorkItem w = a.wide[i];
    wide_insert_bucket<K, NT>(a, w, L, added);
  }
  if (threadIdx.x == 0 && added) atomicAdd((unsigned long long*)&a.ctl->nkeys, added);
}

// ---------------------------------------------------------------------------
// Delete (Section 4.4 TL-Bulk with compaction): for every node of the bucket's
// chain whose range meets the slice, the group stages the node, marks the
// keys present in the slice (binary search in the sorted batch), and moves
// each survivor left by the number of deletions before it (ballot + mbcnt).
// Structure upkeep along the walk: a node that can join its predecessor
// (sizes summing to at most cap/2, or an emptied head) is appended to it and
// returned to the free list; this also unlinks every emptied non-head node
// (Section 4.4 step 5).  The head node is never freed.
// ---------------------------------------------------------------------------
template <typename K, int GL, int NT>
__device__ void delete_items(const UpdArgs<K>& a, u32 lds_items, u32 blk, u32 nblk,
                             unsigned char* s_dyn, UpdShared& sh) {
  unsigned long long& s_removed = sh.counter;
  constexpr int GPB = NT / GL;
  Group<GL> g;
  const u32 gid = threadIdx.x / GL;
  K* ak = reinterpret_cast<K*>(s_dyn) + (size_t)gid * 2 * lds_items;   // node keys [cap]
  K* av = ak + lds_items;                                               // node values [cap]
  K* bk = ak + a.cap;                                                   // slice keys [chunk]
  if (threadIdx.x == 0) s_removed = 0;
  __syncthreads();
  if (a.ctl->call_abort != 0) return;   // an epoch rejected as a whole (uniform)
  const u32 nitems = load_work_map(a.ctl, sh.pre);
  const u32 f = a.cap / 2;
  u64 removed = 0;
  const u32 stride = nblk * GPB;
  u32 it = blk * GPB + gid;
  WorkItem wnext;
  WorkCursor cur;
  cur.seek(sh.pre, it);
  if (it < nitems) wnext = a.work[cur.slot(it, a.rcap)];
  for (; it < nitems; it += stride) {
    const WorkItem w = wnext;
    if (it + stride < nitems) {   // prefetch
      cur.move(sh.pre, it + stride);
      wnext = a.work[cur.slot(it + stride, a.rcap)];
    }
    if (w.head & kWideItem) continue;   // k_delete_wide takes it
    // predecessor state (P), kept in registers; P == kNil before the head
    u32 P = kNil;
    NodeHdr hP;
    hP.fence = 0; hP.size = 0; hP.next = kNil;
    bool p_dirty = false;
    bool p_is_head = false;
    bool p_fence_known = true;
    u32 X = w.b;
    NodeHdr hX;
    bool x_fence_known = true;
    if (w.head & kSingleNode) {   // single-node bucket: header from the work item
      hX.size = w.head & ~kSingleNode;
      hX.next = kNil;
      hX.fence = 0;
      x_fence_known = false;
    } else {
      hX = a.hdr[X];
    }
    u32 j = w.s;
    int freed = 0;
    const bool was_empty = (w.head & kSingleNode) && (w.head & ~kSingleNode) == 0;
    while (true) {
      // the last node of a chain takes every remaining key of the slice
      u32 j2 = (j >= w.e) ? j
               : (hX.next == kNil) ? w.e : upper_bound_idx<K>(a.skeys, j, w.e, (K)hX.fence);
      const bool touched = j2 > j;
      const bool join = (P != kNil) &&
                        ((hP.size + hX.size <= f) || (p_is_head && hP.size == 0));
      u32 sx = hX.size;
      if (sx > a.cap) {   // never on a consistent store
        if (g.lane == 0) atomicCAS(a.status, 0u, kErrInternal);
        break;
      }
      // the node's slice goes to LDS when it fits, else it is searched in place
      const bool slice_lds = touched && (j2 - j) <= a.chunk;
      // One round trip for the slice's first 4*GL keys and the node's first
      // NR*GL items (X's data has not been written by this kernel).  Five
      // rounds of registers cover a bulk-loaded node plus the keys a batch
      // just added (a fourth round left them to a second round trip; a sixth
      // costs a wave per SIMD).
      const bool stage_x = touched || join;
      const K* xsk = a.nkeys + (u64)X * a.cap;
      const K* xsv = a.nvals + (u64)X * a.cap;
      constexpr int NR = 5;
      const u32 first = stage_x ? (sx < (u32)NR * GL ? sx : (u32)NR * GL) : 0u;
      K nk[NR], nv[NR];
      if (slice_lds) {
        for (u32 i0 = j; i0 < j2; i0 += 4 * GL) {
          K kk[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            u32 i = i0 + r * GL + g.lane;
            if (i < j2) kk[r] = a.skeys[i];
          }
          if (i0 == j) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
              const u32 i = r * GL + g.lane;
              if (i < first) {
                nk[r] = xsk[i];
                nv[r] = xsv[i];
              }
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            u32 i = i0 + r * GL + g.lane;
            if (i < j2) bk[i - j] = kk[r];
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const u32 i = r * GL + g.lane;
          if (i < first) {
            nk[r] = xsk[i];
            nv[r] = xsv[i];
          }
        }
      }
      if (stage_x) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const u32 i = r * GL + g.lane;
          if (i < first) {
            ak[i] = nk[r];
            av[i] = nv[r];
          }
        }
        if (sx > first)
          stage_items<K, GL>(ak + first, av + first, xsk + first, xsv + first, sx - first, g.lane,
                             false);
        wave_lds_sync();
      }
      u32 first_gone = sx;   // slot of the first removed item: earlier slots stay
      if (touched) {
        // mark + compact in LDS (survivors only move left); node items below
        // the slice's smallest key survive in place, so the scan starts at
        // the group-aligned run holding the first key >= it
        const K smin = slice_lds ? bk[0] : a.skeys[j];
        const u32 f0 = lower_bound_idx<K>(ak, 0u, sx, smin);
        const u32 i_lo = f0 - f0 % GL;
        u32 kept = i_lo;
        for (u32 i0 = i_lo; i0 < sx; i0 += GL) {
          u32 i = i0 + g.lane;
          bool keep = false;
          K kk = K(0), vv = K(0);
          if (i < sx) {
            kk = ak[i];
            vv = av[i];
            if (slice_lds) {
              u32 p = lower_bound_idx<K>(bk, 0u, j2 - j, kk);
              keep = !(p < j2 - j && bk[p] == kk);
            } else {
              u32 p = lower_bound_idx<K>(a.skeys, j, j2, kk);
              keep = !(p < j2 && a.skeys[p] == kk);
            }
          }
          const u64 gone = g.ballot(i < sx && !keep);
          if (gone && first_gone == sx) first_gone = i0 + (u32)__builtin_ctzll(gone >> g.gbase);
          u32 dst = kept + g.rank(keep);
          kept += g.count(keep);
          if (keep) {
            ak[dst] = kk;
            av[dst] = vv;
          }
        }
        wave_lds_sync();
        removed += sx - kept;
        sx = kept;
      }
      const bool join2 = (P != kNil) &&
                         ((hP.size + sx <= f) || sx == 0 || (p_is_head && hP.size == 0));
      if (join2) {
        // append X's survivors to P, unlink X, free X
        for (u32 i = g.lane; i < sx; i += GL) {
          a.nkeys[(u64)P * a.cap + hP.size + i] = ak[i];
          a.nvals[(u64)P * a.cap + hP.size + i] = av[i];
        }
        hP.size += sx;
        hP.fence = hX.fence;
        hP.next = hX.next;
        p_dirty = true;
        p_fence_known = true;
        if (g.lane == 0) {
          u32 pos = atomicAdd(&a.ctl->free_top, 1u);
          if (pos < a.pool) a.free_ids[pos] = X;
          else atomicCAS(a.status, 0u, kErrInternal);   // more frees than nodes: never expected
        }
        ++freed;
      } else {
        if (touched) {
          for (u32 i = first_gone + g.lane; i < sx; i += GL) {
            a.nkeys[(u64)X * a.cap + i] = ak[i];
            a.nvals[(u64)X * a.cap + i] = av[i];
          }
          hX.size = sx;
        }
        if (P != kNil && p_dirty && g.lane == 0) write_hdr(a.hdr + P, hP, p_fence_known);
        P = X;
        hP = hX;
        p_dirty = touched;
        p_is_head = (X == w.b);
        p_fence_known = x_fence_known;
      }
      wave_lds_sync();
      j = j2;
      const u32 nxt = hP.next;   // next node after the current predecessor
      if (nxt == kNil) break;
      const bool more = j < w.e || (p_is_head && hP.size == 0) || (p_dirty && hP.size <= f);
      if (!more) break;
      if (nxt >= a.pool) {   // a link outside the pool: never expected
        if (g.lane == 0) atomicCAS(a.status, 0u, kErrInternal);
        break;
      }
      X = nxt;
      hX = a.hdr[X];
      x_fence_known = true;
    }
    if (P != kNil && p_dirty && g.lane == 0) write_hdr(a.hdr + P, hP, p_fence_known);
    if (freed && g.lane == 0) a.bnodes[w.b] -= (u32)freed;
    // the head stays the predecessor while it is empty, so an emptied bucket
    // ends with P at its head, size 0 and no link
    if (!was_empty && P == w.b && hP.size == 0 && hP.next == kNil && g.lane == 0)
      occ_clear(a.occ, w.b);
  }
  if (g.lane == 0 && removed) atomicAdd(&s_removed, removed);
  __syncthreads();
  if (threadIdx.x == 0 && s_removed)
    atomicAdd((unsigned long long*)&a.ctl->nkeys, (unsigned long long)(0ull - s_removed));
  __syncthreads();
}

template <typename K, int GL, int NT>
__global__ __launch_bounds__(NT) void k_delete_apply(UpdArgs<K> a, u32 lds_items) {
  extern __shared__ unsigned char s_dyn[];
  __shared__ UpdShared sh;
  delete_items<K, GL, NT>(a, lds_items, blockIdx.x, gridDim.x, s_dyn, sh);
}

// ---------------------------------------------------------------------------
// Workgroup-wide delete (elastic compute for a long chain, Section 3.4): the
// lane-group delete walks a chain node by node, staging, compacting and
// writing each touched node before it reads the next header, so a bucket
// whose chain holds hundreds of nodes (a dense run of inserts makes one) costs
// hundreds of dependent rounds.  Here one workgroup takes such a bucket:
//   1. one lane walks the headers (a window of up to kWideDelNodes nodes);
//   2. every slice key finds its node by its fence (binary search in LDS),
//      which gives each node its part of the slice;
//   3. the waves compact the touched nodes in parallel (a key of the node
//      that is in its part is removed; survivors move left);
//   4. one lane replays the structure rule of the lane-group delete over the
//      new sizes, in chain order (a node joins its predecessor when their
//      sizes sum to at most cap/2, when it is empty, or when the predecessor
//      is the emptied head; the walk ends once the slice is consumed and the
//      predecessor neither is the emptied head nor changed to at most cap/2),
//      writing headers as it goes;
//   5. the waves append every joined node's survivors to its predecessor and
//      the joined nodes go back to the free list.
// The result is the lane-group kernel's, node for node.
// ---------------------------------------------------------------------------
constexpr u32 kWideDelNodes = 512;     // nodes per window
constexpr u32 kWideDelStage = 256;     // slice keys a wave stages per node

constexpr int NTW = 256;   // threads of the wide delete kernel

template <typename K>
struct WideDelLds {
  u32 id[kWideDelNodes];
  u32 next[kWideDelNodes];
  u32 size[kWideDelNodes];      // before compaction, then after
  u32 cnt[kWideDelNodes + 1];   // slice keys per node, then where each node's part starts
  u32 dst[kWideDelNodes];       // node that takes this node's survivors (kNil: none)
  u32 off[kWideDelNodes];       // their first slot there
  u32 tl[kWideDelNodes];        // touched nodes of the window
  u32 jl[kWideDelNodes];        // joined nodes of the window, in chain order
  u64 fence[kWideDelNodes];
  u32 tmp[NTW / 64 + 1];
  u32 ntl;
  K stg[4][kWideDelStage];      // per wave: the part of the slice of its node
  u32 nw;                       // nodes in this window
  u32 j0;                       // slice position where this window's parts begin
  u32 cont;                     // node after the window (kNil: the chain ends in it)
  u32 stop;                     // the structure walk has ended
  u32 nfree;                    // nodes of this window returned to the free list
  u32 free_base;
  u32 bad;
  u32 removed;
  // predecessor, carried across windows
  u32 P, Psize, Pnext, Pdirty, Phead;
  u64 Pfence;
  u32 freed_total;
  u32 was_empty;
  u32 walked;                   // nodes walked so far
};

template <typename K, int NT>
__device__ void wide_delete_bucket(const UpdArgs<K>& a, const WorkItem& w, WideDelLds<K>& L) {
  static_assert(NT == 256, "four waves, one staging row each");
  const u32 tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  constexpr u32 NW = NT / 64;
  const u32 f = a.cap / 2;
  if (tid == 0) {
    L.cont = w.b;
    L.j0 = w.s;
    L.stop = 0;
    L.bad = 0;
    L.removed = 0;
    L.P = kNil;
    L.Psize = 0;
    L.Pnext = kNil;
    L.Pdirty = 0;
    L.Phead = 0;
    L.Pfence = 0;
    L.freed_total = 0;
    L.was_empty = 0;
    L.walked = 0;
  }
  __syncthreads();
  while (true) {
    // 1. walk the next window of the chain (one lane)
    if (tid == 0) {
      u32 X = L.cont;
      u32 nw = 0;
      while (X != kNil && nw < kWideDelNodes) {
        // a link outside the pool, or a chain longer than the pool (a
        // cycle): never on a consistent store
        if (X >= a.pool || ++L.walked > a.pool) {
          L.bad = 1;
          break;
        }
        const NodeHdr h = a.hdr[X];
        if (h.size > a.cap) {
          L.bad = 1;
          break;
        }
        L.id[nw] = X;
        L.next[nw] = h.next;
        L.size[nw] = h.size;
        L.fence[nw] = h.fence;
        ++nw;
        X = h.next;
      }
      L.nw = nw;
      L.cont = X;
      if (L.bad) atomicCAS(a.status, 0u, kErrInternal);
      if (L.P == kNil && nw > 0) L.was_empty = (L.size[0] == 0 && L.next[0] == kNil) ? 1u : 0u;
    }
    for (u32 i = tid; i <= kWideDelNodes; i += NT) L.cnt[i] = 0;
    __syncthreads();
    if (L.bad) return;
    const u32 nw = L.nw;
    const u32 j0 = L.j0;
    const bool last_window = L.cont == kNil;
    // 2. the node of every slice key from j0 on: the first node of the window
    //    whose fence is >= the key; the chain's last node takes the rest;
    //    keys past this window's last fence belong to later windows
    for (u32 j = j0 + tid; j < w.e; j += NT) {
      const K k = a.skeys[j];
      u32 lo = 0, hi = nw;
      while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (L.fence[mid] < (u64)k) lo = mid + 1; else hi = mid;
      }
      if (lo == nw && last_window) lo = nw - 1;
      if (lo < nw) atomicAdd(&L.cnt[lo], 1u);
    }
    if (tid == 0) L.ntl = 0;
    __syncthreads();
    {
      // where every node's part starts (two nodes per thread), and the list
      // of touched nodes
      static_assert(kWideDelNodes == 2 * NT, "two window nodes per thread");
      const u32 c0 = 2 * tid < nw ? L.cnt[2 * tid] : 0u;
      const u32 c1 = 2 * tid + 1 < nw ? L.cnt[2 * tid + 1] : 0u;
      u32 total;
      const u32 ex = block_exclusive_scan<NT>(c0 + c1, L.tmp, &total);
      if (2 * tid < nw) {
        L.cnt[2 * tid] = j0 + ex;
        if (c0) L.tl[atomicAdd(&L.ntl, 1u)] = 2 * tid;
      }
      if (2 * tid + 1 < nw) {
        L.cnt[2 * tid + 1] = j0 + ex + c0;
        if (c1) L.tl[atomicAdd(&L.ntl, 1u)] = 2 * tid + 1;
      }
      if (tid == 0) L.cnt[nw] = j0 + total;
    }
    __syncthreads();
    // 3. compaction of the touched nodes, one wave per node
    u32 removed = 0;
    const u32 ntl = L.ntl;
    for (u32 ti = wv; ti < ntl; ti += NW) {
      const u32 i = L.tl[ti];
      const u32 s = L.cnt[i], e = L.cnt[i + 1];
      const u32 X = L.id[i];
      const u32 S = L.size[i];
      const u32 t = e - s;
      const bool staged = t <= kWideDelStage;
      if (staged)
        for (u32 q = lane; q < t; q += 64) L.stg[wv][q] = a.skeys[s + q];
      wave_lds_sync();
      K* const xk = a.nkeys + (u64)X * a.cap;
      K* const xv = a.nvals + (u64)X * a.cap;
      u32 kept = 0;
      for (u32 i0 = 0; i0 < S; i0 += 64) {
        const u32 p = i0 + lane;
        bool keep = false;
        K kk = K(0), vv = K(0);
        if (p < S) {
          kk = xk[p];
          vv = xv[p];
          u32 q;
          if (staged) {
            q = lower_bound_idx<K>(L.stg[wv], 0u, t, kk);
            keep = !(q < t && L.stg[wv][q] == kk);
          } else {
            q = lower_bound_idx<K>(a.skeys, s, e, kk);
            keep = !(q < e && a.skeys[q] == kk);
          }
        }
        const u64 km = wave_ballot(keep);
        const u32 dstp = kept + rank_below(km);
        // survivors only move left, and every load of this step is complete
        // before its stores (they use the loaded values)
        if (keep && dstp != p) {
          xk[dstp] = kk;
          xv[dstp] = vv;
        }
        kept += (u32)__popcll(km);
      }
      if (lane == 0) L.size[i] = kept;
      removed += S - kept;
    }
    if (lane == 0 && removed) atomicAdd(&L.removed, removed);
    __syncthreads();
    // 4. the structure rule in chain order, from the carried predecessor
    if (tid == 0) {
      u32 P = L.P, Psize = L.Psize, Pnext = L.Pnext, Pdirty = L.Pdirty, Phead = L.Phead;
      u64 Pfence = L.Pfence;
      u32 nfree = 0;
      u32 i = 0;
      bool stop = false;
      for (; i < nw; ++i) {
        if (P != kNil) {
          // the lane-group walk reaches node i only while this holds
          const bool more = L.cnt[i] < w.e || (Phead && Psize == 0) || (Pdirty && Psize <= f);
          if (!more) {
            stop = true;
            break;
          }
        }
        const u32 sx = L.size[i];
        const bool touched = L.cnt[i + 1] > L.cnt[i];
        const bool join = P != kNil && (Psize + sx <= f || sx == 0 || (Phead && Psize == 0));
        if (join) {
          L.dst[i] = P;
          L.off[i] = Psize;
          L.jl[nfree] = i;
          Psize += sx;
          Pfence = L.fence[i];
          Pnext = L.next[i];
          Pdirty = 1;
          ++nfree;
        } else {
          if (P != kNil && Pdirty) {
            NodeHdr h;
            h.fence = Pfence;
            h.size = Psize;
            h.next = Pnext;
            a.hdr[P] = h;
          }
          P = L.id[i];
          Psize = sx;
          Pfence = L.fence[i];
          Pnext = L.next[i];
          Pdirty = touched ? 1u : 0u;
          Phead = P == w.b ? 1u : 0u;
        }
      }
      if (stop || last_window) {
        if (P != kNil && Pdirty) {
          NodeHdr h;
          h.fence = Pfence;
          h.size = Psize;
          h.next = Pnext;
          a.hdr[P] = h;
        }
        stop = true;
      }
      L.P = P;
      L.Psize = Psize;
      L.Pnext = Pnext;
      L.Pdirty = Pdirty;
      L.Phead = Phead;
      L.Pfence = Pfence;
      L.stop = stop ? 1u : 0u;
      L.nfree = nfree;
      if (nfree) {
        const u32 base = atomicAdd(&a.ctl->free_top, nfree);
        L.free_base = base;
        if ((u64)base + nfree > a.pool) {   // more frees than nodes: never expected
          atomicCAS(a.status, 0u, kErrInternal);
          L.nfree = 0;
        }
      }
      L.freed_total += nfree;
      L.j0 = L.cnt[nw];
    }
    __syncthreads();
    // 5. survivors of the joined nodes to their predecessors; freed ids
    const u32 nj = L.nfree;
    for (u32 q0 = wv; q0 < nj; q0 += NW) {
      const u32 i = L.jl[q0];
      const u32 D = L.dst[i];
      const u32 X = L.id[i];
      const u32 sx = L.size[i];
      const u32 o = L.off[i];
      for (u32 q = lane; q < sx; q += 64) {
        a.nkeys[(u64)D * a.cap + o + q] = a.nkeys[(u64)X * a.cap + q];
        a.nvals[(u64)D * a.cap + o + q] = a.nvals[(u64)X * a.cap + q];
      }
      if (lane == 0) a.free_ids[L.free_base + q0] = X;
    }
    __syncthreads();
    if (L.stop) break;
  }
  if (tid == 0) {
    if (L.freed_total) a.bnodes[w.b] -= L.freed_total;
    // an emptied bucket ends with its head as predecessor, size 0, no link
    if (!L.was_empty && L.P == w.b && L.Psize == 0 && L.Pnext == kNil) occ_clear(a.occ, w.b);
    if (L.removed)
      atomicAdd((unsigned long long*)&a.ctl->nkeys, (unsigned long long)(0ull - (u64)L.removed));
  }
  __syncthreads();   // LDS is reused by the next item
}

// The slice kernel lists the wide delete items; workgroup g takes items g,
// g + G, ...
template <typename K, int NT>
__global__ __launch_bounds__(NT) void k_delete_wide(UpdArgs<K> a) {
  __shared__ WideDelLds<K> L;
  const Ctl* ctl = a.ctl;
  if (ctl->call_abort != 0) return;   // an epoch rejected as a whole
  const u32 n = ctl->wide_n < a.wide_cap ? ctl->wide_n : a.wide_cap;
  for (u32 i = blockIdx.x; i < n; i += gridDim.x) {
    const WorkItem w = a.wide[i];
    wide_delete_bucket<K, NT>(a, w, L);
  }
}

}  // namespace flix
