// Persistent fused drain: one co-resident grid executes a whole queue of
// mixed-type batches (lookup, successor, range, insert, delete) in order.
// Every batch runs the same phases as the per-batch launches (histogram,
// onesweep passes, then the read kernel or slices + update kernel), with a
// grid barrier between phases instead of a kernel boundary.  The queue lives
// in device memory, so one launch (or one hipGraph replay) drains it, and the
// batches can change between replays.
//
// Ordering and memory: a grid barrier is arrive (agent-scope release +
// atomic) / wait (generation word) / agent-scope acquire.  Tiles of a pass are
// walked in increasing order by every workgroup, so a tile only waits on
// tiles that are resident or finished.  Look-back words carry an epoch from
// a device counter that every drain advances, so nothing is cleared between
// passes, drains or graph replays.
#pragma once

#include "flix_device.hpp"
#include "flix_read2.hpp"
#include "flix_sort.hpp"
#include "flix_update.hpp"

namespace flix {

constexpr u32 kOpInsert = 3;
constexpr u32 kOpDelete = 4;
constexpr u32 kOpLast = 5;   // predecessor

struct alignas(16) DrainBatch {
  u32 op;
  u32 n;
  u32 maxpq;
  u32 reserved;
  const void* keys;   // keys (range: lo)
  const void* aux;    // insert: values; range: hi
  void* out_v;
  void* out_k;
  u32* counts;
  void* reserved2;
};

// Arrival groups of the grid barrier: workgroup b arrives on counter b % 8,
// which matches the round-robin placement of workgroups on the 8 XCDs, so no
// counter takes more than an eighth of the arrivals.
constexpr u32 kBarGroups = 8;

struct DrainCtl {
  u32 bar_gen;       // barrier generation
  u32 epoch;         // last look-back epoch used by a drain
  u32 err;           // sticky: 1 barrier wait or look-back gave up, 4 bad descriptor
  u32 top_count;     // groups complete at the current barrier
  u32 pad0[28];
  u32 grp[kBarGroups][32];   // arrivals per group, one 128-byte line each
};

// The store's layout as the kernels see it.  Bulk loads reallocate the
// directory and the pool, so a drain captured in a graph must not hold these
// pointers: it reads this record, which every bulk load rewrites, when each
// replay starts.
struct alignas(16) StoreLayout {
  const void* mkba;
  NodeHdr* hdr;
  void* nkeys;
  void* nvals;
  u32* bnodes;
  u32* free_ids;
  u32 nb;
  u32 pool;
  u32 pad[2];
  OccLevels occ;
};

template <typename K>
struct DrainArgs {
  const DrainBatch* batches;
  u32 nbatch;
  // store: layout read from device memory at kernel start
  const StoreLayout* layout;
  u32 cap;
  Ctl* ctl;
  // scratch
  K* bk[2];
  void* bp[2];
  u32* hist;          // [2][P*R]
  u64* status;
  u64* status_cl;
  u64 status_words;
  u64 cluster_words;
  WorkItem* work;
  u32 lds_items;
  u32 chunk;
  DrainCtl* dctl;
  unsigned long long* tstamp;   // [nbatch + 1]: start, then one per batch (may be null)
  u32 max_batch;
};

// Grid-wide barrier for a co-resident grid.  Each workgroup publishes its
// writes (agent-scope release fence: the L2 of its XCD is written back),
// arrives on its group counter; the last arrival of a group arrives on the
// top counter, and the last group flips the generation.  Waiters poll the
// generation with relaxed loads and invalidate their caches once, after the
// flip (an acquire load per poll would invalidate the L2 on every poll).
// Bounded: a workgroup that waits too long records an error.  Returns true
// (in every thread of the workgroup) once the grid has failed, a barrier wait
// or a sort look-back having given up: the caller must then leave the kernel,
// since later phases would read buffers that earlier phases did not finish.
__device__ __forceinline__ bool grid_sync(DrainCtl* c, u32 nblocks) {
  __shared__ u32 s_abort;
  __syncthreads();
  if (threadIdx.x == 0) {
    const u32 g = blockIdx.x % kBarGroups;
    const u32 members = (nblocks - g + kBarGroups - 1) / kBarGroups;
    const u32 ngroups = nblocks < kBarGroups ? nblocks : kBarGroups;
    const u32 gen = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this workgroup's writes
    bool flipped = false;
    const u32 a = __hip_atomic_fetch_add(&c->grp[g][0], 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (a == members) {
      __hip_atomic_store(&c->grp[g][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");   // the group's writes, onward
      const u32 t = __hip_atomic_fetch_add(&c->top_count, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) + 1u;
      if (t == ngroups) {
        __hip_atomic_store(&c->top_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&c->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        flipped = true;
      }
    }
    if (!flipped) {
      // Bounded wait; once any barrier has failed (the grid was not fully
      // resident) no later barrier waits, so the kernel ends promptly.
      u32 polls = 0;
      while (__hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u) break;
        if (++polls > (1u << 22)) {
          atomicOr(&c->err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // everyone's writes
    s_abort = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u;
  }
  __syncthreads();
  return s_abort != 0;
}

template <typename K, int RB, int GL, int KPL>
struct DrainSmemSize {
  static constexpr int U = KPL >= 16 ? 2 : 4;
  static constexpr size_t hist = sizeof(HistSmem<K, RB>);
  static constexpr size_t pass_idx = sizeof(OnesweepSmem<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayIndex>);
  static constexpr size_t pass_val = sizeof(OnesweepSmem<K, K, RB, kDrainSortNT, kDrainSortIPT, kPayValue>);
  static constexpr size_t pass_none = sizeof(OnesweepSmem<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayNone>);
  static constexpr size_t read = sizeof(ReadSmem<K, 512, 256>);
  static constexpr size_t slices = sizeof(SliceSmem<K, (sizeof(K) == 4 ? 1024 : 512), 256>);
  static constexpr size_t fixed() {
    size_t m = hist;
    m = m > pass_idx ? m : pass_idx;
    m = m > pass_val ? m : pass_val;
    m = m > pass_none ? m : pass_none;
    m = m > read ? m : read;
    m = m > slices ? m : slices;
    return m;
  }
};

template <typename K, int RB, int GL, int KPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_drain(DrainArgs<K> a) {
  extern __shared__ unsigned char smem[];
  __shared__ UpdShared s_upd;
  __shared__ u32 s_epoch;
  constexpr int R = RadixShape<K, RB>::R;
  constexpr int P = RadixShape<K, RB>::P;
  constexpr int U = KPL >= 16 ? 2 : 4;
  constexpr int SR = 512;                       // read share
  constexpr int SS = sizeof(K) == 4 ? 1024 : 512;  // slice share
  const u32 G = gridDim.x;
  const u32 blk = blockIdx.x;
  DrainCtl* dc = a.dctl;
  const StoreLayout L = *a.layout;
  const K* const mkba = (const K*)L.mkba;
  K* const nkeys = (K*)L.nkeys;
  K* const nvals = (K*)L.nvals;

  // Epochs: every workgroup reads the base before anyone advances it (the
  // advance happens after the first barrier, by the most this drain can use,
  // so a drain that stops early never leaves epochs to be reused).  Near
  // wrap-around the status words are cleared first.
  if (threadIdx.x == 0) s_epoch = __hip_atomic_load(&dc->epoch, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  u32 epoch = s_epoch;
  const u32 need_epochs = a.nbatch * (u32)P + 1u;
  if (epoch + need_epochs >= (1u << 30) - 1u) {
    for (u64 i = (u64)blk * 256 + threadIdx.x; i < a.status_words; i += (u64)G * 256) a.status[i] = 0;
    for (u64 i = (u64)blk * 256 + threadIdx.x; i < a.cluster_words; i += (u64)G * 256)
      a.status_cl[i] = 0;
    epoch = 0;
  }
  // both histogram slots start at zero
  if (blk == 0)
    for (int i = threadIdx.x; i < 2 * P * R; i += 256) a.hist[i] = 0;
  if (blk == 0 && threadIdx.x == 0 && a.tstamp) a.tstamp[0] = wall_clock64();
  const u32 epoch_end = epoch + need_epochs;
  const bool failed0 = grid_sync(dc, G);
  if (blk == 0 && threadIdx.x == 0)
    __hip_atomic_store(&dc->epoch, epoch_end, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (failed0) return;

  u32 nz = 0;   // batches processed so far: selects the histogram slot
  for (u32 bi = 0; bi < a.nbatch; ++bi) {
    const DrainBatch d = a.batches[bi];
    const u32 n = d.n;
    if (n > a.max_batch || d.op > kOpLast) {   // rewritten descriptor out of range
      if (blk == 0 && threadIdx.x == 0) atomicOr(&dc->err, 4u);
      continue;
    }
    if (n == 0) {
      if (blk == 0 && threadIdx.x == 0 && a.tstamp) a.tstamp[bi + 1] = wall_clock64();
      continue;
    }
    const bool is_update = d.op == kOpInsert || d.op == kOpDelete;
    const u32 slot = nz & 1u;
    ++nz;
    u32* hist = a.hist + slot * (P * R);
    if (is_update && blk == 0) {
      if (threadIdx.x == 0) {
        a.ctl->need = 0;
        a.ctl->call_err = 0;
        a.ctl->call_abort = 0;
      }
      reset_work_regions(a.ctl, threadIdx.x);
    }
    // ---- histogram
    radix_hist_part<K, RB>((const K*)d.keys, n, hist, blk, G,
                           *reinterpret_cast<HistSmem<K, RB>*>(smem));
    if (grid_sync(dc, G)) return;
    // ---- onesweep passes
    const u32 ntiles = (n + kSortTile - 1) / kSortTile;
    for (int p = 0; p < P; ++p) {
      ++epoch;
      // constant indices only: a runtime index into the argument arrays
      // would move them to scratch memory
      K* const bk0 = a.bk[0];
      K* const bk1 = a.bk[1];
      void* const bp0 = a.bp[0];
      void* const bp1 = a.bp[1];
      const K* ki = (p == 0) ? (const K*)d.keys : ((p & 1) ? bk0 : bk1);
      K* ko = (p & 1) ? bk1 : bk0;
      if (d.op == kOpInsert) {
        PassArgs<K, K> pa;
        pa.kin = ki;
        pa.vin = (p == 0) ? (const K*)d.aux : (const K*)((p & 1) ? bp0 : bp1);
        pa.kout = ko;
        pa.vout = (K*)((p & 1) ? bp1 : bp0);
        pa.n = n; pa.shift = (u32)(p * RB); pa.hist_p = hist + p * R;
        pa.status = a.status; pa.status_cl = a.status_cl; pa.epoch = epoch; pa.err = &dc->err;
        for (u32 t = blk; t < ntiles; t += G)
          onesweep_tile<K, K, RB, kDrainSortNT, kDrainSortIPT, kPayValue>(
              pa, t, *reinterpret_cast<OnesweepSmem<K, K, RB, kDrainSortNT, kDrainSortIPT, kPayValue>*>(smem));
      } else if (d.op == kOpDelete) {
        PassArgs<K, u32> pa;
        pa.kin = ki; pa.vin = nullptr; pa.kout = ko; pa.vout = nullptr;
        pa.n = n; pa.shift = (u32)(p * RB); pa.hist_p = hist + p * R;
        pa.status = a.status; pa.status_cl = a.status_cl; pa.epoch = epoch; pa.err = &dc->err;
        for (u32 t = blk; t < ntiles; t += G)
          onesweep_tile<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayNone>(
              pa, t, *reinterpret_cast<OnesweepSmem<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayNone>*>(smem));
      } else {
        PassArgs<K, u32> pa;
        pa.kin = ki;
        pa.vin = (p == 0) ? nullptr : (const u32*)((p & 1) ? bp0 : bp1);
        pa.kout = ko;
        pa.vout = (u32*)((p & 1) ? bp1 : bp0);
        pa.n = n; pa.shift = (u32)(p * RB); pa.hist_p = hist + p * R;
        pa.status = a.status; pa.status_cl = a.status_cl; pa.epoch = epoch; pa.err = &dc->err;
        for (u32 t = blk; t < ntiles; t += G)
          onesweep_tile<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayIndex>(
              pa, t, *reinterpret_cast<OnesweepSmem<K, u32, RB, kDrainSortNT, kDrainSortIPT, kPayIndex>*>(smem));
      }
      if (grid_sync(dc, G)) return;
    }
    const int r = ((P - 1) & 1) ? 1 : 0;
    // the other histogram slot was last used by the previous batch and is
    // next used by the following one, after at least one more barrier
    if (blk == 0)
      for (int i = threadIdx.x; i < P * R; i += 256) a.hist[(slot ^ 1u) * (P * R) + i] = 0;
    // ---- apply
    if (!is_update) {
      ReadArgs<K> ra;
      ra.skeys = a.bk[r];
      ra.sidx = (const u32*)a.bp[r];
      ra.m = n;
      ra.mkba = mkba;
      ra.nb = L.nb;
      ra.hdr = L.hdr;
      ra.nkeys = nkeys;
      ra.nvals = nvals;
      ra.cap = a.cap;
      ra.share = SR;
      ra.out_v = (K*)d.out_v;
      ra.out_k = (K*)d.out_k;
      ra.hi = (const K*)d.aux;
      ra.counts = d.counts;
      ra.maxpq = d.maxpq;
      ra.pool = L.pool;
      ra.err = &a.ctl->status;
      ra.occ = L.occ.w0;
      ra.cuts = nullptr;   // each share searches its own cuts
      const u32 nshares = (u32)(((u64)n + L.nb + SR - 1) / SR);
      for (u32 vb = blk; vb < nshares; vb += G) {
        read_share<K, 256, SR, GL, KPL, U>(ra, (int)d.op, vb,
                                          *reinterpret_cast<ReadSmem<K, SR, 256>*>(smem));
        __syncthreads();
      }
    } else {
      SliceArgs<K> sa;
      sa.skeys = a.bk[r];
      sa.svals = d.op == kOpInsert ? (const K*)a.bp[r] : nullptr;
      sa.m = n;
      sa.mkba = mkba;
      sa.nb = L.nb;
      sa.hdr = L.hdr;
      sa.bnodes = L.bnodes;
      sa.cap = a.cap;
      sa.share = SS;
      sa.work = a.work;
      sa.rcap = work_region_cap(a.max_batch);
      sa.ctl = a.ctl;
      const u32 nshares = (u32)(((u64)n + L.nb + SS - 1) / SS);
      for (u32 vb = blk; vb < nshares; vb += G) {
        if (d.op == kOpInsert)
          slices_share<K, 256, SS, true>(sa, vb, *reinterpret_cast<SliceSmem<K, SS, 256>*>(smem));
        else
          slices_share<K, 256, SS, false>(sa, vb, *reinterpret_cast<SliceSmem<K, SS, 256>*>(smem));
      }
      if (grid_sync(dc, G)) return;
      UpdArgs<K> ua;
      ua.mkba = mkba;
      ua.skeys = a.bk[r];
      ua.svals = d.op == kOpInsert ? (const K*)a.bp[r] : nullptr;
      ua.m = n;
      ua.hdr = L.hdr;
      ua.nkeys = nkeys;
      ua.nvals = nvals;
      ua.bnodes = L.bnodes;
      ua.free_ids = L.free_ids;
      ua.cap = a.cap;
      ua.chunk = a.chunk;
      ua.pool = L.pool;
      ua.work = a.work;
      ua.rcap = work_region_cap(a.max_batch);
      ua.ctl = a.ctl;
      ua.status = &a.ctl->status;
      ua.occ = L.occ;
      if (d.op == kOpInsert)
        insert_items<K, GL, 256>(ua, a.lds_items, blk, G, smem, s_upd);
      else
        delete_items<K, GL, 256>(ua, a.lds_items, blk, G, smem, s_upd);
    }
    if (grid_sync(dc, G)) return;
    if (blk == 0 && threadIdx.x == 0 && a.tstamp) a.tstamp[bi + 1] = wall_clock64();
  }
}

}  // namespace flix
