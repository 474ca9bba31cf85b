// Device-side building blocks shared by the FliX kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace flix {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr int kWave = 64;
constexpr u32 kNil = 0xFFFFFFFFu;

// Per-node metadata (Section 3.2: every node stores its maxKey and its size;
// nodes of one bucket are chained through a node link).  The fence is kept in
// 64 bits for both key widths so the record is always 16 bytes.
struct alignas(16) NodeHdr {
  u64 fence;  // largest key this node may hold (its "maxKey")
  u32 size;   // live keys, stored sorted in slots [0, size)
  u32 next;   // next node of the same bucket, or kNil
};
static_assert(sizeof(NodeHdr) == 16 && offsetof(NodeHdr, size) == 8 && offsetof(NodeHdr, next) == 12,
              "size and next are read together as one 8-byte word");

// Regions of the update work list.  The slice workgroups of one call append
// to kWorkRegions regions (consecutive shares to the same one), each with a
// counter on a line of its own, so the thousands of workgroups of a call do
// not serialise on a single address (same-address device atomics are
// executed one at a time past the L2s).
constexpr u32 kWorkRegions = 64;

// Device control block: counters and status words owned by one store.
struct alignas(128) Ctl {
  u32 free_top;        // number of node ids on the free stack
  u32 status;          // sticky first device-detected error (negative code)
  u32 call_err;        // error raised by the pre-check of the current call
  u32 call_abort;      // an epoch's updates were rejected as a whole: its
                       // delete and insert kernels change nothing
  u64 need;            // pre-check: upper bound of nodes the call may take
  u64 nkeys;           // number of live keys in the store
  u32 free_snapshot;   // free_top as seen before the current apply kernel
  u32 work_ovf;        // work items in the overflow region of the work list
  u32 wide_n;          // items on the list of the workgroup-wide insert kernel
  u32 scan_total;      // output of device-wide compaction scans
  // per region: [0] items claimed, [1] first claim that did not fit (all
  // ones: none), so the region holds min([0], [1]) items
  alignas(128) u32 wreg[kWorkRegions][32];
};

// Work-list slots of a store whose batches hold at most max_batch keys:
// kWorkRegions regions of region_cap slots, then an overflow region of
// max_batch slots (a call never has more work items than keys).
__host__ __device__ inline u32 work_region_cap(u64 max_batch) {
  return (u32)((max_batch + kWorkRegions - 1) / kWorkRegions);
}
__host__ __device__ inline u64 work_slots(u64 max_batch) {
  return (u64)kWorkRegions * work_region_cap(max_batch) + max_batch;
}

// Per-call reset of the work-list counters (region r by thread r).
__device__ __forceinline__ void reset_work_regions(Ctl* ctl, u32 t) {
  if (t < kWorkRegions) {
    ctl->wreg[t][0] = 0;
    ctl->wreg[t][1] = 0xFFFFFFFFu;
  }
  if (t == 0) {
    ctl->work_ovf = 0;
    ctl->wide_n = 0;
  }
}

// Slots of the workgroup-wide insert list, after the work list: every item on
// it holds at least 256 batch keys, and slices are disjoint.
// Wide work items: an insert slice holds at least 256 keys, a wide delete
// slice at least 16.
__host__ __device__ inline u32 wide_slots(u64 max_batch) { return (u32)(max_batch / 16 + 1); }

// Work-list map of an apply workgroup: s_pre[r] = items in regions < r
// (kWorkRegions + 1 entries).  All threads call; returns the item count.
__device__ inline u32 load_work_map(const Ctl* ctl, u32* s_pre) {
  if (threadIdx.x < kWorkRegions) {
    const u32 lane = threadIdx.x;
    const u32 c = ctl->wreg[lane][0], f = ctl->wreg[lane][1];
    u32 x = c < f ? c : f;
    for (u32 o = 1; o < kWorkRegions; o <<= 1) {
      const u32 y = (u32)__shfl_up((int)x, o, 64);
      if (lane >= o) x += y;
    }
    s_pre[lane + 1] = x;
    if (lane == 0) s_pre[0] = 0;
  }
  __syncthreads();
  return s_pre[kWorkRegions] + ctl->work_ovf;
}

// Position of an apply group in the work list: region r (kWorkRegions is the
// overflow region, which starts at slot kWorkRegions * rcap) and the number
// of items before it.  A group visits increasing item indices, so after one
// binary search it only steps forward over the map.
struct WorkCursor {
  u32 r;
  u32 base;   // s_pre[r]
  __device__ void seek(const u32* s_pre, u32 i) {
    if (i >= s_pre[kWorkRegions]) {
      r = kWorkRegions;
      base = s_pre[kWorkRegions];
      return;
    }
    u32 lo = 0, hi = kWorkRegions;   // s_pre[lo] <= i < s_pre[hi]
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (s_pre[mid] <= i) lo = mid; else hi = mid;
    }
    r = lo;
    base = s_pre[lo];
  }
  // advance to item i (not below the current one)
  __device__ void move(const u32* s_pre, u32 i) {
    while (r < kWorkRegions) {
      const u32 next = s_pre[r + 1];
      if (next > i) break;
      ++r;
      base = next;
    }
  }
  __device__ u32 slot(u32 i, u32 rcap) const { return r * rcap + (i - base); }
};

// Sticky status codes written by kernels (the negated C ABI error codes).
constexpr u32 kErrInval = 0xFFFFFFFFu;     // -1
constexpr u32 kErrNomem = 0xFFFFFFFEu;     // -2
constexpr u32 kErrInternal = 0xFFFFFFFBu;  // -5: internal consistency check failed

template <typename K>
__device__ __forceinline__ K key_max() { return ~K(0); }

__device__ __forceinline__ u32 lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// popcount(mask & lanes-below-me)
__device__ __forceinline__ u32 rank_below(u64 m) {
  return __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}

__device__ __forceinline__ u64 wave_ballot(bool p) { return __ballot(p); }

// Lanes (among `valid`) whose RB-bit digit d equals this lane's: a lane
// differs from another where some bit of their digits differs, i.e. where the
// ballot of that bit differs from this lane's bit widened to 0 or all ones;
// OR over the bits, complemented.  (RB ballots; per bit one XOR and one OR per
// 32-bit half.)
template <int RB>
__device__ __forceinline__ u64 match_digit(u32 d, u64 valid) {
  u32 x0 = 0, x1 = 0;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const u32 t = (u32)((int)(d << (31 - b)) >> 31);   // bit b as 0 or all ones
    const u64 bb = wave_ballot(t != 0u);
    x0 |= (u32)bb ^ t;
    x1 |= (u32)(bb >> 32) ^ t;
  }
  return valid & ~(((u64)x1 << 32) | (u64)x0);
}

// Orders a wave's LDS writes before its later LDS reads (by any of its lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Agent-scope relaxed atomics for words other workgroups poll.
__device__ __forceinline__ u64 ld_agent(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_agent32(const u32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First index i in [lo, hi) with a[i] > x (a sorted ascending).
template <typename K, typename Ptr>
__device__ __forceinline__ u32 upper_bound_idx(Ptr a, u32 lo, u32 hi, K x) {
  while (lo < hi) {
    u32 mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First index i in [lo, hi) with a[i] >= x.
template <typename K, typename Ptr>
__device__ __forceinline__ u32 lower_bound_idx(Ptr a, u32 lo, u32 hi, K x) {
  while (lo < hi) {
    u32 mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Block-wide exclusive scan of one u32 per thread (blockDim.x == NT, NT a
// multiple of 64, at most 1024).  `tmp` needs NT/64 + 1 words of LDS.  Returns
// the exclusive prefix; *total receives the block sum.  All threads must call.
template <int NT>
__device__ __forceinline__ u32 block_exclusive_scan(u32 v, u32* tmp, u32* total) {
  const u32 lane = threadIdx.x & 63;
  const u32 w = threadIdx.x >> 6;
  // inclusive wave scan with shuffles
  u32 x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    u32 y = __shfl_up(x, off, 64);
    if (lane >= (u32)off) x += y;
  }
  if (lane == 63) tmp[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 run = 0;
    for (int i = 0; i < NT / 64; ++i) {
      u32 t = tmp[i];
      tmp[i] = run;
      run += t;
    }
    tmp[NT / 64] = run;
  }
  __syncthreads();
  u32 res = tmp[w] + x - v;
  *total = tmp[NT / 64];
  __syncthreads();
  return res;
}

}  // namespace flix
