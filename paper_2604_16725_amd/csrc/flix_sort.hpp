// Onesweep LSD radix sort of (key, payload) pairs for gfx950.
//
// The paper sorts every operation batch on the GPU before the bucket kernels
// run (Section 3.3; sort cost in Table 1 and Section 6.4).  The method used
// here is Onesweep (Adinets & Merrill, 2022): one read of the keys builds the
// digit histograms of every pass, then each pass is a single kernel in which
// every tile ranks its items, publishes per-digit counts and obtains its
// global offsets by decoupled look-back over the preceding tiles.  The sort is
// stable, which gives "last occurrence wins" for duplicate insert keys.
//
// Layout for wave64: tile = NT threads x IPT items, items arranged wave-
// striped (item k of lane l in wave w sits at w*64*IPT + k*64 + l), so ranking
// item slots k = 0..IPT-1 in order, lanes in order, reproduces input order.
//
// Look-back status words are 64 bits: [63:34] epoch, [33:32] flag, [31:0]
// count.  The epoch changes for every pass launch, so the status array never
// needs clearing between passes or calls.
#pragma once

#include <hip/hip_ext.h>

#include "flix_device.hpp"

namespace flix {

constexpr u64 kFlagAgg = 1;   // tile-local count published
constexpr u64 kFlagPre = 2;   // inclusive prefix published

__device__ __forceinline__ u64 pack_status(u32 epoch, u64 flag, u32 v) {
  return ((u64)epoch << 34) | (flag << 32) | (u64)v;
}

template <typename K, int RB>
struct RadixShape {
  static constexpr int R = 1 << RB;
  static constexpr int P = (int)((sizeof(K) * 8 + RB - 1) / RB);
};

template <typename K, int RB>
__device__ __forceinline__ u32 digit_of(K k, u32 shift) {
  return (u32)(k >> shift) & ((1u << RB) - 1u);
}

// Digit histograms of all passes in one read of the keys.  Block 0 also
// clears `hist_next`, the histogram slot the next sort call will use.
template <typename K, int RB>
struct HistSmem {
  u32 sh[RadixShape<K, RB>::P * RadixShape<K, RB>::R];
};

// Keys per thread and chunk of the histogram: one chunk's loads are all
// issued before its first count, so a chunk costs one memory round trip.
constexpr int kHistIPT = 16;

// Histogram part `part` of `nparts` (grid-stride over chunks of 256 x
// kHistIPT keys; each of a chunk's kHistIPT loads is coalesced across the
// workgroup).
template <typename K, int RB>
__device__ void radix_hist_part(const K* __restrict__ keys, u32 n, u32* __restrict__ hist,
                                u32 part, u32 nparts, HistSmem<K, RB>& sm) {
  constexpr int R = RadixShape<K, RB>::R;
  constexpr int P = RadixShape<K, RB>::P;
  constexpr u32 CH = 256u * kHistIPT;
  u32* sh = sm.sh;
  for (int i = threadIdx.x; i < P * R; i += 256) sh[i] = 0;
  __syncthreads();
  for (u64 base = (u64)part * CH; base < n; base += (u64)nparts * CH) {
    K kk[kHistIPT];
#pragma unroll
    for (int c = 0; c < kHistIPT; ++c) {
      const u64 i = base + (u64)c * 256u + threadIdx.x;
      kk[c] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int c = 0; c < kHistIPT; ++c) {
      if (base + (u64)c * 256u + threadIdx.x < n) {
#pragma unroll
        for (int p = 0; p < P; ++p) atomicAdd(&sh[p * R + digit_of<K, RB>(kk[c], p * RB)], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P * R; i += 256)
    if (sh[i]) atomicAdd(&hist[i], sh[i]);
  __syncthreads();
}

template <typename K, int RB>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, u32 n,
                                                    u32* __restrict__ hist,
                                                    u32* __restrict__ hist_next,
                                                    u32* __restrict__ tile_ctr) {
  constexpr int R = RadixShape<K, RB>::R;
  constexpr int P = RadixShape<K, RB>::P;
  __shared__ HistSmem<K, RB> sm;
  if (blockIdx.x == 0 && hist_next != nullptr)
    for (int i = threadIdx.x; i < P * R; i += 256) hist_next[i] = 0;
  (void)tile_ctr;
  radix_hist_part<K, RB>(keys, n, hist, blockIdx.x, gridDim.x, sm);
}

constexpr u32 kSortCluster = 16;   // tiles per look-back cluster
constexpr u32 kLookWindow = 16;    // statuses read per look-back round trip

// Payload modes.
constexpr int kPayNone = 0;    // keys only
constexpr int kPayIndex = 1;   // payload is u32; vin == nullptr means "input index"
constexpr int kPayValue = 2;   // payload read from vin

template <typename K, typename V, int RB, int NT, int IPT, int PAY>
struct OnesweepSmem {
  K k[NT * IPT];
  V v[PAY == kPayNone ? 1 : NT * IPT];
  u32 wc[NT / 64][1 << RB];
  u32 lstart[1 << RB];
  u32 gbase[1 << RB];
  u32 tmp[NT / 64 + 1];
  u32 trivial;
};

template <typename K, typename V>
struct PassArgs {
  const K* kin;
  const V* vin;
  K* kout;
  V* vout;
  u32 n;
  u32 shift;
  const u32* hist_p;
  u64* status;
  u64* status_cl;
  u32 epoch;
  u32* err;
};

// One tile of one onesweep pass.  Tiles must be processed so that every tile
// a tile waits on is resident or finished: in a plain launch tile = workgroup
// id (workgroups are dispatched in id order); in a persistent grid every
// workgroup walks its tiles in increasing order.
template <typename K, typename V, int RB, int NT, int IPT, int PAY>
__device__ void onesweep_tile(const PassArgs<K, V>& pa, u32 tile,
                              OnesweepSmem<K, V, RB, NT, IPT, PAY>& sm) {
  constexpr int R = 1 << RB;
  constexpr int WAVES = NT / 64;
  constexpr int TILE = NT * IPT;
  static_assert(R <= NT, "one look-back thread per digit");
  const K* __restrict__ kin = pa.kin;
  const V* __restrict__ vin = pa.vin;
  K* __restrict__ kout = pa.kout;
  V* __restrict__ vout = pa.vout;
  const u32 n = pa.n, shift = pa.shift, epoch = pa.epoch;
  const u32* __restrict__ hist_p = pa.hist_p;
  u64* status = pa.status;
  u64* status_cl = pa.status_cl;
  u32* err = pa.err;
  K* s_k = sm.k;
  V* s_v = sm.v;
  auto& s_wc = sm.wc;
  u32* s_lstart = sm.lstart;
  u32* s_gbase = sm.gbase;
  u32* s_tmp = sm.tmp;
  u32& s_trivial = sm.trivial;

  const u32 tid = threadIdx.x;
  const u32 lane = tid & 63;
  const u32 w = tid >> 6;

  if (tid == 0) s_trivial = 0;
  for (int i = tid; i < WAVES * R; i += NT) (&s_wc[0][0])[i] = 0;
  __syncthreads();
  const u32 tile0 = tile * (u32)TILE;

  // Load items (wave-striped) and this pass's digit counts in one round.
  K key[IPT];
  V pay[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    if (idx < n) {
      key[k] = kin[idx];
      if (PAY == kPayIndex) pay[k] = vin ? vin[idx] : (V)idx;
      if (PAY == kPayValue) pay[k] = vin[idx];
    } else {
      key[k] = K(0);
      if (PAY != kPayNone) pay[k] = V(0);
    }
  }
  u32 hcount = (tid < (u32)R) ? hist_p[tid] : 0u;

  // Global exclusive digit offsets of this pass, and the trivial-pass test
  // (all keys share one digit: the stable permutation is the identity).
  if (tid < (u32)R && hcount == n) s_trivial = 1;
  u32 htotal;
  u32 hexcl = block_exclusive_scan<NT>(hcount, s_tmp, &htotal);

  if (s_trivial) {  // uniform across the grid: no look-back is needed
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
      if (idx < n) {
        kout[idx] = key[k];
        if (PAY != kPayNone) vout[idx] = pay[k];
      }
    }
    __syncthreads();
    return;
  }

  // Stable rank of every item among the same-digit items of its wave.
  u32 rank[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    bool valid = idx < n;
    u32 d = digit_of<K, RB>(key[k], shift);
    const u64 m = match_digit<RB>(d, wave_ballot(valid));
    u32 below = rank_below(m);
    u32 cnt = __popcll(m);
    u32 base = valid ? s_wc[w][d] : 0u;
    rank[k] = base + below;
    if (valid && below == cnt - 1) s_wc[w][d] = base + cnt;
  }
  __syncthreads();

  // Per-digit totals of the tile; turn the per-wave counts into exclusive
  // prefixes across waves.
  u32 tot = 0;
  if (tid < (u32)R) {
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      u32 c = s_wc[ww][tid];
      s_wc[ww][tid] = tot;
      tot += c;
    }
    // Publish the tile aggregate (tile 0 publishes its inclusive prefix).
    st_agent(&status[(u64)tile * R + tid],
             pack_status(epoch, tile == 0 ? kFlagPre : kFlagAgg, tot));
  }
  u32 dummy;
  u32 lstart = block_exclusive_scan<NT>(tid < (u32)R ? tot : 0u, s_tmp, &dummy);
  if (tid < (u32)R) {
    s_lstart[tid] = lstart;
    // Two-level decoupled look-back for this digit.  Tiles form clusters of
    // CL consecutive tiles; the last tile of a cluster also publishes the
    // cluster's aggregate (or inclusive prefix) once it has read its cluster
    // mates.  A tile sums the published counts of its cluster mates (nearest
    // first, LB per round trip) and then those of earlier clusters, stopping
    // at the first inclusive prefix, so the chain of dependent round trips
    // stays short however many tiles the pass has.
    u32 excl = 0;
    if (tile > 0) {
      const u32 c = tile / kSortCluster;
      const u32 cbeg = c * kSortCluster;
      const bool last_of_cluster = (tile == cbeg + kSortCluster - 1);
      bool done = false;
      bool gave_up = false;
      u32 polls = 0;
      // (1) cluster mates [cbeg, tile)
      u32 pt = tile;
      while (!done && pt > cbeg) {
        u64 win[kLookWindow];
#pragma unroll
        for (u32 w = 0; w < kLookWindow; ++w)
          win[w] = (w < pt - cbeg) ? ld_agent(&status[(u64)(pt - 1 - w) * R + tid]) : 0ull;
        u32 used = 0;
#pragma unroll
        for (u32 w = 0; w < kLookWindow; ++w) {
          if (done || w != used || w >= pt - cbeg) continue;
          u64 s = win[w];
          u32 fl = (u32)(s >> 32) & 3u;
          if ((u32)(s >> 34) != epoch || fl == 0) continue;   // not published yet
          excl += (u32)s;
          ++used;
          if (fl == kFlagPre) done = true;
        }
        pt -= used;
        if (!done && used == 0) {
          // Bounded wait: a predecessor that never publishes is a bug, and the
          // kernel must still end; the error word reports it.
          if (++polls > (1u << 22)) { atomicOr(err, 1u); gave_up = true; break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (last_of_cluster && !gave_up)
        st_agent(&status_cl[(u64)c * R + tid],
                 pack_status(epoch, done ? kFlagPre : kFlagAgg, excl + tot));
      // (2) earlier clusters [0, c)
      u32 pc = c;
      while (!done && !gave_up && pc > 0) {
        u64 win[kLookWindow];
#pragma unroll
        for (u32 w = 0; w < kLookWindow; ++w)
          win[w] = (w < pc) ? ld_agent(&status_cl[(u64)(pc - 1 - w) * R + tid]) : 0ull;
        u32 used = 0;
#pragma unroll
        for (u32 w = 0; w < kLookWindow; ++w) {
          if (done || w != used || w >= pc) continue;
          u64 s = win[w];
          u32 fl = (u32)(s >> 32) & 3u;
          if ((u32)(s >> 34) != epoch || fl == 0) continue;
          excl += (u32)s;
          ++used;
          if (fl == kFlagPre) done = true;
        }
        pc -= used;
        if (!done && used == 0) {
          if (++polls > (1u << 22)) { atomicOr(err, 1u); gave_up = true; break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      st_agent(&status[(u64)tile * R + tid], pack_status(epoch, kFlagPre, excl + tot));
      if (last_of_cluster && !gave_up)
        st_agent(&status_cl[(u64)c * R + tid], pack_status(epoch, kFlagPre, excl + tot));
    }
    s_gbase[tid] = hexcl + excl;
  }
  __syncthreads();

  // Local counting sort of the tile into LDS.
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    if (idx < n) {
      u32 d = digit_of<K, RB>(key[k], shift);
      u32 pos = s_lstart[d] + s_wc[w][d] + rank[k];
      s_k[pos] = key[k];
      if (PAY != kPayNone) s_v[pos] = pay[k];
    }
  }
  __syncthreads();

  // Write out in digit order: consecutive threads write consecutive slots of
  // one digit's run.
  u32 valid_n = (n - tile0) < (u32)TILE ? (n - tile0) : (u32)TILE;
#pragma unroll
  for (u32 r = 0; r < (u32)IPT; ++r) {
    const u32 i = tid + r * (u32)NT;
    if (i < valid_n) {
      K kk = s_k[i];
      u32 d = digit_of<K, RB>(kk, shift);
      u32 g = s_gbase[d] + (i - s_lstart[d]);
      if (g < n) {   // always true for a consistent histogram
        kout[g] = kk;
        if (PAY != kPayNone) vout[g] = s_v[i];
      }
    }
  }
  __syncthreads();
}

template <typename K, typename V, int RB, int NT, int IPT, int PAY>
__global__ __launch_bounds__(NT) void k_onesweep(PassArgs<K, V> pa) {
  __shared__ OnesweepSmem<K, V, RB, NT, IPT, PAY> sm;
  onesweep_tile<K, V, RB, NT, IPT, PAY>(pa, blockIdx.x, sm);
}

// ---------------------------------------------------------------------------
// Batches of at most kLocalMaxItems items with 8-bit digits: one onesweep pass
// on the most significant digit splits the batch into 256 runs (stably), then
// k_local_sort gives every run one workgroup that sorts it on the remaining
// digits.  A run of at most kLocalCap items stays in LDS for all of its
// passes; a longer one (skewed keys) is sorted in global memory, chunk by
// chunk, in the two buffers of its run.  Every pass is a stable counting sort
// whose ranks come from wave ballots over wave-striped items (as in a
// onesweep tile), so the sort stays stable.  This replaces P - 1 device-wide
// passes, each with its look-back, by work that stays inside one CU.
constexpr int kLocalNT = 1024;
constexpr int kLocalIPT = 8;
constexpr u32 kLocalCap = kLocalNT * kLocalIPT;
constexpr u32 kLocalMaxItems = 1u << 22;

constexpr int kLocalMaxPass = 7;   // digits below the top one (64-bit keys)

struct LocalSortHead {
  u32 wc[kLocalNT / 64][256];   // per-wave digit counts, then their prefixes
  u32 dstart[256];              // first slot of every digit in the run or chunk
  u32 off[256];                 // running digit offsets (chunked runs)
  u32 hist[kLocalMaxPass][256]; // digit counts of every pass (chunked runs)
  u32 tmp[kLocalNT / 64 + 1];
  u32 range[2];
};
constexpr size_t kLocalHeadBytes = (sizeof(LocalSortHead) + 15) & ~size_t(15);

template <typename K, typename V, int PAY>
constexpr size_t local_sort_lds() {
  return kLocalHeadBytes + (size_t)kLocalCap * sizeof(K) +
         (PAY == kPayNone ? 0 : (size_t)kLocalCap * sizeof(V));
}

// Stable ranks of the kLocalIPT wave-striped items of each thread among the
// items of its wave with the same digit; per-wave digit counts go to
// h.wc[wave] (cleared by the caller).
template <typename K>
__device__ __forceinline__ void local_rank(const K (&key)[kLocalIPT], u32 nvalid_base, u32 n,
                                           u32 shift, LocalSortHead& h, u32 (&rank)[kLocalIPT]) {
  const u32 w = threadIdx.x >> 6, lane = threadIdx.x & 63u;
#pragma unroll
  for (int k = 0; k < kLocalIPT; ++k) {
    const u32 li = nvalid_base + w * 64u * kLocalIPT + (u32)k * 64u + lane;
    const bool valid = li < n;
    const u32 d = digit_of<K, 8>(key[k], shift);
    const u64 m = match_digit<8>(d, wave_ballot(valid));
    const u32 below = rank_below(m);
    const u32 cnt = (u32)__popcll(m);
    const u32 base = valid ? h.wc[w][d] : 0u;
    rank[k] = base + below;
    if (valid && below == cnt - 1) h.wc[w][d] = base + cnt;
  }
}

// Turns h.wc into exclusive prefixes across waves (per digit) and returns,
// in thread d < 256, the digit's total.  All threads call.
__device__ __forceinline__ u32 local_wave_prefix(LocalSortHead& h) {
  constexpr int WAVES = kLocalNT / 64;
  const u32 tid = threadIdx.x;
  u32 tot = 0;
  if (tid < 256u) {
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      const u32 c = h.wc[ww][tid];
      h.wc[ww][tid] = tot;
      tot += c;
    }
  }
  return tot;
}

// Sorts the cnt (<= kLocalCap) wave-striped items held in registers on digits
// 0..npass-1, leaving them sorted and wave-striped in registers; s_k / s_v
// are the LDS staging arrays.  All threads call.
template <typename K, typename V, int PAY>
__device__ void local_lds_passes(K (&key)[kLocalIPT], V (&pay)[kLocalIPT], u32 cnt, u32 npass,
                                 LocalSortHead& h, K* s_k, V* s_v) {
  constexpr int IPT = kLocalIPT;
  const u32 tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  u32 rank[IPT];
  for (u32 p = 0; p < npass; ++p) {
    const u32 shift = p * 8u;
    for (u32 i = tid; i < (kLocalNT / 64) * 256u; i += kLocalNT) (&h.wc[0][0])[i] = 0;
    __syncthreads();
    local_rank<K>(key, 0u, cnt, shift, h, rank);
    __syncthreads();
    const u32 tot = local_wave_prefix(h);
    u32 dummy;
    const u32 ds = block_exclusive_scan<kLocalNT>(tid < 256u ? tot : 0u, h.tmp, &dummy);
    if (tid < 256u) h.dstart[tid] = ds;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < cnt) {
        const u32 d = digit_of<K, 8>(key[k], shift);
        const u32 pos = h.dstart[d] + h.wc[w][d] + rank[k];
        s_k[pos] = key[k];
        if (PAY != kPayNone) s_v[pos] = pay[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < cnt) {
        key[k] = s_k[li];
        if (PAY != kPayNone) pay[k] = s_v[li];
      }
    }
    __syncthreads();
  }
}

// Stable rank of the flagged wave-striped items of a chunk among the flagged
// items (input order); returns the chunk's flagged count.  All threads call.
__device__ __forceinline__ u32 local_class_rank(const bool (&is)[kLocalIPT],
                                                u32 (&rank)[kLocalIPT], LocalSortHead& h) {
  const u32 tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  u32 run = 0;
#pragma unroll
  for (int k = 0; k < kLocalIPT; ++k) {
    const u64 m = wave_ballot(is[k]);
    rank[k] = run + rank_below(m);
    run += (u32)__popcll(m);
  }
  if (lane == 0) h.wc[0][w] = run;
  __syncthreads();
  u32 pre = 0, total = 0;
  for (u32 ww = 0; ww < kLocalNT / 64; ++ww) {
    const u32 c = h.wc[0][ww];
    if (ww < w) pre += c;
    total += c;
  }
#pragma unroll
  for (int k = 0; k < kLocalIPT; ++k) rank[k] += pre;
  __syncthreads();
  return total;
}

template <typename K, typename V, int PAY>
__global__ __launch_bounds__(kLocalNT) void k_local_sort(K* __restrict__ ka, V* __restrict__ va,
                                                         K* __restrict__ kb, V* __restrict__ vb,
                                                         const u32* __restrict__ top_count,
                                                         u32 npass, u32 n, u32* __restrict__ err) {
  extern __shared__ unsigned char lsm[];
  LocalSortHead& h = *reinterpret_cast<LocalSortHead*>(lsm);
  K* s_k = reinterpret_cast<K*>(lsm + kLocalHeadBytes);
  V* s_v = reinterpret_cast<V*>(lsm + kLocalHeadBytes + (size_t)kLocalCap * sizeof(K));
  constexpr int IPT = kLocalIPT;
  const u32 tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  // this run: the blockIdx.x-th run of the most significant digit
  {
    const u32 c = tid < 256u ? top_count[tid] : 0u;
    u32 total;
    const u32 ex = block_exclusive_scan<kLocalNT>(c, h.tmp, &total);
    if (tid == blockIdx.x) {
      h.range[0] = ex;
      h.range[1] = c;
    }
    __syncthreads();
  }
  const u32 start = h.range[0], cnt = h.range[1];
  if (cnt == 0 || npass > (u32)kLocalMaxPass) return;
  if ((u64)start + cnt > n) {   // histogram inconsistent with the keys: never expected
    if (tid == 0) atomicOr(err, 2u);
    return;
  }
  K key[IPT];
  V pay[IPT];
  u32 rank[IPT];
  if (cnt <= kLocalCap) {
    // the run lives in registers and LDS for all passes
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < cnt) {
        key[k] = ka[start + li];
        if (PAY != kPayNone) pay[k] = va[start + li];
      } else {
        key[k] = K(0);
      }
    }
    local_lds_passes<K, V, PAY>(key, pay, cnt, npass, h, s_k, s_v);
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < cnt) {
        kb[start + li] = key[k];
        if (PAY != kPayNone) vb[start + li] = pay[k];
      }
    }
    return;
  }
  // A long run is usually one repeated key (skewed batches).  With X the key
  // in the middle of the run: the items other than X are gathered in order
  // into LDS; if they fit, they are sorted there and written around the
  // block of X items, which keep their input order (stable).
  {
    const K X = ka[start + cnt / 2];
    u32 nrest = 0;
    bool fits = true;
    for (u32 base = 0; base < cnt; base += kLocalCap) {
      bool rest[IPT];
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base + w * 64u * IPT + (u32)k * 64u + lane;
        const bool valid = li < cnt;
        key[k] = valid ? ka[start + li] : X;
        if (PAY != kPayNone && valid) pay[k] = va[start + li];
        rest[k] = valid && key[k] != X;
      }
      const u32 tot = local_class_rank(rest, rank, h);
      if (nrest + tot > kLocalCap) {   // uniform: tot and nrest are workgroup-wide
        fits = false;
        break;
      }
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        if (rest[k]) {
          s_k[nrest + rank[k]] = key[k];
          if (PAY != kPayNone) s_v[nrest + rank[k]] = pay[k];
        }
      }
      nrest += tot;
    }
    if (fits) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
        if (li < nrest) {
          key[k] = s_k[li];
          if (PAY != kPayNone) pay[k] = s_v[li];
        }
      }
      __syncthreads();
      local_lds_passes<K, V, PAY>(key, pay, nrest, npass, h, s_k, s_v);
      // items below X come first, then the X block, then the rest
      u32 mine = 0;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
        if (li < nrest && key[k] < X) ++mine;
      }
      u32 nlt;
      (void)block_exclusive_scan<kLocalNT>(mine, h.tmp, &nlt);
      const u32 neq = cnt - nrest;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
        if (li < nrest) {
          const u32 o = li < nlt ? li : li + neq;
          kb[start + o] = key[k];
          if (PAY != kPayNone) vb[start + o] = pay[k];
        }
      }
      // the X items in input order
      u32 xbase = 0;
      for (u32 base = 0; base < cnt; base += kLocalCap) {
        bool isx[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 li = base + w * 64u * IPT + (u32)k * 64u + lane;
          const bool valid = li < cnt;
          isx[k] = false;
          if (valid) {
            isx[k] = ka[start + li] == X;
            if (PAY != kPayNone) pay[k] = va[start + li];
          }
        }
        const u32 tot = local_class_rank(isx, rank, h);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          if (isx[k]) {
            kb[start + nlt + xbase + rank[k]] = X;
            if (PAY != kPayNone) vb[start + nlt + xbase + rank[k]] = pay[k];
          }
        }
        xbase += tot;
      }
      return;
    }
    __syncthreads();
  }
  // A long run: each pass reads one buffer of the run and writes the other
  // (npass is odd, so the last pass writes the second buffer), chunk by
  // chunk in order.  The digit counts of every pass come from one sweep over
  // the run first (a pass only permutes the run).
  for (u32 i = tid; i < npass * 256u; i += kLocalNT) (&h.hist[0][0])[i] = 0;
  __syncthreads();
  for (u32 base = 0; base < cnt; base += kLocalCap) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = base + (u32)k * kLocalNT + tid;
      key[k] = li < cnt ? ka[start + li] : K(0);
    }
    // Skewed runs repeat a few keys: the wave's most common case, the first
    // valid lane's digit, is added once with its lane count, the other lanes
    // add one each (LDS atomics on one address would serialise the wave).
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const bool valid = base + (u32)k * kLocalNT + tid < cnt;
      const u64 vm = wave_ballot(valid);
      if (vm == 0) continue;   // uniform across the wave
      const int src = __ffsll((unsigned long long)vm) - 1;
      for (u32 p = 0; p < npass; ++p) {
        const u32 d = digit_of<K, 8>(key[k], p * 8u);
        const u32 d0 = (u32)__shfl((int)d, src, 64);
        const u64 same = wave_ballot(valid && d == d0);
        if ((int)lane == src) atomicAdd(&h.hist[p][d0], (u32)__popcll(same));
        if (valid && d != d0) atomicAdd(&h.hist[p][d], 1u);
      }
    }
  }
  __syncthreads();
  for (u32 p = 0; p < npass; ++p) {
    const u32 shift = p * 8u;
    K* ik = (p & 1u) ? kb + start : ka + start;
    V* iv = (p & 1u) ? vb + start : va + start;
    K* ok = (p & 1u) ? ka + start : kb + start;
    V* ov = (p & 1u) ? va + start : vb + start;
    {
      const u32 c = tid < 256u ? h.hist[p][tid] : 0u;
      u32 dummy;
      const u32 ex = block_exclusive_scan<kLocalNT>(c, h.tmp, &dummy);
      if (tid < 256u) h.off[tid] = ex;
      __syncthreads();
    }
    for (u32 base = 0; base < cnt; base += kLocalCap) {
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base + w * 64u * IPT + (u32)k * 64u + lane;
        if (li < cnt) {
          key[k] = ik[li];
          if (PAY != kPayNone) pay[k] = iv[li];
        } else {
          key[k] = K(0);
        }
      }
      for (u32 i = tid; i < (kLocalNT / 64) * 256u; i += kLocalNT) (&h.wc[0][0])[i] = 0;
      __syncthreads();
      local_rank<K>(key, base, cnt, shift, h, rank);
      __syncthreads();
      const u32 tot = local_wave_prefix(h);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base + w * 64u * IPT + (u32)k * 64u + lane;
        if (li < cnt) {
          const u32 d = digit_of<K, 8>(key[k], shift);
          const u32 pos = h.off[d] + h.wc[w][d] + rank[k];
          ok[pos] = key[k];
          if (PAY != kPayNone) ov[pos] = pay[k];
        }
      }
      __syncthreads();
      if (tid < 256u) h.off[tid] += tot;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Batches of at most kSplitMaxItems items with 8-bit digits: two launches and
// no device-wide look-back chain.
//   k_tile_split: every tile of kSplitTile items is split stably on the most
//     significant digit in LDS and written back in place, digit by digit,
//     with the start of every digit inside the tile (one 256-entry row per
//     tile);
//   k_run_sort: one workgroup per top digit.  It reads its column of the row
//     table (where its digit's segment lies in every tile), publishes the
//     run's length, gathers the segments in tile order (a stable
//     concatenation), sorts the run on the digits that vary inside it
//     (LDS passes when it fits, else the dominant-key or chunked global
//     forms), and writes it at the sum of the lengths published by the lower
//     digits.
// A workgroup only waits on lower digits, whose workgroups were dispatched
// before it and publish before they wait on anything.
constexpr int kSplitNT = 512;
constexpr int kSplitIPT = 4;
constexpr u32 kSplitTile = kSplitNT * kSplitIPT;
constexpr u32 kSplitMaxTiles = 1024;
constexpr u32 kSplitMaxItems = kSplitMaxTiles * kSplitTile;   // 2^21
static_assert(kSplitMaxTiles <= (u32)kLocalNT, "one tile per thread of a run workgroup");
static_assert(kSplitTile <= 65536u, "segment starts are 16-bit");

template <typename K, typename V, int PAY>
struct SplitSmem {
  K k[kSplitTile];
  V v[PAY == kPayNone ? 1 : kSplitTile];
  u32 wc[kSplitNT / 64][256];
  u32 lstart[256];
  u32 tmp[kSplitNT / 64 + 1];
};

template <typename K, typename V, int PAY>
__global__ __launch_bounds__(kSplitNT) void k_tile_split(const K* __restrict__ kin,
                                                         const V* __restrict__ vin,
                                                         K* __restrict__ ks, V* __restrict__ vs,
                                                         u32* __restrict__ toff, u32 n,
                                                         u32 shift) {
  __shared__ SplitSmem<K, V, PAY> sm;
  constexpr int IPT = kSplitIPT;
  constexpr int NT = kSplitNT;
  constexpr int WAVES = NT / 64;
  const u32 tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const u32 tile0 = blockIdx.x * kSplitTile;
  for (u32 i = tid; i < (u32)WAVES * 256u; i += NT) (&sm.wc[0][0])[i] = 0;
  K key[IPT];
  V pay[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    key[k] = K(0);
    if (PAY != kPayNone) pay[k] = V(0);
    if (idx < n) {
      key[k] = kin[idx];
      if (PAY == kPayIndex) pay[k] = vin ? vin[idx] : (V)idx;
      if (PAY == kPayValue) pay[k] = vin[idx];
    }
  }
  __syncthreads();
  // stable rank among the same-digit items of the wave (wave-striped order)
  u32 rank[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    const bool valid = idx < n;
    const u32 d = digit_of<K, 8>(key[k], shift);
    const u64 m = match_digit<8>(d, wave_ballot(valid));
    const u32 below = rank_below(m);
    const u32 cnt = (u32)__popcll(m);
    const u32 base = valid ? sm.wc[w][d] : 0u;
    rank[k] = base + below;
    if (valid && below == cnt - 1) sm.wc[w][d] = base + cnt;
  }
  __syncthreads();
  u32 tot = 0;
  if (tid < 256u) {
    u32 c[WAVES];
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) c[ww] = sm.wc[ww][tid];
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) {
      sm.wc[ww][tid] = tot;
      tot += c[ww];
    }
  }
  u32 dummy;
  const u32 ls = block_exclusive_scan<NT>(tid < 256u ? tot : 0u, sm.tmp, &dummy);
  if (tid < 256u) {
    sm.lstart[tid] = ls;
    toff[(u64)blockIdx.x * 256u + tid] = ls;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 idx = tile0 + w * 64u * IPT + (u32)k * 64u + lane;
    if (idx < n) {
      const u32 d = digit_of<K, 8>(key[k], shift);
      const u32 pos = sm.lstart[d] + sm.wc[w][d] + rank[k];
      sm.k[pos] = key[k];
      if (PAY != kPayNone) sm.v[pos] = pay[k];
    }
  }
  __syncthreads();
  const u32 valid_n = (n - tile0) < kSplitTile ? (n - tile0) : kSplitTile;
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const u32 i = tid + (u32)r * NT;
    if (i < valid_n) {
      ks[tile0 + i] = sm.k[i];
      if (PAY != kPayNone) vs[tile0 + i] = sm.v[i];
    }
  }
}

// Where one top digit's run lies in the split tiles: segment t starts at
// a[t] inside tile t and holds run positions [p[t], p[t+1]).
struct RunMap {
  u32 p[kSplitMaxTiles + 1];
  unsigned short a[kSplitMaxTiles];
  u32 red[4];
};
constexpr size_t kRunMapBytes = (sizeof(RunMap) + 15) & ~size_t(15);

template <typename K, typename V, int PAY>
constexpr size_t run_sort_lds() {
  return kLocalHeadBytes + kRunMapBytes + (size_t)kLocalCap * sizeof(K) +
         (PAY == kPayNone ? 0 : (size_t)kLocalCap * sizeof(V));
}

// Staging index of run position i (0 <= i < run length): the segment is the
// last tile whose first position is <= i (empty segments share positions).
__device__ __forceinline__ u32 run_src(const RunMap& m, u32 ntiles, u32 i) {
  u32 lo = 0, hi = ntiles;   // p[lo] <= i < p[hi]
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (m.p[mid] <= i) lo = mid; else hi = mid;
  }
  return lo * kSplitTile + m.a[lo] + (i - m.p[lo]);
}

// Bit p of the result is set when digit p (below the top one) differs
// between some two of the thread's valid items' keys across the workgroup.
template <typename K>
__device__ __forceinline__ u32 varying_digits(K kand, K kor, u32 npass, u32* red) {
  const u32 tid = threadIdx.x;
  if (tid < 4u) red[tid] = tid < 2u ? 0xFFFFFFFFu : 0u;
  __syncthreads();
  const u64 a = (u64)kand, o = (u64)kor;
  u32 a0 = (u32)a, a1 = (u32)(a >> 32), o0 = (u32)o, o1 = (u32)(o >> 32);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a0 &= (u32)__shfl_xor((int)a0, off, 64);
    a1 &= (u32)__shfl_xor((int)a1, off, 64);
    o0 |= (u32)__shfl_xor((int)o0, off, 64);
    o1 |= (u32)__shfl_xor((int)o1, off, 64);
  }
  if ((tid & 63u) == 0) {
    atomicAnd(&red[0], a0);
    atomicAnd(&red[1], a1);
    atomicOr(&red[2], o0);
    atomicOr(&red[3], o1);
  }
  __syncthreads();
  const u64 diff = (((u64)red[1] << 32) | red[0]) ^ (((u64)red[3] << 32) | red[2]);
  __syncthreads();
  u32 mask = 0;
  for (u32 p = 0; p < npass; ++p)
    if ((diff >> (8u * p)) & 0xFFull) mask |= 1u << p;
  return mask;
}

// LDS passes over the digits set in `passes` for cnt items held wave-striped
// with ipt items per lane (position w*64*ipt + k*64 + lane); leaves them
// sorted in the same layout.  All threads call.
template <typename K, typename V, int PAY>
__device__ void run_lds_passes(K (&key)[kLocalIPT], V (&pay)[kLocalIPT], u32 cnt, u32 ipt,
                               u32 passes, LocalSortHead& h, K* s_k, V* s_v) {
  constexpr int IPT = kLocalIPT;
  constexpr int WAVES = kLocalNT / 64;
  const u32 tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  u32 rank[IPT];
  for (u32 p = 0; p < (u32)kLocalMaxPass; ++p) {
    if (!((passes >> p) & 1u)) continue;
    const u32 shift = p * 8u;
    for (u32 i = tid; i < (u32)WAVES * 256u; i += kLocalNT) (&h.wc[0][0])[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      rank[k] = 0;
      if ((u32)k < ipt) {   // uniform across the workgroup
        const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
        const bool valid = li < cnt;
        const u32 d = digit_of<K, 8>(key[k], shift);
        const u64 vm = wave_ballot(valid);
        if (vm) {
          const u64 m = match_digit<8>(d, vm);
          const u32 below = rank_below(m);
          const u32 c = (u32)__popcll(m);
          const u32 base = valid ? h.wc[w][d] : 0u;
          rank[k] = base + below;
          if (valid && below == c - 1) h.wc[w][d] = base + c;
        }
      }
    }
    __syncthreads();
    u32 tot = 0;
    if (tid < 256u) {
      u32 c[WAVES];
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) c[ww] = h.wc[ww][tid];
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) {
        h.wc[ww][tid] = tot;
        tot += c[ww];
      }
    }
    u32 dummy;
    const u32 ds = block_exclusive_scan<kLocalNT>(tid < 256u ? tot : 0u, h.tmp, &dummy);
    if (tid < 256u) h.dstart[tid] = ds;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
      if ((u32)k < ipt && li < cnt) {
        const u32 d = digit_of<K, 8>(key[k], shift);
        const u32 pos = h.dstart[d] + h.wc[w][d] + rank[k];
        s_k[pos] = key[k];
        if (PAY != kPayNone) s_v[pos] = pay[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
      if ((u32)k < ipt && li < cnt) {
        key[k] = s_k[li];
        if (PAY != kPayNone) pay[k] = s_v[li];
      }
    }
  }
}

// Sum of the run lengths published by the digits below d (all threads call;
// the result is workgroup-uniform).
__device__ __forceinline__ u32 lower_runs_total(const u64* status, u32 d, u32 epoch, u32* err,
                                                u32* tmp) {
  const u32 tid = threadIdx.x;
  u32 v = 0;
  if (tid < d) {
    u32 polls = 0;
    while (true) {
      const u64 s = ld_agent(&status[tid]);
      if ((u32)(s >> 34) == epoch && ((s >> 32) & 3u) != 0u) {
        v = (u32)s;
        break;
      }
      // bounded wait: a lower digit that never publishes is a bug, and the
      // kernel must still end; the error word reports it
      if (++polls > (1u << 22)) {
        atomicOr(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  u32 total;
  (void)block_exclusive_scan<kLocalNT>(v, tmp, &total);
  return total;
}

// Merge-path cuts of the read kernel's shares, written by the run sort: the
// merge of the sorted batch with the directory maxima (MKBA) is, top digit
// by top digit, the merge of one run with the MKBA entries of that digit, so
// the workgroup of digit d finds every cut whose diagonal falls in its block
// [base + mktop[d], base + cnt + mktop[d + 1]) by a binary search over its
// own run and MKBA slice (ties to the keys: a key equal to MKBA[i] belongs
// to bucket i).  This replaces a device-wide search launch per read call.
template <typename K>
struct RunCuts {
  const K* mk;          // MKBA (nb entries); null: no cuts wanted
  const u32* mktop;     // [257] first MKBA entry of every top digit
  u32 nb;
  u32 share;            // merged items per share
  u32 ncuts;            // shares + 1 (the last diagonal is the merge's end)
  u32* cuts;
};

// Cuts of block d (all threads call; run: the sorted run (cnt keys), mks:
// the digit's MKBA entries (nmk), both in LDS or global memory).
template <typename K>
__device__ void write_block_cuts(const RunCuts<K>& rc, u32 d, u32 base, u32 cnt, const K* run,
                                 const K* mks, u32 nmk, u64 total) {
  const u64 b0 = (u64)base + rc.mktop[d];
  const u64 b1 = b0 + cnt + nmk;
  const u32 c0 = (u32)((b0 + rc.share - 1) / rc.share);
  const u32 c1 = d == 255u ? rc.ncuts : (u32)((b1 + rc.share - 1) / rc.share);
  for (u32 c = c0 + threadIdx.x; c < c1; c += kLocalNT) {
    u64 dd = (u64)c * rc.share;
    if (dd > total) dd = total;
    const u32 l = (u32)(dd - b0);   // local diagonal, at most cnt + nmk
    // the run items among the first l items of merge(run, mks): the
    // predicate run[p] <= mks[l - p - 1] holds exactly for p below the cut
    u32 lo = l > nmk ? l - nmk : 0u;
    u32 hi = l < cnt ? l : cnt;
    while (lo < hi) {
      const u32 mid = (lo + hi) >> 1;
      if (run[mid] <= mks[l - mid - 1]) lo = mid + 1; else hi = mid;
    }
    rc.cuts[c] = base + lo;
  }
}

template <typename K, typename V, int PAY>
__global__ __launch_bounds__(kLocalNT) void k_run_sort(const K* __restrict__ ks,
                                                       const V* __restrict__ vs,
                                                       K* __restrict__ ko, V* __restrict__ vo,
                                                       K* __restrict__ kx, V* __restrict__ vx,
                                                       const u32* __restrict__ toff,
                                                       u64* __restrict__ status, u32 epoch,
                                                       u32 npass, u32 n, u32* __restrict__ err,
                                                       RunCuts<K> rcut) {
  extern __shared__ unsigned char lsm[];
  LocalSortHead& h = *reinterpret_cast<LocalSortHead*>(lsm);
  RunMap& m = *reinterpret_cast<RunMap*>(lsm + kLocalHeadBytes);
  K* s_k = reinterpret_cast<K*>(lsm + kLocalHeadBytes + kRunMapBytes);
  V* s_v = reinterpret_cast<V*>(lsm + kLocalHeadBytes + kRunMapBytes +
                                (size_t)kLocalCap * sizeof(K));
  constexpr int IPT = kLocalIPT;
  const u32 tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  const u32 d = blockIdx.x;
  const u32 ntiles = (n + kSplitTile - 1) / kSplitTile;   // <= kSplitMaxTiles = blockDim
  // the read kernel's cuts of this digit's block, once the run is in place
  // (run: its sorted keys in LDS or in the output); the MKBA slice is staged
  // in the payload area of LDS when it fits (the payloads are written out)
  auto block_cuts = [&](u32 base, u32 cnt, const K* run) {
    if (rcut.mk == nullptr) return;
    const u32 m0 = rcut.mktop[d];
    const u32 nmk = rcut.mktop[d + 1] - m0;
    const K* mks = rcut.mk + m0;
    if (PAY != kPayNone && (size_t)nmk * sizeof(K) <= (size_t)kLocalCap * sizeof(V)) {
      K* st = reinterpret_cast<K*>(s_v);
      for (u32 i = threadIdx.x; i < nmk; i += kLocalNT) st[i] = mks[i];
      mks = st;
    }
    __syncthreads();
    write_block_cuts<K>(rcut, d, base, cnt, run, mks, nmk, (u64)n + rcut.nb);
  };
  // this digit's segment in every tile
  u32 c = 0;
  if (tid < ntiles) {
    const u32 tn = (n - tid * kSplitTile) < kSplitTile ? (n - tid * kSplitTile) : kSplitTile;
    const u32 a = toff[(u64)tid * 256u + d];
    const u32 b = d < 255u ? toff[(u64)tid * 256u + d + 1u] : tn;
    if (a <= b && b <= tn) {
      c = b - a;
    } else {   // rows inconsistent with the tiles: never expected
      atomicOr(err, 2u);
    }
    m.a[tid] = (unsigned short)a;
  }
  u32 cnt;
  const u32 pre = block_exclusive_scan<kLocalNT>(c, h.tmp, &cnt);
  if (tid < ntiles) m.p[tid] = pre;
  if (tid == 0) {
    m.p[ntiles] = cnt;
    st_agent(&status[d], pack_status(epoch, kFlagAgg, cnt));
  }
  __syncthreads();
  if (cnt == 0) {
    if (rcut.mk != nullptr) block_cuts(lower_runs_total(status, d, epoch, err, h.tmp), 0u, s_k);
    return;
  }
  K key[IPT];
  V pay[IPT];
  if (cnt <= kLocalCap) {
    // the run lives in registers and LDS for all of its passes
    const u32 ipt = (cnt + kLocalNT - 1) / kLocalNT;
    K kand = ~K(0), kor = K(0);
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
      key[k] = K(0);
      if ((u32)k < ipt && li < cnt) {
        const u32 src = run_src(m, ntiles, li);
        key[k] = ks[src];
        if (PAY != kPayNone) pay[k] = vs[src];
        kand &= key[k];
        kor |= key[k];
      }
    }
    const u32 passes = varying_digits<K>(kand, kor, npass, m.red);
    run_lds_passes<K, V, PAY>(key, pay, cnt, ipt, passes, h, s_k, s_v);
    const u32 base = lower_runs_total(status, d, epoch, err, h.tmp);
    if (base + cnt > n) {   // published lengths inconsistent: never expected
      if (tid == 0) atomicOr(err, 2u);
      return;
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
      if ((u32)k < ipt && li < cnt) {
        ko[base + li] = key[k];
        if (PAY != kPayNone) vo[base + li] = pay[k];
      }
    }
    if (rcut.mk != nullptr) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
        if ((u32)k < ipt && li < cnt) s_k[li] = key[k];
      }
      block_cuts(base, cnt, s_k);
    }
    return;
  }
  const u32 base = lower_runs_total(status, d, epoch, err, h.tmp);
  if (base + cnt > n) {
    if (tid == 0) atomicOr(err, 2u);
    return;
  }
  K* const okr = ko + base;
  V* const ovr = vo + base;
  u32 rank[IPT];
  // A long run is usually one repeated key (skewed batches).  With X the key
  // in the middle of the run: the items other than X are gathered in order
  // into LDS; if they fit, they are sorted there and written around the
  // block of X items, which keep their input order (stable).
  {
    const K X = ks[run_src(m, ntiles, cnt / 2)];
    // the form only pays when X holds a good share of the run (a skewed
    // batch); 64 evenly spaced samples decide, so a run of many distinct
    // keys (a clustered batch) goes straight to the split below
    if (tid < 64u) {
      const u32 li = (u32)(((u64)cnt * tid) / 64u);
      const u64 bm = wave_ballot(ks[run_src(m, ntiles, li)] == X);
      if (tid == 0) m.red[1] = (u32)__popcll(bm);
    }
    __syncthreads();
    // (and only when the samples leave the other items room in LDS: a run
    // of two or three hot keys goes to the split below at once)
    const u32 same = m.red[1];
    const bool try_dominant =
        same >= 16u && (u64)cnt * (64u - same) <= (u64)kLocalCap * 58u;
    // the X items' payloads go to the run's region of the extra buffer in
    // input order as they are met, and are copied behind the smaller keys
    // once their number is known
    V* const xvr0 = vx + base;
    u32 nrest = 0, xbase = 0;
    bool fits = try_dominant;
    K kand = ~K(0), kor = K(0);
    for (u32 base0 = 0; fits && base0 < cnt; base0 += kLocalCap) {
      bool rest[IPT], isx[IPT];
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base0 + w * 64u * IPT + (u32)k * 64u + lane;
        const bool valid = li < cnt;
        key[k] = X;
        if (valid) {
          const u32 src = run_src(m, ntiles, li);
          key[k] = ks[src];
          if (PAY != kPayNone) pay[k] = vs[src];
        }
        rest[k] = valid && key[k] != X;
        isx[k] = valid && key[k] == X;
        if (rest[k]) {
          kand &= key[k];
          kor |= key[k];
        }
      }
      const u32 tot = local_class_rank(rest, rank, h);
      if (nrest + tot > kLocalCap) {   // uniform: tot and nrest are workgroup-wide
        fits = false;
        break;
      }
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        if (rest[k]) {
          s_k[nrest + rank[k]] = key[k];
          if (PAY != kPayNone) s_v[nrest + rank[k]] = pay[k];
        }
      }
      nrest += tot;
      // every valid item is X or not, and valid items are a prefix of the
      // chunk, so an X item's rank among the chunk's X items is its position
      // less the non-X items before it
      if (PAY != kPayNone) {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 pos = w * 64u * IPT + (u32)k * 64u + lane;
          if (isx[k]) xvr0[xbase + pos - rank[k]] = pay[k];
        }
      }
      const u32 valid_n = cnt - base0 < kLocalCap ? cnt - base0 : kLocalCap;
      xbase += valid_n - tot;
    }
    if (fits) {
      __syncthreads();
      const u32 ipt = (nrest + kLocalNT - 1) / kLocalNT;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
        if ((u32)k < ipt && li < nrest) {
          key[k] = s_k[li];
          if (PAY != kPayNone) pay[k] = s_v[li];
        }
      }
      const u32 passes = varying_digits<K>(kand, kor, npass, m.red) & (nrest ? ~0u : 0u);
      run_lds_passes<K, V, PAY>(key, pay, nrest, ipt, passes, h, s_k, s_v);
      // items below X come first, then the X block, then the rest
      u32 mine = 0;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
        if ((u32)k < ipt && li < nrest && key[k] < X) ++mine;
      }
      u32 nlt;
      (void)block_exclusive_scan<kLocalNT>(mine, h.tmp, &nlt);
      const u32 neq = cnt - nrest;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
        if ((u32)k < ipt && li < nrest) {
          const u32 o = li < nlt ? li : li + neq;
          okr[o] = key[k];
          if (PAY != kPayNone) ovr[o] = pay[k];
        }
      }
      // the X block (the payload copies were written by other threads before
      // the barriers above); IPT loads in flight per thread before the stores
      for (u32 i0 = 0; i0 < neq; i0 += kLocalNT * IPT) {
        V xv[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 i = i0 + (u32)k * kLocalNT + tid;
          if (PAY != kPayNone && i < neq) xv[k] = xvr0[i];
        }
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 i = i0 + (u32)k * kLocalNT + tid;
          if (i < neq) {
            okr[nlt + i] = X;
            if (PAY != kPayNone) ovr[nlt + i] = xv[k];
          }
        }
      }
      if (rcut.mk != nullptr) {
        __syncthreads();   // the run is in the output: search it there
        block_cuts(base, cnt, okr);
      }
      return;
    }
    __syncthreads();
  }
  // A long run of many keys.  An AND/OR sweep finds the digits that vary
  // inside it; the run is split stably on the highest of them into the extra
  // buffer (one histogram sweep, one pass), which leaves 256 sub-runs in
  // order.  Consecutive sub-runs are then taken in groups of up to kLocalCap
  // items and sorted in registers and LDS on the digits that vary inside the
  // group (the digits above the split one are constant in the run, so each
  // group only needs its own order); a sub-run longer than kLocalCap is
  // sorted by chunked global passes over its varying digits.  Everything is
  // written at the group's or sub-run's place in the output.
  K* const xkr = kx + base;
  V* const xvr = vx + base;
  // key of item i: from the split tiles (mapped) or a contiguous region
  auto load_key = [&](bool mapped, const K* ik, u32 i) -> K {
    return mapped ? ks[run_src(m, ntiles, i)] : ik[i];
  };
  // digits (below `below`) that vary among n items
  auto sweep_vary = [&](bool mapped, const K* ik, u32 n, u32 below) -> u32 {
    K kand = ~K(0), kor = K(0);
    for (u32 base0 = 0; base0 < n; base0 += kLocalCap) {
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base0 + (u32)k * kLocalNT + tid;
        if (li < n) {
          const K kk = load_key(mapped, ik, li);
          kand &= kk;
          kor |= kk;
        }
      }
    }
    return varying_digits<K>(kand, kor, npass, m.red) & ((1u << below) - 1u);
  };
  // digit histograms (digits in `mask`) of n items into h.hist
  auto sweep_hist = [&](bool mapped, const K* ik, u32 n, u32 mask) {
    for (u32 i = tid; i < npass * 256u; i += kLocalNT)
      if ((mask >> (i / 256u)) & 1u) (&h.hist[0][0])[i] = 0;
    __syncthreads();
    for (u32 base0 = 0; base0 < n; base0 += kLocalCap) {
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base0 + (u32)k * kLocalNT + tid;
        key[k] = li < n ? load_key(mapped, ik, li) : K(0);
      }
      // Skewed runs repeat a few keys: the wave's most common case, the first
      // valid lane's digit, is added once with its lane count, the other lanes
      // add one each (LDS atomics on one address would serialise the wave).
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const bool valid = base0 + (u32)k * kLocalNT + tid < n;
        const u64 vm = wave_ballot(valid);
        if (vm == 0) continue;   // uniform across the wave
        const int src = __ffsll((unsigned long long)vm) - 1;
        for (u32 p = 0; p < npass; ++p) {
          if (!((mask >> p) & 1u)) continue;   // uniform across the workgroup
          const u32 dg = digit_of<K, 8>(key[k], p * 8u);
          const u32 d0 = (u32)__shfl((int)dg, src, 64);
          const u64 same = wave_ballot(valid && dg == d0);
          if ((int)lane == src) atomicAdd(&h.hist[p][d0], (u32)__popcll(same));
          if (valid && dg != d0) atomicAdd(&h.hist[p][dg], 1u);
        }
      }
    }
    __syncthreads();
  };
  // h.off = exclusive prefix of the histogram of digit p
  auto digit_starts = [&](u32 p) {
    const u32 cc = tid < 256u ? h.hist[p][tid] : 0u;
    u32 dummy;
    const u32 ex = block_exclusive_scan<kLocalNT>(cc, h.tmp, &dummy);
    if (tid < 256u) h.off[tid] = ex;
    __syncthreads();
  };
  // one stable counting pass on digit p over n items, chunk by chunk in
  // order, from the tiles or (ik, iv) to (ok, ov); h.off holds the starts
  auto chunk_pass = [&](bool mapped, const K* ik, const V* iv, u32 n, u32 p, K* ok, V* ov) {
    const u32 shift = p * 8u;
    for (u32 base0 = 0; base0 < n; base0 += kLocalCap) {
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base0 + w * 64u * IPT + (u32)k * 64u + lane;
        key[k] = K(0);
        if (li < n) {
          const u32 src = mapped ? run_src(m, ntiles, li) : li;
          key[k] = mapped ? ks[src] : ik[src];
          if (PAY != kPayNone) pay[k] = mapped ? vs[src] : iv[src];
        }
      }
      for (u32 i = tid; i < (kLocalNT / 64) * 256u; i += kLocalNT) (&h.wc[0][0])[i] = 0;
      __syncthreads();
      local_rank<K>(key, base0, n, shift, h, rank);
      __syncthreads();
      const u32 tot = local_wave_prefix(h);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = base0 + w * 64u * IPT + (u32)k * 64u + lane;
        if (li < n) {
          const u32 dg = digit_of<K, 8>(key[k], shift);
          const u32 pos = h.off[dg] + h.wc[w][dg] + rank[k];
          ok[pos] = key[k];
          if (PAY != kPayNone) ov[pos] = pay[k];
        }
      }
      __syncthreads();
      if (tid < 256u) h.off[tid] += tot;
      __syncthreads();
    }
  };
  // n contiguous items copied in order
  auto copy_items = [&](bool mapped, const K* ik, const V* iv, u32 n, K* ok, V* ov) {
    for (u32 li = tid; li < n; li += kLocalNT) {
      const u32 src = mapped ? run_src(m, ntiles, li) : li;
      ok[li] = mapped ? ks[src] : ik[src];
      if (PAY != kPayNone) ov[li] = mapped ? vs[src] : iv[src];
    }
  };

  const u32 vary = sweep_vary(true, nullptr, cnt, npass);
  if (vary == 0) {   // every key of the run is equal: copy it in order
    copy_items(true, nullptr, nullptr, cnt, okr, ovr);
    if (rcut.mk != nullptr) {
      __syncthreads();
      block_cuts(base, cnt, okr);
    }
    return;
  }
  const u32 ph = 31u - (u32)__clz(vary);   // highest varying digit
  // 1. split on digit ph into the extra buffer; h.hist[ph] becomes the
  //    sub-run starts (no later step writes that row)
  sweep_hist(true, nullptr, cnt, 1u << ph);
  digit_starts(ph);
  if (tid < 256u) h.hist[ph][tid] = h.off[tid];
  __syncthreads();
  chunk_pass(true, nullptr, nullptr, cnt, ph, xkr, xvr);
  // 2. the sub-runs in order
  u32 v = 0;
  while (v < 256u) {   // uniform: every thread reads the same LDS row
    const u32 s0 = h.hist[ph][v];
    u32 v2 = v;
    while (v2 < 256u) {
      const u32 e2 = v2 < 255u ? h.hist[ph][v2 + 1] : cnt;
      if (e2 - s0 > kLocalCap) break;
      ++v2;
    }
    if (v2 > v) {
      // sub-runs v .. v2-1 fit LDS together: sort them there
      const u32 n = (v2 < 256u ? h.hist[ph][v2] : cnt) - s0;
      if (n > 0) {
        const u32 ipt = (n + kLocalNT - 1) / kLocalNT;
        K kand = ~K(0), kor = K(0);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
          key[k] = K(0);
          if ((u32)k < ipt && li < n) {
            key[k] = xkr[s0 + li];
            if (PAY != kPayNone) pay[k] = xvr[s0 + li];
            kand &= key[k];
            kor |= key[k];
          }
        }
        const u32 passes = varying_digits<K>(kand, kor, npass, m.red) & ((2u << ph) - 1u);
        run_lds_passes<K, V, PAY>(key, pay, n, ipt, passes, h, s_k, s_v);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
          const u32 li = w * 64u * ipt + (u32)k * 64u + lane;
          if ((u32)k < ipt && li < n) {
            okr[s0 + li] = key[k];
            if (PAY != kPayNone) ovr[s0 + li] = pay[k];
          }
        }
        __syncthreads();
      }
      v = v2;
      continue;
    }
    // sub-run v alone is longer than kLocalCap: chunked passes over the
    // digits (below ph) that vary inside it, from the extra buffer,
    // alternating with the output region, the last one into the output
    const u32 n = (v < 255u ? h.hist[ph][v + 1] : cnt) - s0;
    K* const sxk = xkr + s0;
    V* const sxv = xvr + s0;
    K* const sok = okr + s0;
    V* const sov = ovr + s0;
    const u32 vary2 = sweep_vary(false, sxk, n, ph);
    const u32 np2 = (u32)__popc(vary2);
    if (np2 > 0) sweep_hist(false, sxk, n, vary2);
    u32 done = 0;
    for (u32 p = 0; p < ph; ++p) {
      if (!((vary2 >> p) & 1u)) continue;
      digit_starts(p);
      const bool to_out = (done & 1u) == 0u;   // the input is in the extra buffer
      chunk_pass(false, to_out ? sxk : sok, to_out ? sxv : sov, n, p, to_out ? sok : sxk,
                 to_out ? sov : sxv);
      ++done;
    }
    if ((done & 1u) == 0u) {   // an even number of passes left it in the extra buffer
      copy_items(false, sxk, sxv, n, sok, sov);
      __syncthreads();
    }
    ++v;
  }
  if (rcut.mk != nullptr) {
    __syncthreads();   // the run is in the output: search it there
    block_cuts(base, cnt, okr);
  }
}

// Scratch shared by every sort call of one store.
struct SortScratch {
  u32* hist = nullptr;      // [2][P*R] ping-pong histogram slots
  u64* status = nullptr;    // [max_tiles * R]
  u64* status_cl = nullptr; // [max_tiles / cluster * R]
  u32* tile_ctr = nullptr;  // [16] per-pass tile ticket counters (cleared by k_radix_hist)
  u32* err = nullptr;       // sticky sort error bits (1: look-back wait gave up, 2: runs
                            // that do not fit the batch)
  u32 epoch = 0;            // last epoch used
  u32 parity = 0;           // histogram slot of the next call
  u64 max_items = 0;        // capacity of the status array, in items
  u32* toff = nullptr;      // [kSplitMaxTiles][256] digit starts of the split tiles
  void* xk = nullptr;       // [x_items] keys of long runs between passes (8-byte slots)
  void* xv = nullptr;       // [x_items] their payloads (8-byte slots)
  u64 x_items = 0;
  // optional per-kernel timing hooks (family 0: histogram, 1: one pass or
  // the tile split, 2: the per-run sort):
  // on_begin hands out the start/stop events of the next dispatch
  void (*on_begin)(void* ctx, int family, hipEvent_t* e0, hipEvent_t* e1) = nullptr;
  void (*on_end)(void* ctx, int family, hipEvent_t e0, hipEvent_t e1) = nullptr;
  void* hook_ctx = nullptr;
};

// Kernel launch that, given events, has the dispatch itself stamp them at its
// start and end (hipExtLaunchKernelGGL): timing then adds no marker packets
// between kernels.  Without events it is a plain launch.
template <typename F, typename... Args>
inline void launch_timed(hipEvent_t e0, hipEvent_t e1, F kernel, dim3 grid, dim3 block,
                         uint32_t shm, hipStream_t st, Args... args) {
  if (e0 && e1)
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, e0, e1, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
}

struct SortTimer {
  SortScratch& s;
  int fam;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SortTimer(SortScratch& s_, int fam_) : s(s_), fam(fam_) {
    if (s.on_begin) s.on_begin(s.hook_ctx, fam, &e0, &e1);
  }
  void end() {
    if (s.on_end && e0) s.on_end(s.hook_ctx, fam, e0, e1);
  }
};

// Pass kernel shape: 2048-item tiles of 512 threads x 4 items (eight waves
// share a tile's ranking and scatter; measured faster than 256 x 8 and
// 1024 x 2).  The persistent drain's 256-thread workgroups take the same
// tiles as 256 x 8, so both read the same look-back words.
constexpr int kSortNT = 512;
constexpr int kSortIPT = 4;
constexpr int kSortTile = kSortNT * kSortIPT;
constexpr int kDrainSortNT = 256;
constexpr int kDrainSortIPT = kSortTile / kDrainSortNT;

inline u64 sort_status_words(u64 max_items, int rb) {
  return ((max_items + kSortTile - 1) / kSortTile + 1) * (u64)(1 << rb);
}
inline u64 sort_cluster_words(u64 max_items) {
  return ((max_items + kSortTile - 1) / kSortTile / kSortCluster + 2) * 256ull;
}

// Host driver: sorts n pairs from (kin, vin) using ping-pong buffers
// (k0, v0) / (k1, v1).  Returns which buffer holds the result (0 or 1).
// `reset_status` is called when the epoch counter wraps.
template <typename K, typename V, int RB, int PAY>
hipError_t radix_sort(const K* kin, const V* vin, K* k0, V* v0, K* k1, V* v1, u32 n,
                      SortScratch& s, hipStream_t st, int* result_buf,
                      const RunCuts<K>* cuts = nullptr, bool* cuts_done = nullptr) {
  if (cuts_done) *cuts_done = false;
  constexpr int R = RadixShape<K, RB>::R;
  constexpr int P = RadixShape<K, RB>::P;
  if (n == 0) {
    *result_buf = 0;
    return hipSuccess;
  }
  if ((u64)n > s.max_items) return hipErrorInvalidValue;
  const u32 ntiles = (n + kSortTile - 1) / kSortTile;
  if (RB == 8 && n <= kSplitMaxItems && s.toff && s.xk && s.xv && n <= s.x_items) {
    // two launches: tile split on the top digit, then one workgroup per run
    if (s.epoch >= (1u << 30) - 1u) {
      hipError_t e = hipMemsetAsync(s.status, 0, sort_status_words(s.max_items, RB) * sizeof(u64), st);
      if (e != hipSuccess) return e;
      e = hipMemsetAsync(s.status_cl, 0, sort_cluster_words(s.max_items) * sizeof(u64), st);
      if (e != hipSuccess) return e;
      s.epoch = 0;
    }
    const u32 epoch = ++s.epoch;
    const u32 nsplit = (n + kSplitTile - 1) / kSplitTile;
    {
      SortTimer t(s, 1);
      launch_timed(t.e0, t.e1, k_tile_split<K, V, PAY>, dim3(nsplit), dim3(kSplitNT), 0, st, kin,
                   vin, k0, v0, s.toff, n, (u32)((P - 1) * RB));
      t.end();
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr size_t lds = run_sort_lds<K, V, PAY>();
    static bool lds_set = false;
    if (!lds_set) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_run_sort<K, V, PAY>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      lds_set = true;
    }
    {
      SortTimer t(s, 2);
      RunCuts<K> rc{};
      if (cuts) rc = *cuts;
      launch_timed(t.e0, t.e1, k_run_sort<K, V, PAY>, dim3(R), dim3(kLocalNT), (uint32_t)lds, st,
                   (const K*)k0, (const V*)v0, k1, v1, (K*)s.xk, (V*)s.xv, (const u32*)s.toff,
                   s.status, epoch, (u32)(P - 1), n, s.err, rc);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    *result_buf = 1;
    if (cuts_done && cuts && cuts->mk) *cuts_done = true;
    return hipSuccess;
  }
  u32* hist = s.hist + (size_t)s.parity * (P * R);
  u32* hist_next = s.hist + (size_t)(s.parity ^ 1u) * (P * R);
  s.parity ^= 1u;
  u32 hb = (n + 256u * kHistIPT - 1u) / (256u * kHistIPT);
  if (hb > 1024u) hb = 1024u;
  {
    SortTimer t(s, 0);
    launch_timed(t.e0, t.e1, k_radix_hist<K, RB>, dim3(hb), dim3(256), 0, st, kin, n, hist,
                 hist_next, s.tile_ctr);
    t.end();
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Small batches with 8-bit digits: one onesweep pass on the top digit, then
  // the runs are sorted on the other digits by k_local_sort (result in k1).
  const bool local = RB == 8 && n <= kLocalMaxItems && ((P - 1) & 1) == 1;
  for (int p = local ? P - 1 : 0; p < P; ++p) {
    if (s.epoch >= (1u << 30) - 1u) {
      e = hipMemsetAsync(s.status, 0, sort_status_words(s.max_items, RB) * sizeof(u64), st);
      if (e != hipSuccess) return e;
      e = hipMemsetAsync(s.status_cl, 0, sort_cluster_words(s.max_items) * sizeof(u64), st);
      if (e != hipSuccess) return e;
      s.epoch = 0;
    }
    const u32 epoch = ++s.epoch;
    const bool first = local || p == 0;
    const K* ki = first ? kin : ((p & 1) ? k0 : k1);
    const V* vi = first ? vin : ((p & 1) ? v0 : v1);
    K* ko = (local || !(p & 1)) ? k0 : k1;
    V* vo = (local || !(p & 1)) ? v0 : v1;
    PassArgs<K, V> pa;
    pa.kin = ki;
    pa.vin = vi;
    pa.kout = ko;
    pa.vout = vo;
    pa.n = n;
    pa.shift = (u32)(p * RB);
    pa.hist_p = hist + p * R;
    pa.status = s.status;
    pa.status_cl = s.status_cl;
    pa.epoch = epoch;
    pa.err = s.err;
    SortTimer t(s, 1);
    launch_timed(t.e0, t.e1, k_onesweep<K, V, RB, kSortNT, kSortIPT, PAY>, dim3(ntiles),
                 dim3(kSortNT), 0, st, pa);
    t.end();
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (local) {
    constexpr size_t lds = local_sort_lds<K, V, PAY>();
    static bool lds_set = false;
    if (!lds_set) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_local_sort<K, V, PAY>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      lds_set = true;
    }
    SortTimer t(s, 2);
    launch_timed(t.e0, t.e1, k_local_sort<K, V, PAY>, dim3(R), dim3(kLocalNT), (uint32_t)lds, st,
                 k0, v0, k1, v1, (const u32*)(hist + (P - 1) * R), (u32)(P - 1), n, s.err);
    t.end();
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    *result_buf = 1;
    return hipSuccess;
  }
  *result_buf = ((P - 1) & 1) ? 1 : 0;
  return hipSuccess;
}

}  // namespace flix
