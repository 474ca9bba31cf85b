// Bucket-group read path: the batch sort and the bucket kernel of a read
// batch in two launches.
//
// The paper sorts every batch, and then each bucket binary-searches the sorted
// list for the slice between its neighbour's maxBucket and its own
// (Section 3.3, Section 4.1).  On MI355X the whole sorted batch never has to
// reach HBM for that: the buckets are cut into G groups of consecutive buckets
// (a group's upper bound is the maxBucket of its last bucket), and
//
//   k_part         reads the batch once.  Every 4096-item tile splits its
//                  items stably by group (ballot ranks, as in a radix pass),
//                  writes them back group by group inside the tile, records
//                  the tile's group offsets and adds its group counts to the
//                  group totals.  No look-back and no separate histogram.
//   k_group_read   one workgroup per chunk of at most C items of one group:
//                  it gathers the chunk from the tiles, radix-sorts it in LDS
//                  on the key bits that vary inside the chunk, loads the
//                  group's maxBucket entries and head words, lets every bucket
//                  of the group binary-search its slice of the sorted chunk
//                  and resolves the slices (phases A and B of flix_read2.hpp).
//
// A group with more than C items is cut into several chunks, each sorted and
// resolved on its own: reads do not change the store, so any subset of a
// bucket's slice can be answered independently.  Chunks are numbered group by
// group from the group totals, so extra workgroups take the chunks of large
// (skewed) groups in parallel.
#pragma once

#include "flix_device.hpp"
#include "flix_read2.hpp"
#include "flix_sort.hpp"

namespace flix {

constexpr int kPartNT = 256;
constexpr int kPartIPT = 16;
constexpr u32 kPartTile = kPartNT * kPartIPT;   // items per partition tile
constexpr u32 kGroupBitsMax = 10;
constexpr u32 kGroupMax = 1u << kGroupBitsMax;  // groups per store at most
constexpr u32 kGroupBucketsMax = 1024;          // buckets per group at most
constexpr u32 kGroupTilesMax = 1024;            // tiles per batch at most (2^22 items)

// Groups of a store with nb buckets: at most kGroupMax groups of equal bucket
// counts (the last one may be shorter).  Returns false when a group would
// exceed kGroupBucketsMax buckets (the group path is then not used).
__host__ __device__ inline bool group_shape(u32 nb, u32* ngroups, u32* per_group) {
  u32 bpg = (nb + kGroupMax - 1) / kGroupMax;
  if (bpg == 0) bpg = 1;
  const u32 g = (nb + bpg - 1) / bpg;
  *ngroups = g;
  *per_group = bpg;
  return bpg <= kGroupBucketsMax && g <= kGroupMax;
}

// Bits needed to number g groups (0 for a single group).
__host__ __device__ inline u32 group_bits(u32 g) {
  u32 b = 0;
  while ((1u << b) < g) ++b;
  return b;
}

// Group upper bounds: split[i] = maxBucket of the last bucket of group i, for
// i < G - 1 (the last group ends at KEY_MAX).
template <typename K>
__global__ void k_build_split(const K* __restrict__ mkba, u32 nb, u32 bpg, u32 ngroups,
                              K* __restrict__ split) {
  const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i + 1 < ngroups) {
    u64 last = (u64)(i + 1) * bpg - 1;
    if (last >= nb) last = nb - 1;
    split[i] = mkba[last];
  }
}

template <typename K, typename P>
struct PartArgs {
  const K* keys;      // [n] in input order
  const P* vin;       // values (kPayValue) or nullptr
  u32 n;
  const K* split;     // [G - 1] group upper bounds
  u32 ngroups;        // G
  u32 gbits;          // group_bits(G)
  K* tk;              // [n] keys, grouped inside each tile
  P* tp;              // [n] payload (input position or value), same order
  u32* gpre;          // [ntiles][G + 1] start of every group inside each tile
  u32* gtot;          // [G] group totals (zero before the launch; atomically summed)
  u32* gtot_clear;    // [G] totals slot of the next call, cleared here (may be null)
};

// Dynamic LDS of k_part: splitters, per-wave group counts, the tile's group
// starts, the staged tile and the scan scratch.
template <typename K, typename P, int PAY>
struct PartLds {
  static constexpr size_t split = 0;
  static constexpr size_t wc = (split + (kGroupMax - 1) * sizeof(K) + 15) & ~size_t(15);
  static constexpr size_t gstart = wc + (kPartNT / 64) * kGroupMax * sizeof(u32);
  static constexpr size_t k = (gstart + (kGroupMax + 1) * sizeof(u32) + 15) & ~size_t(15);
  static constexpr size_t p = k + kPartTile * sizeof(K);
  static constexpr size_t tmp = p + (PAY == kPayNone ? 0 : kPartTile * sizeof(P));
  static constexpr size_t bytes = tmp + (kPartNT / 64 + 1) * sizeof(u32);
};

template <typename K, typename P, int PAY>
__global__ __launch_bounds__(kPartNT) void k_part(PartArgs<K, P> a) {
  using L = PartLds<K, P, PAY>;
  extern __shared__ unsigned char lds[];
  K* s_split = reinterpret_cast<K*>(lds + L::split);
  u32(*s_wc)[kGroupMax] = reinterpret_cast<u32(*)[kGroupMax]>(lds + L::wc);
  u32* s_gstart = reinterpret_cast<u32*>(lds + L::gstart);
  K* s_k = reinterpret_cast<K*>(lds + L::k);
  P* s_p = reinterpret_cast<P*>(lds + L::p);
  u32* s_tmp = reinterpret_cast<u32*>(lds + L::tmp);
  constexpr int IPT = kPartIPT;
  constexpr int WAVES = kPartNT / 64;
  const u32 tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const u32 G = a.ngroups;
  const u32 tile = blockIdx.x;
  const u32 tile0 = tile * kPartTile;
  const u32 m = a.n - tile0 < kPartTile ? a.n - tile0 : kPartTile;

  if (tile == 0 && a.gtot_clear)
    for (u32 g = tid; g < G; g += kPartNT) a.gtot_clear[g] = 0;
  // Items (wave-striped) and splitters in one round of loads.
  K key[IPT];
  P pay[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
    if (li < m) {
      key[k] = a.keys[tile0 + li];
      if (PAY == kPayIndex) pay[k] = (P)(tile0 + li);
      if (PAY == kPayValue) pay[k] = a.vin[tile0 + li];
    } else {
      key[k] = K(0);
      if (PAY != kPayNone) pay[k] = P(0);
    }
  }
  for (u32 i = tid; i + 1 < G; i += kPartNT) s_split[i] = a.split[i];
  for (u32 i = tid; i < WAVES * kGroupMax; i += kPartNT) (&s_wc[0][0])[i] = 0;
  __syncthreads();
  // Group of every item: the first group whose upper bound is >= the key.
  u32 grp[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) grp[k] = lower_bound_idx<K>(s_split, 0u, G - 1, key[k]);
  // Stable rank of every item among the same-group items of its wave.
  u32 rank[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
    const bool valid = li < m;
    const u32 d = grp[k];
    u64 msk = wave_ballot(valid);
    for (u32 b = 0; b < a.gbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const u64 bb = wave_ballot(bit);
      msk &= bit ? bb : ~bb;
    }
    const u32 below = rank_below(msk);
    const u32 cnt = (u32)__popcll(msk);
    const u32 base = valid ? s_wc[w][d] : 0u;
    rank[k] = base + below;
    if (valid && below == cnt - 1) s_wc[w][d] = base + cnt;
  }
  __syncthreads();
  // Per-group totals of the tile (exclusive prefixes across waves in s_wc),
  // then the tile's group starts.
  constexpr u32 GPT = kGroupMax / kPartNT;
  u32 tot[GPT];
  u32 sum = 0;
#pragma unroll
  for (u32 r = 0; r < GPT; ++r) {
    const u32 g = tid * GPT + r;
    u32 t = 0;
    if (g < G) {
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) {
        const u32 c = s_wc[ww][g];
        s_wc[ww][g] = t;
        t += c;
      }
    }
    tot[r] = t;
    sum += t;
  }
  u32 total;
  u32 ex = block_exclusive_scan<kPartNT>(sum, s_tmp, &total);
#pragma unroll
  for (u32 r = 0; r < GPT; ++r) {
    const u32 g = tid * GPT + r;
    if (g < G) s_gstart[g] = ex;
    ex += tot[r];
  }
  if (tid == 0) s_gstart[G] = total;
  __syncthreads();
  // Scatter into LDS group by group, then write the tile out in that order.
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
    if (li < m) {
      const u32 pos = s_gstart[grp[k]] + s_wc[w][grp[k]] + rank[k];
      s_k[pos] = key[k];
      if (PAY != kPayNone) s_p[pos] = pay[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const u32 i = tid + (u32)r * kPartNT;
    if (i < m) {
      a.tk[tile0 + i] = s_k[i];
      if (PAY != kPayNone) a.tp[tile0 + i] = s_p[i];
    }
  }
  u32* row = a.gpre + (u64)tile * (G + 1);
  for (u32 g = tid; g <= G; g += kPartNT) row[g] = s_gstart[g];
#pragma unroll
  for (u32 r = 0; r < GPT; ++r) {
    const u32 g = tid * GPT + r;
    if (g < G && tot[r]) atomicAdd(&a.gtot[g], tot[r]);
  }
}

template <typename K>
struct GroupArgs {
  const K* tk;        // k_part output
  const u32* tp;      // input positions, same order
  const u32* gpre;    // [ntiles][G + 1]
  const u32* gtot;    // [G]
  const K* split;     // [G - 1]
  u32 n;
  u32 ntiles;
  u32 ngroups;
  u32 bpg;            // buckets per group
  u32 chunk_items;    // C: items per chunk (NT * IPT of the kernel)
};

// Number of chunks of a group of t items.
__device__ __forceinline__ u32 chunks_of(u32 t, u32 c) { return (t + c - 1) / c; }

// Upper bound of the chunks a batch of n items over G groups can produce.
__host__ __device__ inline u32 group_chunk_bound(u32 n, u32 ngroups, u32 c) {
  const u32 nonempty = n < ngroups ? n : ngroups;
  return nonempty + (n + c - 1) / c;
}

// Dynamic LDS of k_group_read, in bytes, for C items and B buckets per group.
// The region `x` holds, one after another in time: the chunk map (G words),
// the tile segment table (2 * (ntiles + 1) words), the sort's per-wave digit
// counts, and finally the result codes of phase A (C words).
template <typename K>
struct GroupLds {
  size_t q, idx, hi, cnt, x, mk, e, hw, tl, tmp, bytes;
  __host__ __device__ GroupLds(u32 C, u32 NT, u32 B, bool range) {
    size_t o = 0;
    auto take = [&](size_t b) {
      const size_t at = o;
      o = (o + b + 15) & ~size_t(15);
      return at;
    };
    q = take((size_t)C * sizeof(K));
    idx = take((size_t)C * 4);
    hi = range ? take((size_t)C * sizeof(K)) : 0;
    cnt = range ? take((size_t)C * 4) : 0;
    size_t xw = (size_t)C;
    if (xw < kGroupMax + 1) xw = kGroupMax + 1;
    if (xw < 2 * (kGroupTilesMax + 1)) xw = 2 * (kGroupTilesMax + 1);
    if (xw < (NT / 64) * 256) xw = (NT / 64) * 256;
    x = take(xw * 4);
    mk = take((size_t)B * sizeof(K));
    e = take((size_t)(B + 1) * 4);
    hw = take((size_t)(B + 1) * 4);
    tl = take((size_t)(B + 1) * 2);
    tmp = take((NT / 64 + 8) * 4);
    bytes = o;
  }
};

// One chunk of one group: gather, sort in LDS, bound search, resolve.
template <typename K, int NT, int IPT, int GL, int KPL, int U>
__global__ __launch_bounds__(NT) void k_group_read(GroupArgs<K> ga, ReadArgs<K> a, int op) {
  constexpr u32 C = (u32)NT * IPT;
  constexpr int WAVES = NT / 64;
  extern __shared__ unsigned char lds[];
  const GroupLds<K> L(C, NT, kGroupBucketsMax, op == kOpRange);
  K* s_q = reinterpret_cast<K*>(lds + L.q);
  u32* s_idx = reinterpret_cast<u32*>(lds + L.idx);
  K* s_hi = reinterpret_cast<K*>(lds + L.hi);
  u32* s_cnt = reinterpret_cast<u32*>(lds + L.cnt);
  u32* s_x = reinterpret_cast<u32*>(lds + L.x);
  K* s_mk = reinterpret_cast<K*>(lds + L.mk);
  u32* s_e = reinterpret_cast<u32*>(lds + L.e);
  u32* s_hw = reinterpret_cast<u32*>(lds + L.hw);
  unsigned short* s_tl = reinterpret_cast<unsigned short*>(lds + L.tl);
  u32* s_tmp = reinterpret_cast<u32*>(lds + L.tmp);
  u32* s_misc = s_tmp + WAVES + 1;   // [0] group, [1] chunk, [2] ntouch, [3..4] key range
  const u32 tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const u32 G = ga.ngroups;

  // 1. Chunk map: chunks of every group in group order; this workgroup takes
  //    chunk blockIdx.x of that list.
  {
    constexpr u32 GPT = kGroupMax / NT;
    u32 c[GPT];
    u32 sum = 0;
#pragma unroll
    for (u32 r = 0; r < GPT; ++r) {
      const u32 g = tid * GPT + r;
      c[r] = g < G ? chunks_of(ga.gtot[g], C) : 0u;
      sum += c[r];
    }
    u32 total;
    u32 ex = block_exclusive_scan<NT>(sum, s_tmp, &total);
#pragma unroll
    for (u32 r = 0; r < GPT; ++r) {
      const u32 g = tid * GPT + r;
      if (g < G) s_x[g] = ex;
      ex += c[r];
    }
    __syncthreads();
    if (blockIdx.x >= total) return;   // uniform: no chunk for this workgroup
    if (tid == 0) {
      // last group whose first chunk is <= blockIdx.x (groups with no chunk
      // share their start with the next group, so take the last such one)
      const u32 g = upper_bound_idx<u32>(s_x, 0u, G, blockIdx.x) - 1u;
      s_misc[0] = g;
      s_misc[1] = blockIdx.x - s_x[g];
    }
    __syncthreads();
  }
  const u32 g = s_misc[0];
  const u32 chunk = s_misc[1];
  const u32 gt = ga.gtot[g];
  const u32 c0 = chunk * C;
  const u32 m = gt - c0 < C ? gt - c0 : C;   // items of this chunk
  __syncthreads();

  // 2. Segment table of the group: tile t holds its items at
  //    [t*tile + gpre[t][g], t*tile + gpre[t][g+1]).
  const u32 nt = ga.ntiles;
  u32* s_seg = s_x;               // [nt + 1] exclusive prefix of the segment sizes
  u32* s_sbase = s_x + nt + 1;    // [nt] first item of each segment
  {
    constexpr u32 TPT = kGroupTilesMax / NT;
    u32 cnt[TPT], base[TPT];
    u32 sum = 0;
#pragma unroll
    for (u32 r = 0; r < TPT; ++r) {
      const u32 t = tid * TPT + r;
      cnt[r] = 0;
      base[r] = 0;
      if (t < nt) {
        const u32* row = ga.gpre + (u64)t * (G + 1);
        const u32 s0 = row[g], s1 = row[g + 1];
        cnt[r] = s1 > s0 ? s1 - s0 : 0u;
        base[r] = t * kPartTile + s0;
      }
      sum += cnt[r];
    }
    u32 total;
    u32 ex = block_exclusive_scan<NT>(sum, s_tmp, &total);
#pragma unroll
    for (u32 r = 0; r < TPT; ++r) {
      const u32 t = tid * TPT + r;
      if (t < nt) {
        s_seg[t] = ex;
        s_sbase[t] = base[r];
      }
      ex += cnt[r];
    }
    if (tid == 0) s_seg[nt] = total;
    if (total != gt) {   // the tiles disagree with the totals: never expected
      if (tid == 0) atomicCAS(a.err, 0u, kErrInternal);
      return;
    }
    __syncthreads();
  }

  // 3. Gather the chunk (wave-striped) and, in the same round, the group's
  //    maxBucket entries and head words.
  const u32 b0 = g * ga.bpg;
  const u32 nbl = (a.nb - b0) < ga.bpg ? (a.nb - b0) : ga.bpg;
  K key[IPT];
  u32 pay[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
    key[k] = K(0);
    pay[k] = 0;
    if (li < m) {
      const u32 j = c0 + li;
      const u32 t = upper_bound_idx<u32>(s_seg, 0u, nt, j) - 1u;
      const u32 gi = s_sbase[t] + (j - s_seg[t]);
      if (gi < ga.n) {
        key[k] = ga.tk[gi];
        pay[k] = ga.tp[gi];
      }
    }
  }
  constexpr u32 RB = (kGroupBucketsMax + NT - 1) / NT;
  K mk[RB];
  u64 hwr[RB];
#pragma unroll
  for (u32 r = 0; r < RB; ++r) {
    const u32 i = tid + r * NT;
    hwr[r] = (u64)kNil << 32;
    if (i < nbl) {
      mk[r] = a.mkba[b0 + i];
      hwr[r] = *reinterpret_cast<const u64*>(&a.hdr[b0 + i].size);
    }
  }
  // key range of the chunk: the sort only needs the bits that vary
  K kmin = key_max<K>(), kmax = K(0);
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
    if (li < m) {
      kmin = key[k] < kmin ? key[k] : kmin;
      kmax = key[k] > kmax ? key[k] : kmax;
    }
  }
  __syncthreads();   // segment table no longer needed: s_x is reused below
#pragma unroll
  for (u32 r = 0; r < RB; ++r) {
    const u32 i = tid + r * NT;
    if (i < nbl) {
      s_mk[i] = mk[r];
      s_hw[i] = (u32)hwr[r] | ((u32)(hwr[r] >> 32) != kNil ? kChainBit : 0u);
    }
  }
  // reduce the key range over the workgroup
  for (int off = 32; off > 0; off >>= 1) {
    const K a0 = __shfl_xor(kmin, off, 64);
    const K a1 = __shfl_xor(kmax, off, 64);
    kmin = a0 < kmin ? a0 : kmin;
    kmax = a1 > kmax ? a1 : kmax;
  }
  K* s_kr = reinterpret_cast<K*>(s_x);   // [2 * WAVES] per-wave min and max
  if (lane == 0) {
    s_kr[2 * w] = kmin;
    s_kr[2 * w + 1] = kmax;
  }
  __syncthreads();
  kmin = s_kr[0];
  kmax = s_kr[1];
#pragma unroll
  for (int ww = 1; ww < WAVES; ++ww) {
    kmin = s_kr[2 * ww] < kmin ? s_kr[2 * ww] : kmin;
    kmax = s_kr[2 * ww + 1] > kmax ? s_kr[2 * ww + 1] : kmax;
  }
  __syncthreads();
  const K diff = kmin ^ kmax;
  u32 nbits = 0;
  if (diff) nbits = sizeof(K) * 8 - (sizeof(K) == 4 ? (u32)__clz((u32)diff) : (u32)__clzll((u64)diff));
  const u32 npass = (nbits + 7) / 8;

  // 4. Stable LSD radix sort of the chunk in LDS on the varying bits (8-bit
  //    digits, ballot ranks over wave-striped items as in a onesweep tile);
  //    the last pass leaves the sorted keys and positions in s_q / s_idx.
  u32(*s_wc)[256] = reinterpret_cast<u32(*)[256]>(s_x);
  if (npass == 0) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < m) {
        s_q[li] = key[k];
        s_idx[li] = pay[k];
      }
    }
  }
  for (u32 p = 0; p < npass; ++p) {
    const u32 shift = p * 8u;
    for (u32 i = tid; i < WAVES * 256u; i += NT) (&s_wc[0][0])[i] = 0;
    __syncthreads();
    u32 rank[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      const bool valid = li < m;
      const u32 d = digit_of<K, 8>(key[k], shift);
      const u64 msk = match_digit<8>(d, wave_ballot(valid));
      const u32 below = rank_below(msk);
      const u32 cnt = (u32)__popcll(msk);
      const u32 base = valid ? s_wc[w][d] : 0u;
      rank[k] = base + below;
      if (valid && below == cnt - 1) s_wc[w][d] = base + cnt;
    }
    __syncthreads();
    u32 tot = 0;
    if (tid < 256u) {
#pragma unroll
      for (int ww = 0; ww < WAVES; ++ww) {
        const u32 c = s_wc[ww][tid];
        s_wc[ww][tid] = tot;
        tot += c;
      }
    }
    u32 dummy;
    const u32 ds = block_exclusive_scan<NT>(tid < 256u ? tot : 0u, s_tmp, &dummy);
    // digit starts go to s_e (free until the bound search)
    if (tid < 256u) s_e[tid] = ds;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
      if (li < m) {
        const u32 d = digit_of<K, 8>(key[k], shift);
        const u32 pos = s_e[d] + s_wc[w][d] + rank[k];
        s_q[pos] = key[k];
        s_idx[pos] = pay[k];
      }
    }
    __syncthreads();
    if (p + 1 < npass) {
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const u32 li = w * 64u * IPT + (u32)k * 64u + lane;
        if (li < m) {
          key[k] = s_q[li];
          pay[k] = s_idx[li];
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // range upper bounds follow their queries' input positions
  if (op == kOpRange) {
    K hv[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 j = tid + (u32)k * NT;
      if (j < m) hv[k] = a.hi[s_idx[j]];
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const u32 j = tid + (u32)k * NT;
      if (j < m) s_hi[j] = hv[k];
    }
  }

  // 5. Bound search: bucket lb's slice ends at the first key above its
  //    maxBucket; then the touched buckets are listed.
  for (u32 lb = tid; lb < nbl; lb += NT)
    s_e[lb] = (lb + 1 < nbl) ? upper_bound_idx<K>(s_q, 0u, m, s_mk[lb]) : m;
  __syncthreads();
  constexpr u32 PER = (kGroupBucketsMax + NT - 1) / NT;
  u32 flags = 0, ntc = 0;
#pragma unroll
  for (u32 r = 0; r < PER; ++r) {
    const u32 lb = tid * PER + r;
    if (lb < nbl) {
      const u32 s = lb ? s_e[lb - 1] : 0u;
      if (s_e[lb] > s) {
        flags |= 1u << r;
        ++ntc;
      }
    }
  }
  u32 ntot;
  u32 wpos = block_exclusive_scan<NT>(ntc, s_tmp, &ntot);
#pragma unroll
  for (u32 r = 0; r < PER; ++r)
    if (flags & (1u << r)) s_tl[wpos++] = (unsigned short)(tid * PER + r);
  __syncthreads();

  // 6. Phases A and B.
  SliceView<K> v;
  v.q = s_q;
  v.hi = s_hi;
  v.idx = s_idx;
  v.pos = s_x;
  v.cnt = s_cnt;
  v.e = s_e;
  v.hw = s_hw;
  v.tl = s_tl;
  v.list = nullptr;   // ranges past their node take the one-lane path here
  v.list_cap = 0;
  v.nlist = nullptr;
  v.lnode = nullptr;
  v.lbk = nullptr;
  resolve_slices<K, NT, GL, KPL, U, IPT>(a, op, v, b0, m, ntot);
}

}  // namespace flix
