// Epochs: a coalesced group of requests with mixed reads and updates.
//
// Order inside an epoch: every read (lookup, range) observes the store as it
// was before the epoch; then the updates take effect, and for a key updated
// more than once the entry that comes last in the epoch's update array wins.
// An update whose value is the reserved all-ones pattern is a delete.
//
// The updates are sorted by key with a stable sort (so entries of one key stay
// in array order), folded to the last entry of every key, and split into a
// sorted upsert list and a sorted delete list whose lengths stay on the
// device.  The bucket kernels then run on those lists with the length read
// from device memory, so preparing an epoch never waits for the host.
#pragma once

#include "flix_build.hpp"
#include "flix_device.hpp"
#include "flix_update.hpp"

namespace flix {

// 0: superseded by a later entry of the same key, 1: upsert, 2: delete.
template <typename K>
__device__ __forceinline__ u32 fold_class(const K* k, const K* v, u64 i, u64 n) {
  if (i + 1 < n && k[i] == k[i + 1]) return 0u;
  return v[i] == ~K(0) ? 2u : 1u;
}

template <typename K>
__global__ __launch_bounds__(kCompactNT) void k_fold_count(const K* __restrict__ k,
                                                          const K* __restrict__ v, u64 n,
                                                          u32* __restrict__ bsum_ins,
                                                          u32* __restrict__ bsum_del) {
  __shared__ u32 s_tmp[kCompactNT / 64 + 1];
  const u64 base = (u64)blockIdx.x * kCompactTile + (u64)threadIdx.x * kCompactIPT;
  u32 ci = 0, cd = 0;
  for (int j = 0; j < kCompactIPT; ++j) {
    const u64 i = base + j;
    if (i < n) {
      const u32 c = fold_class(k, v, i, n);
      ci += c == 1u;
      cd += c == 2u;
    }
  }
  u32 ti, td;
  block_exclusive_scan<kCompactNT>(ci, s_tmp, &ti);
  block_exclusive_scan<kCompactNT>(cd, s_tmp, &td);
  if (threadIdx.x == 0) {
    bsum_ins[blockIdx.x] = ti;
    bsum_del[blockIdx.x] = td;
  }
}

template <typename K>
__global__ __launch_bounds__(kCompactNT) void k_fold_scatter(
    const K* __restrict__ k, const K* __restrict__ v, u64 n, const u32* __restrict__ off_ins,
    const u32* __restrict__ off_del, K* __restrict__ ins_k, K* __restrict__ ins_v,
    K* __restrict__ del_k) {
  __shared__ u32 s_tmp[kCompactNT / 64 + 1];
  const u64 base = (u64)blockIdx.x * kCompactTile + (u64)threadIdx.x * kCompactIPT;
  u32 cls[kCompactIPT];
  u32 ci = 0, cd = 0;
  for (int j = 0; j < kCompactIPT; ++j) {
    const u64 i = base + j;
    cls[j] = i < n ? fold_class(k, v, i, n) : 0u;
    ci += cls[j] == 1u;
    cd += cls[j] == 2u;
  }
  u32 ti, td;
  u32 pi = block_exclusive_scan<kCompactNT>(ci, s_tmp, &ti) + off_ins[blockIdx.x];
  u32 pd = block_exclusive_scan<kCompactNT>(cd, s_tmp, &td) + off_del[blockIdx.x];
  for (int j = 0; j < kCompactIPT; ++j) {
    const u64 i = base + j;
    if (cls[j] == 1u) {
      ins_k[pi] = k[i];
      ins_v[pi] = v[i];
      ++pi;
    } else if (cls[j] == 2u) {
      del_k[pd++] = k[i];
    }
  }
}

// Slice discovery over a sorted list whose length is in device memory; the
// grid is sized for the largest possible length.
template <typename K, int NT, int S, bool INSERT>
__global__ __launch_bounds__(NT) void k_slices_counted(SliceArgs<K> a, const u32* __restrict__ m_dev) {
  __shared__ SliceSmem<K, S, NT> sm;
  const u32 m = *m_dev;
  if (m == 0) return;
  if ((u64)blockIdx.x * S >= (u64)m + a.nb) return;
  a.m = m;
  slices_share<K, NT, S, INSERT>(a, blockIdx.x, sm);
}

template <typename K, int GL, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(sizeof(K) == 4 ? 6 : 1))) void k_insert_counted(
    UpdArgs<K> a, u32 lds_items, const u32* __restrict__ m_dev) {
  extern __shared__ unsigned char s_dyn[];
  __shared__ UpdShared sh;
  a.m = *m_dev;
  if (a.m == 0) return;
  insert_items<K, GL, NT>(a, lds_items, blockIdx.x, gridDim.x, s_dyn, sh);
}

template <typename K, int GL, int NT>
__global__ __launch_bounds__(NT) void k_delete_counted(UpdArgs<K> a, u32 lds_items,
                                                       const u32* __restrict__ m_dev) {
  extern __shared__ unsigned char s_dyn[];
  __shared__ UpdShared sh;
  a.m = *m_dev;
  if (a.m == 0) return;
  delete_items<K, GL, NT>(a, lds_items, blockIdx.x, gridDim.x, s_dyn, sh);
}

}  // namespace flix
