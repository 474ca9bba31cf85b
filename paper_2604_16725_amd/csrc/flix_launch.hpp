// Launchers of the kernel families that live in translation units of their
// own (compiled in parallel): the read kernels (flix_read_tu.hip) and the
// persistent drain (flix_drain_tu.hip).  The host code of the C ABI
// (flix.hip) calls them through these plain functions.
#pragma once

#include <hip/hip_runtime.h>

#include "flix_drain.hpp"
#include "flix_group.hpp"
#include "flix_read2.hpp"

namespace flix {

// Read kernel over sorted shares (k_merge_cuts + k_read_apply2 form) with GL
// lanes per bucket and node capacity `cap`; e0/e1 (may be null) are stamped
// by the dispatch.
template <typename K>
void launch_read2(u32 gl, u32 cap, const ReadArgs<K>& a, int op, u32 grid, hipStream_t st,
                  hipEvent_t e0, hipEvent_t e1);

// Bucket-group read kernel (k_group_read); `chunk` items per workgroup.
template <typename K>
void launch_group(u32 gl, u32 cap, const GroupArgs<K>& ga, const ReadArgs<K>& a, int op,
                  u32 grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1);

// Everything one persistent drain launch needs.
struct DrainLaunch {
  int key_bits;
  u32 radix_bits, gl, cap, lds_items, chunk, max_batch;
  const DrainBatch* batches;
  u32 nbatch;
  const StoreLayout* layout;
  Ctl* ctl;
  void* bk[2];
  void* bp[2];
  u32* hist;
  u64* status;
  u64* status_cl;
  u64 status_words, cluster_words;
  WorkItem* work;
  DrainCtl* dctl;
  unsigned long long* tstamp;
  int* grid;        // in/out: co-resident workgroups (0: not sized yet)
  size_t* shm;      // in/out: dynamic LDS the grid was sized for
};

// Sizes the co-resident grid on first use, then launches the drain.  Returns
// hipSuccess, a runtime error, or hipErrorInvalidConfiguration when not even
// one workgroup fits a CU.
hipError_t drain_launch(const DrainLaunch& d, hipStream_t st);

}  // namespace flix
