// Host side of the FliX C ABI (include/flix.h): store allocation, the batch
// pipelines (sort -> bucket kernels) and the test/ops aids.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/flix.h"
#include "flix_build.hpp"
#include "flix_device.hpp"
#include "flix_drain.hpp"
#include "flix_epoch.hpp"
#include "flix_group.hpp"
#include "flix_launch.hpp"
#include "flix_read.hpp"
#include "flix_read2.hpp"
#include "flix_sort.hpp"
#include "flix_update.hpp"

using namespace flix;

// Scratch of flix_dump_noalloc: per-bucket totals, their offsets, the block
// sums of the offset scan and the scan total, for stores of at most
// kNoAllocBuckets buckets (16 MiB, held by every GPU the library runs on
// until the process ends).
constexpr u64 kNoAllocBuckets = 1ull << 21;
constexpr u64 kNoAllocBlocks = kNoAllocBuckets / 256;
constexpr u64 kNoAllocWords = 2 * kNoAllocBuckets + kNoAllocBlocks + 64;
static __device__ __align__(256) u32 scratch[kNoAllocWords];

namespace {

constexpr int kFamilies = 13;
const char* kFamilyNames[kFamilies] = {"sort_hist", "sort_pass", "read_apply", "slices",
                                       "insert_apply", "delete_apply", "read_cuts", "sort_local",
                                       "part", "group_read", "insert_st", "insert_wide",
                                       "delete_wide"};
enum Family {
  F_HIST = 0, F_PASS = 1, F_READ = 2, F_PRE = 3, F_INSERT = 4, F_DELETE = 5, F_CUTS = 6,
  F_LOCAL = 7, F_PART = 8, F_GROUP = 9, F_INSERT_ST = 10, F_INSERT_WIDE = 11,
  F_DELETE_WIDE = 12
};
int sort_family(int fam) { return fam == 0 ? F_HIST : fam == 1 ? F_PASS : F_LOCAL; }

struct Timing {
  bool on = false;
  u32 mask = 0;   // bit f: family f is timed
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[kFamilies] = {};
  uint64_t count[kFamilies] = {};
};

}  // namespace

// Scratch of one epoch slot: the sorted read lists, the sorted and folded
// update lists and a sort scratch of its own, so that one slot can be
// prepared while another slot's epoch is applied.
struct EpochSlot {
  u64 cap = 0;                         // items per list
  void* lk[2] = {nullptr, nullptr};    // lookups: keys, original index
  void* lp[2] = {nullptr, nullptr};
  void* rk[2] = {nullptr, nullptr};    // ranges: lo, original index
  void* rp[2] = {nullptr, nullptr};
  void* uk[2] = {nullptr, nullptr};    // updates: keys, values
  void* up[2] = {nullptr, nullptr};
  void* ins_k = nullptr;               // folded upserts (sorted, distinct)
  void* ins_v = nullptr;
  void* del_k = nullptr;               // folded deletes (sorted, distinct)
  u32* bsum = nullptr;                 // [2][blocks] fold block counts
  u32* counts = nullptr;               // [0] upserts, [1] deletes, [2..3] spare
  SortScratch ss;
  int rl = 0, rr = 0, ru = 0;          // which ping-pong buffer holds each sorted list
  bool prepared = false;
  u64 n_lookup = 0, n_range = 0, n_update = 0;
};

struct flix_store {
  flix_config cfg{};
  int kb = 32;
  u32 ksz = 4;
  u32 cap = 64, fill = 32, rb = 8, gl = 16;
  u64 max_batch = 0;
  // directory and node pool
  u32 nb = 0;          // buckets
  u32 nb_alloc = 0;    // capacity of the directory arrays
  u32 pool = 0;        // nodes
  void* mkba = nullptr;
  NodeHdr* hdr = nullptr;
  void* nkeys = nullptr;
  void* nvals = nullptr;
  u32* bnodes = nullptr;
  u64* occ = nullptr;    // bucket occupancy summary [occ_words(nb_alloc)]
  OccLevels occl{};      // its three levels for the current bucket count
  u32* cuts = nullptr;   // read-share cuts [(max_batch + nb_alloc) / 512 + 2]
  u32* mktop = nullptr;  // [257] first MKBA entry of every top key digit
  // bucket groups of the read path (flix_group.hpp)
  bool grp_ok = false;   // the store's shape fits the group kernels
  u32 ngrp = 1, bpg = 1;
  void* split = nullptr; // [kGroupMax] group upper bounds
  u32* gpre = nullptr;   // [tiles(max_batch)][kGroupMax + 1] tile group starts
  u32* gtot = nullptr;   // [2][kGroupMax] group totals, two slots
  u32 gslot = 0;         // totals slot of the next read call
  u32* free_ids = nullptr;
  Ctl* ctl = nullptr;
  // scratch
  void* bk[2] = {nullptr, nullptr};   // sort keys ping-pong [max_batch]
  void* bp[2] = {nullptr, nullptr};   // sort payload ping-pong [max_batch] (8-byte slots)
  WorkItem* work = nullptr;           // [work_slots(max_batch) + wide_slots(max_batch)]
  SortScratch ss;
  Timing tm;
  // persistent drain: its own look-back words, histogram slots and control
  u64* d_status = nullptr;
  u64* d_status_cl = nullptr;
  u64 d_status_words = 0, d_cluster_words = 0;
  u32* d_hist = nullptr;
  DrainCtl* dctl = nullptr;
  int drain_grid = 0;                 // co-resident workgroups of the drain kernel
  size_t drain_shm = 0;
  StoreLayout* d_layout = nullptr;    // layout record read by drains (graph replays)
  u32 upd_resident[4] = {0, 0, 0, 0}; // resident workgroups of each update kernel
  // epoch slots (allocated by the first epoch call)
  EpochSlot* ep[2] = {nullptr, nullptr};
};

namespace {

thread_local char g_last_error[256] = "";

int note_hip_error(hipError_t e, const char* what, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s", what, line,
                hipGetErrorString(e));
  return FLIX_EHIP;
}

#define HIP_TRY(x)                                               \
  do {                                                           \
    hipError_t e_ = (x);                                         \
    if (e_ != hipSuccess) return note_hip_error(e_, #x, __LINE__); \
  } while (0)

inline hipStream_t S(void* st) { return reinterpret_cast<hipStream_t>(st); }

u64 node_bytes(const flix_store* s) { return (u64)s->cap * 2 * s->ksz + sizeof(NodeHdr); }

// ---- timing -----------------------------------------------------------------
// Timing token: the start/stop events of one kernel dispatch (both null while
// timing is off); the launch stamps them (launch_timed).
struct TmTok {
  hipEvent_t b = nullptr, e = nullptr;
};
TmTok tm_arm(flix_store* s, int fam) {
  TmTok t;
  if (!s->tm.on || !(s->tm.mask & (1u << fam))) return t;
  if (s->tm.used + 2 > s->tm.pool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return t;
      s->tm.pool.push_back(e);
    }
  }
  t.b = s->tm.pool[s->tm.used++];
  t.e = s->tm.pool[s->tm.used++];
  return t;
}
void tm_done(flix_store* s, int fam, const TmTok& t) {
  if (t.b && t.e) s->tm.pending.push_back({fam, {t.b, t.e}});
}
void tm_collect(flix_store* s) {
  for (auto& p : s->tm.pending) {
    (void)hipEventSynchronize(p.second.second);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.second.first, p.second.second);
    s->tm.ms[p.first] += ms;
    s->tm.count[p.first] += 1;
  }
  s->tm.pending.clear();
  s->tm.used = 0;
}

// ---- allocation -------------------------------------------------------------
// Optional allocator hook (flix_set_allocator): device buffers come from it
// instead of hipMalloc / hipFree.
struct AllocHook {
  flix_alloc_fn alloc = nullptr;
  flix_free_fn free = nullptr;
  void* ctx = nullptr;
};
AllocHook g_alloc;

template <typename T>
int dev_alloc(T** p, u64 bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (g_alloc.alloc) {
    void* q = g_alloc.alloc(bytes, g_alloc.ctx);
    if (!q) {
      std::snprintf(g_last_error, sizeof(g_last_error), "allocator hook failed for %llu bytes",
                    (unsigned long long)bytes);
      return FLIX_ENOMEM;
    }
    *p = static_cast<T*>(q);
    return FLIX_OK;
  }
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    std::snprintf(g_last_error, sizeof(g_last_error), "hipMalloc of %llu bytes: %s",
                  (unsigned long long)bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    return FLIX_ENOMEM;
  }
  return FLIX_OK;
}
template <typename T>
void dev_free(T** p) {
  if (*p && g_alloc.free) {
    // hipFree waits for the device; a hook's free may not, so wait here
    (void)hipDeviceSynchronize();
    g_alloc.free(static_cast<void*>(*p), g_alloc.ctx);
    *p = nullptr;
    return;
  }
  if (*p) (void)hipFree(*p);
  *p = nullptr;
}

// Row table and long-run buffers of the two-launch sort (batches of up to
// kSplitMaxItems items).
int alloc_split_scratch(SortScratch& ss, u64 items) {
  const u64 want = items < kSplitMaxItems ? items : kSplitMaxItems;
  int rc;
  if (!ss.toff && (rc = dev_alloc(&ss.toff, (u64)kSplitMaxTiles * 256u * sizeof(u32)))) return rc;
  if (want <= ss.x_items) return FLIX_OK;
  dev_free(&ss.xk);
  dev_free(&ss.xv);
  ss.x_items = 0;
  if ((rc = dev_alloc(&ss.xk, want * 8)) || (rc = dev_alloc(&ss.xv, want * 8))) return rc;
  ss.x_items = want;
  return FLIX_OK;
}

int ensure_sort_capacity(flix_store* s, u64 items) {
  if (items <= s->ss.max_items) return FLIX_OK;
  HIP_TRY(hipDeviceSynchronize());
  dev_free(&s->ss.status);
  u64 words = sort_status_words(items, 8);  // sized for the widest digit
  int rc = dev_alloc(&s->ss.status, words * sizeof(u64));
  if (rc) return rc;
  HIP_TRY(hipMemset(s->ss.status, 0, words * sizeof(u64)));
  dev_free(&s->ss.status_cl);
  u64 cwords = sort_cluster_words(items);
  rc = dev_alloc(&s->ss.status_cl, cwords * sizeof(u64));
  if (rc) return rc;
  HIP_TRY(hipMemset(s->ss.status_cl, 0, cwords * sizeof(u64)));
  s->ss.epoch = 0;
  s->ss.max_items = items;
  return alloc_split_scratch(s->ss, items);
}

int alloc_pool(flix_store* s, u32 pool) {
  dev_free(&s->hdr);
  dev_free(&s->nkeys);
  dev_free(&s->nvals);
  dev_free(&s->free_ids);
  s->pool = 0;
  int rc;
  if ((rc = dev_alloc(&s->hdr, (u64)pool * sizeof(NodeHdr)))) return rc;
  if ((rc = dev_alloc(&s->nkeys, (u64)pool * s->cap * s->ksz))) return rc;
  if ((rc = dev_alloc(&s->nvals, (u64)pool * s->cap * s->ksz))) return rc;
  if ((rc = dev_alloc(&s->free_ids, (u64)pool * sizeof(u32)))) return rc;
  s->pool = pool;
  return FLIX_OK;
}

// Entries of the read-share cut list for batches of up to n keys over nb buckets.
u64 cuts_for(u64 n, u64 nb) { return (n + nb) / 512u + 2u; }

// Partition tiles of a batch of up to n items, capped at the group kernels' limit.
u64 group_tiles(u64 n) {
  const u64 t = (n + kPartTile - 1) / kPartTile;
  return t < kGroupTilesMax ? t : kGroupTilesMax;
}

// Directory arrays for nb buckets.  The new arrays are allocated before the
// old ones are freed, so a failed allocation leaves the directory as it was.
int alloc_dir(flix_store* s, u32 nb) {
  if (nb <= s->nb_alloc) return FLIX_OK;
  void* mk = nullptr;
  u32* bn = nullptr;
  u64* oc = nullptr;
  u32* cu = nullptr;
  int rc;
  if ((rc = dev_alloc(&mk, (u64)nb * s->ksz)) || (rc = dev_alloc(&bn, (u64)nb * sizeof(u32))) ||
      (rc = dev_alloc(&oc, occ_words(nb) * sizeof(u64))) ||
      (rc = dev_alloc(&cu, (cuts_for(s->max_batch, nb) * sizeof(u32))))) {
    dev_free(&mk); dev_free(&bn); dev_free(&oc); dev_free(&cu);
    return rc;
  }
  dev_free(&s->mkba);
  dev_free(&s->bnodes);
  dev_free(&s->cuts);
  dev_free(&s->occ);
  s->mkba = mk;
  s->bnodes = bn;
  s->occ = oc;
  s->cuts = cu;
  s->nb_alloc = nb;
  return FLIX_OK;
}

u32 auto_pool(const flix_store* s, u64 nbuckets) {
  u64 f = s->cap / 2;
  u64 p = 2 * nbuckets + 2 * ((s->max_batch + f - 1) / f) + 64;
  if (p > 0xFFFFFFF0ull) p = 0xFFFFFFF0ull;
  return (u32)p;
}

// ---- sort dispatch ----------------------------------------------------------
// payload: 0 none, 1 index, 2 value.  Result in s->bk[r], s->bp[r].
template <typename K>
int sort_batch_t(flix_store* s, const K* keys, const K* vals, u32 n, int pay, hipStream_t st,
                 int* r, const RunCuts<K>* cuts = nullptr, bool* cuts_done = nullptr) {
  hipError_t e;
  K* k0 = (K*)s->bk[0];
  K* k1 = (K*)s->bk[1];
  if (cuts_done) *cuts_done = false;
  if (pay == kPayIndex) {
    u32* p0 = (u32*)s->bp[0];
    u32* p1 = (u32*)s->bp[1];
    e = s->rb == 4 ? radix_sort<K, u32, 4, kPayIndex>(keys, nullptr, k0, p0, k1, p1, n, s->ss, st, r)
                   : radix_sort<K, u32, 8, kPayIndex>(keys, nullptr, k0, p0, k1, p1, n, s->ss, st, r,
                                                      cuts, cuts_done);
  } else if (pay == kPayValue) {
    K* p0 = (K*)s->bp[0];
    K* p1 = (K*)s->bp[1];
    e = s->rb == 4 ? radix_sort<K, K, 4, kPayValue>(keys, vals, k0, p0, k1, p1, n, s->ss, st, r)
                   : radix_sort<K, K, 8, kPayValue>(keys, vals, k0, p0, k1, p1, n, s->ss, st, r);
  } else {
    e = s->rb == 4
            ? radix_sort<K, u32, 4, kPayNone>(keys, nullptr, k0, nullptr, k1, nullptr, n, s->ss, st, r)
            : radix_sort<K, u32, 8, kPayNone>(keys, nullptr, k0, nullptr, k1, nullptr, n, s->ss, st, r);
  }
  return e == hipSuccess ? FLIX_OK : note_hip_error(e, "sort", __LINE__);
}

// Per-call counters are cleared by a one-block kernel at the start of every
// update call (they are read by the kernels that follow on the stream).
__global__ void k_reset_call(Ctl* ctl, u32 clear_abort) {
  if (threadIdx.x == 0) {
    ctl->need = 0;
    ctl->call_err = 0;
    if (clear_abort) ctl->call_abort = 0;
  }
  reset_work_regions(ctl, threadIdx.x);
}

// Epoch gate: the node bound of the epoch's upserts, summed on the store as
// it is before the epoch's deletes, decides for the whole update list.  The
// deletes only shrink buckets and chains and return nodes, so a list that
// passes here also passes the insert kernel's own check after the deletes;
// a list that fails is rejected before any node changes.
__global__ void k_epoch_gate(Ctl* ctl) {
  if (threadIdx.x == 0) {
    const u32 err = ctl->call_err;
    const bool abort = err != 0 || ctl->need > (u64)ctl->free_top;
    ctl->call_abort = abort ? 1u : 0u;
    if (abort) atomicCAS(&ctl->status, 0u, err != 0 ? err : kErrNomem);
  }
}

void sort_hook_begin(void* ctx, int fam, hipEvent_t* e0, hipEvent_t* e1) {
  const TmTok t = tm_arm(static_cast<flix_store*>(ctx), sort_family(fam));
  *e0 = t.b;
  *e1 = t.e;
}
void sort_hook_end(void* ctx, int fam, hipEvent_t e0, hipEvent_t e1) {
  TmTok t;
  t.b = e0;
  t.e = e1;
  tm_done(static_cast<flix_store*>(ctx), sort_family(fam), t);
}

template <typename K>
int sort_batch(flix_store* s, const void* keys, const void* vals, u64 n, int pay, hipStream_t st,
               int* r, const RunCuts<K>* cuts = nullptr, bool* cuts_done = nullptr) {
  return sort_batch_t<K>(s, (const K*)keys, (const K*)vals, (u32)n, pay, st, r, cuts, cuts_done);
}

// ---- read path --------------------------------------------------------------
template <typename K>
struct ReadCfg;
template <>
struct ReadCfg<u32> {
  static constexpr int S = 512;
};
template <>
struct ReadCfg<u64> {
  static constexpr int S = 512;
};

// Bucket kernel over an already sorted read list (keys + original index).
template <typename K>
int read_apply_sorted(flix_store* s, int op, const K* skeys, const u32* sidx, u64 n, void* out_k,
                      void* out_v, const void* hi, u32* counts, u32 maxpq, hipStream_t st,
                      bool cuts_ready = false) {
  ReadArgs<K> a;
  a.skeys = skeys;
  a.sidx = sidx;
  a.m = (u32)n;
  a.mkba = (const K*)s->mkba;
  a.nb = s->nb;
  a.hdr = s->hdr;
  a.nkeys = (const K*)s->nkeys;
  a.nvals = (const K*)s->nvals;
  a.cap = s->cap;
  a.share = ReadCfg<K>::S;
  a.out_v = (K*)out_v;
  a.out_k = (K*)out_k;
  a.hi = (const K*)hi;
  a.counts = counts;
  a.maxpq = maxpq;
  a.pool = s->pool;
  a.err = &s->ctl->status;
  a.occ = s->occl.w0;
  u64 grid = ((u64)n + s->nb + a.share - 1) / a.share;
  // cut list: half a wave per share boundary (the list holds cuts_for(max_batch,
  // nb_alloc) >= grid + 1 entries)
  a.cuts = nullptr;
  if (cuts_ready) {
    a.cuts = s->cuts;   // written by the batch sort
  } else if (s->cuts && grid + 1 <= cuts_for(s->max_batch, s->nb_alloc)) {
    const u32 ncuts = (u32)grid + 1u;
    const TmTok tc = tm_arm(s, F_CUTS);
    launch_timed(tc.b, tc.e, k_merge_cuts<K>, dim3((ncuts + 7) / 8), dim3(256), 0, st, skeys,
                 (u32)n, (const K*)s->mkba, s->nb, a.share, ncuts, s->cuts);
    tm_done(s, F_CUTS, tc);
    a.cuts = s->cuts;
  }
  const TmTok t = tm_arm(s, F_READ);
  launch_read2<K>(s->gl, s->cap, a, op, (u32)grid, st, t.b, t.e);
  tm_done(s, F_READ, t);
  HIP_TRY(hipGetLastError());
  return FLIX_OK;
}

// Read batch on the bucket-group path: k_part, then k_group_read.
template <typename K>
int read_batch_groups(flix_store* s, int op, const K* keys, u64 n, void* out_k, void* out_v,
                      const void* hi, u32* counts, u32 maxpq, hipStream_t st) {
  const u32 ntiles = (u32)((n + kPartTile - 1) / kPartTile);
  u32* gtot = s->gtot + (size_t)s->gslot * kGroupMax;
  u32* gnext = s->gtot + (size_t)(s->gslot ^ 1u) * kGroupMax;
  s->gslot ^= 1u;
  PartArgs<K, u32> pa;
  pa.keys = keys;
  pa.vin = nullptr;
  pa.n = (u32)n;
  pa.split = (const K*)s->split;
  pa.ngroups = s->ngrp;
  pa.gbits = group_bits(s->ngrp);
  pa.tk = (K*)s->bk[0];
  pa.tp = (u32*)s->bp[0];
  pa.gpre = s->gpre;
  pa.gtot = gtot;
  pa.gtot_clear = gnext;
  {
    using L = PartLds<K, u32, kPayIndex>;
    static bool attr = false;
    if (!attr && L::bytes > 65536) {
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part<K, u32, kPayIndex>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::bytes));
      attr = true;
    }
    const TmTok t = tm_arm(s, F_PART);
    launch_timed(t.b, t.e, k_part<K, u32, kPayIndex>, dim3(ntiles), dim3(kPartNT),
                 (uint32_t)L::bytes, st, pa);
    tm_done(s, F_PART, t);
    HIP_TRY(hipGetLastError());
  }
  GroupArgs<K> ga;
  ga.tk = (const K*)s->bk[0];
  ga.tp = (const u32*)s->bp[0];
  ga.gpre = s->gpre;
  ga.gtot = gtot;
  ga.split = (const K*)s->split;
  ga.n = (u32)n;
  ga.ntiles = ntiles;
  ga.ngroups = s->ngrp;
  ga.bpg = s->bpg;
  ga.chunk_items = 2048;
  ReadArgs<K> a;
  a.skeys = nullptr;
  a.sidx = nullptr;
  a.m = (u32)n;
  a.mkba = (const K*)s->mkba;
  a.nb = s->nb;
  a.hdr = s->hdr;
  a.nkeys = (const K*)s->nkeys;
  a.nvals = (const K*)s->nvals;
  a.cap = s->cap;
  a.share = 0;
  a.out_v = (K*)out_v;
  a.out_k = (K*)out_k;
  a.hi = (const K*)hi;
  a.counts = counts;
  a.maxpq = maxpq;
  a.pool = s->pool;
  a.err = &s->ctl->status;
  a.occ = s->occl.w0;
  a.cuts = nullptr;
  const u32 grid = group_chunk_bound((u32)n, s->ngrp, 2048);
  const TmTok t = tm_arm(s, F_GROUP);
  launch_group<K>(s->gl, s->cap, ga, a, op, grid, st, t.b, t.e);
  tm_done(s, F_GROUP, t);
  HIP_TRY(hipGetLastError());
  return FLIX_OK;
}

template <typename K>
int read_batch(flix_store* s, int op, const void* keys, u64 n, void* out_k, void* out_v,
               const void* hi, u32* counts, u32 maxpq, hipStream_t st) {
  if (s->cfg.read_path == FLIX_READ_GROUPS && s->grp_ok && n <= (u64)kGroupTilesMax * kPartTile)
    return read_batch_groups<K>(s, op, (const K*)keys, n, out_k, out_v, hi, counts, maxpq, st);
  int r;
  // the run sort also writes the read kernel's share cuts when it can
  RunCuts<K> rc_args{};
  const u64 grid = ((u64)n + s->nb + ReadCfg<K>::S - 1) / ReadCfg<K>::S;
  const bool want = s->cuts && s->mktop && grid + 1 <= cuts_for(s->max_batch, s->nb_alloc);
  if (want) {
    rc_args.mk = (const K*)s->mkba;
    rc_args.mktop = s->mktop;
    rc_args.nb = s->nb;
    rc_args.share = ReadCfg<K>::S;
    rc_args.ncuts = (u32)grid + 1u;
    rc_args.cuts = s->cuts;
  }
  bool cuts_done = false;
  int rc = sort_batch<K>(s, keys, nullptr, n, kPayIndex, st, &r, want ? &rc_args : nullptr,
                         &cuts_done);
  if (rc) return rc;
  return read_apply_sorted<K>(s, op, (const K*)s->bk[r], (const u32*)s->bp[r], n, out_k, out_v, hi,
                              counts, maxpq, st, cuts_done);
}

// ---- update path ------------------------------------------------------------
template <typename K>
struct SliceCfg;
template <>
struct SliceCfg<u32> {
  static constexpr int S = 1024;
};
template <>
struct SliceCfg<u64> {
  static constexpr int S = 512;
};

constexpr int kUpdNT = 256;

// Slice length up to which the adaptive insert gives a bucket one lane: the
// single-lane kernel moves up to a node of keys per insert, so it only pays
// for nodes of at most 16 keys.
u32 adaptive_st_max(u32 cap) { return cap <= 16 ? (u32)FLIX_ST_MAX_KEYS : 0u; }

// Slice length from which a single-node bucket is merged by a whole workgroup
// (k_insert_wide): the lane-group kernel would walk such a slice in more than
// eight node-sized chunks, one after another.
u32 wide_min_keys(u32 cap) { return std::max<u32>(4 * cap, 256u); }

// Batch items staged per merge step: half a node (at least 64).  With
// capacity 128 a group's LDS is then 1.5 KB, so six workgroups fit a CU.
u32 upd_chunk(const flix_store* s) { return std::max<u32>(s->cap / 2, 64u); }
u32 upd_lds_items(const flix_store* s) { return s->cap + upd_chunk(s); }

// m_dev: null for a list of host-known length n; otherwise the length is read
// from device memory and n is its upper bound (grid sizing only).
// The grid gives every lane group one work item when there are few and is
// capped at the resident workgroup count when there are many, so each group
// then walks a run of items with the next one's loads in flight.
template <typename K, int GL>
void launch_update(flix_store* s, bool insert, const UpdArgs<K>& a, u64 items, hipStream_t st,
                   u32 lds_items, const u32* m_dev, const TmTok& t) {
  size_t shm = (size_t)(kUpdNT / GL) * 2 * lds_items * sizeof(K);
  static size_t attr_set[4] = {0, 0, 0, 0};
  const int which = (insert ? 1 : 0) + (m_dev ? 2 : 0);
  const void* fn;
  switch (which) {
    case 0: fn = reinterpret_cast<const void*>(&k_delete_apply<K, GL, kUpdNT>); break;
    case 1: fn = reinterpret_cast<const void*>(&k_insert_apply<K, GL, kUpdNT>); break;
    case 2: fn = reinterpret_cast<const void*>(&k_delete_counted<K, GL, kUpdNT>); break;
    default: fn = reinterpret_cast<const void*>(&k_insert_counted<K, GL, kUpdNT>); break;
  }
  if (shm > 65536 && shm > attr_set[which]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e == hipSuccess) attr_set[which] = shm;
    (void)hipGetLastError();
  }
  if (s->upd_resident[which] == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kUpdNT, shm) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu < 1 || cus < 1) {
      per_cu = 4;
      cus = 256;
    }
    (void)hipGetLastError();
    s->upd_resident[which] = (u32)(per_cu * cus);
  }
  const u32 gpb = kUpdNT / GL;
  u64 g2 = (items + gpb - 1) / gpb;
  if (g2 < 1) g2 = 1;
  if (g2 > s->upd_resident[which]) g2 = s->upd_resident[which];
  const u32 grid = (u32)g2;
  const dim3 g(grid), blk(kUpdNT);
  const uint32_t sh = (uint32_t)shm;
  switch (which) {
    case 0:
      launch_timed(t.b, t.e, k_delete_apply<K, GL, kUpdNT>, g, blk, sh, st, a, lds_items);
      break;
    case 1:
      launch_timed(t.b, t.e, k_insert_apply<K, GL, kUpdNT>, g, blk, sh, st, a, lds_items);
      break;
    case 2:
      launch_timed(t.b, t.e, k_delete_counted<K, GL, kUpdNT>, g, blk, sh, st, a, lds_items, m_dev);
      break;
    default:
      launch_timed(t.b, t.e, k_insert_counted<K, GL, kUpdNT>, g, blk, sh, st, a, lds_items, m_dev);
      break;
  }
}

// Slice discovery and the bucket kernel over an already sorted update list
// (the per-call counters must have been reset on the stream before).
template <typename K>
int update_apply_sorted(flix_store* s, bool insert, const K* skeys, const K* svals, u64 n,
                        const u32* m_dev, hipStream_t st) {
  SliceArgs<K> sa;
  sa.skeys = skeys;
  sa.svals = insert ? svals : nullptr;
  sa.m = (u32)n;
  sa.mkba = (const K*)s->mkba;
  sa.nb = s->nb;
  sa.hdr = s->hdr;
  sa.bnodes = s->bnodes;
  sa.cap = s->cap;
  sa.share = SliceCfg<K>::S;
  sa.work = s->work;
  sa.rcap = work_region_cap(s->max_batch);
  sa.ctl = s->ctl;
  // a long slice into a single-node bucket (a dense run of new keys) is merged
  // by a whole workgroup: the slice kernel lists those items
  const bool wide = insert && !m_dev &&
                    (s->cfg.insert_algo == FLIX_INSERT_TL_BULK ||
                     s->cfg.insert_algo == FLIX_INSERT_ADAPTIVE) &&
                    n >= wide_min_keys(s->cap);
  // a long slice or a long chain of a delete goes to the workgroup-wide
  // delete kernel
  const bool wide_del = !insert && !m_dev && n >= kWideDelKeys;
  if (wide || wide_del) {
    sa.wide_min = wide_min_keys(s->cap);
    sa.wide_cap = wide_slots(s->max_batch);
    sa.wide = s->work + work_slots(s->max_batch);
  }
  constexpr int SS = SliceCfg<K>::S;
  u64 grid = ((u64)n + s->nb + sa.share - 1) / sa.share;
  TmTok t = tm_arm(s, F_PRE);
  if (m_dev) {
    if (insert)
      launch_timed(t.b, t.e, k_slices_counted<K, 256, SS, true>, dim3(grid), dim3(256), 0, st, sa,
                   m_dev);
    else
      launch_timed(t.b, t.e, k_slices_counted<K, 256, SS, false>, dim3(grid), dim3(256), 0, st, sa,
                   m_dev);
  } else {
    if (insert)
      launch_timed(t.b, t.e, k_slices<K, 256, SS, true>, dim3(grid), dim3(256), 0, st, sa);
    else
      launch_timed(t.b, t.e, k_slices<K, 256, SS, false>, dim3(grid), dim3(256), 0, st, sa);
  }
  tm_done(s, F_PRE, t);
  HIP_TRY(hipGetLastError());

  UpdArgs<K> ua;
  ua.mkba = (const K*)s->mkba;
  ua.skeys = skeys;
  ua.svals = insert ? svals : nullptr;
  ua.m = (u32)n;
  ua.hdr = s->hdr;
  ua.nkeys = (K*)s->nkeys;
  ua.nvals = (K*)s->nvals;
  ua.bnodes = s->bnodes;
  ua.free_ids = s->free_ids;
  ua.cap = s->cap;
  ua.chunk = upd_chunk(s);
  ua.pool = s->pool;
  ua.work = s->work;
  ua.rcap = work_region_cap(s->max_batch);
  ua.ctl = s->ctl;
  ua.status = &s->ctl->status;
  ua.occ = s->occl;
  u32 lds_items = upd_lds_items(s);
  u64 items = std::min<u64>(n, s->nb);
  // insert kernel choice: the single-lane kernel takes the items its selector
  // names, the lane-group kernel the complement
  u32 algo = (insert && !m_dev) ? s->cfg.insert_algo : (u32)FLIX_INSERT_TL_BULK;
  // the listed long slices go to the workgroup-wide kernel; the lane-group
  // kernel skips them
  if (wide) {
    ua.wide_min = sa.wide_min;
    ua.wide_cap = sa.wide_cap;
    ua.wide = sa.wide;
    const u32 grid = (u32)std::min<u64>(1024, n / sa.wide_min + 1);
    const TmTok tw = tm_arm(s, F_INSERT_WIDE);
    launch_timed(tw.b, tw.e, k_insert_wide<K, 256>, dim3(grid), dim3(256), 0, st, ua);
    tm_done(s, F_INSERT_WIDE, tw);
    HIP_TRY(hipGetLastError());
  }
  if (algo == FLIX_INSERT_ADAPTIVE && adaptive_st_max(s->cap) == 0) algo = FLIX_INSERT_TL_BULK;
  if (algo != FLIX_INSERT_TL_BULK) {
    UpdArgs<K> us = ua;
    us.sel = algo == FLIX_INSERT_ST_SHIFT_RIGHT ? kSelAll
           : algo == FLIX_INSERT_ST_TL_MIXED    ? kSelRound
                                                : kSelShort;
    // adaptive: one lane per bucket only where a node is a few cache lines
    // (a lane shifts the node serially); larger nodes keep the lane group
    us.st_max = algo == FLIX_INSERT_ADAPTIVE ? adaptive_st_max(s->cap) : (u32)FLIX_ST_MAX_KEYS;
    const u32 grid = (u32)std::max<u64>(1, (items + 255) / 256);
    const TmTok ts = tm_arm(s, F_INSERT_ST);
    launch_timed(ts.b, ts.e, k_insert_st<K, 256>, dim3(grid), dim3(256), 0, st, us);
    tm_done(s, F_INSERT_ST, ts);
    HIP_TRY(hipGetLastError());
    if (algo == FLIX_INSERT_ST_SHIFT_RIGHT) return FLIX_OK;
    ua.sel = algo == FLIX_INSERT_ST_TL_MIXED ? kSelRoundL : kSelLong;
    ua.st_max = us.st_max;
  }
  t = tm_arm(s, insert ? F_INSERT : F_DELETE);
  switch (s->gl) {
    case 16: launch_update<K, 16>(s, insert, ua, items, st, lds_items, m_dev, t); break;
    case 32: launch_update<K, 32>(s, insert, ua, items, st, lds_items, m_dev, t); break;
    default: launch_update<K, 64>(s, insert, ua, items, st, lds_items, m_dev, t); break;
  }
  tm_done(s, insert ? F_INSERT : F_DELETE, t);
  HIP_TRY(hipGetLastError());
  if (wide_del) {
    ua.wide_min = sa.wide_min;
    ua.wide_cap = sa.wide_cap;
    ua.wide = sa.wide;
    const u32 grid = (u32)std::min<u64>(1024, n / kWideDelKeys + 1);
    const TmTok tw = tm_arm(s, F_DELETE_WIDE);
    launch_timed(tw.b, tw.e, k_delete_wide<K, 256>, dim3(grid), dim3(256), 0, st, ua);
    tm_done(s, F_DELETE_WIDE, tw);
    HIP_TRY(hipGetLastError());
  }
  return FLIX_OK;
}

// The insert slice kernel alone, for a device-counted list (the epoch gate's
// node bound on the store before the epoch's deletes).
template <typename K>
int update_slices_only(flix_store* s, const K* skeys, const K* svals, u64 n, const u32* m_dev,
                       hipStream_t st) {
  SliceArgs<K> sa;
  sa.skeys = skeys;
  sa.svals = svals;
  sa.m = (u32)n;
  sa.mkba = (const K*)s->mkba;
  sa.nb = s->nb;
  sa.hdr = s->hdr;
  sa.bnodes = s->bnodes;
  sa.cap = s->cap;
  sa.share = SliceCfg<K>::S;
  sa.work = s->work;
  sa.rcap = work_region_cap(s->max_batch);
  sa.ctl = s->ctl;
  constexpr int SS = SliceCfg<K>::S;
  const u64 grid = ((u64)n + s->nb + sa.share - 1) / sa.share;
  hipLaunchKernelGGL((k_slices_counted<K, 256, SS, true>), dim3(grid), dim3(256), 0, st, sa, m_dev);
  HIP_TRY(hipGetLastError());
  return FLIX_OK;
}

template <typename K>
int update_batch(flix_store* s, bool insert, const void* keys, const void* vals, u64 n,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_reset_call, dim3(1), dim3(kWorkRegions), 0, st, s->ctl, 1u);
  int r;
  int rc = sort_batch<K>(s, keys, vals, n, insert ? kPayValue : kPayNone, st, &r);
  if (rc) return rc;
  return update_apply_sorted<K>(s, insert, (const K*)s->bk[r],
                                insert ? (const K*)s->bp[r] : nullptr, n, nullptr, st);
}

// ---- epochs -----------------------------------------------------------------
void free_slot(EpochSlot* e) {
  for (int i = 0; i < 2; ++i) {
    dev_free(&e->lk[i]); dev_free(&e->lp[i]);
    dev_free(&e->rk[i]); dev_free(&e->rp[i]);
    dev_free(&e->uk[i]); dev_free(&e->up[i]);
  }
  dev_free(&e->ins_k); dev_free(&e->ins_v); dev_free(&e->del_k);
  dev_free(&e->bsum); dev_free(&e->counts);
  dev_free(&e->ss.hist); dev_free(&e->ss.status); dev_free(&e->ss.status_cl);
  dev_free(&e->ss.tile_ctr); dev_free(&e->ss.err);
  dev_free(&e->ss.toff); dev_free(&e->ss.xk); dev_free(&e->ss.xv);
  e->ss.x_items = 0;
}

int alloc_slot(flix_store* s, EpochSlot* e) {
  const u64 n = s->max_batch;
  const u64 K = s->ksz;
  const u64 nblk = (n + kCompactTile - 1) / kCompactTile;
  int rc;
  for (int i = 0; i < 2; ++i) {
    if ((rc = dev_alloc(&e->lk[i], n * K)) || (rc = dev_alloc(&e->lp[i], n * 4)) ||
        (rc = dev_alloc(&e->rk[i], n * K)) || (rc = dev_alloc(&e->rp[i], n * 4)) ||
        (rc = dev_alloc(&e->uk[i], n * K)) || (rc = dev_alloc(&e->up[i], n * K)))
      return rc;
  }
  if ((rc = dev_alloc(&e->ins_k, n * K)) || (rc = dev_alloc(&e->ins_v, n * K)) ||
      (rc = dev_alloc(&e->del_k, n * K)) || (rc = dev_alloc(&e->bsum, 2 * nblk * 4)) ||
      (rc = dev_alloc(&e->counts, 16)))
    return rc;
  const u64 words = sort_status_words(n, 8);
  const u64 cwords = sort_cluster_words(n);
  if ((rc = dev_alloc(&e->ss.hist, 2 * 2048 * sizeof(u32))) ||
      (rc = dev_alloc(&e->ss.status, words * 8)) || (rc = dev_alloc(&e->ss.status_cl, cwords * 8)) ||
      (rc = dev_alloc(&e->ss.tile_ctr, 64)) || (rc = dev_alloc(&e->ss.err, 16)))
    return rc;
  HIP_TRY(hipMemset(e->ss.hist, 0, 2 * 2048 * sizeof(u32)));
  HIP_TRY(hipMemset(e->ss.status, 0, words * 8));
  HIP_TRY(hipMemset(e->ss.status_cl, 0, cwords * 8));
  HIP_TRY(hipMemset(e->ss.tile_ctr, 0, 64));
  HIP_TRY(hipMemset(e->ss.err, 0, 16));
  HIP_TRY(hipMemset(e->counts, 0, 16));
  e->ss.max_items = n;
  e->ss.epoch = 0;
  e->ss.parity = 0;
  if ((rc = alloc_split_scratch(e->ss, n))) return rc;
  e->cap = n;
  return FLIX_OK;
}

int ensure_slots(flix_store* s) {
  if (s->ep[0]) return FLIX_OK;
  HIP_TRY(hipDeviceSynchronize());
  for (int i = 0; i < 2; ++i) {
    EpochSlot* e = new (std::nothrow) EpochSlot;
    if (!e) return FLIX_ENOMEM;
    int rc = alloc_slot(s, e);
    if (rc) {
      free_slot(e);
      delete e;
      for (int j = 0; j < i; ++j) {
        free_slot(s->ep[j]);
        delete s->ep[j];
        s->ep[j] = nullptr;
      }
      return rc;
    }
    s->ep[i] = e;
  }
  return FLIX_OK;
}

template <typename K, int RB>
int epoch_prepare_rb(EpochSlot* es, const flix_epoch* e, hipStream_t st) {
  hipError_t err = hipSuccess;
  if (e->n_lookup)
    err = radix_sort<K, u32, RB, kPayIndex>((const K*)e->d_lookup_keys, nullptr, (K*)es->lk[0],
                                            (u32*)es->lp[0], (K*)es->lk[1], (u32*)es->lp[1],
                                            (u32)e->n_lookup, es->ss, st, &es->rl);
  if (err == hipSuccess && e->n_range)
    err = radix_sort<K, u32, RB, kPayIndex>((const K*)e->d_range_lo, nullptr, (K*)es->rk[0],
                                            (u32*)es->rp[0], (K*)es->rk[1], (u32*)es->rp[1],
                                            (u32)e->n_range, es->ss, st, &es->rr);
  if (err == hipSuccess && e->n_update)
    err = radix_sort<K, K, RB, kPayValue>((const K*)e->d_update_keys, (const K*)e->d_update_vals,
                                          (K*)es->uk[0], (K*)es->up[0], (K*)es->uk[1],
                                          (K*)es->up[1], (u32)e->n_update, es->ss, st, &es->ru);
  if (err != hipSuccess) return note_hip_error(err, "epoch sort", __LINE__);
  if (e->n_update) {
    const u64 n = e->n_update;
    const u32 nblk = (u32)((n + kCompactTile - 1) / kCompactTile);
    const K* sk = (const K*)es->uk[es->ru];
    const K* sv = (const K*)es->up[es->ru];
    u32* bi = es->bsum;
    u32* bd = es->bsum + nblk;
    hipLaunchKernelGGL((k_fold_count<K>), dim3(nblk), dim3(kCompactNT), 0, st, sk, sv, n, bi, bd);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, bi, nblk, es->counts);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, bd, nblk, es->counts + 1);
    hipLaunchKernelGGL((k_fold_scatter<K>), dim3(nblk), dim3(kCompactNT), 0, st, sk, sv, n, bi, bd,
                       (K*)es->ins_k, (K*)es->ins_v, (K*)es->del_k);
    HIP_TRY(hipGetLastError());
  }
  return FLIX_OK;
}

template <typename K>
int epoch_apply_t(flix_store* s, EpochSlot* es, const flix_epoch* e, hipStream_t st) {
  int rc;
  if (e->n_lookup &&
      (rc = read_apply_sorted<K>(s, kOpLookup, (const K*)es->lk[es->rl], (const u32*)es->lp[es->rl],
                                 e->n_lookup, nullptr, e->d_lookup_vals, nullptr, nullptr, 0, st)))
    return rc;
  if (e->n_range &&
      (rc = read_apply_sorted<K>(s, kOpRange, (const K*)es->rk[es->rr], (const u32*)es->rp[es->rr],
                                 e->n_range, e->d_range_keys, e->d_range_vals, e->d_range_hi,
                                 e->d_range_counts, e->range_max, st)))
    return rc;
  if (e->n_update) {
    // the folded lists hold distinct keys, so deletes and upserts commute;
    // deletes go first and return nodes to the free list.  The upserts' node
    // bound is checked first, on the store before the deletes, so a rejected
    // epoch leaves the store unchanged.
    hipLaunchKernelGGL(k_reset_call, dim3(1), dim3(kWorkRegions), 0, st, s->ctl, 1u);
    if ((rc = update_slices_only<K>(s, (const K*)es->ins_k, (const K*)es->ins_v, e->n_update,
                                    es->counts, st)))
      return rc;
    hipLaunchKernelGGL(k_epoch_gate, dim3(1), dim3(64), 0, st, s->ctl);
    hipLaunchKernelGGL(k_reset_call, dim3(1), dim3(kWorkRegions), 0, st, s->ctl, 0u);
    if ((rc = update_apply_sorted<K>(s, false, (const K*)es->del_k, nullptr, e->n_update,
                                     es->counts + 1, st)))
      return rc;
    hipLaunchKernelGGL(k_reset_call, dim3(1), dim3(kWorkRegions), 0, st, s->ctl, 0u);
    if ((rc = update_apply_sorted<K>(s, true, (const K*)es->ins_k, (const K*)es->ins_v,
                                     e->n_update, es->counts, st)))
      return rc;
  }
  return FLIX_OK;
}

int epoch_validate(flix_store* s, uint32_t slot, const flix_epoch* e) {
  if (!s) return FLIX_ESTATE;
  if (!e || slot >= 2) return FLIX_EINVAL;
  if (e->reserved != 0) return FLIX_EINVAL;
  if (e->n_lookup > s->max_batch || e->n_range > s->max_batch || e->n_update > s->max_batch)
    return FLIX_EINVAL;
  if (e->n_lookup && (!e->d_lookup_keys || !e->d_lookup_vals)) return FLIX_EINVAL;
  if (e->n_range && (!e->d_range_lo || !e->d_range_hi || !e->d_range_counts)) return FLIX_EINVAL;
  if (e->n_range && e->range_max && !e->d_range_vals && !e->d_range_keys) return FLIX_EINVAL;
  if (e->n_update && (!e->d_update_keys || !e->d_update_vals)) return FLIX_EINVAL;
  return FLIX_OK;
}

// ---- bulk load --------------------------------------------------------------
// Rewrite the device layout record that drains read (after every change of
// the directory or the pool).  Synchronous: the store is idle at this point.
int publish_layout(flix_store* s) {
  if (!s->d_layout) return FLIX_OK;
  StoreLayout L{};
  L.mkba = s->mkba;
  L.hdr = s->hdr;
  L.nkeys = s->nkeys;
  L.nvals = s->nvals;
  L.bnodes = s->bnodes;
  L.free_ids = s->free_ids;
  L.nb = s->nb;
  L.pool = s->pool;
  L.occ = s->occl;
  HIP_TRY(hipMemcpy(s->d_layout, &L, sizeof(L), hipMemcpyHostToDevice));
  return FLIX_OK;
}

// Device address of `scratch` on each GPU (in host code the array's name is
// not a device address), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
u32* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(u32** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FLIX_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return note_hip_error(e, "scratch symbol address", __LINE__);
    g_scratch_ptr[dev] = static_cast<u32*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FLIX_OK;
}

// Dump kernels on caller-provided scratch: tot and off [nb], bs [ceil(nb/256)],
// total [1].  Asynchronous on st.
int dump_launch(flix_store* s, void* ko, void* vo, u64 capacity, u32* tot, u32* off, u32* bs,
                u32* total, hipStream_t st) {
  const u32 nb = s->nb;
  const u32 nblk = (nb + 255) / 256;
  const u32 g = std::min<u32>(nblk, 65535);
  hipLaunchKernelGGL(k_bucket_totals, dim3(g), dim3(256), 0, st, s->hdr, nb, s->pool, tot);
  hipLaunchKernelGGL(k_scan_blocks_u32, dim3(nblk), dim3(256), 0, st, tot, nb, off, bs);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, bs, nblk, total);
  hipLaunchKernelGGL(k_scan_addback, dim3(nblk), dim3(256), 0, st, off, nb, bs);
  const u32 gw = std::min<u32>((nb + 3) / 4, 65535);
  if (s->kb == 32)
    hipLaunchKernelGGL((k_dump_copy<u32>), dim3(gw), dim3(256), 0, st, s->hdr, (const u32*)s->nkeys,
                       (const u32*)s->nvals, nb, s->cap, s->pool, off, (u32*)ko, (u32*)vo,
                       (u64)capacity);
  else
    hipLaunchKernelGGL((k_dump_copy<u64>), dim3(gw), dim3(256), 0, st, s->hdr, (const u64*)s->nkeys,
                       (const u64*)s->nvals, nb, s->cap, s->pool, off, (u64*)ko, (u64*)vo,
                       (u64)capacity);
  HIP_TRY(hipGetLastError());
  return FLIX_OK;
}

// Every pair in ascending key order into ko / vo (at most `capacity` of them):
// per-bucket totals, their scan, then one wave per bucket copies its chain.
// Synchronizes st.
int dump_body(flix_store* s, void* ko, void* vo, u64 capacity, hipStream_t st) {
  const u32 nb = s->nb;
  const u32 nblk = (nb + 255) / 256;
  u32 *tot = nullptr, *off = nullptr, *bs = nullptr, *total = nullptr;
  int rc;
  if ((rc = dev_alloc(&tot, (u64)nb * 4)) || (rc = dev_alloc(&off, (u64)nb * 4)) ||
      (rc = dev_alloc(&bs, (u64)nblk * 4)) || (rc = dev_alloc(&total, 16))) {
    dev_free(&tot); dev_free(&off); dev_free(&bs); dev_free(&total);
    return rc;
  }
  rc = dump_launch(s, ko, vo, capacity, tot, off, bs, total, st);
  const hipError_t e2 = hipStreamSynchronize(st);
  dev_free(&tot); dev_free(&off); dev_free(&bs); dev_free(&total);
  if (rc) return rc;
  return e2 == hipSuccess ? FLIX_OK : note_hip_error(e2, "dump", __LINE__);
}

// Nodes, directory, occupancy summary and free stack from nd sorted, distinct
// pairs (Section 3.2 build rule: groups of `fill` consecutive keys, one node
// per bucket, the last key of a group is its maxBucket, KEY_MAX for the last
// bucket).  The pool and a directory of at least nbk buckets are allocated.
// Asynchronous on st.
// First MKBA entry of every top key digit (the block boundaries of the read
// cuts that the run sort writes).
template <typename K>
__global__ void k_mk_top(const K* __restrict__ mk, u32 nb, u32* __restrict__ top) {
  const u32 t = threadIdx.x;
  const K x = (K)((K)t << (sizeof(K) * 8 - 8));
  u32 lo = 0, hi = nb;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if (mk[mid] < x) lo = mid + 1; else hi = mid;
  }
  top[t] = lo;
  if (t == 0) top[256] = nb;
}

template <typename K>
int build_layout(flix_store* s, const K* ck, const K* cv, u64 nd, u32 nbk, hipStream_t st) {
  const u32 pool = s->pool;
  HIP_TRY(hipGetLastError());
  s->nb = nbk;
  if (nd) {
    u64 g = std::min<u64>((nd + 255) / 256, 65536);
    hipLaunchKernelGGL((k_build_nodes<K>), dim3(g), dim3(256), 0, st, ck, cv, nd, s->fill, s->cap,
                       (K*)s->nkeys, (K*)s->nvals);
    HIP_TRY(hipGetLastError());
  }
  u64 g = std::min<u64>((nbk + 255) / 256, 65536);
  hipLaunchKernelGGL((k_build_dir<K>), dim3(g), dim3(256), 0, st, ck, nd, s->fill, nbk,
                     (K*)s->mkba, s->hdr, s->bnodes);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL((k_mk_top<K>), dim3(1), dim3(256), 0, st, (const K*)s->mkba, nbk, s->mktop);
  HIP_TRY(hipGetLastError());
  // occupancy summary of the new directory
  s->occl.w0 = s->occ;
  s->occl.w1 = s->occ + occ_words0(nbk);
  s->occl.w2 = s->occl.w1 + occ_words1(nbk);
  hipLaunchKernelGGL(k_occ_build0, dim3((u32)((occ_words0(nbk) + 255) / 256)), dim3(256), 0, st,
                     s->hdr, nbk, s->occl.w0);
  hipLaunchKernelGGL(k_occ_build_up, dim3((u32)((occ_words1(nbk) + 255) / 256)), dim3(256), 0,
                     st, (const u64*)s->occl.w0, occ_words0(nbk), s->occl.w1, occ_words1(nbk));
  hipLaunchKernelGGL(k_occ_build_up, dim3((u32)((occ_words2(nbk) + 255) / 256)), dim3(256), 0,
                     st, (const u64*)s->occl.w1, occ_words1(nbk), s->occl.w2, occ_words2(nbk));
  HIP_TRY(hipGetLastError());
  u64 g2 = std::min<u64>((pool - nbk + 255) / 256 + 1, 65536);
  hipLaunchKernelGGL(k_build_free, dim3(g2), dim3(256), 0, st, nbk, pool, nd, s->free_ids, s->ctl);
  HIP_TRY(hipGetLastError());
  return FLIX_OK;
}

template <typename K>
int bulk_load_body(flix_store* s, const K* keys, const K* vals, u64 n, hipStream_t st) {
  if (n > 0xFFFFFFF0ull) return FLIX_EINVAL;
  // reserved value check before anything changes
  if (n) {
    HIP_TRY(hipMemsetAsync(&s->ctl->call_err, 0, sizeof(u32), st));
    u64 g = std::min<u64>((n + 255) / 256, 4096);
    hipLaunchKernelGGL((k_check_reserved<K>), dim3(g), dim3(256), 0, st, vals, n, &s->ctl->call_err);
    HIP_TRY(hipGetLastError());
    u32 err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &s->ctl->call_err, sizeof(u32), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (err) return FLIX_EINVAL;
  }
  // sorted, deduplicated pairs in temporary buffers
  K *tk0 = nullptr, *tk1 = nullptr, *tv0 = nullptr, *tv1 = nullptr, *ck = nullptr, *cv = nullptr;
  u32* bsum = nullptr;
  u64 nd = 0;
  int rc = FLIX_OK;
  auto cleanup = [&]() {
    dev_free(&tk0); dev_free(&tk1); dev_free(&tv0); dev_free(&tv1);
    dev_free(&ck); dev_free(&cv); dev_free(&bsum);
  };
  if (n) {
    if ((rc = ensure_sort_capacity(s, n))) return rc;
    if ((rc = dev_alloc(&tk0, n * sizeof(K))) || (rc = dev_alloc(&tk1, n * sizeof(K))) ||
        (rc = dev_alloc(&tv0, n * sizeof(K))) || (rc = dev_alloc(&tv1, n * sizeof(K))) ||
        (rc = dev_alloc(&ck, n * sizeof(K))) || (rc = dev_alloc(&cv, n * sizeof(K)))) {
      cleanup();
      return rc;
    }
    int r = 0;
    hipError_t e = s->rb == 4
        ? radix_sort<K, K, 4, kPayValue>(keys, vals, tk0, tv0, tk1, tv1, (u32)n, s->ss, st, &r)
        : radix_sort<K, K, 8, kPayValue>(keys, vals, tk0, tv0, tk1, tv1, (u32)n, s->ss, st, &r);
    if (e != hipSuccess) { cleanup(); return note_hip_error(e, "bulk load sort", __LINE__); }
    const K* sk = r ? tk1 : tk0;
    const K* sv = r ? tv1 : tv0;
    u32 nblk = (u32)((n + kCompactTile - 1) / kCompactTile);
    if ((rc = dev_alloc(&bsum, (u64)nblk * sizeof(u32)))) { cleanup(); return rc; }
    hipLaunchKernelGGL((k_compact_count<K>), dim3(nblk), dim3(kCompactNT), 0, st, sk, n, bsum);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, bsum, nblk, &s->ctl->scan_total);
    hipLaunchKernelGGL((k_compact_scatter<K>), dim3(nblk), dim3(kCompactNT), 0, st, sk, sv, n, bsum,
                       ck, cv);
    if ((e = hipGetLastError()) != hipSuccess) { cleanup(); return note_hip_error(e, "bulk load compaction", __LINE__); }
    u32 tot = 0;
    if (hipMemcpyAsync(&tot, &s->ctl->scan_total, sizeof(u32), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      cleanup();
      return FLIX_EHIP;
    }
    nd = tot;
  }
  u64 nbk = nd ? (nd + s->fill - 1) / s->fill : 1;
  if (nbk > 0xFFFFFF00ull) { cleanup(); return FLIX_EINVAL; }
  u32 pool = s->cfg.pool_bytes ? (u32)std::min<u64>(s->cfg.pool_bytes / node_bytes(s), 0xFFFFFFF0ull)
                               : auto_pool(s, nbk);
  if (nbk > pool) { cleanup(); return FLIX_ENOMEM; }
  if (pool != s->pool) {
    HIP_TRY(hipStreamSynchronize(st));
    if ((rc = alloc_pool(s, pool))) { cleanup(); return rc; }
  }
  if ((rc = alloc_dir(s, (u32)nbk))) { cleanup(); return rc; }
  if ((rc = build_layout<K>(s, ck, cv, nd, (u32)nbk, st))) { cleanup(); return rc; }
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  cleanup();
  if (e1 != hipSuccess) return note_hip_error(e1, "bulk load kernels", __LINE__);
  if (e2 != hipSuccess) return note_hip_error(e2, "bulk load sync", __LINE__);
  return FLIX_OK;
}

// Bucket groups of the read path for the current directory: their shape,
// upper bounds and cleared totals.  Synchronous (the store is idle).
template <typename K>
int rebuild_groups(flix_store* s, hipStream_t st) {
  u32 g = 1, bpg = 1;
  s->grp_ok = group_shape(s->nb, &g, &bpg) && s->gpre && s->split && s->gtot;
  s->ngrp = g;
  s->bpg = bpg;
  s->gslot = 0;
  if (!s->grp_ok) return FLIX_OK;
  if (g > 1)
    hipLaunchKernelGGL((k_build_split<K>), dim3((g + 255) / 256), dim3(256), 0, st,
                       (const K*)s->mkba, s->nb, bpg, g, (K*)s->split);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemsetAsync(s->gtot, 0, 2ull * kGroupMax * sizeof(u32), st));
  HIP_TRY(hipStreamSynchronize(st));
  return FLIX_OK;
}

// Bulk load, then the layout record and the bucket groups, also after a
// failure part way (the directory or the pool may have been reallocated).
template <typename K>
int bulk_load_t(flix_store* s, const K* keys, const K* vals, u64 n, hipStream_t st) {
  const int rc = bulk_load_body<K>(s, keys, vals, n, st);
  (void)hipStreamSynchronize(st);
  const int rp = publish_layout(s);
  const int rg = rebuild_groups<K>(s, st);
  return rc ? rc : (rp ? rp : rg);
}

// Restructuring (Section 3.5): the live pairs are read out in key order and laid
// out again by the build rule, so every bucket is one node at the bulk-load
// fill, chains are gone, underfull nodes are merged and maxBucket follows the
// current key distribution.  The pool keeps its size; a pool smaller than the
// new bucket count -> FLIX_ENOMEM with nothing changed.  Synchronizes.
template <typename K>
int restructure_t(flix_store* s, hipStream_t st, u64* before, u64* after) {
  Ctl hctl;
  HIP_TRY(hipMemcpyAsync(&hctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const u64 n = hctl.nkeys;
  if (before) *before = (u64)s->pool - hctl.free_top;
  const u64 nbk = n ? (n + s->fill - 1) / s->fill : 1;
  if (nbk > 0xFFFFFF00ull) return FLIX_EINVAL;
  if (nbk > s->pool) return FLIX_ENOMEM;
  K *ck = nullptr, *cv = nullptr;
  auto cleanup = [&]() { dev_free(&ck); dev_free(&cv); };
  int rc = FLIX_OK;
  if (n) {
    if ((rc = dev_alloc(&ck, n * sizeof(K))) || (rc = dev_alloc(&cv, n * sizeof(K))) ||
        (rc = dump_body(s, ck, cv, n, st))) {
      cleanup();
      return rc;
    }
  }
  // the old layout is no longer read: the directory may be replaced
  if ((rc = alloc_dir(s, (u32)nbk))) { cleanup(); return rc; }
  rc = build_layout<K>(s, ck, cv, n, (u32)nbk, st);
  const hipError_t e = hipStreamSynchronize(st);
  cleanup();
  const int rp = publish_layout(s);
  const int rg = rebuild_groups<K>(s, st);
  if (rc) return rc;
  if (e != hipSuccess) return note_hip_error(e, "restructure", __LINE__);
  if (rp || rg) return rp ? rp : rg;
  if (after) *after = nbk;
  return FLIX_OK;
}

int check_args(flix_store* s, u64 n, std::initializer_list<const void*> ptrs) {
  if (!s) return FLIX_ESTATE;
  if (n == 0) return 1;  // no-op
  if (n > s->max_batch) return FLIX_EINVAL;
  for (const void* p : ptrs)
    if (!p) return FLIX_EINVAL;
  return FLIX_OK;
}

void destroy_all(flix_store* s) {
  dev_free(&s->mkba);
  dev_free(&s->cuts);
  dev_free(&s->split);
  dev_free(&s->gpre);
  dev_free(&s->gtot);
  dev_free(&s->occ);
  dev_free(&s->hdr);
  dev_free(&s->nkeys);
  dev_free(&s->nvals);
  dev_free(&s->bnodes);
  dev_free(&s->free_ids);
  dev_free(&s->ctl);
  for (int i = 0; i < 2; ++i) {
    dev_free(&s->bk[i]);
    dev_free(&s->bp[i]);
  }
  dev_free(&s->work);
  dev_free(&s->ss.hist);
  dev_free(&s->ss.status);
  dev_free(&s->ss.status_cl);
  dev_free(&s->ss.tile_ctr);
  dev_free(&s->ss.toff);
  dev_free(&s->ss.xk);
  dev_free(&s->ss.xv);
  s->ss.x_items = 0;
  dev_free(&s->mktop);
  dev_free(&s->d_status);
  dev_free(&s->d_status_cl);
  dev_free(&s->d_hist);
  dev_free(&s->dctl);
  dev_free(&s->d_layout);
  dev_free(&s->ss.err);
  for (auto e : s->tm.pool) (void)hipEventDestroy(e);
  s->tm.pool.clear();
  for (int i = 0; i < 2; ++i) {
    if (s->ep[i]) {
      free_slot(s->ep[i]);
      delete s->ep[i];
      s->ep[i] = nullptr;
    }
  }
}

// ---- persistent drain -------------------------------------------------------
int drain_launch(flix_store* s, const DrainBatch* b, u32 nb, unsigned long long* ts,
                 hipStream_t st) {
  DrainLaunch d;
  d.key_bits = s->kb;
  d.radix_bits = s->rb;
  d.gl = s->gl;
  d.cap = s->cap;
  d.lds_items = upd_lds_items(s);
  d.chunk = upd_chunk(s);
  d.max_batch = (u32)s->max_batch;
  d.batches = b;
  d.nbatch = nb;
  d.layout = s->d_layout;
  d.ctl = s->ctl;
  d.bk[0] = s->bk[0];
  d.bk[1] = s->bk[1];
  d.bp[0] = s->bp[0];
  d.bp[1] = s->bp[1];
  d.hist = s->d_hist;
  d.status = s->d_status;
  d.status_cl = s->d_status_cl;
  d.status_words = s->d_status_words;
  d.cluster_words = s->d_cluster_words;
  d.work = s->work;
  d.dctl = s->dctl;
  d.tstamp = ts;
  d.grid = &s->drain_grid;
  d.shm = &s->drain_shm;
  const hipError_t e = flix::drain_launch(d, st);
  if (e == hipErrorInvalidConfiguration) return FLIX_EINVAL;
  if (e != hipSuccess) return note_hip_error(e, "drain launch", __LINE__);
  return FLIX_OK;
}

int drain_validate(flix_store* s, const flix_batch* h, u32 nbatch) {
  // look-back epochs of one drain must fit the 30-bit epoch field
  if (nbatch > (1u << 24)) return FLIX_EINVAL;
  for (u32 i = 0; i < nbatch; ++i) {
    const flix_batch& b = h[i];
    if (b.op > FLIX_OP_PREDECESSOR) return FLIX_EINVAL;
    if (b.n == 0) continue;
    if (b.n > s->max_batch || !b.d_keys) return FLIX_EINVAL;
    if ((b.op == FLIX_OP_INSERT || b.op == FLIX_OP_RANGE) && !b.d_aux) return FLIX_EINVAL;
    const bool keyed = b.op == FLIX_OP_SUCCESSOR || b.op == FLIX_OP_PREDECESSOR;
    if ((b.op == FLIX_OP_LOOKUP || keyed) && !b.d_vals_out) return FLIX_EINVAL;
    if (keyed && !b.d_keys_out) return FLIX_EINVAL;
    if (b.op == FLIX_OP_RANGE && !b.d_counts) return FLIX_EINVAL;
  }
  return FLIX_OK;
}

static_assert(sizeof(flix_batch) == sizeof(DrainBatch), "descriptor layouts must match");

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

int flix_create(const flix_config* cfg, void* stream, flix_store** out) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!out) return FLIX_EINVAL;
  *out = nullptr;
  if (!cfg) return FLIX_EINVAL;
  if (cfg->key_bits != 32 && cfg->key_bits != 64) return FLIX_EINVAL;
  u32 cap = cfg->bucket_capacity;
  if (cap < 8 || cap > 256 || (cap & (cap - 1))) return FLIX_EINVAL;
  u32 gl = cfg->lanes_per_bucket ? cfg->lanes_per_bucket : 16;
  if (gl != 16 && gl != 32 && gl != 64) return FLIX_EINVAL;
  u32 rb = cfg->radix_bits ? cfg->radix_bits : 8;
  if (rb != 4 && rb != 8) return FLIX_EINVAL;
  u32 fill = cfg->fill ? cfg->fill : cap / 2;
  if (fill > cap || fill == 0) return FLIX_EINVAL;
  if (cfg->max_batch == 0 || cfg->max_batch > 0x7FFFFFFFull) return FLIX_EINVAL;
  if (cfg->insert_algo > FLIX_INSERT_ADAPTIVE) return FLIX_EINVAL;
  if (cfg->read_path > FLIX_READ_GROUPS || cfg->reserved != 0) return FLIX_EINVAL;
  {
    // device address of the allocation-free entry point's scratch on this GPU;
    // a failed lookup is reported by that entry point (it retries), stores
    // do not depend on it
    u32* sc = nullptr;
    if (noalloc_scratch(&sc) != FLIX_OK) (void)hipGetLastError();
  }
  flix_store* s = new (std::nothrow) flix_store;
  if (!s) return FLIX_ENOMEM;
  s->cfg = *cfg;
  s->kb = (int)cfg->key_bits;
  s->ksz = cfg->key_bits / 8;
  s->cap = cap;
  s->gl = gl;
  s->rb = rb;
  s->fill = fill;
  s->max_batch = cfg->max_batch;
  int rc = FLIX_OK;
  u64 mb = cfg->max_batch;
  if ((rc = dev_alloc(&s->ctl, sizeof(Ctl))) || (rc = dev_alloc(&s->mktop, 257 * sizeof(u32))) ||
      (rc = dev_alloc(&s->bk[0], mb * s->ksz)) ||
      (rc = dev_alloc(&s->bk[1], mb * s->ksz)) || (rc = dev_alloc(&s->bp[0], mb * 8)) ||
      (rc = dev_alloc(&s->bp[1], mb * 8)) || (rc = dev_alloc(&s->work, ((u64)work_slots(mb) + wide_slots(mb)) * sizeof(WorkItem))) ||
      (rc = dev_alloc(&s->ss.hist, 2 * 2048 * sizeof(u32))) ||
      (rc = dev_alloc(&s->ss.tile_ctr, 64)) || (rc = dev_alloc(&s->ss.err, 16)) ||
      (rc = dev_alloc(&s->split, (u64)kGroupMax * s->ksz)) ||
      (rc = dev_alloc(&s->gpre, group_tiles(mb) * (kGroupMax + 1) * sizeof(u32))) ||
      (rc = dev_alloc(&s->gtot, 2ull * kGroupMax * sizeof(u32)))) {
    destroy_all(s);
    delete s;
    return rc;
  }
  if (hipMemset(s->gtot, 0, 2ull * kGroupMax * sizeof(u32)) != hipSuccess) {
    destroy_all(s);
    delete s;
    return FLIX_EHIP;
  }
  std::snprintf(g_last_error, sizeof(g_last_error), "flix_create: initial memset");
  if (hipMemset(s->ctl, 0, sizeof(Ctl)) != hipSuccess ||
      hipMemset(s->ss.hist, 0, 2 * 2048 * sizeof(u32)) != hipSuccess ||
      hipMemset(s->ss.tile_ctr, 0, 64) != hipSuccess ||
      hipMemset(s->ss.err, 0, 16) != hipSuccess) {
    destroy_all(s);
    delete s;
    return FLIX_EHIP;
  }
  s->ss.max_items = 0;
  s->ss.epoch = 0;
  s->ss.parity = 0;
  if ((rc = ensure_sort_capacity(s, mb))) {
    destroy_all(s);
    delete s;
    return rc;
  }
  s->d_status_words = sort_status_words(mb, 8);
  s->d_cluster_words = sort_cluster_words(mb);
  if ((rc = dev_alloc(&s->d_status, s->d_status_words * 8)) ||
      (rc = dev_alloc(&s->d_status_cl, s->d_cluster_words * 8)) ||
      (rc = dev_alloc(&s->d_hist, 2 * 2048 * sizeof(u32))) ||
      (rc = dev_alloc(&s->dctl, sizeof(DrainCtl))) ||
      (rc = dev_alloc(&s->d_layout, sizeof(StoreLayout)))) {
    destroy_all(s);
    delete s;
    return rc;
  }
  if (hipMemset(s->d_status, 0, s->d_status_words * 8) != hipSuccess ||
      hipMemset(s->d_status_cl, 0, s->d_cluster_words * 8) != hipSuccess ||
      hipMemset(s->dctl, 0, sizeof(DrainCtl)) != hipSuccess) {
    destroy_all(s);
    delete s;
    return FLIX_EHIP;
  }
  rc = s->kb == 32 ? bulk_load_t<u32>(s, nullptr, nullptr, 0, S(stream))
                   : bulk_load_t<u64>(s, nullptr, nullptr, 0, S(stream));
  if (rc) {
    destroy_all(s);
    delete s;
    return rc;
  }
  *out = s;
  return FLIX_OK;
}

int flix_set_allocator(flix_alloc_fn alloc, flix_free_fn free, void* ctx) {
  if ((alloc == nullptr) != (free == nullptr)) return FLIX_EINVAL;
  g_alloc.alloc = alloc;
  g_alloc.free = free;
  g_alloc.ctx = ctx;
  return FLIX_OK;
}

int flix_destroy(flix_store* s) {
  if (!s) return FLIX_ESTATE;
  (void)hipDeviceSynchronize();
  destroy_all(s);
  delete s;
  return FLIX_OK;
}

int flix_bulk_load(flix_store* s, const void* d_keys, const void* d_vals, uint64_t n,
                   void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!s) return FLIX_ESTATE;
  if (n && (!d_keys || !d_vals)) return FLIX_EINVAL;
  return s->kb == 32 ? bulk_load_t<u32>(s, (const u32*)d_keys, (const u32*)d_vals, n, S(stream))
                     : bulk_load_t<u64>(s, (const u64*)d_keys, (const u64*)d_vals, n, S(stream));
}

int flix_restructure(flix_store* s, uint64_t* nodes_before, uint64_t* nodes_after, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!s) return FLIX_ESTATE;
  return s->kb == 32 ? restructure_t<u32>(s, S(stream), nodes_before, nodes_after)
                     : restructure_t<u64>(s, S(stream), nodes_before, nodes_after);
}

int flix_insert(flix_store* s, const void* d_keys, const void* d_vals, uint64_t n,
                void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys, d_vals});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32 ? update_batch<u32>(s, true, d_keys, d_vals, n, S(stream))
                     : update_batch<u64>(s, true, d_keys, d_vals, n, S(stream));
}

int flix_delete(flix_store* s, const void* d_keys, uint64_t n, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32 ? update_batch<u32>(s, false, d_keys, nullptr, n, S(stream))
                     : update_batch<u64>(s, false, d_keys, nullptr, n, S(stream));
}

int flix_lookup(flix_store* s, const void* d_keys, uint64_t n, void* d_vals_out, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys, d_vals_out});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32
             ? read_batch<u32>(s, kOpLookup, d_keys, n, nullptr, d_vals_out, nullptr, nullptr, 0, S(stream))
             : read_batch<u64>(s, kOpLookup, d_keys, n, nullptr, d_vals_out, nullptr, nullptr, 0, S(stream));
}

int flix_successor(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                   void* d_vals_out, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys, d_keys_out, d_vals_out});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32 ? read_batch<u32>(s, kOpSuccessor, d_keys, n, d_keys_out, d_vals_out, nullptr,
                                       nullptr, 0, S(stream))
                     : read_batch<u64>(s, kOpSuccessor, d_keys, n, d_keys_out, d_vals_out, nullptr,
                                       nullptr, 0, S(stream));
}

int flix_predecessor(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                     void* d_vals_out, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys, d_keys_out, d_vals_out});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32 ? read_batch<u32>(s, kOpPredecessor, d_keys, n, d_keys_out, d_vals_out,
                                       nullptr, nullptr, 0, S(stream))
                     : read_batch<u64>(s, kOpPredecessor, d_keys, n, d_keys_out, d_vals_out,
                                       nullptr, nullptr, 0, S(stream));
}

int flix_range(flix_store* s, const void* d_lo, const void* d_hi, uint64_t n,
               uint32_t max_per_query, uint32_t* d_counts, void* d_keys_out, void* d_vals_out,
               void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_lo, d_hi, d_counts});
  if (c) return c > 0 ? FLIX_OK : c;
  return s->kb == 32 ? read_batch<u32>(s, kOpRange, d_lo, n, d_keys_out, d_vals_out, d_hi, d_counts,
                                       max_per_query, S(stream))
                     : read_batch<u64>(s, kOpRange, d_lo, n, d_keys_out, d_vals_out, d_hi, d_counts,
                                       max_per_query, S(stream));
}

int flix_size(flix_store* s, uint64_t* out, void* stream) {
  if (!s) return FLIX_ESTATE;
  if (!out) return FLIX_EINVAL;
  u64 v = 0;
  HIP_TRY(hipMemcpyAsync(&v, &s->ctl->nkeys, sizeof(u64), hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  *out = v;
  return FLIX_OK;
}

int flix_status(flix_store* s, void* stream) {
  if (!s) return FLIX_ESTATE;
  u32 v = 0, se = 0;
  HIP_TRY(hipMemcpyAsync(&v, &s->ctl->status, sizeof(u32), hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemcpyAsync(&se, s->ss.err, sizeof(u32), hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemsetAsync(&s->ctl->status, 0, sizeof(u32), S(stream)));
  HIP_TRY(hipMemsetAsync(s->ss.err, 0, sizeof(u32), S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  u32 de = 0;
  HIP_TRY(hipMemcpyAsync(&de, &s->dctl->err, sizeof(u32), hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipMemsetAsync(&s->dctl->err, 0, sizeof(u32), S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  if (de & 1u) {
    // a drain stopped part way: its barrier counters are left mid-count
    HIP_TRY(hipMemset(&s->dctl->top_count, 0, sizeof(u32)));
    HIP_TRY(hipMemset(&s->dctl->grp[0][0], 0, sizeof(s->dctl->grp)));
  }
  for (int i = 0; i < 2; ++i) {
    if (!s->ep[i]) continue;
    u32 x = 0;
    HIP_TRY(hipMemcpyAsync(&x, s->ep[i]->ss.err, sizeof(u32), hipMemcpyDeviceToHost, S(stream)));
    HIP_TRY(hipMemsetAsync(s->ep[i]->ss.err, 0, sizeof(u32), S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));
    se |= x;
  }
  if (v == 0 && (se != 0 || de != 0)) return FLIX_EINTERNAL;
  return (int)v;
}

int flix_dump(flix_store* s, void* d_keys_out, void* d_vals_out, uint64_t capacity,
              uint64_t* out_n, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!s) return FLIX_ESTATE;
  if (!out_n) return FLIX_EINVAL;
  hipStream_t st = S(stream);
  u64 n = 0;
  HIP_TRY(hipMemcpyAsync(&n, &s->ctl->nkeys, sizeof(u64), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out_n = n;
  if (n > capacity) return FLIX_EINVAL;
  if (n == 0) return FLIX_OK;
  if (!d_keys_out || !d_vals_out) return FLIX_EINVAL;
  return dump_body(s, d_keys_out, d_vals_out, capacity, st);
}

int flix_dump_noalloc(flix_store* s, void* d_keys_out, void* d_vals_out, uint64_t capacity,
                      uint64_t* out_n, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!s) return FLIX_ESTATE;
  if (!out_n) return FLIX_EINVAL;
  if (s->nb > kNoAllocBuckets) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "flix_dump_noalloc: %u buckets, at most %llu supported", s->nb,
                  (unsigned long long)kNoAllocBuckets);
    return FLIX_EINVAL;
  }
  u32* sc = nullptr;
  int rc = noalloc_scratch(&sc);
  if (rc) return rc;
  hipStream_t st = S(stream);
  u64 n = 0;
  HIP_TRY(hipMemcpyAsync(&n, &s->ctl->nkeys, sizeof(u64), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out_n = n;
  if (n > capacity) return FLIX_EINVAL;
  if (n == 0) return FLIX_OK;
  if (!d_keys_out || !d_vals_out) return FLIX_EINVAL;
  u32* tot = sc;
  u32* off = sc + kNoAllocBuckets;
  u32* bs = sc + 2 * kNoAllocBuckets;
  u32* total = bs + kNoAllocBlocks;
  if ((rc = dump_launch(s, d_keys_out, d_vals_out, capacity, tot, off, bs, total, st))) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return FLIX_OK;
}

int flix_check(flix_store* s, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  if (!s) return FLIX_ESTATE;
  hipStream_t st = S(stream);
  u32* mark = nullptr;
  u32* err = nullptr;
  unsigned long long* counters = nullptr;
  int rc;
  if ((rc = dev_alloc(&mark, (u64)s->pool * 4)) || (rc = dev_alloc(&err, 16)) ||
      (rc = dev_alloc(&counters, 16))) {
    dev_free(&mark); dev_free(&err); dev_free(&counters);
    return rc;
  }
  (void)hipMemsetAsync(mark, 0, (u64)s->pool * 4, st);
  (void)hipMemsetAsync(err, 0, 16, st);
  (void)hipMemsetAsync(counters, 0, 16, st);
  u32 g = std::min<u32>((s->nb + 255) / 256, 65535);
  if (s->kb == 32)
    hipLaunchKernelGGL((k_check_buckets<u32>), dim3(g), dim3(256), 0, st, (const u32*)s->mkba,
                       s->hdr, (const u32*)s->nkeys, s->bnodes, s->nb, s->cap, s->pool, mark,
                       counters, err);
  else
    hipLaunchKernelGGL((k_check_buckets<u64>), dim3(g), dim3(256), 0, st, (const u64*)s->mkba,
                       s->hdr, (const u64*)s->nkeys, s->bnodes, s->nb, s->cap, s->pool, mark,
                       counters, err);
  hipLaunchKernelGGL(k_check_free, dim3(std::min<u32>((s->pool + 255) / 256, 65535)), dim3(256), 0,
                     st, s->free_ids, s->ctl, s->pool, mark, err);
  hipLaunchKernelGGL(k_occ_check, dim3((u32)std::min<u64>((occ_words(s->nb) + 255) / 256, 65535)),
                     dim3(256), 0, st, s->hdr, s->nb, s->occl, err);
  u32 herr = 0;
  unsigned long long hc[2] = {0, 0};
  Ctl hctl;
  (void)hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(hc, counters, 16, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(&hctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
  hipError_t e = hipStreamSynchronize(st);
  dev_free(&mark); dev_free(&err); dev_free(&counters);
  if (e != hipSuccess) return FLIX_EHIP;
  if (herr) return (int)herr;
  if (hc[0] != hctl.nkeys) return 9;
  if (hc[1] + hctl.free_top != s->pool) return 10;
  return FLIX_OK;
}

int flix_get_stats(flix_store* s, flix_stats* out, void* stream) {
  if (!s) return FLIX_ESTATE;
  if (!out) return FLIX_EINVAL;
  Ctl hctl;
  HIP_TRY(hipMemcpyAsync(&hctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, S(stream)));
  HIP_TRY(hipStreamSynchronize(S(stream)));
  out->buckets = s->nb;
  out->pool_nodes = s->pool;
  out->live_nodes = s->pool - hctl.free_top;
  out->capacity = s->cap;
  out->keys = hctl.nkeys;
  return FLIX_OK;
}

int flix_copy_layout(flix_store* s, void* h_mkba, void* h_hdr, void* h_keys, void* h_vals,
                     uint32_t* h_free, uint64_t* h_free_top, void* stream) {
  if (!s) return FLIX_ESTATE;
  hipStream_t st = S(stream);
  if (h_mkba) HIP_TRY(hipMemcpyAsync(h_mkba, s->mkba, (u64)s->nb * s->ksz, hipMemcpyDeviceToHost, st));
  if (h_hdr) HIP_TRY(hipMemcpyAsync(h_hdr, s->hdr, (u64)s->pool * sizeof(NodeHdr), hipMemcpyDeviceToHost, st));
  if (h_keys) HIP_TRY(hipMemcpyAsync(h_keys, s->nkeys, (u64)s->pool * s->cap * s->ksz, hipMemcpyDeviceToHost, st));
  if (h_vals) HIP_TRY(hipMemcpyAsync(h_vals, s->nvals, (u64)s->pool * s->cap * s->ksz, hipMemcpyDeviceToHost, st));
  if (h_free) HIP_TRY(hipMemcpyAsync(h_free, s->free_ids, (u64)s->pool * 4, hipMemcpyDeviceToHost, st));
  Ctl hctl;
  HIP_TRY(hipMemcpyAsync(&hctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h_free_top) *h_free_top = hctl.free_top;
  return FLIX_OK;
}

int flix_sort_pairs(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                    uint32_t* d_idx_out, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int c = check_args(s, n, {d_keys, d_keys_out, d_idx_out});
  if (c) return c > 0 ? FLIX_OK : c;
  hipStream_t st = S(stream);
  int r;
  int rc = s->kb == 32 ? sort_batch<u32>(s, d_keys, nullptr, n, kPayIndex, st, &r)
                       : sort_batch<u64>(s, d_keys, nullptr, n, kPayIndex, st, &r);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(d_keys_out, s->bk[r], n * s->ksz, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_idx_out, s->bp[r], n * 4, hipMemcpyDeviceToDevice, st));
  return FLIX_OK;
}

const char* flix_last_error(void) { return g_last_error; }

int flix_epoch_prepare(flix_store* s, uint32_t slot, const flix_epoch* e, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int rc = epoch_validate(s, slot, e);
  if (rc) return rc;
  if ((rc = ensure_slots(s))) return rc;
  EpochSlot* es = s->ep[slot];
  es->prepared = false;
  hipStream_t st = S(stream);
  if (s->kb == 32)
    rc = s->rb == 4 ? epoch_prepare_rb<u32, 4>(es, e, st) : epoch_prepare_rb<u32, 8>(es, e, st);
  else
    rc = s->rb == 4 ? epoch_prepare_rb<u64, 4>(es, e, st) : epoch_prepare_rb<u64, 8>(es, e, st);
  if (rc) return rc;
  es->prepared = true;
  es->n_lookup = e->n_lookup;
  es->n_range = e->n_range;
  es->n_update = e->n_update;
  return FLIX_OK;
}

int flix_epoch_apply(flix_store* s, uint32_t slot, const flix_epoch* e, void* stream) {
  (void)hipGetLastError();  // drop errors left by other code on this thread
  int rc = epoch_validate(s, slot, e);
  if (rc) return rc;
  EpochSlot* es = s->ep[slot];
  if (!es || !es->prepared || es->n_lookup != e->n_lookup || es->n_range != e->n_range ||
      es->n_update != e->n_update)
    return FLIX_EINVAL;
  es->prepared = false;
  hipStream_t st = S(stream);
  return s->kb == 32 ? epoch_apply_t<u32>(s, es, e, st) : epoch_apply_t<u64>(s, es, e, st);
}

int flix_drain(flix_store* s, const flix_batch* h_batches, const flix_batch* d_batches,
               uint32_t nbatch, uint64_t* d_timestamps, void* stream) {
  if (!s) return FLIX_ESTATE;
  (void)hipGetLastError();
  if (nbatch == 0) return FLIX_OK;
  if (!h_batches || !d_batches) return FLIX_EINVAL;
  int rc = drain_validate(s, h_batches, nbatch);
  if (rc) return rc;
  return drain_launch(s, reinterpret_cast<const DrainBatch*>(d_batches), nbatch,
                      reinterpret_cast<unsigned long long*>(d_timestamps), S(stream));
}

int flix_drain_graph(flix_store* s, const flix_batch* h_batches, const flix_batch* d_batches,
                     uint32_t nbatch, uint64_t* d_timestamps, void** graph_exec, void* stream) {
  if (!s) return FLIX_ESTATE;
  if (!graph_exec || !stream) return FLIX_EINVAL;
  (void)hipGetLastError();
  *graph_exec = nullptr;
  int rc = drain_validate(s, h_batches, nbatch);
  if (rc) return rc;
  hipStream_t st = S(stream);
  // size the grid outside the capture (occupancy queries are not captured)
  if (s->drain_grid == 0) {
    rc = drain_launch(s, reinterpret_cast<const DrainBatch*>(d_batches), 0, nullptr, st);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  rc = drain_launch(s, reinterpret_cast<const DrainBatch*>(d_batches), nbatch,
                    reinterpret_cast<unsigned long long*>(d_timestamps), st);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return note_hip_error(e, "hipStreamEndCapture", __LINE__);
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return note_hip_error(e, "hipGraphInstantiate", __LINE__);
  *graph_exec = ex;
  return FLIX_OK;
}

int flix_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return FLIX_EINVAL;
  HIP_TRY(hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph_exec), S(stream)));
  return FLIX_OK;
}

int flix_graph_destroy(void* graph_exec) {
  if (!graph_exec) return FLIX_EINVAL;
  HIP_TRY(hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph_exec)));
  return FLIX_OK;
}

int flix_drain_info(flix_store* s, uint32_t* grid_blocks, uint64_t* timestamp_hz) {
  if (!s) return FLIX_ESTATE;
  if (grid_blocks) *grid_blocks = (uint32_t)s->drain_grid;
  if (timestamp_hz) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *timestamp_hz = (uint64_t)khz * 1000ull;
  }
  return FLIX_OK;
}

static int set_timing_mask(flix_store* s, u32 mask) {
  if (!s) return FLIX_ESTATE;
  tm_collect(s);
  s->tm.on = mask != 0;
  s->tm.mask = mask;
  s->ss.on_begin = s->tm.on ? sort_hook_begin : nullptr;
  s->ss.on_end = s->tm.on ? sort_hook_end : nullptr;
  s->ss.hook_ctx = s;
  for (int i = 0; i < kFamilies; ++i) {
    s->tm.ms[i] = 0;
    s->tm.count[i] = 0;
  }
  return FLIX_OK;
}

int flix_set_timing(flix_store* s, int enable) {
  return set_timing_mask(s, enable ? (1u << kFamilies) - 1u : 0u);
}

int flix_set_timing_only(flix_store* s, const char* family) {
  if (!s) return FLIX_ESTATE;
  if (!family) return set_timing_mask(s, (1u << kFamilies) - 1u);
  for (int i = 0; i < kFamilies; ++i)
    if (std::strcmp(family, kFamilyNames[i]) == 0) return set_timing_mask(s, 1u << i);
  return FLIX_EINVAL;
}

int flix_kernel_time(flix_store* s, const char* family, double* ms, uint64_t* launches) {
  if (!s) return FLIX_ESTATE;
  if (!family || !ms || !launches) return FLIX_EINVAL;
  tm_collect(s);
  for (int i = 0; i < kFamilies; ++i) {
    if (std::strcmp(family, kFamilyNames[i]) == 0) {
      *ms = s->tm.ms[i];
      *launches = s->tm.count[i];
      return FLIX_OK;
    }
  }
  return FLIX_EINVAL;
}

}  // extern "C"
