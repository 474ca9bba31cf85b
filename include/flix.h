/*
 * flix.h - C ABI of the FliX flipped-index ordered key-value store on MI355X.
 *
 * FliX ("Flipped-Indexing for Scalable GPU Queries and Updates", arXiv
 * 2604.16725) keeps an ordered map entirely in GPU memory with no index
 * layer.  Keys live in buckets; bucket i holds the keys in
 * (maxBucket[i-1], maxBucket[i]] as a chain of fixed-capacity sorted nodes
 * (Section 3.2).  Every operation batch is sorted on the device; then each
 * bucket binary-searches the sorted batch for its own slice and applies it in
 * place (Sections 3.3 and 4.1): point lookup, successor, range, merge-insert
 * with node split (Section 4.3.2), compact-delete with node reclamation
 * (Section 4.4).
 *
 * Conventions for every entry point
 *  - Keys and values have the same width: 32 or 64 bits (flix_config.key_bits).
 *    Device buffers hold uint32_t or uint64_t elements accordingly.
 *  - NOT_FOUND is the all-ones value of the value width.  It is returned for
 *    misses and may not be inserted.  KEY_MAX is the all-ones key; 0 and
 *    KEY_MAX are ordinary keys.
 *  - Pointers named d_* are device pointers owned by the caller.  They must
 *    stay valid until the work enqueued on `stream` has completed.  Inputs are
 *    never modified; the library sorts copies in its own scratch memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    calls are asynchronous and stream-ordered unless marked "synchronizes".
 *    A store may be used from one host thread at a time; when the caller
 *    switches streams between calls it must order them (event + wait).
 *  - n == 0 is a no-op returning FLIX_OK; null pointers are then allowed.
 *  - Batch semantics equal applying the batch sequentially in input order:
 *    within one insert batch the last occurrence of a key wins; deleting an
 *    absent key is a no-op; read batches answer every element.
 *
 * Errors (return values)
 *  FLIX_OK      0  success (for asynchronous calls: successfully enqueued)
 *  FLIX_EINVAL -1  bad argument: null pointer with n > 0, n > max_batch, bad
 *                  config, or (detected on the device) a value equal to
 *                  NOT_FOUND in an insert batch
 *  FLIX_ENOMEM -2  node pool exhausted (checked on the device before any
 *                  node is touched) or a host allocation failed
 *  FLIX_EHIP   -3  HIP runtime error
 *  FLIX_ESTATE -4  null store handle
 *  FLIX_EINTERNAL -5  (status only) a device-side consistency guard fired;
 *                  never expected on a store the library itself maintains
 *  Errors found on the device (reserved value, pool exhausted) cancel the
 *  whole batch: the store is left exactly as before the call.  They are
 *  recorded in a sticky status word that flix_status() returns and clears.
 */
#ifndef FLIX_H
#define FLIX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLIX_OK 0
#define FLIX_EINVAL (-1)
#define FLIX_ENOMEM (-2)
#define FLIX_EHIP (-3)
#define FLIX_ESTATE (-4)
#define FLIX_EINTERNAL (-5)

typedef struct flix_store flix_store; /* opaque; owns all memory it allocates */

typedef struct {
  uint32_t key_bits;        /* 32 or 64; values have the same width */
  uint32_t bucket_capacity; /* node capacity NS (Section 5.3.1): power of 2 in [8, 256] */
  uint32_t lanes_per_bucket;/* lanes cooperating on one bucket: 16, 32 or 64 (0 = 16) */
  uint32_t radix_bits;      /* sort digit width: 4 or 8 (0 = 8) */
  uint64_t max_batch;       /* largest n accepted by batch calls; sizes the scratch */
  uint64_t pool_bytes;      /* node pool budget in bytes; 0 = automatic (see below) */
  uint32_t fill;            /* keys per node at bulk load (Section 3.2: p = NS/2);
                               0 = bucket_capacity/2; at most bucket_capacity */
  uint32_t insert_algo;     /* insert kernel, one of FLIX_INSERT_* (0 = TL-Bulk) */
  uint32_t read_path;       /* read batches: FLIX_READ_SORTED (0) or FLIX_READ_GROUPS */
  uint32_t reserved;        /* must be 0 */
} flix_config;

/* Read-batch pipelines (both Section 3.3 / 4.1: sort, per-bucket slice search,
 * per-bucket resolve; same results).  SORTED sorts the whole batch on the
 * device (onesweep + per-run sort), then merge-path shares resolve it.  GROUPS
 * splits the batch by groups of consecutive buckets in one pass and sorts each
 * group's items in LDS inside the resolving workgroup (no device-wide sort). */
#define FLIX_READ_SORTED 0
#define FLIX_READ_GROUPS 1

/* Insert kernels (Section 4.2.1 ST-Shift-Right, Section 4.3.2 TL-Bulk,
 * Section 5.3.5 ST-TL-Mixed, Section 3.4 adaptive compute per bucket).  All
 * give the same contents; they differ in how lanes are assigned to buckets. */
#define FLIX_INSERT_TL_BULK 0        /* a group of lanes_per_bucket lanes per bucket; a
                                        bucket receiving at least max(4 * capacity, 256)
                                        batch keys (a dense run) is merged by a whole
                                        workgroup, node by node along its chain */
#define FLIX_INSERT_ST_SHIFT_RIGHT 1 /* one lane per bucket, key by key */
#define FLIX_INSERT_ST_TL_MIXED 2    /* per call: ST-Shift-Right when the call averages at
                                        most FLIX_ST_MAX_KEYS batch keys per touched
                                        bucket, TL-Bulk otherwise */
#define FLIX_INSERT_ADAPTIVE 3       /* per bucket: one lane for a slice of at most
                                        FLIX_ST_MAX_KEYS batch keys when nodes hold at most
                                        16 keys, a lane group otherwise */
#define FLIX_ST_MAX_KEYS 4

/* Create an empty store (Section 3.2 layout: a maxBucket directory over
 * buckets of chained fixed-capacity nodes; empty, it is one bucket covering
 * every key).  Allocates the
 * directory, the node pool and scratch sized by cfg->max_batch.  With
 * pool_bytes == 0 the pool is sized automatically: 2x the nodes a bulk load
 * needs plus room for one max_batch of inserts, re-sized by flix_bulk_load.
 * Synchronizes.  *out receives the handle (NULL on error). */
int flix_create(const flix_config* cfg, void* stream, flix_store** out);

/* Replace the contents with the n pairs (d_keys[i], d_vals[i]) (Section 3.2
 * initial build: sort, cut into groups of `fill`, one node per bucket, the last
 * key of a group is its maxBucket).  Duplicate keys: last occurrence wins.  n
 * is not limited by max_batch.  A value equal to NOT_FOUND -> FLIX_EINVAL and
 * the previous contents are kept.  Pool too small for a fixed pool_bytes ->
 * FLIX_ENOMEM.  Synchronizes. */
int flix_bulk_load(flix_store* s, const void* d_keys, const void* d_vals, uint64_t n,
                   void* stream);

/* Upsert n pairs (Section 4.3.2 TL-Bulk merge; full nodes split into halves,
 * Section 5.3.1).  An existing key takes the new value. */
int flix_insert(flix_store* s, const void* d_keys, const void* d_vals, uint64_t n,
                void* stream);

/* Delete n keys (Section 4.4 TL-Bulk delete with compaction; empty nodes are
 * unlinked and returned to the free list; adjacent underfull nodes merge). */
int flix_delete(flix_store* s, const void* d_keys, uint64_t n, void* stream);

/* Point lookups (Section 3.3): d_vals_out[i] = value of d_keys[i] or NOT_FOUND. */
int flix_lookup(flix_store* s, const void* d_keys, uint64_t n, void* d_vals_out, void* stream);

/* Successor queries (Section 6.5): smallest stored key k' >= d_keys[i] and its
 * value; (KEY_MAX, NOT_FOUND) when none exists. */
int flix_successor(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                   void* d_vals_out, void* stream);

/* Predecessor queries (ordered-map ADT, Section 2.1, the mirror of the
 * successor): largest stored key k' <= d_keys[i] and its value; (0, NOT_FOUND)
 * when none exists (NOT_FOUND tells the miss apart from a stored key 0). */
int flix_predecessor(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                     void* d_vals_out, void* stream);

/* Range queries (ordered-map ADT, Section 2.1): all pairs with
 * d_lo[i] <= k <= d_hi[i], ascending.  d_counts[i] = exact number of such
 * pairs (0 when lo > hi); the first min(count, max_per_query) keys/values are
 * written to d_keys_out / d_vals_out at [i*max_per_query + r].  Either output
 * may be NULL.  Slots beyond min(count, max_per_query) are not written. */
int flix_range(flix_store* s, const void* d_lo, const void* d_hi, uint64_t n,
               uint32_t max_per_query, uint32_t* d_counts, void* d_keys_out, void* d_vals_out,
               void* stream);

/* Restructuring (Section 3.5, evaluated in Section 6.6): the live pairs are
 * laid out again by the initial-build rule (Section 3.2) at the bulk-load fill,
 * so every bucket is one node again: chains are flattened, underfull nodes are
 * merged into nodes of `fill` keys, and maxBucket follows the current key
 * distribution.  Contents are unchanged.  The pool keeps its size.
 * *nodes_before / *nodes_after (either may be NULL) receive the nodes in use
 * before and after.  A pool with fewer than ceil(keys / fill) nodes ->
 * FLIX_ENOMEM, nothing changed.  Synchronizes; the store must be idle. */
int flix_restructure(flix_store* s, uint64_t* nodes_before, uint64_t* nodes_after, void* stream);

/* Optional device-memory allocator hook: every device buffer the library
 * allocates afterwards (directory, node pool, scratch, the temporaries of
 * bulk load, dump, check and restructure) comes from alloc(bytes, ctx) and
 * goes back through free(ptr, ctx) instead of hipMalloc / hipFree, so a
 * framework's caching allocator can back a store.  alloc returns NULL on
 * failure (-> FLIX_ENOMEM).  The library frees a buffer only when no work of
 * its own on the store's stream still uses it (after a synchronisation).
 * Process-wide: set it before creating stores, and destroy a store while the
 * hook it was created under is still set.  (NULL, NULL) restores hipMalloc /
 * hipFree; exactly one NULL -> FLIX_EINVAL. */
typedef void* (*flix_alloc_fn)(uint64_t bytes, void* ctx);
typedef void (*flix_free_fn)(void* ptr, void* ctx);
int flix_set_allocator(flix_alloc_fn alloc, flix_free_fn free, void* ctx);

/* Free every resource of the store (Section 3.2 lists what a store holds: the
 * maxBucket directory and the node pool; here also the scratch).
 * Synchronizes with the device. */
int flix_destroy(flix_store* s);

/* Number of stored keys.  Synchronizes `stream`. */
int flix_size(flix_store* s, uint64_t* out, void* stream);

/* Copy all pairs in ascending key order to d_keys_out / d_vals_out (device
 * buffers of at least `capacity` elements).  *out_n = number of pairs; if it
 * exceeds `capacity` nothing is copied and FLIX_EINVAL is returned.
 * Synchronizes `stream`. */
int flix_dump(flix_store* s, void* d_keys_out, void* d_vals_out, uint64_t capacity,
              uint64_t* out_n, void* stream);

/* flix_dump without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid it).
 * Same arguments, results and errors as flix_dump.  Its per-bucket scratch is
 * a fixed 16 MiB device array of the library on each GPU (looked up by
 * flix_create or by the first call on that GPU), so stores of more than 2^21
 * buckets -> FLIX_EINVAL.  Calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must not
 * be issued.  Synchronizes `stream`. */
int flix_dump_noalloc(flix_store* s, void* d_keys_out, void* d_vals_out, uint64_t capacity,
                      uint64_t* out_n, void* stream);

/* Device invariant checker: node keys strictly increasing and inside their
 * node's (previous maxKey, maxKey] range, chain fences increasing and ending at
 * maxBucket, sizes within capacity, no empty non-head node, chain lengths,
 * total key count, live + free nodes == pool, free list without duplicates.
 * Returns FLIX_OK or a positive code naming the first violated invariant (see
 * flix_build.hpp).  Synchronizes `stream`. */
int flix_check(flix_store* s, void* stream);

/* Return and clear the sticky device error (FLIX_OK if none).  Synchronizes. */
int flix_status(flix_store* s, void* stream);

/* Layout statistics (for tests and the benchmark's byte model): number of
 * buckets, pool nodes, nodes in use, node capacity.  Synchronizes. */
typedef struct {
  uint64_t buckets;
  uint64_t pool_nodes;
  uint64_t live_nodes;
  uint64_t capacity;
  uint64_t keys;
} flix_stats;
int flix_get_stats(flix_store* s, flix_stats* out, void* stream);

/* Copy the raw layout to HOST buffers (tests only; any pointer may be NULL):
 * maxBucket array [buckets], node headers as {fence u64, size u32, next u32}
 * [pool_nodes], node keys and values [pool_nodes * capacity], free stack
 * [pool_nodes] and its height.  Synchronizes. */
int flix_copy_layout(flix_store* s, void* h_mkba, void* h_hdr, void* h_keys, void* h_vals,
                     uint32_t* h_free, uint64_t* h_free_top, void* stream);

/* Stable device radix sort of (key, index) used by every batch call, exposed
 * for verification: d_keys_out = keys ascending, d_idx_out = input position of
 * each output key (ties keep input order).  n <= max_batch.  Asynchronous. */
int flix_sort_pairs(flix_store* s, const void* d_keys, uint64_t n, void* d_keys_out,
                    uint32_t* d_idx_out, void* stream);

/* ---- Persistent fused drain (a queue of mixed batches in one launch) ----
 * One co-resident grid executes the batches in order with the same phases as
 * the per-batch calls (sort, bound search, apply) separated by grid barriers,
 * so a whole queue costs one launch (or one hipGraph replay).  Results are
 * identical to issuing the batches one by one with the calls above. */
#define FLIX_OP_LOOKUP 0
#define FLIX_OP_SUCCESSOR 1
#define FLIX_OP_RANGE 2
#define FLIX_OP_INSERT 3
#define FLIX_OP_DELETE 4
#define FLIX_OP_PREDECESSOR 5
typedef struct {
  uint32_t op;            /* FLIX_OP_* */
  uint32_t n;             /* operations in the batch, <= max_batch (0: skipped) */
  uint32_t max_per_query; /* range only */
  uint32_t reserved;      /* must be 0 */
  const void* d_keys;     /* keys (range: lo) */
  const void* d_aux;      /* insert: values; range: hi; otherwise NULL */
  void* d_vals_out;       /* lookup / successor / predecessor / range values */
  void* d_keys_out;       /* successor / predecessor / range keys (range: may be NULL) */
  uint32_t* d_counts;     /* range counts */
  void* reserved2;        /* must be NULL */
} flix_batch;             /* 64 bytes */

/* Execute nbatch (<= 2^24) batches in order in one persistent kernel launch on `stream`.
 * h_batches (host) is validated like the per-batch calls; d_batches is the
 * same array in device memory, read by the kernel.  d_timestamps (device,
 * nbatch+1 entries, may be NULL) receives the device wall clock at the start
 * and after each batch (rate: flix_drain_info).  Device-detected update
 * errors behave as in flix_insert (batch cancelled, sticky status). */
int flix_drain(flix_store* s, const flix_batch* h_batches, const flix_batch* d_batches,
               uint32_t nbatch, uint64_t* d_timestamps, void* stream);

/* Capture one flix_drain launch into an instantiated hipGraph (returned as an
 * opaque hipGraphExec_t in *graph_exec).  Replays read the descriptor array in
 * device memory again, so the caller may rewrite it between replays (same
 * nbatch), and they read the store's current layout, so bulk loads between
 * replays are allowed (ordered on the stream like any other call).  The store
 * must outlive the graph.  `stream` must not be the null stream.  Synchronizes. */
int flix_drain_graph(flix_store* s, const flix_batch* h_batches, const flix_batch* d_batches,
                     uint32_t nbatch, uint64_t* d_timestamps, void** graph_exec, void* stream);
int flix_graph_launch(void* graph_exec, void* stream);
int flix_graph_destroy(void* graph_exec);

/* Workgroups of the co-resident drain grid (0 before the first drain) and the
 * tick rate of the drain timestamps. */
int flix_drain_info(flix_store* s, uint32_t* grid_blocks, uint64_t* timestamp_hz);

/* ---- Epochs: coalesced mixed requests (the serving form) ----
 * An epoch is a group of requests merged into three lists: lookups, ranges
 * and updates.  Its order is defined as follows (the paper only has
 * single-type batches): every read of the epoch observes the store as it was
 * before the epoch; then the updates take effect, and for each key the entry
 * that comes LAST in d_update_keys decides: a value equal to the reserved
 * all-ones pattern deletes the key, any other value upserts it.
 *
 * Two slots let one epoch be prepared while the previous one is applied:
 * flix_epoch_prepare sorts the epoch's three lists into the slot and folds
 * the updates (it reads only the epoch's inputs, never the store), and
 * flix_epoch_apply runs the bucket kernels of the prepared slot: lookups,
 * ranges (as flix_lookup / flix_range), then the folded deletes and upserts.
 * The caller orders the two streams with events: a slot's apply after its
 * prepare, a slot's next prepare after its previous apply, and all applies
 * in epoch order on one stream.  apply must get the same descriptor as the
 * prepare of that slot (EINVAL otherwise).  All buffers are device memory
 * owned by the caller and must stay valid until the apply completes.
 * Errors: EINVAL for a slot >= FLIX_EPOCH_SLOTS, counts above max_batch,
 * null buffers with a non-zero count, reserved != 0.  Device-detected
 * ENOMEM (an upper bound of the nodes the upserts may take, summed on the
 * store before the epoch's deletes, exceeds the free nodes) cancels the
 * epoch's updates as a whole, deletes included, and sets the sticky status;
 * the epoch's reads are answered.  The first call allocates the slots'
 * scratch. */
#define FLIX_EPOCH_SLOTS 2
typedef struct {
  uint64_t n_lookup;
  const void* d_lookup_keys;   /* [n_lookup] */
  void* d_lookup_vals;         /* [n_lookup] out: value or all-ones */
  uint64_t n_range;
  uint32_t range_max;          /* result slots per range */
  uint32_t reserved;           /* must be 0 */
  const void* d_range_lo;      /* [n_range] */
  const void* d_range_hi;      /* [n_range] */
  uint32_t* d_range_counts;    /* [n_range] out: keys in [lo, hi] */
  void* d_range_keys;          /* [n_range * range_max] out, may be NULL */
  void* d_range_vals;          /* [n_range * range_max] out, may be NULL */
  uint64_t n_update;
  const void* d_update_keys;   /* [n_update] in request order */
  const void* d_update_vals;   /* [n_update] all-ones = delete */
} flix_epoch;

int flix_epoch_prepare(flix_store* s, uint32_t slot, const flix_epoch* e, void* stream);
int flix_epoch_apply(flix_store* s, uint32_t slot, const flix_epoch* e, void* stream);

/* Text describing the last HIP runtime error a call of this host thread hit
 * (which call and the runtime's message); "" if none.  Never NULL. */
const char* flix_last_error(void);

/* Per-kernel timing with HIP events (for the benchmark).  While enabled,
 * every launch of a timed kernel family carries a start and a stop event that
 * the dispatch itself stamps (no marker packets between kernels);
 * flix_kernel_time returns the summed milliseconds and launch count since the
 * last reset.  Each family is one kernel: "sort_hist" (digit histograms),
 * "sort_pass" (one onesweep pass), "sort_local" (the per-run sort of batches
 * of up to 2^22 keys after their top-digit pass), "read_apply"
 * (lookup/successor/range bucket kernel), "read_cuts" (merge-path cuts of the
 * read shares), "slices" (update slice discovery and node budget),
 * "insert_apply", "delete_apply".  flix_set_timing(s, enable) times every
 * family (enable != 0) or none; flix_set_timing_only(s, family) times only
 * the named family, leaving the other launches uninstrumented (FLIX_EINVAL
 * for an unknown name).  Both reset the sums.  Host-side and synchronous with
 * respect to earlier timed launches (their events are collected first). */
int flix_set_timing(flix_store* s, int enable);
int flix_set_timing_only(flix_store* s, const char* family);
int flix_kernel_time(flix_store* s, const char* family, double* ms, uint64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* FLIX_H */
