/*
 * sivf.h -- C ABI of the streaming IVF index for AMD Instinct MI355X (gfx950).
 *
 * The index keeps every inverted list in fixed-capacity device slabs and
 * mutates them in place (Sec. 3 of "SIVF: GPU-Resident IVF Index for
 * Streaming Vector Search"): insertion takes slabs from a device free stack
 * (Sec. 3.1, Alg. 1; Sec. 3.2, Alg. 2), deletion finds an id's slot through an
 * address translation table in O(1) (Sec. 3.4, Alg. 4), and search scans the
 * slabs of the probed lists (Sec. 3.3, Alg. 3).  The operations follow the
 * paper's statement of the problem: add_with_ids / remove_ids / search on a
 * GPU-resident index (Sec. 1 and Sec. 4.1), plus the sliding-window step of
 * Sec. 5.5.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns a sivf_status; nothing throws across the ABI.
 *  - Memory: the library never allocates device memory.  The caller passes
 *    one device workspace of sivf_workspace_bytes() bytes to sivf_create and
 *    keeps it, and every input/output buffer, alive until the stream has
 *    passed the call.  Pointers marked "device" are HIP device pointers;
 *    pointers marked "host" are ordinary host memory.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *    enqueue work and return at once; only sivf_sync, sivf_stats, sivf_dump
 *    and sivf_dump_info wait.
 *  - Errors: argument errors are detected on the host and return
 *    SIVF_ERR_ARG with nothing enqueued.  Errors that depend on device data
 *    (pool exhausted, id out of range) are recorded in a device status word;
 *    the failing call changes no index state, and sivf_sync returns the first
 *    such error since the previous sivf_sync.
 *  - Ids are int64 at the ABI and dense in [0, id_capacity) (Sec. 3, Data
 *    Model).  Adding a live id replaces it (delete-then-insert, Sec. 3, Data
 *    Model); if one add batch holds an id twice, the last occurrence wins.
 *    Removing an absent id is a no-op (idempotent delete, Alg. 4, Theorem 3).
 *  - Distances: squared L2 (ascending) or inner product (descending); ties
 *    go to the smaller id.  Missing results are label -1 with +inf (L2) or
 *    -inf (IP).  nprobe is clamped to nlist.
 *  - Determinism: index membership and every search result are identical
 *    to a sequential contiguous-array IVF with the same centroids; the slot
 *    layout inside the slabs is implementation-defined.
 *  - A handle is used from one host thread at a time.
 */
#ifndef SIVF_H
#define SIVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sivf_index sivf_index;

typedef enum {
    SIVF_OK = 0,
    SIVF_ERR_ARG = -1,      /* invalid argument (host check; nothing enqueued)   */
    SIVF_ERR_NOSPACE = -2,  /* slab pool too small for the add batch (Sec. 3.2)  */
    SIVF_ERR_ID_RANGE = -3, /* an id outside [0, id_capacity)                    */
    SIVF_ERR_DEVICE = -4,   /* a HIP runtime call failed                         */
    SIVF_ERR_STATE = -5,    /* handle unusable (e.g. after a device error)       */
    SIVF_ERR_LIVE_ID = -6,  /* a server insert named an id that is live          */
    SIVF_ERR_TOO_LARGE = -7 /* request exceeds the fixed scratch of sivf_probe_noalloc */
} sivf_status;

typedef enum { SIVF_L2 = 0, SIVF_IP = 1 } sivf_metric;
typedef enum { SIVF_F32 = 0, SIVF_BF16 = 1, SIVF_F16 = 2 } sivf_dtype;

/* How sivf_remove deletes (both give the same membership and search results):
 *  SIVF_DELETE_COMPACT: the list's tail entry moves into the hole at once, so
 *    lists stay dense and emptied tail slabs return to the pool in the call;
 *  SIVF_DELETE_LAZY: the paper's eviction (Sec. 3.4, Alg. 4): a validity bit
 *    per slot is cleared with an atomic AND (the 1 -> 0 transition counts the
 *    removal exactly once, Theorem 3) and nothing moves, so a delete never
 *    waits for searches; inserts publish their slots with a release fence and
 *    an atomic OR (Alg. 2).  Dead slots keep their space until
 *    sivf_compact. */
typedef enum { SIVF_DELETE_COMPACT = 0, SIVF_DELETE_LAZY = 1 } sivf_delete_mode;

/* Index configuration.  The slab pool and id space are fixed at creation
 * (the paper pre-allocates a monolithic slab pool, Sec. 3.1 and Sec. 4.1). */
typedef struct {
    int32_t dim;           /* vector dimension d, 1..2048                          */
    int32_t nlist;         /* number of lists / centroids, 1..65536                */
    int32_t slab_capacity; /* C, vectors per slab (Sec. 3.1): a power of two <= 128;
                            * 32, 64 and 128 are the performance settings        */
    int32_t metric;        /* sivf_metric                                          */
    int32_t storage;       /* sivf_dtype of the scanned copy of each vector: with
                            * SIVF_BF16 / SIVF_F16 the slabs hold a rounded copy
                            * (round to nearest even) scanned on MFMA, beside the
                            * exact fp32 copy used for the final re-rank; needs
                            * dim <= 256 and slab_capacity >= 16               */
    int32_t rerank_factor; /* R: reduced precision keeps the best R * k candidates
                            * per query by approximate distance, then re-ranks them
                            * by the exact fp32 distance; R * max_k <= 64.  Must be
                            * 0 with SIVF_F32                                      */
    int64_t num_slabs;     /* slabs in the pool, 1..2^31/C                         */
    int64_t id_capacity;   /* N_max: ids are dense in [0, id_capacity), <= 2^31    */
    int32_t max_batch;     /* largest n of one sivf_add / sivf_remove call         */
    int32_t max_queries;   /* largest nq of one sivf_search call                   */
    int32_t max_k;         /* largest k, 1..128 (fp32 storage)                     */
    int32_t max_nprobe;    /* largest nprobe, 1..1024                              */
    int32_t delete_mode;   /* sivf_delete_mode                                     */
    int32_t reserved;      /* must be 0                                            */
} sivf_config;

/* Bytes of device workspace the configuration needs (0 if invalid). */
size_t sivf_workspace_bytes(const sivf_config *cfg);

/* Create an index.  centroids: device, nlist x dim fp32 row-major, copied into
 * the workspace (the caller may free its copy after the stream passes the
 * call).  workspace: device, ws_bytes >= sivf_workspace_bytes(cfg), owned by
 * the caller.  The pool starts empty with every slab on the free stack.
 * Returns SIVF_ERR_ARG for an invalid configuration or a short workspace. */
sivf_status sivf_create(const sivf_config *cfg, const float *centroids, void *workspace,
                        size_t ws_bytes, void *stream, sivf_index **out);

/* Release the host handle.  The workspace is not freed. */
sivf_status sivf_destroy(sivf_index *ix);

/* Insert n vectors (Sec. 3.2, Alg. 2; delete-then-insert for live ids, Sec. 3).
 * x: device, n x dim fp32 row-major; ids: device, n int64.  Each vector goes
 * to the list of its nearest centroid.  If any id is outside the id range
 * (SIVF_ERR_ID_RANGE), the final state would need more slabs than the pool
 * holds (SIVF_ERR_NOSPACE) or a vector has a non-finite coordinate
 * (SIVF_ERR_ARG, as the device status), the whole batch is rejected and
 * nothing changes.  0 <= n <= max_batch. */
sivf_status sivf_add(sivf_index *ix, int64_t n, const float *x, const int64_t *ids, void *stream);

/* Delete ids (Sec. 3.4, Alg. 4): O(1) address-table lookup per id; the hole
 * is filled with the list's tail entry and emptied tail slabs return to the
 * free stack.  ids: device, n int64; absent and repeated ids are no-ops.
 * n_removed: device int64 scalar or NULL; receives the number of ids that
 * were live.  An id outside the id range rejects the whole batch
 * (SIVF_ERR_ID_RANGE).  0 <= n <= max_batch. */
sivf_status sivf_remove(sivf_index *ix, int64_t n, const int64_t *ids, int64_t *n_removed,
                        void *stream);

/* k-nearest-neighbour search over the nprobe nearest lists (Sec. 3.3, Alg. 3).
 * q: device, nq x dim fp32.  k: row stride of the outputs, 1 <= k <= max_k.
 * k_per_query: device nq int32 in [0, k], or NULL (every query uses k).
 * nprobe: 1..max_nprobe, used when nprobe_per_query is NULL; otherwise
 * nprobe_per_query: device nq int32 in [1, max_nprobe].
 * dist: device nq x k fp32; labels: device nq x k int64.  Row i holds query i's
 * results best first; entries past the query's own k are padding.
 * 0 <= nq <= max_queries. */
sivf_status sivf_search(sivf_index *ix, int64_t nq, const float *q, int32_t k,
                        const int32_t *k_per_query, int32_t nprobe,
                        const int32_t *nprobe_per_query, float *dist, int64_t *labels,
                        void *stream);

/* Search schedule autotuner (for uneven batches: skewed list lengths,
 * per-query nprobe and k).  Runs sivf_search on this sample batch once per
 * candidate schedule -- queries per work item (fp32 storage: 8 and 4, and
 * 16 where the certified matrix-core scan applies: dim <= 256,
 * slab_capacity >= 4; the reduced-precision scan always takes 16) x
 * positions per work item (2^10
 * .. 2^17; longer lists are split into chunks scanned in parallel) x wave
 * schedule (one wave per work item, or resident waves pulling items from
 * per-XCD counters) -- times each with HIP events and keeps the fastest for
 * every later search of this index (and graphs captured afterwards).  When
 * the certified scan wins and the batch asks for k > 64, the schedule of
 * the k > 64 pass (sivf_set_deep_schedule) is tuned after it the same way.
 * Results do not depend on the schedule.  Arguments as sivf_search;
 * dist/labels receive the last run's results.  Blocks until done.  tile,
 * chunk_shift, persistent: host int32 or NULL, receive the chosen values. */
sivf_status sivf_tune_search(sivf_index *ix, int64_t nq, const float *q, int32_t k, const int32_t *k_per_query,
                             int32_t nprobe, const int32_t *nprobe_per_query, float *dist, int64_t *labels,
                             void *stream, int32_t *tile, int32_t *chunk_shift, int32_t *persistent);

/* Set the search schedule directly (e.g. one found earlier by
 * sivf_tune_search): tile = queries per work item (fp32 storage: 4, 8
 * when dim <= 1024, or 16 -- the certified matrix-core scan, identical
 * results -- when dim <= 256 and slab_capacity >= 4; reduced
 * precision: 16), 2^chunk_shift = positions per
 * work item (6..31), persistent = 0 (one wave per item) or 1 (resident
 * waves).  SIVF_ERR_ARG for other values.  Applies to later calls. */
sivf_status sivf_set_search_schedule(sivf_index *ix, int32_t tile, int32_t chunk_shift, int32_t persistent);

/* Schedule of the k > 64 pass (fp32 storage).  Under the certified scan
 * (tile 16) a search whose k exceeds 64 runs in two passes over the same
 * probes and the same snapshot of list lengths: the queries with k <= 64 on
 * the certified scan with 64-key lists, then those with k > 64 on this
 * schedule (tile 4 or 8: the VALU scan; 16: the certified scan with 128-key
 * lists); without per-query k every query takes the second.  Arguments and
 * errors as sivf_set_search_schedule (SIVF_ERR_ARG on reduced-precision
 * indexes too); default 16 queries x 2^14 positions, resident waves.  Set by
 * sivf_tune_search as well.  Results do not depend on it. */
sivf_status sivf_set_deep_schedule(sivf_index *ix, int32_t tile, int32_t chunk_shift, int32_t persistent);

/* The schedules in force: sched (host, 6 int32) receives tile, chunk_shift,
 * persistent of the search schedule, then those of the k > 64 pass. */
sivf_status sivf_get_search_schedule(const sivf_index *ix, int32_t *sched);

/* One sliding-window step in the order of the paper's mixed loop
 * (Sec. 5.5: insert, then search, then delete).  Any part with a zero count
 * is skipped.  Same argument rules as the three calls (k_per_query and
 * nprobe_per_query as in sivf_search, NULL for uniform values). */
typedef struct {
    int64_t n_add;
    const float *x;          /* device n_add x dim                  */
    const int64_t *add_ids;  /* device n_add                        */
    int64_t nq;
    const float *q;          /* device nq x dim                     */
    int32_t k, nprobe;
    float *dist;             /* device nq x k                       */
    int64_t *labels;         /* device nq x k                       */
    const int32_t *k_per_query;      /* device nq or NULL           */
    const int32_t *nprobe_per_query; /* device nq or NULL           */
    int64_t n_remove;
    const int64_t *remove_ids; /* device n_remove                   */
    int64_t *n_removed;      /* device scalar or NULL               */
} sivf_step_args;

sivf_status sivf_step(sivf_index *ix, const sivf_step_args *args, void *stream);

/* A window step captured once as a HIP graph and replayed: the ~30 kernel
 * launches of a step are recorded once and replayed as one graph launch
 * (the paper finds that amortising kernel-launch overhead is a major factor in
 * mutation latency, Sec. 5.2.3).  The graph records the pointers in `args`:
 * before each launch, write the new batch into the same buffers.  Counts
 * (n_add, nq, k, nprobe, n_remove) are fixed per graph, so create one graph
 * per shape.  Profiling events are not recorded inside a graph.  The capture
 * uses a private stream of default priority; `sivf_graph_launch` enqueues the
 * whole step on `stream`.  A graph must be destroyed before its index. */
typedef struct sivf_graph sivf_graph;
sivf_status sivf_graph_create(sivf_index *ix, const sivf_step_args *args, sivf_graph **out);
sivf_status sivf_graph_launch(sivf_graph *g, void *stream);
sivf_status sivf_graph_destroy(sivf_graph *g);

/* Reclaim the slots of lazy deletes (SIVF_DELETE_LAZY; a no-op otherwise):
 * every list whose dead slots are at least min_dead_fraction of its length
 * (0 = any dead slot) is compacted -- its tail entries move into the dead
 * slots below the new length, as a dense delete does, and emptied tail slabs
 * return to the pool with cleared validity words (reset before the push).
 * The adaptive background compaction the paper plans (Sec. 6): call it when
 * fragmentation passes a threshold.  Entries move, so no search may overlap
 * the call (the server orders it after earlier searches).  At most max_batch
 * dead slots are reclaimed per call; n_compacted (device int64 scalar or
 * NULL) receives the number reclaimed; call again while it is positive. */
sivf_status sivf_compact(sivf_index *ix, float min_dead_fraction, int64_t *n_compacted, void *stream);

/* ---- Host tier: cold lists in host memory (the hierarchical storage the
 * paper plans as future work, Sec. 6: cold slabs offloaded to host memory so
 * that the window may outgrow device memory).
 *
 * A second slab pool, in the device pool's layout, whose rows and ids live in
 * caller-provided pinned host memory (the GPU reads and writes it in place
 * over the host link) and whose bookkeeping -- validity bits, slab directory,
 * free stacks, per-list cold lengths and dead counts, per-list probe counts --
 * lives in a caller-provided device buffer.  Offloading a list moves every
 * position of it (live or dead) to the end of its cold segment and returns its
 * device slabs to the pool; later inserts into the list go to device slabs as
 * usual.  Results are unchanged: a search scans each probed list's cold
 * segment too (the VALU scan, reading host memory; profile class
 * SIVF_PROF_SCAN_COLD) and merges both; a delete of a cold entry clears its
 * validity bit in the device-resident cold bitmap (Alg. 4 as for device
 * slots); sivf_get_rows, sivf_save and the live count of sivf_stats include cold
 * entries; sivf_dump shows the device pool only (sivf_tier_dump the rest).
 * Requires fp32 storage and SIVF_DELETE_LAZY; host_slabs >= 1 with
 * (num_slabs + host_slabs) * slab_capacity < 2^31.  The management calls
 * (attach, offload, reclaim, maintain) wait for the index's stream and must
 * not overlap other calls on the index. */

/* Bytes of the two tier buffers for host_slabs cold slabs (SIVF_ERR_ARG if
 * the index cannot take a tier). */
sivf_status sivf_tier_bytes(const sivf_index *ix, int64_t host_slabs, size_t *host_bytes, size_t *dev_bytes);

/* Attach an empty host tier (once per index).  host_buf: pinned host memory
 * the device can address (hipHostMalloc), 256-byte aligned; dev_buf: device
 * memory, 256-byte aligned; both owned by the caller and kept until
 * sivf_destroy.  SIVF_ERR_ARG for other buffers or sizes, SIVF_ERR_STATE if
 * a tier is already attached. */
sivf_status sivf_tier_attach(sivf_index *ix, int64_t host_slabs, void *host_buf, size_t host_bytes, void *dev_buf,
                             size_t dev_bytes, void *stream);

/* Move the n lists in `lists` (host int32, distinct list ids) to the tier:
 * every position of each goes to the end of its cold segment (dead slots stay
 * dead) and its device slabs return to the pool.  *moved (host, or NULL) =
 * positions moved.  SIVF_ERR_NOSPACE (nothing moved) if the cold pool lacks
 * the slabs; SIVF_ERR_STATE without a tier.  Waits. */
sivf_status sivf_tier_offload(sivf_index *ix, int32_t n, const int32_t *lists, int64_t *moved, void *stream);

/* Release every cold segment with no live entry left (a sliding window's old
 * entries die together); *released (host, or NULL) = positions released.
 * Partly dead segments stay until they die.  Waits. */
sivf_status sivf_tier_reclaim(sivf_index *ix, int64_t *released, void *stream);

/* Counts of the tier (host int64 each, any may be NULL; zeros without a
 * tier): live cold entries, cold positions, cold slabs in use, free cold
 * slabs.  Waits. */
sivf_status sivf_tier_stats(sivf_index *ix, int64_t *cold_live, int64_t *cold_positions, int64_t *cold_used_slabs,
                            int64_t *cold_free_slabs);

/* Host copy of the cold segments: cold_len[nlist] and, list after list in
 * position order, each cold position's id (-1 for a dead slot) in
 * cold_ids_by_list[sum of cold_len] (either may be NULL).  Waits. */
sivf_status sivf_tier_dump(sivf_index *ix, int32_t *cold_len, int64_t *cold_ids_by_list);

/* Per-list probe counts since the tier was attached (host int32[nlist]): a
 * search's first pass adds each list's (query, probe) pairs, saturating.
 * halve != 0 halves the stored counts after reading them (decay).  Waits. */
sivf_status sivf_list_heat(sivf_index *ix, int32_t *heat, int halve);

typedef struct {
    int64_t compacted;            /* dead device slots reclaimed by compaction */
    int64_t reclaimed;            /* cold positions released (dead segments) */
    int64_t offloaded_positions;  /* positions moved to the tier */
    int32_t offloaded_lists;      /* lists moved to the tier */
    int32_t reserved;
} sivf_maintain_report;

/* Adaptive maintenance (the background compaction policy of Sec. 6), for an
 * idle moment of the index: (1) with lazy deletes, sivf_compact at
 * min_dead_fraction until a call reclaims nothing; (2) with a tier, release
 * dead cold segments; (3) with a tier, while the device pool has fewer than
 * min_free_slabs free slabs, offload non-empty lists in ascending probe count
 * (at most max_offload lists), then halve the probe counts.  rep (host, or
 * NULL) receives what was done.  Waits. */
sivf_status sivf_maintain(sivf_index *ix, float min_dead_fraction, int64_t min_free_slabs, int32_t max_offload,
                          sivf_maintain_report *rep, void *stream);

/* Nearest list of each vector (the coarse assignment used by sivf_add).
 * x: device n x dim fp32; lists: device n int32.  n <= max(max_batch, max_queries). */
sivf_status sivf_assign(sivf_index *ix, int64_t n, const float *x, int32_t *lists, void *stream);

/* The nprobe nearest lists of each query (the probe set used by sivf_search),
 * nearest first, ties to the smaller list id.  probes: device nq x nprobe
 * int32; entries past nlist are -1.  1 <= nprobe <= max_nprobe. */
sivf_status sivf_probe(sivf_index *ix, int64_t nq, const float *q, int32_t nprobe,
                       int32_t *probes, void *stream);

/* sivf_probe for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same probe sets, with the approximate-distance scratch in a fixed 16 MiB
 * device array of the library instead of the index workspace.  Each device
 * holds one copy of that array until the process ends; every call on a
 * device shares it and leaves its contents behind (nothing in it needs to
 * start at zero), so calls that overlap on one device -- on two streams, or
 * from two threads -- race and must not be issued.  nq x nlist floats
 * (when nprobe == 1: nq x ceil(nlist / 16) for more than 2,048 lists of at
 * most 128 dimensions, else twice that) must fit in 16 MiB and nq may not
 * exceed max(max_batch, max_queries): larger requests return
 * SIVF_ERR_TOO_LARGE with nothing enqueued.  The calling thread's device may
 * differ from the index's; the kernels run on the stream given.  Allocates
 * nothing, ever (the array is set up on the first call on a device). */
sivf_status sivf_probe_noalloc(sivf_index *ix, int64_t nq, const float *q, int32_t nprobe,
                               int32_t *probes, void *stream);

/* Approximate coarse distances of the quantizer's MFMA stage:
 * |x|^2 + |c|^2 - 2 x.c (L2) or -x.c (IP), before the exact re-check.  For
 * validating the error bound |approx - exact| <= (4d+16) 2^-24 (|x|+|c|)^2
 * (L2) or (4d+16) 2^-24 |x||c| (IP) that the re-check relies on.  Indexes
 * with bf16/fp16 storage multiply bf16-rounded operands (bf16 MFMA); their
 * bound adds 2 (2u + u^2) |x||c| (L2) or (2u + u^2) |x||c| (IP), u = 2^-8.
 * x: device n x dim fp32; scores: device n x nlist fp32.
 * n <= max(max_batch, max_queries). */
sivf_status sivf_coarse_scores(sivf_index *ix, int64_t n, const float *x, float *scores, void *stream);

/* Stored vectors of ids.  ids: device n int64; rows: device n x dim fp32.
 * Rows of absent or out-of-range ids are filled with NaN.  n <= 2^26. */
sivf_status sivf_get_rows(sivf_index *ix, int64_t n, const int64_t *ids, float *rows, void *stream);

/* Wait for all work enqueued on the handle's streams; *device_status (may be
 * NULL) receives the first data-dependent error since the previous
 * sivf_sync (SIVF_OK if none), which is then cleared.  Returns
 * SIVF_ERR_DEVICE if a HIP call fails. */
sivf_status sivf_sync(sivf_index *ix, sivf_status *device_status);

/* Counters (waits for the handle's last stream).  Any pointer may be NULL.
 * live = entries in all lists (host-tier entries included); used = device
 * slabs held by lists; free = slabs on the free stack.  used + free =
 * num_slabs. */
sivf_status sivf_stats(sivf_index *ix, int64_t *live, int64_t *used_slabs, int64_t *free_slabs);

/* Sizes of the arrays sivf_dump fills (waits for the handle's last stream). */
typedef struct {
    int64_t live;        /* entries in all lists' device slabs           */
    int64_t used_slabs;  /* sum over lists of ceil(len / C)              */
    int64_t free_slabs;  /* entries on the free stack                    */
    int64_t num_slabs;
    int64_t id_capacity;
    int32_t nlist;
    int32_t slab_capacity;
    int64_t positions;   /* sum of list lengths: live plus dead slots (lazy deletes) */
} sivf_dump_info;

sivf_status sivf_dump_info_get(sivf_index *ix, sivf_dump_info *info);

/* Copy the index state to host arrays for validation (waits).  All host.
 *   list_len     [nlist]        entries per list
 *   list_slabs   [used_slabs]   slab ids of list 0 by ordinal, then list 1, ...
 *   ids_by_list  [positions]    ids of list 0 by position, then list 1, ...
 *                               (-1 for a slot deleted lazily, not yet compacted)
 *   free_slabs   [free_slabs]   the free stack, bottom first
 *   slab_owner   [num_slabs]    list holding each slab, or -1
 *   slab_ordinal [num_slabs]    position of the slab in its list's table
 *   att          [id_capacity]  address table: slab * C + slot, or 0xFFFFFFFF
 * Any pointer may be NULL to skip that array. */
sivf_status sivf_dump(sivf_index *ix, int32_t *list_len, int32_t *list_slabs, int64_t *ids_by_list,
                      int32_t *free_slabs, int32_t *slab_owner, int32_t *slab_ordinal,
                      uint32_t *att);

/* Device time per operation class, from HIP events recorded on the call's
 * stream around each class of work while profiling is on (in the spirit of
 * the paper's GPU time breakdown, Sec. 5.6, Tab. 3). */
typedef enum {
    SIVF_PROF_ADD = 0,     /* a whole sivf_add                               */
    SIVF_PROF_REMOVE = 1,  /* a whole sivf_remove                            */
    SIVF_PROF_SEARCH = 2,  /* a whole sivf_search                            */
    SIVF_PROF_COARSE = 3,  /* probe selection of a search (MFMA + re-check)  */
    SIVF_PROF_SCAN = 4,    /* the slab scan kernel of a search (its first pass) */
    SIVF_PROF_MERGE = 5,   /* the final top-k merge kernels of a search      */
    SIVF_PROF_SCAN_DEEP = 6, /* the k > 64 pass's scan of a two-pass search  */
    SIVF_PROF_SCAN_COLD = 7, /* the host-tier scan of a search               */
    SIVF_PROF_KINDS = 8
} sivf_prof_kind;

/* Turn event recording on (on != 0) or off. */
sivf_status sivf_profile_enable(sivf_index *ix, int on);

/* Wait for the recorded work, then write the summed device milliseconds and
 * the number of timed calls of each class (host arrays of SIVF_PROF_KINDS
 * entries, either may be NULL) and reset the sums.  In a two-pass search
 * (see sivf_set_deep_schedule) the first pass's scan counts as SCAN and the
 * second's as SCAN_DEEP; the merges of both add to one MERGE call. */
sivf_status sivf_profile_read(sivf_index *ix, double *total_ms, int64_t *count);

/* Serving: a request loop over one index whose requests overlap on the GPU
 * (the paper's mixed workload, Sec. 5.5, as continuous batching).  Searches
 * run on one stream and inserts/removes on another:
 *   - a search waits for every mutation submitted before it, then records
 *     the length of every list and scans only those entries;
 *   - an insert waits only until the most recent earlier search has recorded
 *     the lengths: inserts append past them, so the two overlap;
 *   - a remove (it moves entries inside lists) waits for every earlier search.
 * Each request therefore returns what it returns when the requests run one
 * at a time in submission order.  Server inserts must use ids that are not
 * live (else the call fails with SIVF_ERR_LIVE_ID and changes nothing).
 * Continuous batching: a search is not launched on its own while a search
 * batch is in flight; it joins the pending batch, and the pending batch
 * (every search submitted since the last launch, in submission order, with
 * its own k and nprobe) goes out as one search launch as soon as the search
 * stream is free -- checked by every server call (submit, poll, wait) -- or
 * before the next insert or remove is enqueued, which therefore never
 * overtakes an earlier search.  A batch holds at most max_queries rows
 * (batch slots): a search that does not fit starts the next batch, and is
 * refused with SIVF_ERR_NOSPACE (nothing enqueued; retry after a poll) while
 * two batches are already in flight.
 * Admission: an insert of n vectors is refused at once with SIVF_ERR_NOSPACE
 * (nothing enqueued) unless the host's view of the free-slab count, minus
 * the slabs reserved by inserts in flight, covers ceil(n/C) + min(n, nlist)
 * slabs.  The free-slab count is copied back after every mutation without
 * blocking.  Every submit returns a ticket; sivf_server_poll (non-blocking)
 * and sivf_server_wait (blocking) observe its completion.  Buffers stay owned
 * by the caller until the ticket completes; outputs are valid once it has.
 * input_stream (a hipStream_t, NULL = the legacy default stream) is the
 * stream whose work so far produces the request's device inputs: the request
 * starts after it.  One host thread per server; do not use the index
 * directly while a server is in use. */
typedef struct sivf_server sivf_server;
sivf_status sivf_server_create(sivf_index *ix, sivf_server **out);
sivf_status sivf_server_destroy(sivf_server *s);   /* waits for every request */
sivf_status sivf_server_add(sivf_server *s, int64_t n, const float *x, const int64_t *ids, void *input_stream,
                            int64_t *ticket);
sivf_status sivf_server_remove(sivf_server *s, int64_t n, const int64_t *ids, int64_t *n_removed,
                               void *input_stream, int64_t *ticket);
sivf_status sivf_server_search(sivf_server *s, int64_t nq, const float *q, int32_t k, int32_t nprobe,
                               float *dist, int64_t *labels, void *input_stream, int64_t *ticket);
sivf_status sivf_server_poll(sivf_server *s, int64_t ticket, int *done);
sivf_status sivf_server_wait(sivf_server *s, int64_t ticket);
/* Host view of free slabs and the slabs reserved by inserts in flight. */
sivf_status sivf_server_free_slabs(sivf_server *s, int64_t *free_slabs, int64_t *reserved);
/* Search batches launched so far and the search requests they carried
 * (host int64, either may be NULL). */
sivf_status sivf_server_batches(sivf_server *s, int64_t *batches, int64_t *requests);

/* ------------------------------------------------------------ checkpoint
 * Save the index to a file and load it into a new workspace (the paper keeps
 * host and device views of its index consistent, Sec. 1 and Sec. 4.1; this
 * is the persistent view).  The file holds the logical content: the
 * configuration, the centroids, each list's length and, list after list in
 * position order, every entry's id and exact fp32 row.  Rounded copies and
 * norms are recomputed on load and the slab layout is not kept, so a
 * checkpoint loads into any configuration with the same dim, nlist, metric,
 * storage and rerank_factor whose pool, id range and batch limits hold it;
 * the loaded index has the same lists, and every search returns what it
 * returned before the save.  Both calls block; sivf_save waits for the
 * handle's last stream and must not overlap other calls on the index.  File
 * errors and a mismatched configuration return SIVF_ERR_ARG; a pool or id
 * range too small returns SIVF_ERR_NOSPACE / SIVF_ERR_ID_RANGE (no index is
 * created).  Staging goes through the index's own workspace. */
sivf_status sivf_save(sivf_index *ix, const char *path);
/* Configuration and live count stored in a checkpoint (live may be NULL). */
sivf_status sivf_checkpoint_config(const char *path, sivf_config *cfg, int64_t *live);
/* Create an index from a checkpoint: workspace and stream as sivf_create. */
sivf_status sivf_load(const char *path, const sivf_config *cfg, void *workspace, size_t ws_bytes, void *stream,
                      sivf_index **out);

/* ------------------------------------------------------ external id registry
 * Sparse 64-bit external ids (UUIDs, hashes) on top of the dense internal
 * id range [0, id_capacity) (the paper maps them through a registry in front
 * of its dense identifier space, Sec. 3, Data Model).  The registry lives in
 * its own device workspace: a hash table (external -> internal), the reverse
 * map (internal -> external) and a stack of free internal ids, so batches of
 * external ids are resolved on the device with no host round trip.  While a
 * registry is attached, use the index only through it (it owns the internal
 * ids).  External ids may be any int64 except INT64_MIN and INT64_MIN + 1
 * (reserved table markers; such an id fails the call with SIVF_ERR_ARG as the
 * device status).  Semantics are those of the dense calls: add of a held id
 * is an upsert, the last duplicate in a batch wins, removing an absent id is
 * a no-op; a failed add maps no new id.  Search labels are external ids (-1
 * for missing results).  Device status: sivf_registry_sync (the registry's
 * first error, else the index's).  Workspace: device, caller-owned, of
 * sivf_registry_workspace_bytes(ix) bytes, 256-byte aligned. */
typedef struct sivf_registry sivf_registry;
size_t sivf_registry_workspace_bytes(const sivf_index *ix);
sivf_status sivf_registry_create(sivf_index *ix, void *workspace, size_t ws_bytes, void *stream,
                                 sivf_registry **out);
sivf_status sivf_registry_destroy(sivf_registry *r);   /* does not free the workspace */
/* x: device n x dim fp32; ext_ids: device n int64.  n <= max_batch. */
sivf_status sivf_registry_add(sivf_registry *r, int64_t n, const float *x, const int64_t *ext_ids, void *stream);
/* ext_ids: device n int64; n_removed: device int64 scalar or NULL. */
sivf_status sivf_registry_remove(sivf_registry *r, int64_t n, const int64_t *ext_ids, int64_t *n_removed,
                                 void *stream);
/* As sivf_search; labels (device nq x k int64) receive external ids. */
sivf_status sivf_registry_search(sivf_registry *r, int64_t nq, const float *q, int32_t k, int32_t nprobe,
                                 float *dist, int64_t *labels, void *stream);
/* Internal id of each external id (device n int64 out; -1 if not held). */
sivf_status sivf_registry_lookup(sivf_registry *r, int64_t n, const int64_t *ext_ids, int64_t *internal,
                                 void *stream);
sivf_status sivf_registry_sync(sivf_registry *r, sivf_status *device_status);
/* The registry's reverse map to / from a file (blocks).  Load into a fresh
 * registry created over the index loaded from the matching sivf_save. */
sivf_status sivf_registry_save(sivf_registry *r, const char *path);
sivf_status sivf_registry_load(sivf_registry *r, const char *path, void *stream);

/* Static text for a status code. */
const char *sivf_status_string(sivf_status s);

#ifdef __cplusplus
}
#endif

#endif /* SIVF_H */
