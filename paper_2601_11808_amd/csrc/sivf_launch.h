// Host-side launch wrappers of the SIVF kernels (internal to libsivf).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sivf_dev.h"

namespace sivf {

// ---- setup (setup.hip)
void launch_init_state(hipStream_t st, const Dev &S, const float *centroids);

// ---- coarse quantizer (coarse.hip)
size_t coarse_select_smem(int dpad, int mmax);
int coarse_groups(int nlist);   // group minima per row of the nearest-list GEMM: ceil(nlist / 16)
void launch_coarse_gemm(hipStream_t st, const float *X, int n, int d, const float *cent, const uint16_t *cent_h, int dpad,
                        const float *cn2, int nlist, int metric, float *out, const int32_t *ctl,
                        int gated, int bf);
// m = 1 (nearest list per row): group-minimum GEMM into scratch (n x
// ceil(nlist / 16) floats), then the exact argmin; rows with a non-finite
// coordinate get -1.
int coarse_assign_words(int nlist, int dpad);
void launch_coarse_assign(hipStream_t st, float *scratch, const float *X, int n, int d, const float *cent,
                          const uint16_t *cent_h, int dpad, const float *cn2, const double *cmax, int nlist, int metric, int32_t *out,
                          int out_stride, const int32_t *ctl, int gated, int bf);
void launch_coarse_select(hipStream_t st, const float *dt, const float *X, int n, int d, const float *cent,
                          int dpad, const double *cnorm, const double *cmax, int nlist, int metric,
                          int m_uniform, const int32_t *m_per_row, int mmax, int32_t *out, int out_stride,
                          const int32_t *ctl, int gated, int bf);

// ---- mutation (mutate.hip)
struct Batch {
    int32_t *assign, *rank, *seg, *inv;   // inv: source row of each new entry, entry-major (adds);
                                          // the list of each tail-window entry (removes)
    uint32_t *rec;
};
void launch_add_prepare(hipStream_t st, const Dev &S, int n, const int64_t *ids);
void launch_add_count(hipStream_t st, const Dev &S, int n, const int64_t *ids, const Batch &B, int fresh_only);
void launch_add_admit(hipStream_t st, const Dev &S);
void launch_add_alloc(hipStream_t st, const Dev &S);
void launch_add_scatter(hipStream_t st, const Dev &S, int n, const float *x, const int64_t *ids,
                        const Batch &B);
void launch_add_cleanup(hipStream_t st, const Dev &S, int n, const int64_t *ids);
// mode 0: a remove call; mode 1: the delete half of an upsert inside an add call;
// mode 2: a remove call whose ids are not validated and skipped when outside
// [0, id_capacity) (the registry passes -1 for keys it does not hold)
void launch_remove(hipStream_t st, const Dev &S, int n, const int64_t *ids, int64_t *n_removed,
                   const Batch &B, int mode);
void launch_call_end(hipStream_t st, const Dev &S);
// lazy deletes: clear validity bits (mode 0: a remove call, ids validated;
// mode 1: the delete half of an upsert; mode 2: ids outside the range skipped)
void launch_remove_lazy(hipStream_t st, const Dev &S, int n, const int64_t *ids, int64_t *n_removed, int mode);
// compaction of lazily deleted slots: at most `budget` dead slots per call
void launch_compact(hipStream_t st, const Dev &S, float min_dead_fraction, int budget, int64_t *n_compacted,
                    const Batch &B);
void launch_get_rows(hipStream_t st, const Dev &S, int n, const int64_t *ids, float *rows);
// checkpoint: entries [e0, e0 + n) in list order (off = per-list first entry) -> rows and ids; with a
// host tier (Sc: the cold pool's view, else NULL) each list's cold segment follows its device positions
void launch_pack(hipStream_t st, const Dev &S, const Dev *Sc, const int32_t *off, int64_t e0, int n, float *rows,
                 uint32_t *ids);
// host tier: move every position of the n lists in olist (device array) to the end of their cold
// segments (longest: the most positions of one of them); lazy deletes only
void launch_tier_offload(hipStream_t st, const Dev &S, const Dev &Sc, const int32_t *olist, int n, int longest);
// host tier: release the cold segments with no live entry; *n_out (device) = positions released
void launch_tier_reclaim(hipStream_t st, const Dev &Sc, int64_t *n_out);
void launch_fill_i64(hipStream_t st, int64_t *p, int64_t n, int64_t v);
void launch_fill_i32(hipStream_t st, int32_t *p, int64_t n, int32_t v);

// ---- search (search.hip)
struct SearchBufs {
    int32_t *probes, *pair_rank, *list_pairs, *item_list, *item_tile, *item_chunk;
    uint64_t *partials;
    int64_t slot_cap;    // partial-result slots (kcap keys each) in partials
    int64_t item_cap;    // entries of item_list / item_tile / item_chunk
    float *rr_dist;      // reduced precision: approximate candidates per query
    int64_t *rr_lab;
    uint32_t *gthr;      // MFMA scans: per query, the best published k-th (R k-th) key's high word
};
// One pass of a search over the queries whose k, clamped to [0, k], lies in
// (lo, hi]: its plan, scan and merge skip the other queries.  A search whose
// per-query k straddles 64 on a certified-scan schedule runs two passes (k up
// to 64 on the certified scan, the rest on the deep schedule) that share the
// coarse probes and the list-length snapshot.
struct KClass {
    const int32_t *kpq;   // per-query k or null (every query asks for k)
    int k, np_stride, lo, hi;
};
inline KClass kclass_all(int np_stride) { return KClass{nullptr, 0, np_stride, -1, 0x7FFFFFFF}; }
int search_tile(const Dev &S);
// Default queries per work item: 16 (reduced precision, or the certified
// matrix-core scan where it applies), else 8 (4 past 1024 dimensions).
int default_tile(int storage, int d, int C, int kcap);
// Whether the certified FP32 MFMA scan (tile 16 on fp32 slabs) applies.
bool cert_ok(int storage, int d, int C, int kcap);
// Default search chunk: 2^14 positions per work item (a list is split only
// when the plan's buffers allow; into longer chunks otherwise).
constexpr int DEFAULT_CHUNK_SHIFT = 14;
// snap = 1: record every list's length (the scan reads only these entries);
// snap = 0: keep the lengths an earlier pass of the same search recorded.
// heat (or NULL): per-list probe counts to add this pass's pairs to
void launch_search_plan(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const KClass &cls, int snap,
                        int32_t *heat = nullptr);
void launch_search_scan(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const float *q, int np_stride,
                        int kcap, int k, const int32_t *k_per_query);
// prior (or NULL): per query, prior_stride sorted keys merged in as one more source;
// keys_out (or NULL): sorted keys (stride out_stride) instead of dist / labels
void launch_search_merge(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const KClass &cls, int kcap,
                         int out_stride, int k, int kmul, const int32_t *k_per_query, float *dist,
                         int64_t *labels, const uint64_t *prior = nullptr, int prior_stride = 0,
                         uint64_t *keys_out = nullptr);
void launch_search_scan_mfma(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const float *q,
                             int np_stride, int kcap, int k, int kmul, const int32_t *k_per_query);
void launch_rerank(hipStream_t st, const Dev &S, int nq, const float *q, int kc, const int64_t *cand, int k,
                   int kmul, const int32_t *k_per_query, float *dist, int64_t *labels);

// ---- external id registry (registry.hip)
constexpr int64_t REG_EMPTY = (int64_t)0x8000000000000000ull;   // table marker: never used
constexpr int64_t REG_TOMB = (int64_t)0x8000000000000001ull;    // table marker: key removed
enum RegCtl { REG_CTL_STATUS = 0, REG_CTL_TOP = 1, REG_CTL_WORDS = 64 };
struct RegDev {
    int64_t *keys;      // [cap] external id, REG_EMPTY or REG_TOMB
    int32_t *vals;      // [cap] internal id of the key
    int64_t *ext_of;    // [id_cap] external id held by each internal id, or REG_EMPTY
    int32_t *free_ids;  // [id_cap] stack of free internal ids (count in ctl[REG_CTL_TOP])
    int64_t cap, id_cap;
};
void launch_reg_add_pre(hipStream_t st, const RegDev &R, int n, const int64_t *ext, int64_t *slot, int32_t *fresh,
                        int64_t *internal, int32_t *ctl);
void launch_reg_add_post(hipStream_t st, const RegDev &R, const Dev &S, int n, const int64_t *slot,
                         const int32_t *fresh, int32_t *ctl);
void launch_reg_lookup(hipStream_t st, const RegDev &R, int n, const int64_t *ext, int64_t *slot, int64_t *internal);
void launch_reg_release(hipStream_t st, const RegDev &R, const Dev &S, int n, const int64_t *ext,
                        const int64_t *slot, int32_t *ctl);
void launch_reg_labels(hipStream_t st, const RegDev &R, int64_t n, int64_t *labels);
void launch_reg_rebuild(hipStream_t st, const RegDev &R, int32_t *ctl);
void launch_reg_free_stack(hipStream_t st, const RegDev &R, int32_t *ctl);

// ---- serving, continuous batching (serve.hip)
// One request of a coalesced search batch: its rows are batch rows
// [row0, row0 + nq); q, dist and labels are the request's own buffers.
struct SrvSeg {
    const float *q;
    float *dist;
    int64_t *labels;
    int32_t row0, nq, k, nprobe;
};
void launch_srv_gather(hipStream_t st, const SrvSeg *segs, int nseg, int nrows, int d, float *q, int32_t *kq,
                       int32_t *npq);
void launch_srv_scatter(hipStream_t st, const SrvSeg *segs, int nseg, int nrows, int kstride, const float *dist,
                        const int64_t *labels);

}  // namespace sivf
