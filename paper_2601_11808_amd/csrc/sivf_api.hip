// Host runtime of libsivf: workspace layout, argument checks and the order in
// which each C-ABI call enqueues its kernels.  All index state lives in the
// caller's device workspace; the host handle holds pointers, sizes and a call
// sequence number (data-dependent failures are recorded on the device against
// the sequence number of the failing call, so the rest of that call's kernels
// skip their work and the index is left unchanged).
#include <stdlib.h>
#include <string.h>

#include <new>
#include <deque>
#include <unordered_map>
#include <vector>

#include "sivf.h"
#include "sivf_launch.h"

using namespace sivf;

namespace {

constexpr size_t ALIGN = 256;
constexpr int64_t COARSE_BYTES = 256ll << 20;   // scratch for approximate coarse distances

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int kcap_for(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : (k <= 64 ? 64 : 128)); }

struct Layout {
    int dp4, kcap, coarse_rows;
    int64_t num_pages, dir_cap, max_items, slot_cap;
    size_t total;
    size_t cent, cent_h, cn2, cnorm, cmax, data, sids, sowner, sord, free_slabs, free_pages, pages, dir, len, att, mark,
        ctl, lists, b_assign, b_rank, b_rec, b_seg, b_inv, dt, probes, pair_rank, list_pairs, item_list, item_tile,
        item_chunk, partials, hdata, xnorm, rr_dist, rr_lab, dt_s;
};

bool config_ok(const sivf_config *c) {
    if (!c) return false;
    if (c->dim < 1 || c->dim > 2048) return false;
    if (c->nlist < 1 || c->nlist > 65536) return false;
    if (c->slab_capacity < 1 || c->slab_capacity > 128 || (c->slab_capacity & (c->slab_capacity - 1))) return false;
    if (c->metric != SIVF_L2 && c->metric != SIVF_IP) return false;
    if (c->storage != SIVF_F32 && c->storage != SIVF_BF16 && c->storage != SIVF_F16) return false;
    if (c->storage == SIVF_F32 && c->rerank_factor != 0) return false;
    if (c->storage != SIVF_F32 &&
        (c->dim > 256 || c->slab_capacity < 16 || c->rerank_factor < 1 ||
         (int64_t)c->rerank_factor * c->max_k > 64))
        return false;
    if (c->num_slabs < 1 || c->num_slabs * (int64_t)c->slab_capacity >= (1ll << 31)) return false;
    if (c->id_capacity < 1 || c->id_capacity >= (1ll << 31)) return false;
    if (c->max_batch < 1 || c->max_queries < 1) return false;
    if (c->max_k < 1 || c->max_k > 128) return false;
    if (c->max_nprobe < 1 || c->max_nprobe > 1024) return false;
    if ((int64_t)c->max_queries * c->max_nprobe >= (1ll << 31) / 64) return false;
    return true;
}

Layout make_layout(const sivf_config *c) {
    Layout L{};
    L.dp4 = (c->dim + 3) / 4;
    L.kcap = kcap_for(c->storage == SIVF_F32 ? c->max_k : c->rerank_factor * c->max_k);
    const int64_t nl = c->nlist, ns = c->num_slabs, C = c->slab_capacity;
    L.dir_cap = (ns + PAGE - 1) / PAGE + 1;
    L.num_pages = (ns + PAGE - 1) / PAGE + nl;
    const int64_t rows_cap = COARSE_BYTES / (4 * nl) > 64 ? COARSE_BYTES / (4 * nl) : 64;
    const int64_t rows_need = c->max_batch > c->max_queries ? c->max_batch : c->max_queries;
    L.coarse_rows = (int)(rows_need < rows_cap ? rows_need : rows_cap);
    const int64_t npairs = (int64_t)c->max_queries * c->max_nprobe;
    L.max_items = npairs + nl;
    L.slot_cap = npairs + npairs / 2;   // partial results: one per (pair, list chunk)
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = cur;
        cur = align_up(cur + (bytes ? bytes : 1));
        return o;
    };
    L.cent = take((size_t)nl * L.dp4 * 16);
    L.cent_h = take(c->storage != SIVF_F32 ? (size_t)nl * L.dp4 * 8 : 0);
    L.cn2 = take((size_t)nl * 4);
    L.cnorm = take((size_t)nl * 8);
    L.cmax = take(8);
    L.data = take((size_t)ns * L.dp4 * C * 16);
    L.sids = take((size_t)ns * C * 4);
    L.sowner = take((size_t)ns * 4);
    L.sord = take((size_t)ns * 4);
    L.free_slabs = take((size_t)ns * 4);
    L.free_pages = take((size_t)L.num_pages * 4);
    L.pages = take((size_t)L.num_pages * PAGE * 4);
    L.dir = take((size_t)nl * L.dir_cap * 4);
    L.len = take((size_t)nl * 4);
    L.att = take((size_t)c->id_capacity * 4);
    L.mark = take((size_t)c->id_capacity * 4);
    L.ctl = take(CTL_WORDS * 4);
    L.lists = take((size_t)16 * nl * 4);
    L.b_assign = take((size_t)c->max_batch * 4);
    L.b_rank = take((size_t)c->max_batch * 4);
    L.b_rec = take((size_t)c->max_batch * 4);
    L.b_seg = take((size_t)c->max_batch * 4);
    L.b_inv = take((size_t)c->max_batch * 4);
    L.dt = take((size_t)L.coarse_rows * nl * 4);     // coarse scratch of inserts
    L.dt_s = take((size_t)L.coarse_rows * nl * 4);   // coarse scratch of searches (they may overlap inserts)
    L.probes = take((size_t)npairs * 4);
    L.pair_rank = take((size_t)npairs * 4);
    L.list_pairs = take((size_t)npairs * 4);
    L.item_list = take((size_t)L.max_items * 4);
    L.item_tile = take((size_t)L.max_items * 4);
    L.item_chunk = take((size_t)L.max_items * 4);
    L.partials = take((size_t)L.slot_cap * L.kcap * 8);
    const bool reduced = c->storage != SIVF_F32;
    L.hdata = take(reduced ? (size_t)ns * ((c->dim + 7) / 8) * C * 16 : 0);
    // squared row norms: the rounded rows' (reduced precision, L2 scan) or the fp32 rows' (the
    // certified FP32 MFMA scan's error bound and approximate distance)
    L.xnorm = take((reduced && c->metric == SIVF_L2) || !reduced ? (size_t)ns * C * 4 : 0);
    L.rr_dist = take(reduced ? (size_t)c->max_queries * L.kcap * 4 : 0);
    L.rr_lab = take(reduced ? (size_t)c->max_queries * L.kcap * 8 : 0);
    L.total = cur;
    return L;
}

bool dev_ok(hipError_t e) { return e == hipSuccess; }

}  // namespace

// Event pairs recorded around one class of work while profiling is on.
struct ProfClass {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
    double ms = 0.0;
    int64_t count = 0;
};

struct sivf_index {
    sivf_config cfg{};
    Layout L{};
    Dev S{};
    Batch B{};
    SearchBufs W{};
    float *dt = nullptr;     // coarse scratch: inserts
    float *dt_s = nullptr;   // coarse scratch: searches
    char *ws = nullptr;
    hipStream_t last = nullptr;
    bool broken = false;
    bool prof = false;
    ProfClass pc[SIVF_PROF_KINDS];
};

namespace {

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

sivf_status launched(sivf_index *ix) {
    if (!dev_ok(hipGetLastError())) {
        ix->broken = true;
        return SIVF_ERR_DEVICE;
    }
    return SIVF_OK;
}

// Fold finished intervals of one class into its sum.
bool prof_fold(sivf_index *ix, ProfClass &c) {
    for (size_t i = 0; i < c.used; i++) {
        if (!dev_ok(hipEventSynchronize(c.stop[i]))) return false;
        float ms = 0.f;
        if (!dev_ok(hipEventElapsedTime(&ms, c.start[i], c.stop[i]))) return false;
        c.ms += ms;
        c.count++;
    }
    c.used = 0;
    return true;
}

// Returns the slot of an interval whose start was recorded, or -1.
int prof_begin(sivf_index *ix, int kind, hipStream_t st) {
    if (!ix->prof) return -1;
    ProfClass &c = ix->pc[kind];
    if (c.used == 4096 && !prof_fold(ix, c)) return -1;
    if (c.used == c.start.size()) {
        hipEvent_t a, b;
        if (!dev_ok(hipEventCreate(&a))) return -1;
        if (!dev_ok(hipEventCreate(&b))) {
            (void)hipEventDestroy(a);
            return -1;
        }
        c.start.push_back(a);
        c.stop.push_back(b);
    }
    if (!dev_ok(hipEventRecord(c.start[c.used], st))) return -1;
    return (int)c.used++;
}

void prof_end(sivf_index *ix, int kind, int slot, hipStream_t st) {
    if (slot < 0) return;
    if (!dev_ok(hipEventRecord(ix->pc[kind].stop[slot], st))) ix->pc[kind].used = (size_t)slot;
}

// Coarse selection over rows [0, n) in chunks that fit the scratch.
void coarse(sivf_index *ix, hipStream_t st, float *dt, const float *x, int64_t n, int m, const int32_t *m_per_row,
            int mmax, int32_t *out, int out_stride, int gated) {
    const Dev &S = ix->S;
    const int dpad = S.dp4 * 4;
    const int bf = S.storage != SIVF_F32;   // reduced-precision indexes run the coarse GEMM on bf16 MFMA
    for (int64_t r0 = 0; r0 < n; r0 += ix->L.coarse_rows) {
        const int nr = (int)((n - r0) < ix->L.coarse_rows ? (n - r0) : ix->L.coarse_rows);
        const float *xr = x + r0 * S.d;
        if (m == 1 && !m_per_row && mmax == 1) {
            launch_coarse_assign(st, dt, xr, nr, S.d, S.cent, S.cent_h, dpad, S.cn2, S.cmax, S.nlist, S.metric,
                                 out + r0 * out_stride, out_stride, S.ctl, gated, bf);
            continue;
        }
        launch_coarse_gemm(st, xr, nr, S.d, S.cent, S.cent_h, dpad, S.cn2, S.nlist, S.metric, dt, S.ctl, gated, bf);
        launch_coarse_select(st, dt, xr, nr, S.d, S.cent, dpad, S.cnorm, S.cmax, S.nlist, S.metric, m,
                             m_per_row ? m_per_row + r0 : nullptr, mmax, out + r0 * out_stride, out_stride,
                             S.ctl, gated, bf);
    }
}

sivf_status do_add(sivf_index *ix, int64_t n, const float *x, const int64_t *ids, hipStream_t st,
                   bool fresh_only = false) {
    if (n < 0 || n > ix->cfg.max_batch) return SIVF_ERR_ARG;
    if (n > 0 && (!x || !ids)) return SIVF_ERR_ARG;
    if (n == 0) return SIVF_OK;
    const Dev &S = ix->S;
    const int nn = (int)n;
    const int ps = prof_begin(ix, SIVF_PROF_ADD, st);
    launch_add_prepare(st, S, nn, ids);
    coarse(ix, st, ix->dt, x, n, 1, nullptr, 1, ix->B.assign, 1, 1);
    launch_add_count(st, S, nn, ids, ix->B, fresh_only ? 1 : 0);
    launch_add_admit(st, S);
    if (!fresh_only) launch_remove(st, S, nn, ids, nullptr, ix->B, 1);   // delete half of an upsert
    launch_add_alloc(st, S);
    launch_add_scatter(st, S, nn, x, ids, ix->B);
    launch_add_cleanup(st, S, nn, ids);
    launch_call_end(st, S);
    prof_end(ix, SIVF_PROF_ADD, ps, st);
    return launched(ix);
}

sivf_status do_remove(sivf_index *ix, int64_t n, const int64_t *ids, int64_t *n_removed, hipStream_t st) {
    if (n < 0 || n > ix->cfg.max_batch) return SIVF_ERR_ARG;
    if (n > 0 && !ids) return SIVF_ERR_ARG;
    if (n == 0) {
        if (n_removed) launch_fill_i64(st, n_removed, 1, 0);
        return launched(ix);
    }
    const int ps = prof_begin(ix, SIVF_PROF_REMOVE, st);
    launch_remove(st, ix->S, (int)n, ids, n_removed, ix->B, 0);
    launch_call_end(st, ix->S);
    prof_end(ix, SIVF_PROF_REMOVE, ps, st);
    return launched(ix);
}

sivf_status do_search(sivf_index *ix, int64_t nq, const float *q, int32_t k, const int32_t *kpq, int32_t nprobe,
                      const int32_t *npq, float *dist, int64_t *labels, hipStream_t st,
                      hipEvent_t snapshot_taken = nullptr) {
    const sivf_config &c = ix->cfg;
    if (nq < 0 || nq > c.max_queries) return SIVF_ERR_ARG;
    if (k < 1 || k > c.max_k) return SIVF_ERR_ARG;
    if (!npq && (nprobe < 1 || nprobe > c.max_nprobe)) return SIVF_ERR_ARG;
    if (nq == 0) return SIVF_OK;
    if (!q || !dist || !labels) return SIVF_ERR_ARG;
    const int mmax = npq ? c.max_nprobe : nprobe;
    const int stride = mmax < c.nlist ? mmax : c.nlist;
    const int ps = prof_begin(ix, SIVF_PROF_SEARCH, st);
    const int pc = prof_begin(ix, SIVF_PROF_COARSE, st);
    coarse(ix, st, ix->dt_s, q, nq, npq ? 0 : stride, npq, stride, ix->W.probes, stride, 0);
    prof_end(ix, SIVF_PROF_COARSE, pc, st);
    launch_search_plan(st, ix->S, ix->W, (int)nq, stride);   // records the list lengths it will scan
    if (snapshot_taken && !dev_ok(hipEventRecord(snapshot_taken, st))) return SIVF_ERR_DEVICE;
    const int pk = prof_begin(ix, SIVF_PROF_SCAN, st);
    if (c.storage == SIVF_F32)
        launch_search_scan(st, ix->S, ix->W, (int)nq, q, stride, ix->L.kcap, k, kpq);
    else
        launch_search_scan_mfma(st, ix->S, ix->W, (int)nq, q, stride, ix->L.kcap, k, c.rerank_factor, kpq);
    prof_end(ix, SIVF_PROF_SCAN, pk, st);
    const int pm = prof_begin(ix, SIVF_PROF_MERGE, st);
    if (c.storage == SIVF_F32) {
        launch_search_merge(st, ix->S, ix->W, (int)nq, stride, ix->L.kcap, k, k, 1, kpq, dist, labels);
    } else {
        // approximate candidates, then the exact fp32 re-rank of R * k per query
        const int kc = c.rerank_factor * k;
        launch_search_merge(st, ix->S, ix->W, (int)nq, stride, ix->L.kcap, kc, k, c.rerank_factor, kpq,
                            ix->W.rr_dist, ix->W.rr_lab);
        launch_rerank(st, ix->S, (int)nq, q, kc, ix->W.rr_lab, k, c.rerank_factor, kpq, dist, labels);
    }
    prof_end(ix, SIVF_PROF_MERGE, pm, st);
    prof_end(ix, SIVF_PROF_SEARCH, ps, st);
    return launched(ix);
}

}  // namespace

extern "C" {

size_t sivf_workspace_bytes(const sivf_config *cfg) {
    if (!config_ok(cfg)) return 0;
    return make_layout(cfg).total;
}

sivf_status sivf_create(const sivf_config *cfg, const float *centroids, void *workspace, size_t ws_bytes,
                        void *stream, sivf_index **out) {
    if (!out) return SIVF_ERR_ARG;
    *out = nullptr;
    if (!config_ok(cfg) || !centroids || !workspace) return SIVF_ERR_ARG;
    const Layout L = make_layout(cfg);
    if (ws_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0) return SIVF_ERR_ARG;
    sivf_index *ix = new (std::nothrow) sivf_index();
    if (!ix) return SIVF_ERR_STATE;
    ix->cfg = *cfg;
    ix->L = L;
    ix->ws = (char *)workspace;
    char *w = ix->ws;
    Dev &S = ix->S;
    S.d = cfg->dim;
    S.dp4 = L.dp4;
    S.nlist = cfg->nlist;
    S.C = cfg->slab_capacity;
    S.metric = cfg->metric;
    S.storage = cfg->storage;
    S.dp8 = (cfg->dim + 7) / 8;
    S.tile = default_tile(cfg->storage, cfg->dim, cfg->slab_capacity, L.kcap);
    S.chunk_shift = DEFAULT_CHUNK_SHIFT;
    S.persistent = 0;
    S.hdata = cfg->storage != SIVF_F32 ? (uint4 *)(w + L.hdata) : nullptr;
    S.xnorm = (cfg->storage == SIVF_F32 || cfg->metric == SIVF_L2) ? (float *)(w + L.xnorm) : nullptr;
    ix->W.rr_dist = cfg->storage != SIVF_F32 ? (float *)(w + L.rr_dist) : nullptr;
    ix->W.rr_lab = cfg->storage != SIVF_F32 ? (int64_t *)(w + L.rr_lab) : nullptr;
    S.num_slabs = cfg->num_slabs;
    S.num_pages = L.num_pages;
    S.dir_cap = L.dir_cap;
    S.id_capacity = cfg->id_capacity;
    S.cent = (const float *)(w + L.cent);
    S.cent_h = cfg->storage != SIVF_F32 ? (const uint16_t *)(w + L.cent_h) : nullptr;
    S.cn2 = (const float *)(w + L.cn2);
    S.cnorm = (const double *)(w + L.cnorm);
    S.cmax = (const double *)(w + L.cmax);
    S.data = (float4 *)(w + L.data);
    S.sids = (uint32_t *)(w + L.sids);
    S.sowner = (int32_t *)(w + L.sowner);
    S.sord = (int32_t *)(w + L.sord);
    S.free_slabs = (int32_t *)(w + L.free_slabs);
    S.free_pages = (int32_t *)(w + L.free_pages);
    S.pages = (int32_t *)(w + L.pages);
    S.dir = (int32_t *)(w + L.dir);
    S.len = (int32_t *)(w + L.len);
    S.att = (uint32_t *)(w + L.att);
    S.mark = (int32_t *)(w + L.mark);
    S.ctl = (int32_t *)(w + L.ctl);
    int32_t *lists = (int32_t *)(w + L.lists);
    int32_t **lp[] = {&S.l_acnt, &S.l_prem, &S.l_base, &S.l_eoff, &S.l_m, &S.l_off, &S.l_newlen,
                      &S.l_q, &S.l_s, &S.l_h, &S.l_qc, &S.l_qcs, &S.l_qoff, &S.l_snap, &S.l_pbase, &S.l_ioff};
    for (int i = 0; i < 16; i++) *lp[i] = lists + (size_t)i * cfg->nlist;
    ix->B.assign = (int32_t *)(w + L.b_assign);
    ix->B.rank = (int32_t *)(w + L.b_rank);
    ix->B.rec = (uint32_t *)(w + L.b_rec);
    ix->B.seg = (int32_t *)(w + L.b_seg);
    ix->B.inv = (int32_t *)(w + L.b_inv);
    ix->dt = (float *)(w + L.dt);
    ix->dt_s = (float *)(w + L.dt_s);
    ix->W.probes = (int32_t *)(w + L.probes);
    ix->W.pair_rank = (int32_t *)(w + L.pair_rank);
    ix->W.list_pairs = (int32_t *)(w + L.list_pairs);
    ix->W.item_list = (int32_t *)(w + L.item_list);
    ix->W.item_tile = (int32_t *)(w + L.item_tile);
    ix->W.item_chunk = (int32_t *)(w + L.item_chunk);
    ix->W.partials = (uint64_t *)(w + L.partials);
    ix->W.slot_cap = L.slot_cap;
    ix->W.item_cap = L.max_items;
    ix->last = as_stream(stream);
    launch_init_state(as_stream(stream), S, centroids);
    if (!dev_ok(hipGetLastError())) {
        delete ix;
        return SIVF_ERR_DEVICE;
    }
    *out = ix;
    return SIVF_OK;
}

sivf_status sivf_destroy(sivf_index *ix) {
    if (!ix) return SIVF_ERR_ARG;
    for (ProfClass &c : ix->pc) {
        for (hipEvent_t e : c.start) (void)hipEventDestroy(e);
        for (hipEvent_t e : c.stop) (void)hipEventDestroy(e);
    }
    delete ix;
    return SIVF_OK;
}

sivf_status sivf_profile_enable(sivf_index *ix, int on) {
    if (!ix) return SIVF_ERR_ARG;
    ix->prof = on != 0;
    return SIVF_OK;
}

sivf_status sivf_profile_read(sivf_index *ix, double *total_ms, int64_t *count) {
    if (!ix) return SIVF_ERR_ARG;
    for (int k = 0; k < SIVF_PROF_KINDS; k++) {
        ProfClass &c = ix->pc[k];
        if (!prof_fold(ix, c)) return SIVF_ERR_DEVICE;
        if (total_ms) total_ms[k] = c.ms;
        if (count) count[k] = c.count;
        c.ms = 0.0;
        c.count = 0;
    }
    return SIVF_OK;
}

sivf_status sivf_add(sivf_index *ix, int64_t n, const float *x, const int64_t *ids, void *stream) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    ix->last = as_stream(stream);
    return do_add(ix, n, x, ids, as_stream(stream));
}

sivf_status sivf_remove(sivf_index *ix, int64_t n, const int64_t *ids, int64_t *n_removed, void *stream) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    ix->last = as_stream(stream);
    return do_remove(ix, n, ids, n_removed, as_stream(stream));
}

sivf_status sivf_search(sivf_index *ix, int64_t nq, const float *q, int32_t k, const int32_t *k_per_query,
                        int32_t nprobe, const int32_t *nprobe_per_query, float *dist, int64_t *labels,
                        void *stream) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    ix->last = as_stream(stream);
    return do_search(ix, nq, q, k, k_per_query, nprobe, nprobe_per_query, dist, labels, as_stream(stream));
}

sivf_status sivf_tune_search(sivf_index *ix, int64_t nq, const float *q, int32_t k, const int32_t *k_per_query,
                             int32_t nprobe, const int32_t *nprobe_per_query, float *dist, int64_t *labels,
                             void *stream, int32_t *tile, int32_t *chunk_shift, int32_t *persistent) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    std::vector<int> tiles;
    if (ix->cfg.storage != SIVF_F32) tiles = {16};
    else if (ix->cfg.dim <= 1024) tiles = {8, 4};
    else tiles = {4};
    if (cert_ok(ix->cfg.storage, ix->cfg.dim, ix->cfg.slab_capacity, ix->L.kcap)) tiles.push_back(16);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!dev_ok(hipEventCreate(&e0)) || !dev_ok(hipEventCreate(&e1))) {
        if (e0) (void)hipEventDestroy(e0);
        return SIVF_ERR_DEVICE;
    }
    const bool prof = ix->prof;
    ix->prof = false;
    int bt = ix->S.tile, bs = ix->S.chunk_shift, bp = ix->S.persistent;
    float best = -1.f;
    sivf_status s = SIVF_OK;
    for (int pm = 0; pm < 2; pm++)
    for (int T : tiles) {
        for (int sh = 10; sh <= 17 && s == SIVF_OK; sh++) {
            ix->S.tile = T;
            ix->S.chunk_shift = sh;
            ix->S.persistent = pm;
            s = do_search(ix, nq, q, k, k_per_query, nprobe, nprobe_per_query, dist, labels, st);   // warm-up
            if (s != SIVF_OK) break;
            if (!dev_ok(hipEventRecord(e0, st))) s = SIVF_ERR_DEVICE;
            for (int r = 0; r < 2 && s == SIVF_OK; r++)
                s = do_search(ix, nq, q, k, k_per_query, nprobe, nprobe_per_query, dist, labels, st);
            float ms = 0.f;
            if (s == SIVF_OK && (!dev_ok(hipEventRecord(e1, st)) || !dev_ok(hipEventSynchronize(e1)) ||
                                 !dev_ok(hipEventElapsedTime(&ms, e0, e1))))
                s = SIVF_ERR_DEVICE;
            if (s == SIVF_OK && (best < 0.f || ms < best)) {
                best = ms;
                bt = T;
                bs = sh;
                bp = pm;
            }
        }
    }
    ix->S.tile = bt;
    ix->S.chunk_shift = bs;
    ix->S.persistent = bp;
    ix->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (tile) *tile = bt;
    if (chunk_shift) *chunk_shift = bs;
    if (persistent) *persistent = bp;
    return s;
}

sivf_status sivf_set_search_schedule(sivf_index *ix, int32_t tile, int32_t chunk_shift, int32_t persistent) {
    if (!ix) return SIVF_ERR_ARG;
    const bool reduced = ix->cfg.storage != SIVF_F32;
    const bool cert = tile == 16 && cert_ok(ix->cfg.storage, ix->cfg.dim, ix->cfg.slab_capacity, ix->L.kcap);
    if (reduced ? tile != 16 : (tile != 4 && (tile != 8 || ix->cfg.dim > 1024) && !cert)) return SIVF_ERR_ARG;
    if (chunk_shift < 6 || chunk_shift > 31 || (persistent != 0 && persistent != 1)) return SIVF_ERR_ARG;
    ix->S.tile = tile;
    ix->S.chunk_shift = chunk_shift;
    ix->S.persistent = persistent;
    return SIVF_OK;
}

static bool step_args_ok(const sivf_index *ix, const sivf_step_args *a) {
    const sivf_config &c = ix->cfg;
    if (a->n_add < 0 || a->n_add > c.max_batch || a->n_remove < 0 || a->n_remove > c.max_batch) return false;
    if (a->nq < 0 || a->nq > c.max_queries) return false;
    if (a->nq > 0 && (a->k < 1 || a->k > c.max_k)) return false;
    if (a->nq > 0 && !a->nprobe_per_query && (a->nprobe < 1 || a->nprobe > c.max_nprobe)) return false;
    return true;
}

static sivf_status enqueue_step(sivf_index *ix, const sivf_step_args *a, hipStream_t st) {
    sivf_status s = do_add(ix, a->n_add, a->x, a->add_ids, st);
    if (s != SIVF_OK) return s;
    if (a->nq > 0) {
        s = do_search(ix, a->nq, a->q, a->k, a->k_per_query, a->nprobe, a->nprobe_per_query, a->dist, a->labels,
                      st);
        if (s != SIVF_OK) return s;
    }
    return do_remove(ix, a->n_remove, a->remove_ids, a->n_removed, st);
}

struct sivf_graph {
    sivf_index *ix;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

sivf_status sivf_graph_create(sivf_index *ix, const sivf_step_args *a, sivf_graph **out) {
    if (!ix || !a || !out) return SIVF_ERR_ARG;
    *out = nullptr;
    if (ix->broken) return SIVF_ERR_STATE;
    if (!step_args_ok(ix, a)) return SIVF_ERR_ARG;
    hipStream_t cs;
    if (!dev_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) return SIVF_ERR_DEVICE;
    const bool prof = ix->prof;
    ix->prof = false;
    hipGraph_t graph = nullptr;
    sivf_status s = SIVF_OK;
    if (!dev_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal))) {
        s = SIVF_ERR_DEVICE;
    } else {
        s = enqueue_step(ix, a, cs);
        if (!dev_ok(hipStreamEndCapture(cs, &graph)) && s == SIVF_OK) s = SIVF_ERR_DEVICE;
    }
    ix->prof = prof;
    (void)hipStreamDestroy(cs);
    if (s != SIVF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    hipGraphExec_t exec;
    if (!dev_ok(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0))) {
        (void)hipGraphDestroy(graph);
        return SIVF_ERR_DEVICE;
    }
    sivf_graph *g = new (std::nothrow) sivf_graph{ix, graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return SIVF_ERR_STATE;
    }
    *out = g;
    return SIVF_OK;
}

sivf_status sivf_graph_launch(sivf_graph *g, void *stream) {
    if (!g) return SIVF_ERR_ARG;
    if (g->ix->broken) return SIVF_ERR_STATE;
    g->ix->last = as_stream(stream);
    return dev_ok(hipGraphLaunch(g->exec, as_stream(stream))) ? SIVF_OK : SIVF_ERR_DEVICE;
}

sivf_status sivf_graph_destroy(sivf_graph *g) {
    if (!g) return SIVF_ERR_ARG;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return SIVF_OK;
}

sivf_status sivf_step(sivf_index *ix, const sivf_step_args *a, void *stream) {
    if (!ix || !a) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    if (!step_args_ok(ix, a)) return SIVF_ERR_ARG;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    return enqueue_step(ix, a, st);
}

sivf_status sivf_assign(sivf_index *ix, int64_t n, const float *x, int32_t *lists, void *stream) {
    if (!ix || n < 0 || (n > 0 && (!x || !lists))) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    const int64_t cap = ix->cfg.max_batch > ix->cfg.max_queries ? ix->cfg.max_batch : ix->cfg.max_queries;
    if (n > cap) return SIVF_ERR_ARG;
    ix->last = as_stream(stream);
    if (n == 0) return SIVF_OK;
    coarse(ix, as_stream(stream), ix->dt, x, n, 1, nullptr, 1, lists, 1, 0);
    return launched(ix);
}

sivf_status sivf_probe(sivf_index *ix, int64_t nq, const float *q, int32_t nprobe, int32_t *probes, void *stream) {
    if (!ix || nq < 0 || (nq > 0 && (!q || !probes))) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    if (nprobe < 1 || nprobe > ix->cfg.max_nprobe) return SIVF_ERR_ARG;
    const int64_t cap = ix->cfg.max_batch > ix->cfg.max_queries ? ix->cfg.max_batch : ix->cfg.max_queries;
    if (nq > cap) return SIVF_ERR_ARG;
    ix->last = as_stream(stream);
    if (nq == 0) return SIVF_OK;
    const int m = nprobe < ix->cfg.nlist ? nprobe : ix->cfg.nlist;
    coarse(ix, as_stream(stream), ix->dt_s, q, nq, m, nullptr, nprobe, probes, nprobe, 0);
    return launched(ix);
}

sivf_status sivf_coarse_scores(sivf_index *ix, int64_t n, const float *x, float *scores, void *stream) {
    if (!ix || n < 0 || (n > 0 && (!x || !scores))) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    const int64_t cap = ix->cfg.max_batch > ix->cfg.max_queries ? ix->cfg.max_batch : ix->cfg.max_queries;
    if (n > cap) return SIVF_ERR_ARG;
    ix->last = as_stream(stream);
    if (n == 0) return SIVF_OK;
    const Dev &S = ix->S;
    launch_coarse_gemm(as_stream(stream), x, (int)n, S.d, S.cent, S.cent_h, S.dp4 * 4, S.cn2, S.nlist, S.metric, scores,
                       S.ctl, 0, S.storage != SIVF_F32);
    return launched(ix);
}

sivf_status sivf_get_rows(sivf_index *ix, int64_t n, const int64_t *ids, float *rows, void *stream) {
    if (!ix || n < 0 || n > (1 << 26) || (n > 0 && (!ids || !rows))) return SIVF_ERR_ARG;   // no scratch used
    if (ix->broken) return SIVF_ERR_STATE;
    ix->last = as_stream(stream);
    if (n == 0) return SIVF_OK;
    launch_get_rows(as_stream(stream), ix->S, (int)n, ids, rows);
    return launched(ix);
}

sivf_status sivf_sync(sivf_index *ix, sivf_status *device_status) {
    if (!ix) return SIVF_ERR_ARG;
    if (!dev_ok(hipStreamSynchronize(ix->last))) return SIVF_ERR_DEVICE;
    int32_t st = 0, zero = 0;
    if (!dev_ok(hipMemcpyAsync(&st, ix->S.ctl + CTL_STATUS, 4, hipMemcpyDeviceToHost, ix->last))) return SIVF_ERR_DEVICE;
    if (!dev_ok(hipMemcpyAsync(ix->S.ctl + CTL_STATUS, &zero, 4, hipMemcpyHostToDevice, ix->last)))
        return SIVF_ERR_DEVICE;
    if (!dev_ok(hipStreamSynchronize(ix->last))) return SIVF_ERR_DEVICE;
    if (device_status) *device_status = (sivf_status)st;
    return SIVF_OK;
}

static sivf_status read_counts(sivf_index *ix, std::vector<int32_t> &len, int32_t *ctl) {
    len.resize(ix->cfg.nlist);
    if (!dev_ok(hipStreamSynchronize(ix->last))) return SIVF_ERR_DEVICE;
    if (!dev_ok(hipMemcpy(len.data(), ix->S.len, sizeof(int32_t) * len.size(), hipMemcpyDeviceToHost)))
        return SIVF_ERR_DEVICE;
    if (!dev_ok(hipMemcpy(ctl, ix->S.ctl, sizeof(int32_t) * CTL_WORDS, hipMemcpyDeviceToHost))) return SIVF_ERR_DEVICE;
    return SIVF_OK;
}

sivf_status sivf_dump_info_get(sivf_index *ix, sivf_dump_info *info) {
    if (!ix || !info) return SIVF_ERR_ARG;
    std::vector<int32_t> len;
    int32_t ctl[CTL_WORDS];
    sivf_status s = read_counts(ix, len, ctl);
    if (s != SIVF_OK) return s;
    int64_t live = 0, used = 0;
    const int C = ix->cfg.slab_capacity;
    for (int32_t v : len) {
        live += v;
        used += (v + C - 1) / C;
    }
    info->live = live;
    info->used_slabs = used;
    info->free_slabs = ctl[CTL_SLAB_TOP];
    info->num_slabs = ix->cfg.num_slabs;
    info->id_capacity = ix->cfg.id_capacity;
    info->nlist = ix->cfg.nlist;
    info->slab_capacity = C;
    return SIVF_OK;
}

sivf_status sivf_stats(sivf_index *ix, int64_t *live, int64_t *used_slabs, int64_t *free_slabs) {
    sivf_dump_info info;
    sivf_status s = sivf_dump_info_get(ix, &info);
    if (s != SIVF_OK) return s;
    if (live) *live = info.live;
    if (used_slabs) *used_slabs = info.used_slabs;
    if (free_slabs) *free_slabs = info.free_slabs;
    return SIVF_OK;
}

sivf_status sivf_dump(sivf_index *ix, int32_t *list_len, int32_t *list_slabs, int64_t *ids_by_list,
                      int32_t *free_slabs, int32_t *slab_owner, int32_t *slab_ordinal, uint32_t *att) {
    if (!ix) return SIVF_ERR_ARG;
    std::vector<int32_t> len;
    int32_t ctl[CTL_WORDS];
    sivf_status s = read_counts(ix, len, ctl);
    if (s != SIVF_OK) return s;
    const sivf_config &c = ix->cfg;
    const int C = c.slab_capacity;
    const Dev &S = ix->S;
    auto d2h = [&](void *dst, const void *src, size_t bytes) { return dev_ok(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost)); };
    if (list_len) memcpy(list_len, len.data(), sizeof(int32_t) * len.size());
    if (list_slabs || ids_by_list) {
        std::vector<int32_t> dir((size_t)c.nlist * S.dir_cap), pages((size_t)S.num_pages * PAGE);
        std::vector<uint32_t> sids;
        if (!d2h(dir.data(), S.dir, dir.size() * 4) || !d2h(pages.data(), S.pages, pages.size() * 4))
            return SIVF_ERR_DEVICE;
        if (ids_by_list) {
            sids.resize((size_t)c.num_slabs * C);
            if (!d2h(sids.data(), S.sids, sids.size() * 4)) return SIVF_ERR_DEVICE;
        }
        int64_t so = 0, io = 0;
        for (int l = 0; l < c.nlist; l++) {
            const int ns = (len[l] + C - 1) / C;
            for (int o = 0; o < ns; o++) {
                const int page = dir[(size_t)l * S.dir_cap + o / PAGE];
                if (page < 0 || page >= S.num_pages) return SIVF_ERR_STATE;
                const int slab = pages[(size_t)page * PAGE + o % PAGE];
                if (list_slabs) list_slabs[so++] = slab;
                if (ids_by_list) {
                    if (slab < 0 || slab >= c.num_slabs) return SIVF_ERR_STATE;
                    const int cnt = (o == ns - 1) ? len[l] - o * C : C;
                    for (int t = 0; t < cnt; t++) {
                        const uint32_t v = sids[(size_t)slab * C + t];
                        ids_by_list[io++] = v == INVALID ? -1 : (int64_t)v;
                    }
                }
            }
        }
    }
    if (free_slabs && ctl[CTL_SLAB_TOP] > 0 && !d2h(free_slabs, S.free_slabs, (size_t)ctl[CTL_SLAB_TOP] * 4))
        return SIVF_ERR_DEVICE;
    if (slab_owner && !d2h(slab_owner, S.sowner, (size_t)c.num_slabs * 4)) return SIVF_ERR_DEVICE;
    if (slab_ordinal && !d2h(slab_ordinal, S.sord, (size_t)c.num_slabs * 4)) return SIVF_ERR_DEVICE;
    if (att && !d2h(att, S.att, (size_t)c.id_capacity * 4)) return SIVF_ERR_DEVICE;
    return SIVF_OK;
}

// ------------------------------------------------------------------ server

struct ServerReq {
    int64_t ticket;
    hipEvent_t done;
    int64_t reserve;     // slabs reserved by an insert until it completes
};

struct sivf_server {
    sivf_index *ix = nullptr;
    hipStream_t s_search = nullptr, s_mut = nullptr;
    hipEvent_t last_mut = nullptr, last_snap = nullptr, last_search = nullptr, inputs = nullptr;
    bool any_mut = false, any_search = false;
    std::vector<hipEvent_t> pool;
    // Requests in flight per stream, in submission order (they complete in
    // that order, so only the oldest of each queue needs a query).
    std::deque<ServerReq> q_search, q_mut;
    std::unordered_map<int64_t, hipEvent_t> inflight;   // ticket -> completion event
    int32_t *mirror = nullptr;     // pinned: free-slab count copied after each mutation
    int64_t free_view = 0, reserved = 0, next_ticket = 1;
};

static hipEvent_t server_event(sivf_server *s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (!dev_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming))) return nullptr;
    return e;
}

// Retire completed requests: recycle events, release reservations, refresh
// the host view of free slabs from the last completed copy.
static void server_reap(sivf_server *s) {
    bool mut_done = false;
    for (std::deque<ServerReq> *q : {&s->q_search, &s->q_mut}) {
        while (!q->empty() && hipEventQuery(q->front().done) == hipSuccess) {
            const ServerReq &r = q->front();
            s->reserved -= r.reserve;
            mut_done |= (q == &s->q_mut);
            s->pool.push_back(r.done);
            s->inflight.erase(r.ticket);
            q->pop_front();
        }
    }
    if (mut_done) s->free_view = *(volatile int32_t *)s->mirror;
}

// The request's inputs come from work enqueued on input_stream: start after it.
static bool server_inputs(sivf_server *s, void *input_stream, hipStream_t st) {
    return dev_ok(hipEventRecord(s->inputs, as_stream(input_stream))) && dev_ok(hipStreamWaitEvent(st, s->inputs, 0));
}

static sivf_status server_finish(sivf_server *s, hipStream_t st, bool mutation, int64_t reserve, int64_t *ticket) {
    if (mutation) {
        if (!dev_ok(hipMemcpyAsync(s->mirror, s->ix->S.ctl + CTL_SLAB_TOP, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   st)))
            return SIVF_ERR_DEVICE;
    }
    hipEvent_t e = server_event(s);
    if (!e || !dev_ok(hipEventRecord(e, st))) return SIVF_ERR_DEVICE;
    if (mutation) {
        if (!dev_ok(hipEventRecord(s->last_mut, st))) return SIVF_ERR_DEVICE;
        s->any_mut = true;
    }
    const int64_t t = s->next_ticket++;
    (mutation ? s->q_mut : s->q_search).push_back(ServerReq{t, e, reserve});
    s->inflight[t] = e;
    s->reserved += reserve;
    if (ticket) *ticket = t;
    return SIVF_OK;
}

sivf_status sivf_server_create(sivf_index *ix, sivf_server **out) {
    if (!ix || !out) return SIVF_ERR_ARG;
    *out = nullptr;
    if (ix->broken) return SIVF_ERR_STATE;
    if (!dev_ok(hipStreamSynchronize(ix->last))) return SIVF_ERR_DEVICE;
    sivf_server *s = new (std::nothrow) sivf_server();
    if (!s) return SIVF_ERR_STATE;
    s->ix = ix;
    bool ok = dev_ok(hipStreamCreateWithFlags(&s->s_search, hipStreamNonBlocking)) &&
              dev_ok(hipStreamCreateWithFlags(&s->s_mut, hipStreamNonBlocking)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_mut, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_snap, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_search, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->inputs, hipEventDisableTiming)) &&
              dev_ok(hipHostMalloc((void **)&s->mirror, sizeof(int32_t), hipHostMallocDefault));
    if (ok) {
        ok = dev_ok(hipMemcpy(s->mirror, ix->S.ctl + CTL_SLAB_TOP, sizeof(int32_t), hipMemcpyDeviceToHost));
        s->free_view = *s->mirror;
    }
    if (!ok) {
        sivf_server_destroy(s);
        return SIVF_ERR_DEVICE;
    }
    *out = s;
    return SIVF_OK;
}

sivf_status sivf_server_destroy(sivf_server *s) {
    if (!s) return SIVF_ERR_ARG;
    if (s->s_search) (void)hipStreamSynchronize(s->s_search);
    if (s->s_mut) (void)hipStreamSynchronize(s->s_mut);
    for (auto &kv : s->inflight) (void)hipEventDestroy(kv.second);
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : {s->last_mut, s->last_snap, s->last_search, s->inputs})
        if (e) (void)hipEventDestroy(e);
    if (s->s_search) (void)hipStreamDestroy(s->s_search);
    if (s->s_mut) (void)hipStreamDestroy(s->s_mut);
    if (s->mirror) (void)hipHostFree(s->mirror);
    delete s;
    return SIVF_OK;
}

sivf_status sivf_server_add(sivf_server *s, int64_t n, const float *x, const int64_t *ids, void *input_stream,
                            int64_t *ticket) {
    if (!s) return SIVF_ERR_ARG;
    sivf_index *ix = s->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    if (n < 0 || n > ix->cfg.max_batch || (n > 0 && (!x || !ids))) return SIVF_ERR_ARG;
    server_reap(s);
    const int64_t C = ix->cfg.slab_capacity;
    const int64_t need = (n + C - 1) / C + (n < ix->cfg.nlist ? n : ix->cfg.nlist);
    if (need > s->free_view - s->reserved) return SIVF_ERR_NOSPACE;
    if (s->any_search && !dev_ok(hipStreamWaitEvent(s->s_mut, s->last_snap, 0))) return SIVF_ERR_DEVICE;
    if (!server_inputs(s, input_stream, s->s_mut)) return SIVF_ERR_DEVICE;
    sivf_status st = do_add(ix, n, x, ids, s->s_mut, true);
    if (st != SIVF_OK) return st;
    return server_finish(s, s->s_mut, true, need, ticket);
}

sivf_status sivf_server_remove(sivf_server *s, int64_t n, const int64_t *ids, int64_t *n_removed,
                               void *input_stream, int64_t *ticket) {
    if (!s) return SIVF_ERR_ARG;
    sivf_index *ix = s->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    if (n < 0 || n > ix->cfg.max_batch || (n > 0 && !ids)) return SIVF_ERR_ARG;
    server_reap(s);
    if (s->any_search && !dev_ok(hipStreamWaitEvent(s->s_mut, s->last_search, 0))) return SIVF_ERR_DEVICE;
    if (!server_inputs(s, input_stream, s->s_mut)) return SIVF_ERR_DEVICE;
    sivf_status st = do_remove(ix, n, ids, n_removed, s->s_mut);
    if (st != SIVF_OK) return st;
    return server_finish(s, s->s_mut, true, 0, ticket);
}

sivf_status sivf_server_search(sivf_server *s, int64_t nq, const float *q, int32_t k, int32_t nprobe,
                               float *dist, int64_t *labels, void *input_stream, int64_t *ticket) {
    if (!s) return SIVF_ERR_ARG;
    sivf_index *ix = s->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    server_reap(s);
    if (s->any_mut && !dev_ok(hipStreamWaitEvent(s->s_search, s->last_mut, 0))) return SIVF_ERR_DEVICE;
    if (!server_inputs(s, input_stream, s->s_search)) return SIVF_ERR_DEVICE;
    sivf_status st = do_search(ix, nq, q, k, nullptr, nprobe, nullptr, dist, labels, s->s_search, s->last_snap);
    if (st != SIVF_OK) return st;
    if (!dev_ok(hipEventRecord(s->last_search, s->s_search))) return SIVF_ERR_DEVICE;
    s->any_search = true;
    return server_finish(s, s->s_search, false, 0, ticket);
}

sivf_status sivf_server_poll(sivf_server *s, int64_t ticket, int *done) {
    if (!s || !done) return SIVF_ERR_ARG;
    server_reap(s);
    *done = (ticket > 0 && ticket < s->next_ticket && s->inflight.find(ticket) == s->inflight.end()) ? 1 : 0;
    return SIVF_OK;
}

sivf_status sivf_server_wait(sivf_server *s, int64_t ticket) {
    if (!s) return SIVF_ERR_ARG;
    auto it = s->inflight.find(ticket);
    if (it != s->inflight.end() && !dev_ok(hipEventSynchronize(it->second))) return SIVF_ERR_DEVICE;
    server_reap(s);
    return SIVF_OK;
}

sivf_status sivf_server_free_slabs(sivf_server *s, int64_t *free_slabs, int64_t *reserved) {
    if (!s) return SIVF_ERR_ARG;
    server_reap(s);
    if (free_slabs) *free_slabs = s->free_view;
    if (reserved) *reserved = s->reserved;
    return SIVF_OK;
}

const char *sivf_status_string(sivf_status s) {
    switch (s) {
        case SIVF_OK: return "ok";
        case SIVF_ERR_ARG: return "invalid argument";
        case SIVF_ERR_NOSPACE: return "slab pool exhausted";
        case SIVF_ERR_ID_RANGE: return "id outside [0, id_capacity)";
        case SIVF_ERR_DEVICE: return "HIP runtime error";
        case SIVF_ERR_STATE: return "index state unusable";
        case SIVF_ERR_LIVE_ID: return "a server insert named a live id";
    }
    return "unknown status";
}

}  // extern "C"
