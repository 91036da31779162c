// Host runtime of libsivf: workspace layout, argument checks and the order in
// which each C-ABI call enqueues its kernels.  All index state lives in the
// caller's device workspace; the host handle holds pointers, sizes and a call
// sequence number (data-dependent failures are recorded on the device against
// the sequence number of the failing call, so the rest of that call's kernels
// skip their work and the index is left unchanged).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "sivf.h"
#include "sivf_launch.h"

using namespace sivf;

namespace {

constexpr size_t ALIGN = 256;
constexpr int64_t COARSE_BYTES = 256ll << 20;   // scratch for approximate coarse distances

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

constexpr int NLISTS = 17;   // per-list scratch arrays

int kcap_for(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : (k <= 64 ? 64 : 128)); }

struct Layout {
    int dp4, kcap, coarse_rows;
    int64_t num_pages, dir_cap, max_items, slot_cap;
    size_t total;
    size_t cent, cent_h, cn2, cnorm, cmax, data, sids, sowner, sord, free_slabs, free_pages, pages, dir, len, att, mark,
        ctl, lists, b_assign, b_rank, b_rec, b_seg, b_inv, dt, probes, pair_rank, list_pairs, item_list, item_tile,
        item_chunk, partials, hdata, xnorm, rr_dist, rr_lab, gthr, dt_s, srv_q, srv_k, srv_np, srv_dist, srv_lab,
        srv_seg, bits;
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
    if (c->delete_mode != SIVF_DELETE_COMPACT && c->delete_mode != SIVF_DELETE_LAZY) return false;
    if (c->reserved != 0) return false;
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
    L.cent_h = take((size_t)nl * L.dp4 * 8);   // bf16 centroids: insert assignment (every storage)
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
    L.lists = take((size_t)NLISTS * nl * 4);
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
    L.gthr = take((size_t)c->max_queries * 4);   // per-query shared thresholds of the MFMA scans
    // serving: one coalesced search batch (query rows, per-row k and nprobe,
    // results at stride max_k, one segment per request)
    L.srv_q = take((size_t)c->max_queries * c->dim * 4);
    L.srv_k = take((size_t)c->max_queries * 4);
    L.srv_np = take((size_t)c->max_queries * 4);
    L.srv_dist = take((size_t)c->max_queries * c->max_k * 4);
    L.srv_lab = take((size_t)c->max_queries * c->max_k * 8);
    L.srv_seg = take((size_t)c->max_queries * sizeof(SrvSeg));
    // lazy deletes: one validity bit per slot, ceil(C / 64) words per slab
    L.bits = take(c->delete_mode == SIVF_DELETE_LAZY ? (size_t)ns * ((C + 63) / 64) * 8 : 0);
    L.total = cur;
    return L;
}

bool dev_ok(hipError_t e) { return e == hipSuccess; }

}  // namespace

// Event pairs recorded around one class of work while profiling is on.
struct ProfClass {
    std::vector<hipEvent_t> start, stop;
    std::vector<char> more;   // the interval continues the previous one's call (not counted again)
    size_t used = 0;
    double ms = 0.0;
    int64_t count = 0;
};

struct sivf_index {
    int device = 0;          // the device current at creation (the workspace's)
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
    // schedule of the k > 64 pass of a certified-scan search (tile, chunk shift, persistent): by
    // default the certified scan with 128-key lists
    int deep_tile = 16, deep_shift = 14, deep_pers = 1;
    // host tier (slabs == 0: none): V views the cold pool; its rows and ids sit in
    // caller-provided pinned host memory, the rest in a caller-provided device buffer
    struct {
        int64_t slabs = 0;
        Dev V{};
        int32_t *heat = nullptr;     // per-list probe counts (searches add theirs)
        uint64_t *prior = nullptr;   // [max_queries][kcap] keys of a search's cold pass
        int32_t *olist = nullptr;    // [nlist] lists of an offload
        int64_t *nout = nullptr;     // positions released by a reclaim
        int64_t positions = 0;       // cold positions held (0: searches skip the cold pass)
    } tier;
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
        if (!c.more[i]) c.count++;
    }
    c.used = 0;
    return true;
}

// Returns the slot of an interval whose start was recorded, or -1.
int prof_begin(sivf_index *ix, int kind, hipStream_t st, bool more = false) {
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
        c.more.push_back(0);
    }
    if (!dev_ok(hipEventRecord(c.start[c.used], st))) return -1;
    c.more[c.used] = more ? 1 : 0;
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
    // inserts are assigned on bf16 MFMA (every storage): the nearest list is almost always separated
    // from the rest by more than the certified bound, and then needs no FP64 re-check; probes stay on
    // FP32 MFMA: a probe batch is small, and the 64 times tighter bound leaves the exact re-check of
    // nprobe lists few candidates
    const int bf = m == 1 && !m_per_row && mmax == 1;
    // the nearest-list path keeps one or two words per group of 16 lists: 8 or 16 times the rows fit
    const bool assign = m == 1 && !m_per_row && mmax == 1;
    const int64_t chunk = assign ? (int64_t)ix->L.coarse_rows * S.nlist /
                                       ((int64_t)coarse_assign_words(S.nlist, dpad) * coarse_groups(S.nlist))
                                 : ix->L.coarse_rows;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int nr = (int)((n - r0) < chunk ? (n - r0) : chunk);
        const float *xr = x + r0 * S.d;
        if (assign) {
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
    if (!fresh_only) {   // delete half of an upsert
        if (S.bits) launch_remove_lazy(st, S, nn, ids, nullptr, 1);
        else launch_remove(st, S, nn, ids, nullptr, ix->B, 1);
    }
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
    if (ix->S.bits) launch_remove_lazy(st, ix->S, (int)n, ids, n_removed, 0);
    else launch_remove(st, ix->S, (int)n, ids, n_removed, ix->B, 0);
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
    if (c.storage != SIVF_F32) {
        const KClass all = kclass_all(stride);
        launch_search_plan(st, ix->S, ix->W, (int)nq, all, 1);   // records the list lengths it will scan
        if (snapshot_taken && !dev_ok(hipEventRecord(snapshot_taken, st))) return SIVF_ERR_DEVICE;
        const int pk = prof_begin(ix, SIVF_PROF_SCAN, st);
        launch_search_scan_mfma(st, ix->S, ix->W, (int)nq, q, stride, ix->L.kcap, k, c.rerank_factor, kpq);
        prof_end(ix, SIVF_PROF_SCAN, pk, st);
        // approximate candidates, then the exact fp32 re-rank of R * k per query
        const int pm = prof_begin(ix, SIVF_PROF_MERGE, st);
        const int kc = c.rerank_factor * k;
        launch_search_merge(st, ix->S, ix->W, (int)nq, all, ix->L.kcap, kc, k, c.rerank_factor, kpq,
                            ix->W.rr_dist, ix->W.rr_lab);
        launch_rerank(st, ix->S, (int)nq, q, kc, ix->W.rr_lab, k, c.rerank_factor, kpq, dist, labels);
        prof_end(ix, SIVF_PROF_MERGE, pm, st);
        prof_end(ix, SIVF_PROF_SEARCH, ps, st);
        return launched(ix);
    }
    // fp32: partial lists as wide as the call's k needs.  On the certified
    // scan, queries with k > 64 form a pass of their own on the deep schedule
    // (its lists of 128 keys cost the certified scan more than the VALU scan
    // pays); the k <= 64 queries keep the certified scan with 64-key lists.
    const int kw = kcap_for(k);
    const bool split = ix->S.tile == 16 && kw > 64;
    Dev Sd = ix->S;
    Sd.tile = ix->deep_tile;
    Sd.chunk_shift = ix->deep_shift;
    Sd.persistent = ix->deep_pers;
    struct Pass {
        const Dev *S;
        KClass cls;
        int kw;
    } passes[2];
    int np = 0;
    if (!split) {
        passes[np++] = {&ix->S, kclass_all(stride), kw};
    } else {
        if (kpq) passes[np++] = {&ix->S, KClass{kpq, k, stride, -1, 64}, 64};
        passes[np++] = {&Sd, kpq ? KClass{kpq, k, stride, 64, 0x7FFFFFFF} : kclass_all(stride), 128};
    }
    // host tier first: the probed lists' cold segments, scanned in host memory
    // by the VALU scan; their sorted keys join each query's merge below
    const uint64_t *prior = nullptr;
    if (ix->tier.slabs > 0 && ix->tier.positions > 0) {
        Dev Sv = ix->tier.V;
        Sv.tile = ix->S.tile == 16 ? (c.dim <= 1024 ? 8 : 4) : ix->S.tile;
        Sv.chunk_shift = ix->S.chunk_shift;
        Sv.persistent = ix->S.persistent;
        const KClass all = kclass_all(stride);
        launch_search_plan(st, Sv, ix->W, (int)nq, all, 1);
        const int pk = prof_begin(ix, SIVF_PROF_SCAN_COLD, st);
        launch_search_scan(st, Sv, ix->W, (int)nq, q, stride, kw, k, kpq);
        prof_end(ix, SIVF_PROF_SCAN_COLD, pk, st);
        launch_search_merge(st, Sv, ix->W, (int)nq, all, kw, kw, k, 1, kpq, nullptr, nullptr, nullptr, 0,
                            ix->tier.prior);
        prior = ix->tier.prior;
    }
    for (int i = 0; i < np; i++) {
        const Pass &P = passes[i];
        launch_search_plan(st, *P.S, ix->W, (int)nq, P.cls, i == 0 ? 1 : 0, i == 0 ? ix->tier.heat : nullptr);
        if (i == 0 && snapshot_taken && !dev_ok(hipEventRecord(snapshot_taken, st))) return SIVF_ERR_DEVICE;
        const int sk = (split && P.S == &Sd) ? SIVF_PROF_SCAN_DEEP : SIVF_PROF_SCAN;
        const int pk = prof_begin(ix, sk, st);
        launch_search_scan(st, *P.S, ix->W, (int)nq, q, stride, P.kw, k, kpq);
        prof_end(ix, sk, pk, st);
        const int pm = prof_begin(ix, SIVF_PROF_MERGE, st, i > 0);
        launch_search_merge(st, *P.S, ix->W, (int)nq, P.cls, P.kw, k, k, 1, kpq, dist, labels, prior, kw);
        prof_end(ix, SIVF_PROF_MERGE, pm, st);
    }
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
    int device = 0;
    if (!dev_ok(hipGetDevice(&device))) return SIVF_ERR_DEVICE;
    sivf_index *ix = new (std::nothrow) sivf_index();
    if (!ix) return SIVF_ERR_STATE;
    ix->device = device;
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
    ix->W.gthr = (uint32_t *)(w + L.gthr);
    S.num_slabs = cfg->num_slabs;
    S.num_pages = L.num_pages;
    S.dir_cap = L.dir_cap;
    S.id_capacity = cfg->id_capacity;
    S.cent = (const float *)(w + L.cent);
    S.cent_h = (const uint16_t *)(w + L.cent_h);
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
    int32_t **lp[NLISTS] = {&S.l_acnt, &S.l_prem, &S.l_base, &S.l_eoff, &S.l_m, &S.l_off, &S.l_newlen, &S.l_q, &S.l_s,
                            &S.l_h, &S.l_qc, &S.l_qcs, &S.l_qoff, &S.l_snap, &S.l_pbase, &S.l_ioff, &S.l_dead};
    for (int i = 0; i < NLISTS; i++) *lp[i] = lists + (size_t)i * cfg->nlist;
    S.bw = (cfg->slab_capacity + 63) / 64;
    S.bits = cfg->delete_mode == SIVF_DELETE_LAZY ? (uint64_t *)(w + L.bits) : nullptr;
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

// Tile of a schedule the index admits: fp32 slabs take 4, 8 (dim <= 1024) or
// 16 (the certified scan, where it applies); reduced precision takes 16.
static bool tile_ok(const sivf_index *ix, int tile) {
    const bool reduced = ix->cfg.storage != SIVF_F32;
    const bool cert = tile == 16 && cert_ok(ix->cfg.storage, ix->cfg.dim, ix->cfg.slab_capacity, ix->L.kcap);
    return reduced ? tile == 16 : (tile == 4 || (tile == 8 && ix->cfg.dim <= 1024) || cert);
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
    sivf_status s = SIVF_OK;
    // device time of two searches after a warm-up one (negative on failure)
    auto timed = [&]() -> float {
        s = do_search(ix, nq, q, k, k_per_query, nprobe, nprobe_per_query, dist, labels, st);
        if (s != SIVF_OK) return -1.f;
        if (!dev_ok(hipEventRecord(e0, st))) s = SIVF_ERR_DEVICE;
        for (int r = 0; r < 2 && s == SIVF_OK; r++)
            s = do_search(ix, nq, q, k, k_per_query, nprobe, nprobe_per_query, dist, labels, st);
        float ms = 0.f;
        if (s == SIVF_OK && (!dev_ok(hipEventRecord(e1, st)) || !dev_ok(hipEventSynchronize(e1)) ||
                             !dev_ok(hipEventElapsedTime(&ms, e0, e1))))
            s = SIVF_ERR_DEVICE;
        return s == SIVF_OK ? ms : -1.f;
    };
    int bt = ix->S.tile, bs = ix->S.chunk_shift, bp = ix->S.persistent;
    float best = -1.f;
    for (int pm = 0; pm < 2 && s == SIVF_OK; pm++)
        for (int T : tiles)
            for (int sh = 10; sh <= 17 && s == SIVF_OK; sh++) {
                ix->S.tile = T;
                ix->S.chunk_shift = sh;
                ix->S.persistent = pm;
                const float ms = timed();
                if (ms >= 0.f && (best < 0.f || ms < best)) {
                    best = ms;
                    bt = T;
                    bs = sh;
                    bp = pm;
                }
            }
    ix->S.tile = bt;
    ix->S.chunk_shift = bs;
    ix->S.persistent = bp;
    // a certified-scan schedule runs queries with k > 64 as a pass of their own: tune its schedule too
    if (s == SIVF_OK && ix->cfg.storage == SIVF_F32 && bt == 16 && kcap_for(k) > 64) {
        int dt = ix->deep_tile, ds = ix->deep_shift, dp = ix->deep_pers;
        float dbest = -1.f;
        for (int pm = 0; pm < 2 && s == SIVF_OK; pm++)
            for (int T : tiles)
                for (int sh = 10; sh <= 17 && s == SIVF_OK; sh++) {
                    ix->deep_tile = T;
                    ix->deep_shift = sh;
                    ix->deep_pers = pm;
                    const float ms = timed();
                    if (ms >= 0.f && (dbest < 0.f || ms < dbest)) {
                        dbest = ms;
                        dt = T;
                        ds = sh;
                        dp = pm;
                    }
                }
        ix->deep_tile = dt;
        ix->deep_shift = ds;
        ix->deep_pers = dp;
    }
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
    if (!tile_ok(ix, tile)) return SIVF_ERR_ARG;
    if (chunk_shift < 6 || chunk_shift > 31 || (persistent != 0 && persistent != 1)) return SIVF_ERR_ARG;
    ix->S.tile = tile;
    ix->S.chunk_shift = chunk_shift;
    ix->S.persistent = persistent;
    return SIVF_OK;
}

sivf_status sivf_set_deep_schedule(sivf_index *ix, int32_t tile, int32_t chunk_shift, int32_t persistent) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->cfg.storage != SIVF_F32 || !tile_ok(ix, tile)) return SIVF_ERR_ARG;
    if (chunk_shift < 6 || chunk_shift > 31 || (persistent != 0 && persistent != 1)) return SIVF_ERR_ARG;
    ix->deep_tile = tile;
    ix->deep_shift = chunk_shift;
    ix->deep_pers = persistent;
    return SIVF_OK;
}

sivf_status sivf_get_search_schedule(const sivf_index *ix, int32_t *sched) {
    if (!ix || !sched) return SIVF_ERR_ARG;
    const int32_t v[6] = {ix->S.tile, ix->S.chunk_shift, ix->S.persistent, ix->deep_tile, ix->deep_shift,
                          ix->deep_pers};
    for (int i = 0; i < 6; i++) sched[i] = v[i];
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

sivf_status sivf_compact(sivf_index *ix, float min_dead_fraction, int64_t *n_compacted, void *stream) {
    if (!ix || !(min_dead_fraction >= 0.f && min_dead_fraction <= 1.f)) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    if (!ix->S.bits) {
        if (n_compacted) launch_fill_i64(st, n_compacted, 1, 0);
        return launched(ix);
    }
    launch_compact(st, ix->S, min_dead_fraction, ix->cfg.max_batch, n_compacted, ix->B);
    launch_call_end(st, ix->S);
    return launched(ix);
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

// ------------------------------------------- probe without workspace scratch
//
// For callers that cannot allocate device memory per call (code under graph
// capture, tight serving loops): the approximate-distance scratch of the
// probe lives in a fixed device array of this library, one copy per device,
// held until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)(16u << 20) / sizeof(float);   // 16 MiB
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[MAX_DEVICES] = {};

float *scratch_on(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        if (!dev_ok(hipGetDevice(&cur))) return nullptr;
        if (cur != device && !dev_ok(hipSetDevice(device))) return nullptr;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (!dev_ok(e) || !p) return nullptr;
        g_scratch_ptr[device] = (float *)p;
    }
    return g_scratch_ptr[device];
}
}  // namespace

sivf_status sivf_probe_noalloc(sivf_index *ix, int64_t nq, const float *q, int32_t nprobe, int32_t *probes,
                               void *stream) {
    if (!ix || nq < 0 || (nq > 0 && (!q || !probes))) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    if (nprobe < 1 || nprobe > ix->cfg.max_nprobe) return SIVF_ERR_ARG;
    const int m = nprobe < ix->cfg.nlist ? nprobe : ix->cfg.nlist;
    // nprobe 1 takes the nearest-list path: group minima, and second-minimum words where that path keeps them
    const int per_row = (m == 1 && nprobe == 1)
                            ? coarse_groups(ix->cfg.nlist) * coarse_assign_words(ix->cfg.nlist, ix->S.dp4 * 4)
                            : ix->cfg.nlist;
    if ((size_t)nq * (size_t)per_row > NOALLOC_SCRATCH_FLOATS) return SIVF_ERR_TOO_LARGE;
    const int64_t cap = ix->cfg.max_batch > ix->cfg.max_queries ? ix->cfg.max_batch : ix->cfg.max_queries;
    if (nq > cap) return SIVF_ERR_TOO_LARGE;
    float *sp = scratch_on(ix->device);
    if (!sp) return SIVF_ERR_DEVICE;
    ix->last = as_stream(stream);
    if (nq == 0) return SIVF_OK;
    coarse(ix, as_stream(stream), sp, q, nq, m, nullptr, nprobe, probes, nprobe, 0);
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

static sivf_status read_counts(sivf_index *ix, std::vector<int32_t> &len, int32_t *ctl,
                               std::vector<int32_t> *dead = nullptr) {
    len.resize(ix->cfg.nlist);
    if (!dev_ok(hipStreamSynchronize(ix->last))) return SIVF_ERR_DEVICE;
    if (!dev_ok(hipMemcpy(len.data(), ix->S.len, sizeof(int32_t) * len.size(), hipMemcpyDeviceToHost)))
        return SIVF_ERR_DEVICE;
    if (dead) {
        dead->assign(ix->cfg.nlist, 0);
        if (ix->S.bits &&
            !dev_ok(hipMemcpy(dead->data(), ix->S.l_dead, sizeof(int32_t) * dead->size(), hipMemcpyDeviceToHost)))
            return SIVF_ERR_DEVICE;
    }
    if (!dev_ok(hipMemcpy(ctl, ix->S.ctl, sizeof(int32_t) * CTL_WORDS, hipMemcpyDeviceToHost))) return SIVF_ERR_DEVICE;
    return SIVF_OK;
}

sivf_status sivf_dump_info_get(sivf_index *ix, sivf_dump_info *info) {
    if (!ix || !info) return SIVF_ERR_ARG;
    std::vector<int32_t> len, dead;
    int32_t ctl[CTL_WORDS];
    sivf_status s = read_counts(ix, len, ctl, &dead);
    if (s != SIVF_OK) return s;
    int64_t pos = 0, nd = 0, used = 0;
    const int C = ix->cfg.slab_capacity;
    for (int l = 0; l < ix->cfg.nlist; l++) {
        pos += len[l];
        nd += dead[l];
        used += (len[l] + C - 1) / C;
    }
    info->live = pos - nd;
    info->positions = pos;
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
    int64_t cold_live = 0;   // entries in the host tier count as live too
    if (ix->tier.slabs > 0 && (s = sivf_tier_stats(ix, &cold_live, nullptr, nullptr, nullptr)) != SIVF_OK) return s;
    if (live) *live = info.live + cold_live;
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
        std::vector<uint64_t> bits;
        if (ids_by_list) {
            sids.resize((size_t)c.num_slabs * C);
            if (!d2h(sids.data(), S.sids, sids.size() * 4)) return SIVF_ERR_DEVICE;
            if (S.bits) {
                bits.resize((size_t)c.num_slabs * S.bw);
                if (!d2h(bits.data(), S.bits, bits.size() * 8)) return SIVF_ERR_DEVICE;
            }
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
                        const bool dead = S.bits && !((bits[(size_t)slab * S.bw + (t >> 6)] >> (t & 63)) & 1ull);
                        ids_by_list[io++] = (v == INVALID || dead) ? -1 : (int64_t)v;
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

// ------------------------------------------------------------------ host tier

namespace {

// Byte layout of a host tier: rows and ids in host memory, bookkeeping on the device.
struct TierLayout {
    int64_t num_pages, dir_cap;
    size_t host_total, data, sids;
    size_t dev_total, bits, sowner, sord, free_slabs, free_pages, pages, dir, len, dead, heat, ctl, prior, olist, nout;
};

TierLayout tier_layout(const sivf_index *ix, int64_t hs) {
    TierLayout T{};
    const sivf_config &c = ix->cfg;
    const int64_t C = c.slab_capacity, nl = c.nlist;
    T.dir_cap = (hs + PAGE - 1) / PAGE + 1;
    T.num_pages = (hs + PAGE - 1) / PAGE + nl;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = cur;
        cur = align_up(cur + (bytes ? bytes : 1));
        return o;
    };
    T.data = take((size_t)hs * ix->L.dp4 * C * 16);
    T.sids = take((size_t)hs * C * 4);
    T.host_total = cur;
    cur = 0;
    T.bits = take((size_t)hs * ix->S.bw * 8);
    T.sowner = take((size_t)hs * 4);
    T.sord = take((size_t)hs * 4);
    T.free_slabs = take((size_t)hs * 4);
    T.free_pages = take((size_t)T.num_pages * 4);
    T.pages = take((size_t)T.num_pages * PAGE * 4);
    T.dir = take((size_t)nl * T.dir_cap * 4);
    T.len = take((size_t)nl * 4);
    T.dead = take((size_t)nl * 4);
    T.heat = take((size_t)nl * 4);
    T.ctl = take(CTL_WORDS * 4);
    T.prior = take((size_t)c.max_queries * ix->L.kcap * 8);
    T.olist = take((size_t)nl * 4);
    T.nout = take(8);
    T.dev_total = cur;
    return T;
}

// fp32 slabs with lazy deletes; cold positions fit the address table's 31 bits and all
// positions of both pools fit the int32 list offsets of a checkpoint
bool tier_cfg_ok(const sivf_index *ix, int64_t hs) {
    return ix->cfg.storage == SIVF_F32 && ix->S.bits && hs >= 1 &&
           (hs + ix->cfg.num_slabs) * (int64_t)ix->cfg.slab_capacity < (1ll << 31);
}

// Cold lengths, dead counts and the cold pool's free-slab count (waits).
sivf_status tier_counts(sivf_index *ix, std::vector<int32_t> &clen, std::vector<int32_t> &cdead, int32_t *cfree) {
    const Dev &V = ix->tier.V;
    clen.resize(ix->cfg.nlist);
    cdead.resize(ix->cfg.nlist);
    if (!dev_ok(hipStreamSynchronize(ix->last)) ||
        !dev_ok(hipMemcpy(clen.data(), V.len, clen.size() * 4, hipMemcpyDeviceToHost)) ||
        !dev_ok(hipMemcpy(cdead.data(), V.l_dead, cdead.size() * 4, hipMemcpyDeviceToHost)) ||
        (cfree && !dev_ok(hipMemcpy(cfree, V.ctl + CTL_SLAB_TOP, 4, hipMemcpyDeviceToHost))))
        return SIVF_ERR_DEVICE;
    int64_t pos = 0;
    for (int32_t v : clen) pos += v;
    ix->tier.positions = pos;
    return SIVF_OK;
}

}  // namespace

sivf_status sivf_tier_bytes(const sivf_index *ix, int64_t host_slabs, size_t *host_bytes, size_t *dev_bytes) {
    if (!ix || !tier_cfg_ok(ix, host_slabs)) return SIVF_ERR_ARG;
    const TierLayout T = tier_layout(ix, host_slabs);
    if (host_bytes) *host_bytes = T.host_total;
    if (dev_bytes) *dev_bytes = T.dev_total;
    return SIVF_OK;
}

sivf_status sivf_tier_attach(sivf_index *ix, int64_t host_slabs, void *host_buf, size_t host_bytes, void *dev_buf,
                             size_t dev_bytes, void *stream) {
    if (!ix || !host_buf || !dev_buf || !tier_cfg_ok(ix, host_slabs)) return SIVF_ERR_ARG;
    if (ix->broken || ix->tier.slabs > 0) return SIVF_ERR_STATE;
    const TierLayout T = tier_layout(ix, host_slabs);
    if (host_bytes < T.host_total || dev_bytes < T.dev_total || ((uintptr_t)host_buf % ALIGN) != 0 ||
        ((uintptr_t)dev_buf % ALIGN) != 0)
        return SIVF_ERR_ARG;
    // the host buffer must be pinned host memory the device reads and writes
    hipPointerAttribute_t a{};
    if (!dev_ok(hipPointerGetAttributes(&a, host_buf)) || a.type != hipMemoryTypeHost || !a.devicePointer)
        return SIVF_ERR_ARG;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    char *h = (char *)a.devicePointer, *w = (char *)dev_buf;
    Dev V = ix->S;   // geometry, scratch and centroids shared; pool arrays replaced
    V.num_slabs = host_slabs;
    V.num_pages = T.num_pages;
    V.dir_cap = T.dir_cap;
    V.data = (float4 *)(h + T.data);
    V.sids = (uint32_t *)(h + T.sids);
    V.hdata = nullptr;
    V.xnorm = nullptr;
    V.bits = (uint64_t *)(w + T.bits);
    V.sowner = (int32_t *)(w + T.sowner);
    V.sord = (int32_t *)(w + T.sord);
    V.free_slabs = (int32_t *)(w + T.free_slabs);
    V.free_pages = (int32_t *)(w + T.free_pages);
    V.pages = (int32_t *)(w + T.pages);
    V.dir = (int32_t *)(w + T.dir);
    V.len = (int32_t *)(w + T.len);
    V.l_dead = (int32_t *)(w + T.dead);
    V.ctl = (int32_t *)(w + T.ctl);
    V.cdata = nullptr;
    V.cbits = nullptr;
    V.csowner = nullptr;
    V.cdead = nullptr;
    // an empty cold pool: every slab and page free (the device pool's initial state)
    std::vector<int32_t> iota((size_t)(host_slabs > T.num_pages ? host_slabs : T.num_pages));
    for (size_t i = 0; i < iota.size(); i++) iota[i] = (int32_t)i;
    std::vector<int32_t> ctl(CTL_WORDS, 0);
    ctl[CTL_GATE] = -1;
    ctl[CTL_UPSERT] = -1;
    ctl[CTL_SLAB_TOP] = (int32_t)host_slabs;
    ctl[CTL_PAGE_TOP] = (int32_t)T.num_pages;
    const int nl = ix->cfg.nlist;
    if (!dev_ok(hipStreamSynchronize(st)) ||
        !dev_ok(hipMemcpy(V.free_slabs, iota.data(), (size_t)host_slabs * 4, hipMemcpyHostToDevice)) ||
        !dev_ok(hipMemcpy(V.free_pages, iota.data(), (size_t)T.num_pages * 4, hipMemcpyHostToDevice)) ||
        !dev_ok(hipMemcpy(V.ctl, ctl.data(), CTL_WORDS * 4, hipMemcpyHostToDevice)))
        return SIVF_ERR_DEVICE;
    launch_fill_i64(st, (int64_t *)V.bits, host_slabs * V.bw, 0);
    launch_fill_i32(st, V.sowner, host_slabs, -1);
    launch_fill_i32(st, V.sord, host_slabs, 0);
    launch_fill_i32(st, V.len, nl, 0);
    launch_fill_i32(st, V.l_dead, nl, 0);
    launch_fill_i32(st, (int32_t *)(w + T.heat), nl, 0);
    if (!dev_ok(hipGetLastError()) || !dev_ok(hipStreamSynchronize(st))) return SIVF_ERR_DEVICE;
    ix->tier.V = V;
    ix->tier.slabs = host_slabs;
    ix->tier.heat = (int32_t *)(w + T.heat);
    ix->tier.prior = (uint64_t *)(w + T.prior);
    ix->tier.olist = (int32_t *)(w + T.olist);
    ix->tier.nout = (int64_t *)(w + T.nout);
    ix->tier.positions = 0;
    ix->S.cdata = V.data;
    ix->S.cbits = V.bits;
    ix->S.csowner = V.sowner;
    ix->S.cdead = V.l_dead;
    return SIVF_OK;
}

sivf_status sivf_tier_offload(sivf_index *ix, int32_t n, const int32_t *lists, int64_t *moved, void *stream) {
    if (!ix || n < 0 || (n > 0 && !lists)) return SIVF_ERR_ARG;
    if (ix->broken || ix->tier.slabs == 0) return SIVF_ERR_STATE;
    const int nl = ix->cfg.nlist, C = ix->cfg.slab_capacity;
    std::vector<char> seen(nl, 0);
    for (int i = 0; i < n; i++) {
        if (lists[i] < 0 || lists[i] >= nl || seen[lists[i]]) return SIVF_ERR_ARG;
        seen[lists[i]] = 1;
    }
    ix->last = as_stream(stream);
    std::vector<int32_t> len, dead, clen, cdead;
    int32_t ctl[CTL_WORDS], cfree = 0;
    sivf_status s = read_counts(ix, len, ctl, &dead);
    if (s == SIVF_OK) s = tier_counts(ix, clen, cdead, &cfree);
    if (s != SIVF_OK) return s;
    if (ctl[CTL_GATE] == ctl[CTL_SEQ]) return SIVF_ERR_STATE;   // a failed call is still open
    std::vector<int32_t> ol;
    int64_t need = 0, pos = 0;
    int longest = 0;
    for (int i = 0; i < n; i++) {
        const int l = lists[i];
        if (len[l] == 0) continue;
        ol.push_back(l);
        need += (clen[l] + len[l] + C - 1) / C - (clen[l] + C - 1) / C;
        pos += len[l];
        longest = len[l] > longest ? len[l] : longest;
    }
    if (need > cfree) return SIVF_ERR_NOSPACE;   // nothing moved
    if (moved) *moved = pos;
    if (ol.empty()) return SIVF_OK;
    hipStream_t st = ix->last;
    if (!dev_ok(hipMemcpy(ix->tier.olist, ol.data(), ol.size() * 4, hipMemcpyHostToDevice))) return SIVF_ERR_DEVICE;
    launch_tier_offload(st, ix->S, ix->tier.V, ix->tier.olist, (int)ol.size(), longest);
    s = launched(ix);
    if (s != SIVF_OK) return s;
    return tier_counts(ix, clen, cdead, nullptr);
}

sivf_status sivf_tier_reclaim(sivf_index *ix, int64_t *released, void *stream) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->broken || ix->tier.slabs == 0) return SIVF_ERR_STATE;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    launch_tier_reclaim(st, ix->tier.V, ix->tier.nout);
    sivf_status s = launched(ix);
    if (s != SIVF_OK) return s;
    int64_t r = 0;
    if (!dev_ok(hipStreamSynchronize(st)) || !dev_ok(hipMemcpy(&r, ix->tier.nout, 8, hipMemcpyDeviceToHost)))
        return SIVF_ERR_DEVICE;
    if (released) *released = r;
    std::vector<int32_t> clen, cdead;
    return tier_counts(ix, clen, cdead, nullptr);
}

sivf_status sivf_tier_stats(sivf_index *ix, int64_t *cold_live, int64_t *cold_positions, int64_t *cold_used_slabs,
                            int64_t *cold_free_slabs) {
    if (!ix) return SIVF_ERR_ARG;
    int64_t live = 0, pos = 0, used = 0;
    int32_t cfree = 0;
    if (ix->tier.slabs > 0) {
        std::vector<int32_t> clen, cdead;
        sivf_status s = tier_counts(ix, clen, cdead, &cfree);
        if (s != SIVF_OK) return s;
        const int C = ix->cfg.slab_capacity;
        for (int l = 0; l < ix->cfg.nlist; l++) {
            pos += clen[l];
            live += clen[l] - cdead[l];
            used += (clen[l] + C - 1) / C;
        }
    }
    if (cold_live) *cold_live = live;
    if (cold_positions) *cold_positions = pos;
    if (cold_used_slabs) *cold_used_slabs = used;
    if (cold_free_slabs) *cold_free_slabs = cfree;
    return SIVF_OK;
}

sivf_status sivf_tier_dump(sivf_index *ix, int32_t *cold_len, int64_t *cold_ids_by_list) {
    if (!ix) return SIVF_ERR_ARG;
    if (ix->tier.slabs == 0) return SIVF_ERR_STATE;
    std::vector<int32_t> clen, cdead;
    sivf_status s = tier_counts(ix, clen, cdead, nullptr);
    if (s != SIVF_OK) return s;
    const Dev &V = ix->tier.V;
    const int C = ix->cfg.slab_capacity, nl = ix->cfg.nlist;
    if (cold_len) memcpy(cold_len, clen.data(), (size_t)nl * 4);
    if (!cold_ids_by_list) return SIVF_OK;
    std::vector<int32_t> dir((size_t)nl * V.dir_cap), pages((size_t)V.num_pages * PAGE);
    std::vector<uint64_t> bits((size_t)V.num_slabs * V.bw);
    std::vector<uint32_t> sids((size_t)V.num_slabs * C);
    if (!dev_ok(hipMemcpy(dir.data(), V.dir, dir.size() * 4, hipMemcpyDeviceToHost)) ||
        !dev_ok(hipMemcpy(pages.data(), V.pages, pages.size() * 4, hipMemcpyDeviceToHost)) ||
        !dev_ok(hipMemcpy(bits.data(), V.bits, bits.size() * 8, hipMemcpyDeviceToHost)) ||
        !dev_ok(hipMemcpy(sids.data(), V.sids, sids.size() * 4, hipMemcpyDeviceToHost)))
        return SIVF_ERR_DEVICE;
    int64_t io = 0;
    for (int l = 0; l < nl; l++)
        for (int p = 0; p < clen[l]; p++) {
            const int o = p / C, t = p % C;
            const int page = dir[(size_t)l * V.dir_cap + o / PAGE];
            if (page < 0 || page >= V.num_pages) return SIVF_ERR_STATE;
            const int slab = pages[(size_t)page * PAGE + o % PAGE];
            if (slab < 0 || slab >= V.num_slabs) return SIVF_ERR_STATE;
            const bool live = (bits[(size_t)slab * V.bw + (t >> 6)] >> (t & 63)) & 1ull;
            cold_ids_by_list[io++] = live ? (int64_t)sids[(size_t)slab * C + t] : -1;
        }
    return SIVF_OK;
}

sivf_status sivf_list_heat(sivf_index *ix, int32_t *heat, int halve) {
    if (!ix || !heat) return SIVF_ERR_ARG;
    if (ix->tier.slabs == 0) return SIVF_ERR_STATE;
    const int nl = ix->cfg.nlist;
    if (!dev_ok(hipStreamSynchronize(ix->last)) ||
        !dev_ok(hipMemcpy(heat, ix->tier.heat, (size_t)nl * 4, hipMemcpyDeviceToHost)))
        return SIVF_ERR_DEVICE;
    if (halve) {
        std::vector<int32_t> h(heat, heat + nl);
        for (int32_t &v : h) v >>= 1;
        if (!dev_ok(hipMemcpy(ix->tier.heat, h.data(), (size_t)nl * 4, hipMemcpyHostToDevice))) return SIVF_ERR_DEVICE;
    }
    return SIVF_OK;
}

sivf_status sivf_maintain(sivf_index *ix, float min_dead_fraction, int64_t min_free_slabs, int32_t max_offload,
                          sivf_maintain_report *rep, void *stream) {
    if (!ix || !(min_dead_fraction >= 0.f && min_dead_fraction <= 1.f) || min_free_slabs < 0 || max_offload < 0)
        return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    sivf_maintain_report r{};
    hipStream_t st = as_stream(stream);
    ix->last = st;
    const bool lazy = ix->S.bits != nullptr;
    // 1. compaction of dead slots, max_batch per call, while it makes progress
    if (lazy) {
        for (int it = 0; it < 1024; it++) {
            launch_compact(st, ix->S, min_dead_fraction, ix->cfg.max_batch, nullptr, ix->B);
            launch_call_end(st, ix->S);
            sivf_status s = launched(ix);
            if (s != SIVF_OK) return s;
            int32_t c = 0;   // the compaction plan leaves its count in the remove-total word
            if (!dev_ok(hipStreamSynchronize(st)) ||
                !dev_ok(hipMemcpy(&c, ix->S.ctl + CTL_RMTOT, 4, hipMemcpyDeviceToHost)))
                return SIVF_ERR_DEVICE;
            r.compacted += c;
            if (c == 0) break;
        }
    }
    if (ix->tier.slabs > 0) {
        // 2. cold segments with no live entry left
        sivf_status s = sivf_tier_reclaim(ix, &r.reclaimed, stream);
        if (s != SIVF_OK) return s;
        // 3. below the free-slab mark: offload the least probed lists, then halve the probe counts
        std::vector<int32_t> len, dead;
        int32_t ctl[CTL_WORDS];
        s = read_counts(ix, len, ctl, &dead);
        if (s != SIVF_OK) return s;
        int64_t free_slabs = ctl[CTL_SLAB_TOP];
        if (free_slabs < min_free_slabs && max_offload > 0) {
            const int nl = ix->cfg.nlist, C = ix->cfg.slab_capacity;
            std::vector<int32_t> heat(nl);
            s = sivf_list_heat(ix, heat.data(), 1);
            if (s != SIVF_OK) return s;
            std::vector<int32_t> order;
            for (int l = 0; l < nl; l++)
                if (len[l] > 0) order.push_back(l);
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return heat[a] < heat[b]; });
            std::vector<int32_t> pick;
            for (int l : order) {
                if (free_slabs >= min_free_slabs || (int)pick.size() >= max_offload) break;
                pick.push_back(l);
                free_slabs += (len[l] + C - 1) / C;
            }
            s = sivf_tier_offload(ix, (int32_t)pick.size(), pick.data(), &r.offloaded_positions, stream);
            if (s != SIVF_OK) return s;
            r.offloaded_lists = (int32_t)pick.size();
        }
    }
    if (rep) *rep = r;
    return SIVF_OK;
}

// ------------------------------------------------------------------ server

// Work in flight on one server stream: a mutation (one ticket) or a
// coalesced search batch (one ticket per request); it completes when `done`
// has been reached.
struct ServerReq {
    std::vector<int64_t> tickets;
    hipEvent_t done;
    int64_t reserve;     // slabs reserved by an insert until it completes
};

// A search request waiting for the next batch.
struct PendingSearch {
    int64_t ticket;
    SrvSeg seg;
    hipEvent_t inputs;   // recorded on the request's input stream at submission
};

constexpr int SRV_MAX_BATCHES = 2;   // search batches in flight before new searches are refused

struct sivf_server {
    sivf_index *ix = nullptr;
    hipStream_t s_search = nullptr, s_mut = nullptr;
    hipEvent_t last_mut = nullptr, last_snap = nullptr, last_search = nullptr, inputs = nullptr;
    bool any_mut = false, any_search = false;
    std::vector<hipEvent_t> pool;
    // Work in flight per stream, in submission order (it completes in that
    // order, so only the oldest entry of each queue needs a query).
    std::deque<ServerReq> q_search, q_mut;
    std::unordered_map<int64_t, hipEvent_t> inflight;   // ticket -> completion event (null while pending)
    std::vector<PendingSearch> pending;                  // the next search batch
    int64_t pending_rows = 0;
    SrvSeg *seg_host[2] = {nullptr, nullptr};            // pinned: segment tables, alternating
    hipEvent_t seg_used[2] = {nullptr, nullptr};         // the copy out of each table has been done
    int seg_next = 0;
    int64_t batches = 0, batched_requests = 0;
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

// Retire completed work: recycle events, release reservations, refresh the
// host view of free slabs from the last completed copy.
static void server_reap(sivf_server *s) {
    bool mut_done = false;
    for (std::deque<ServerReq> *q : {&s->q_search, &s->q_mut}) {
        while (!q->empty() && hipEventQuery(q->front().done) == hipSuccess) {
            const ServerReq &r = q->front();
            s->reserved -= r.reserve;
            mut_done |= (q == &s->q_mut);
            s->pool.push_back(r.done);
            for (int64_t t : r.tickets) s->inflight.erase(t);
            q->pop_front();
        }
    }
    if (mut_done) s->free_view = *(volatile int32_t *)s->mirror;
}

// The request's inputs come from work enqueued on input_stream: start after it.
static bool server_inputs(sivf_server *s, void *input_stream, hipStream_t st) {
    return dev_ok(hipEventRecord(s->inputs, as_stream(input_stream))) && dev_ok(hipStreamWaitEvent(st, s->inputs, 0));
}

static sivf_status server_finish(sivf_server *s, hipStream_t st, bool mutation, int64_t reserve,
                                 std::vector<int64_t> tickets) {
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
    for (int64_t t : tickets) s->inflight[t] = e;
    (mutation ? s->q_mut : s->q_search).push_back(ServerReq{std::move(tickets), e, reserve});
    s->reserved += reserve;
    return SIVF_OK;
}

// Launch the pending searches as one batch on the search stream: it starts
// after every request's inputs and after the last mutation (every pending
// search was submitted after it: a mutation flushes the pending batch before
// it is enqueued), so each request sees the state of its submission.
static sivf_status server_dispatch(sivf_server *s) {
    if (s->pending.empty()) return SIVF_OK;
    sivf_index *ix = s->ix;
    hipStream_t st = s->s_search;
    const int slot = s->seg_next;
    s->seg_next ^= 1;
    // the table in this pinned slot may still feed a copy two batches back
    if (!dev_ok(hipEventSynchronize(s->seg_used[slot]))) return SIVF_ERR_DEVICE;
    SrvSeg *tab = s->seg_host[slot];
    const int nseg = (int)s->pending.size();
    int kmax = 1;
    std::vector<int64_t> tickets;
    tickets.reserve(nseg);
    for (int i = 0; i < nseg; i++) {
        const PendingSearch &p = s->pending[i];
        tab[i] = p.seg;
        kmax = p.seg.k > kmax ? p.seg.k : kmax;
        tickets.push_back(p.ticket);
        if (!dev_ok(hipStreamWaitEvent(st, p.inputs, 0))) return SIVF_ERR_DEVICE;
    }
    const int nrows = (int)s->pending_rows;
    for (PendingSearch &p : s->pending) s->pool.push_back(p.inputs);
    s->pending.clear();
    s->pending_rows = 0;
    if (s->any_mut && !dev_ok(hipStreamWaitEvent(st, s->last_mut, 0))) return SIVF_ERR_DEVICE;
    const Layout &L = ix->L;
    char *w = ix->ws;
    SrvSeg *dseg = (SrvSeg *)(w + L.srv_seg);
    float *bq = (float *)(w + L.srv_q), *bdist = (float *)(w + L.srv_dist);
    int32_t *bk = (int32_t *)(w + L.srv_k), *bnp = (int32_t *)(w + L.srv_np);
    int64_t *blab = (int64_t *)(w + L.srv_lab);
    if (!dev_ok(hipMemcpyAsync(dseg, tab, sizeof(SrvSeg) * nseg, hipMemcpyHostToDevice, st))) return SIVF_ERR_DEVICE;
    if (!dev_ok(hipEventRecord(s->seg_used[slot], st))) return SIVF_ERR_DEVICE;
    launch_srv_gather(st, dseg, nseg, nrows, ix->cfg.dim, bq, bk, bnp);
    sivf_status r = do_search(ix, nrows, bq, kmax, bk, 0, bnp, bdist, blab, st, s->last_snap);
    if (r != SIVF_OK) return r;
    launch_srv_scatter(st, dseg, nseg, nrows, kmax, bdist, blab);
    if (!dev_ok(hipGetLastError())) return SIVF_ERR_DEVICE;
    if (!dev_ok(hipEventRecord(s->last_search, st))) return SIVF_ERR_DEVICE;
    s->any_search = true;
    s->batches++;
    s->batched_requests += nseg;
    return server_finish(s, st, false, 0, std::move(tickets));
}

// Dispatch the pending batch when no search batch is in flight.
static sivf_status server_pump(sivf_server *s) {
    server_reap(s);
    if (!s->pending.empty() && s->q_search.empty()) return server_dispatch(s);
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
    const size_t tab = sizeof(SrvSeg) * (size_t)ix->cfg.max_queries;
    bool ok = dev_ok(hipStreamCreateWithFlags(&s->s_search, hipStreamNonBlocking)) &&
              dev_ok(hipStreamCreateWithFlags(&s->s_mut, hipStreamNonBlocking)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_mut, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_snap, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->last_search, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->inputs, hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->seg_used[0], hipEventDisableTiming)) &&
              dev_ok(hipEventCreateWithFlags(&s->seg_used[1], hipEventDisableTiming)) &&
              dev_ok(hipHostMalloc((void **)&s->seg_host[0], tab, hipHostMallocDefault)) &&
              dev_ok(hipHostMalloc((void **)&s->seg_host[1], tab, hipHostMallocDefault)) &&
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
    sivf_status r = SIVF_OK;
    if (!s->pending.empty() && s->s_search) r = server_dispatch(s);
    if (s->s_search) (void)hipStreamSynchronize(s->s_search);
    if (s->s_mut) (void)hipStreamSynchronize(s->s_mut);
    for (auto &q : {&s->q_search, &s->q_mut})
        for (ServerReq &e : *q) (void)hipEventDestroy(e.done);
    for (PendingSearch &p : s->pending) (void)hipEventDestroy(p.inputs);
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : {s->last_mut, s->last_snap, s->last_search, s->inputs, s->seg_used[0], s->seg_used[1]})
        if (e) (void)hipEventDestroy(e);
    if (s->s_search) (void)hipStreamDestroy(s->s_search);
    if (s->s_mut) (void)hipStreamDestroy(s->s_mut);
    for (SrvSeg *t : s->seg_host)
        if (t) (void)hipHostFree(t);
    if (s->mirror) (void)hipHostFree(s->mirror);
    delete s;
    return r;
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
    sivf_status st = server_dispatch(s);   // earlier searches go first
    if (st != SIVF_OK) return st;
    if (s->any_search && !dev_ok(hipStreamWaitEvent(s->s_mut, s->last_snap, 0))) return SIVF_ERR_DEVICE;
    if (!server_inputs(s, input_stream, s->s_mut)) return SIVF_ERR_DEVICE;
    st = do_add(ix, n, x, ids, s->s_mut, true);
    if (st != SIVF_OK) return st;
    const int64_t t = s->next_ticket++;
    if (ticket) *ticket = t;
    return server_finish(s, s->s_mut, true, need, {t});
}

sivf_status sivf_server_remove(sivf_server *s, int64_t n, const int64_t *ids, int64_t *n_removed,
                               void *input_stream, int64_t *ticket) {
    if (!s) return SIVF_ERR_ARG;
    sivf_index *ix = s->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    if (n < 0 || n > ix->cfg.max_batch || (n > 0 && !ids)) return SIVF_ERR_ARG;
    server_reap(s);
    sivf_status st = server_dispatch(s);   // earlier searches go first
    if (st != SIVF_OK) return st;
    // a compacting delete moves entries that earlier searches may still read;
    // a lazy delete only clears validity bits and overlaps them
    if (!ix->S.bits && s->any_search && !dev_ok(hipStreamWaitEvent(s->s_mut, s->last_search, 0)))
        return SIVF_ERR_DEVICE;
    if (!server_inputs(s, input_stream, s->s_mut)) return SIVF_ERR_DEVICE;
    st = do_remove(ix, n, ids, n_removed, s->s_mut);
    if (st != SIVF_OK) return st;
    const int64_t t = s->next_ticket++;
    if (ticket) *ticket = t;
    return server_finish(s, s->s_mut, true, 0, {t});
}

sivf_status sivf_server_search(sivf_server *s, int64_t nq, const float *q, int32_t k, int32_t nprobe,
                               float *dist, int64_t *labels, void *input_stream, int64_t *ticket) {
    if (!s) return SIVF_ERR_ARG;
    sivf_index *ix = s->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    const sivf_config &c = ix->cfg;
    if (nq < 0 || nq > c.max_queries || k < 1 || k > c.max_k || nprobe < 1 || nprobe > c.max_nprobe)
        return SIVF_ERR_ARG;
    if (nq > 0 && (!q || !dist || !labels)) return SIVF_ERR_ARG;
    server_reap(s);
    if (s->pending_rows + nq > c.max_queries) {
        // the pending batch is full: it goes out now unless the search slots are taken
        if ((int)s->q_search.size() >= SRV_MAX_BATCHES) return SIVF_ERR_NOSPACE;
        sivf_status st = server_dispatch(s);
        if (st != SIVF_OK) return st;
    }
    const int64_t t = s->next_ticket++;
    if (ticket) *ticket = t;
    if (nq == 0) return SIVF_OK;   // nothing to do: complete at once
    hipEvent_t in = server_event(s);
    if (!in || !dev_ok(hipEventRecord(in, as_stream(input_stream)))) return SIVF_ERR_DEVICE;
    PendingSearch p;
    p.ticket = t;
    p.seg = SrvSeg{q, dist, labels, (int32_t)s->pending_rows, (int32_t)nq, k, nprobe};
    p.inputs = in;
    s->pending.push_back(p);
    s->pending_rows += nq;
    s->inflight[t] = nullptr;
    return server_pump(s);
}

sivf_status sivf_server_poll(sivf_server *s, int64_t ticket, int *done) {
    if (!s || !done) return SIVF_ERR_ARG;
    sivf_status st = server_pump(s);
    *done = (ticket > 0 && ticket < s->next_ticket && s->inflight.find(ticket) == s->inflight.end()) ? 1 : 0;
    return st;
}

sivf_status sivf_server_wait(sivf_server *s, int64_t ticket) {
    if (!s) return SIVF_ERR_ARG;
    auto it = s->inflight.find(ticket);
    if (it != s->inflight.end() && it->second == nullptr) {   // still pending: launch its batch now
        sivf_status st = server_dispatch(s);
        if (st != SIVF_OK) return st;
        it = s->inflight.find(ticket);
    }
    if (it != s->inflight.end() && !dev_ok(hipEventSynchronize(it->second))) return SIVF_ERR_DEVICE;
    return server_pump(s);
}

sivf_status sivf_server_free_slabs(sivf_server *s, int64_t *free_slabs, int64_t *reserved) {
    if (!s) return SIVF_ERR_ARG;
    server_reap(s);
    if (free_slabs) *free_slabs = s->free_view;
    if (reserved) *reserved = s->reserved;
    return SIVF_OK;
}

sivf_status sivf_server_batches(sivf_server *s, int64_t *batches, int64_t *requests) {
    if (!s) return SIVF_ERR_ARG;
    if (batches) *batches = s->batches;
    if (requests) *requests = s->batched_requests;
    return SIVF_OK;
}

// ------------------------------------------------------------------ checkpoint
//
// A checkpoint holds the logical content of the index: its configuration,
// the centroids, every list's length and, list after list in position order,
// each entry's id and exact fp32 row.  Reduced-precision copies and norms
// are derived data and are recomputed on load, and the slab layout is not
// kept: a checkpoint loads into any pool large enough (num_slabs, slab
// capacity, id and batch limits may change; dim, nlist, metric, storage and
// re-rank factor may not), and the loaded index has the same lists, so every
// search returns the same result as before the save.
//
// File layout (little-endian):
//   header  CkptHeader (magic, version, configuration, live count, record size)
//   float   centroids [nlist][dim]
//   int32   list lengths [nlist]
//   records of up to `record` entries: uint32 ids [m], then float rows [m][dim]

namespace {

struct CkptHeader {
    char magic[8];        // "SIVFCKP1"
    uint32_t version;     // 1
    uint32_t header_bytes;
    sivf_config cfg;
    int64_t live;
    int64_t record;       // entries per record
};

constexpr uint32_t CKPT_VERSION = 1;

bool write_all(FILE *f, const void *p, size_t bytes) { return bytes == 0 || fwrite(p, 1, bytes, f) == bytes; }
bool read_all(FILE *f, void *p, size_t bytes) { return bytes == 0 || fread(p, 1, bytes, f) == bytes; }

struct FileCloser {
    FILE *f;
    ~FileCloser() {
        if (f) fclose(f);
    }
};

// Entries per record: what fits in the staging area (the insert coarse
// scratch, idle between calls) and in one add batch.
int64_t stage_entries(const sivf_index *ix) {
    const int64_t bytes = (int64_t)ix->L.coarse_rows * ix->cfg.nlist * 4;
    int64_t m = bytes / (4 * (int64_t)ix->cfg.dim + 8);
    if (m > ix->cfg.max_batch) m = ix->cfg.max_batch;
    return m;
}

bool same_shape(const sivf_config &a, const sivf_config &b) {
    return a.dim == b.dim && a.nlist == b.nlist && a.metric == b.metric && a.storage == b.storage &&
           a.rerank_factor == b.rerank_factor;
}

}  // namespace

sivf_status sivf_save(sivf_index *ix, const char *path) {
    if (!ix || !path) return SIVF_ERR_ARG;
    if (ix->broken) return SIVF_ERR_STATE;
    std::vector<int32_t> len, dead;
    int32_t ctl[CTL_WORDS];
    sivf_status s = read_counts(ix, len, ctl, &dead);
    if (s != SIVF_OK) return s;
    const sivf_config &c = ix->cfg;
    // with a host tier each list's cold segment follows its device positions
    std::vector<int32_t> clen(c.nlist, 0), cdead(c.nlist, 0);
    if (ix->tier.slabs > 0 && (s = tier_counts(ix, clen, cdead, nullptr)) != SIVF_OK) return s;
    std::vector<int32_t> off(c.nlist), live_len(c.nlist);
    int64_t positions = 0, live = 0;
    for (int l = 0; l < c.nlist; l++) {
        off[l] = (int32_t)positions;
        positions += len[l] + clen[l];
        live_len[l] = len[l] - dead[l] + clen[l] - cdead[l];   // lazily deleted slots are not saved
        live += live_len[l];
    }
    FILE *f = fopen(path, "wb");
    if (!f) return SIVF_ERR_ARG;
    FileCloser fc{f};
    const int64_t rec = stage_entries(ix);
    if (rec < 1) return SIVF_ERR_STATE;
    CkptHeader h{};
    memcpy(h.magic, "SIVFCKP1", 8);
    h.version = CKPT_VERSION;
    h.header_bytes = sizeof(CkptHeader);
    h.cfg = c;
    h.live = live;
    h.record = rec;
    if (!write_all(f, &h, sizeof h)) return SIVF_ERR_ARG;
    const int dpad = ix->S.dp4 * 4;
    std::vector<float> cent((size_t)c.nlist * dpad);
    if (!dev_ok(hipMemcpy(cent.data(), ix->S.cent, cent.size() * 4, hipMemcpyDeviceToHost))) return SIVF_ERR_DEVICE;
    for (int l = 0; l < c.nlist; l++)
        if (!write_all(f, cent.data() + (size_t)l * dpad, (size_t)c.dim * 4)) return SIVF_ERR_ARG;
    if (!write_all(f, live_len.data(), (size_t)c.nlist * 4)) return SIVF_ERR_ARG;
    // list offsets into the (idle) per-list scratch of removes, rows and ids into the insert coarse scratch
    hipStream_t st = ix->last;
    if (!dev_ok(hipMemcpy(ix->S.l_off, off.data(), (size_t)c.nlist * 4, hipMemcpyHostToDevice))) return SIVF_ERR_DEVICE;
    float *rows_d = ix->dt;
    uint32_t *ids_d = (uint32_t *)(rows_d + (size_t)rec * c.dim);
    std::vector<float> rows((size_t)rec * c.dim), orows((size_t)rec * c.dim);
    std::vector<uint32_t> ids((size_t)rec), oids((size_t)rec);
    int64_t nout = 0, written = 0;   // live entries waiting in orows / oids, and those already written
    auto flush = [&](bool all) {
        while (nout == rec || (all && nout > 0)) {
            if (!write_all(f, oids.data(), (size_t)nout * 4) || !write_all(f, orows.data(), (size_t)nout * c.dim * 4))
                return false;
            written += nout;
            nout = 0;
        }
        return true;
    };
    for (int64_t e0 = 0; e0 < positions; e0 += rec) {
        const int n = (int)(positions - e0 < rec ? positions - e0 : rec);
        launch_pack(st, ix->S, ix->tier.slabs > 0 ? &ix->tier.V : nullptr, ix->S.l_off, e0, n, rows_d, ids_d);
        if (!dev_ok(hipGetLastError()) || !dev_ok(hipStreamSynchronize(st))) return SIVF_ERR_DEVICE;
        if (!dev_ok(hipMemcpy(ids.data(), ids_d, (size_t)n * 4, hipMemcpyDeviceToHost)) ||
            !dev_ok(hipMemcpy(rows.data(), rows_d, (size_t)n * c.dim * 4, hipMemcpyDeviceToHost)))
            return SIVF_ERR_DEVICE;
        for (int i = 0; i < n; i++) {
            if (ids[i] == INVALID) continue;   // a dead slot
            oids[nout] = ids[i];
            memcpy(orows.data() + (size_t)nout * c.dim, rows.data() + (size_t)i * c.dim, (size_t)c.dim * 4);
            nout++;
            if (!flush(false)) return SIVF_ERR_ARG;
        }
    }
    if (!flush(true) || written != live) return written != live ? SIVF_ERR_STATE : SIVF_ERR_ARG;
    if (fflush(f) != 0) return SIVF_ERR_ARG;
    return SIVF_OK;
}

sivf_status sivf_checkpoint_config(const char *path, sivf_config *cfg, int64_t *live) {
    if (!path || !cfg) return SIVF_ERR_ARG;
    FILE *f = fopen(path, "rb");
    if (!f) return SIVF_ERR_ARG;
    FileCloser fc{f};
    CkptHeader h{};
    if (!read_all(f, &h, sizeof h) || memcmp(h.magic, "SIVFCKP1", 8) != 0 || h.version != CKPT_VERSION ||
        h.header_bytes != sizeof(CkptHeader))
        return SIVF_ERR_ARG;
    *cfg = h.cfg;
    if (live) *live = h.live;
    return SIVF_OK;
}

sivf_status sivf_load(const char *path, const sivf_config *cfg, void *workspace, size_t ws_bytes, void *stream,
                      sivf_index **out) {
    if (!path || !cfg || !out) return SIVF_ERR_ARG;
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return SIVF_ERR_ARG;
    FileCloser fc{f};
    CkptHeader h{};
    if (!read_all(f, &h, sizeof h) || memcmp(h.magic, "SIVFCKP1", 8) != 0 || h.version != CKPT_VERSION ||
        h.header_bytes != sizeof(CkptHeader) || h.record < 1 || h.live < 0)
        return SIVF_ERR_ARG;
    if (!config_ok(cfg) || !same_shape(h.cfg, *cfg) || !workspace) return SIVF_ERR_ARG;
    const Layout L = make_layout(cfg);
    if (ws_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0) return SIVF_ERR_ARG;
    const int d = cfg->dim, nlist = cfg->nlist;
    hipStream_t st = as_stream(stream);
    // centroids go through the workspace's insert coarse scratch (not touched by creation)
    std::vector<float> cent((size_t)nlist * d);
    if (!read_all(f, cent.data(), cent.size() * 4)) return SIVF_ERR_ARG;
    float *cent_d = (float *)((char *)workspace + L.dt);
    if ((size_t)L.coarse_rows * nlist < cent.size()) return SIVF_ERR_STATE;
    if (!dev_ok(hipMemcpyAsync(cent_d, cent.data(), cent.size() * 4, hipMemcpyHostToDevice, st)))
        return SIVF_ERR_DEVICE;
    sivf_index *ix = nullptr;
    sivf_status s = sivf_create(cfg, cent_d, workspace, ws_bytes, stream, &ix);
    if (s != SIVF_OK) return s;
    if (!dev_ok(hipStreamSynchronize(st))) {
        sivf_destroy(ix);
        return SIVF_ERR_DEVICE;
    }
    std::vector<int32_t> len(nlist);
    if (!read_all(f, len.data(), (size_t)nlist * 4)) {
        sivf_destroy(ix);
        return SIVF_ERR_ARG;
    }
    int64_t live = 0;
    bool bad = false;
    for (int32_t v : len) {
        bad |= v < 0;
        live += v;
    }
    if (bad || live != h.live) {
        sivf_destroy(ix);
        return SIVF_ERR_ARG;
    }
    // Entries are inserted in file order with their saved lists (no coarse
    // step), staged through the insert coarse scratch.
    const int64_t m = stage_entries(ix);
    std::vector<uint32_t> ids((size_t)h.record);
    std::vector<int64_t> ids64((size_t)h.record);
    std::vector<float> rows((size_t)h.record * d);
    std::vector<int32_t> lists((size_t)h.record);
    float *rows_d = ix->dt;
    int64_t *ids_d = (int64_t *)(rows_d + (size_t)m * d);
    int lcur = 0;
    int64_t lleft = nlist > 0 ? len[0] : 0;
    for (int64_t e0 = 0; e0 < live && s == SIVF_OK; e0 += h.record) {
        const int64_t n = live - e0 < h.record ? live - e0 : h.record;
        if (!read_all(f, ids.data(), (size_t)n * 4) || !read_all(f, rows.data(), (size_t)n * d * 4)) {
            s = SIVF_ERR_ARG;
            break;
        }
        for (int64_t i = 0; i < n; i++) {
            while (lleft == 0) lleft = len[++lcur];
            lists[i] = lcur;
            lleft--;
            ids64[i] = ids[i];
        }
        for (int64_t p0 = 0; p0 < n && s == SIVF_OK; p0 += m) {
            const int nn = (int)(n - p0 < m ? n - p0 : m);
            if (!dev_ok(hipMemcpyAsync(rows_d, rows.data() + (size_t)p0 * d, (size_t)nn * d * 4, hipMemcpyHostToDevice,
                                       st)) ||
                !dev_ok(hipMemcpyAsync(ids_d, ids64.data() + p0, (size_t)nn * 8, hipMemcpyHostToDevice, st)) ||
                !dev_ok(hipMemcpyAsync(ix->B.assign, lists.data() + p0, (size_t)nn * 4, hipMemcpyHostToDevice, st))) {
                s = SIVF_ERR_DEVICE;
                break;
            }
            const Dev &S = ix->S;
            launch_add_prepare(st, S, nn, ids_d);
            launch_add_count(st, S, nn, ids_d, ix->B, 1);
            launch_add_admit(st, S);
            launch_add_alloc(st, S);
            launch_add_scatter(st, S, nn, rows_d, ids_d, ix->B);
            launch_add_cleanup(st, S, nn, ids_d);
            launch_call_end(st, S);
            sivf_status ds = SIVF_OK;
            if (!dev_ok(hipGetLastError())) s = SIVF_ERR_DEVICE;
            else if ((s = sivf_sync(ix, &ds)) == SIVF_OK && ds != SIVF_OK) s = ds;
        }
    }
    if (s != SIVF_OK) {
        sivf_destroy(ix);
        return s;
    }
    *out = ix;
    return SIVF_OK;
}

// ------------------------------------------------------------------ registry

struct sivf_registry {
    sivf_index *ix = nullptr;
    RegDev R{};
    int32_t *ctl = nullptr;
    int64_t *slot = nullptr;     // per batch row: table slot (-1 if none)
    int32_t *fresh = nullptr;    // per batch row: this row claimed a new slot
    int64_t *internal = nullptr; // per batch row: internal id (-1 if none)
    int64_t used_bound = 0;      // upper bound on used table slots (live keys + tombstones)
};

namespace {

struct RegLayout {
    int64_t cap;
    size_t keys, vals, ext_of, free_ids, ctl, slot, fresh, internal, total;
};

RegLayout reg_layout(const sivf_config &c) {
    RegLayout L{};
    int64_t cap = 1024;
    while (cap < 4 * c.id_capacity) cap <<= 1;
    L.cap = cap;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t o = cur;
        cur = align_up(cur + (bytes ? bytes : 1));
        return o;
    };
    L.keys = take((size_t)cap * 8);
    L.vals = take((size_t)cap * 4);
    L.ext_of = take((size_t)c.id_capacity * 8);
    L.free_ids = take((size_t)c.id_capacity * 4);
    L.ctl = take(REG_CTL_WORDS * 4);
    L.slot = take((size_t)c.max_batch * 8);
    L.fresh = take((size_t)c.max_batch * 4);
    L.internal = take((size_t)c.max_batch * 8);
    L.total = cur;
    return L;
}

// Rebuild the table from the reverse map when the used slots could pass half
// of the table (tombstones are never reused, so they accumulate).
void reg_maybe_rebuild(sivf_registry *r, hipStream_t st, int64_t n) {
    if (r->used_bound + n <= r->R.cap / 2) return;
    launch_reg_rebuild(st, r->R, r->ctl);
    r->used_bound = r->ix->cfg.id_capacity;   // live keys after the rebuild: at most one per internal id
}

}  // namespace

size_t sivf_registry_workspace_bytes(const sivf_index *ix) {
    if (!ix) return 0;
    return reg_layout(ix->cfg).total;
}

sivf_status sivf_registry_create(sivf_index *ix, void *workspace, size_t ws_bytes, void *stream,
                                 sivf_registry **out) {
    if (!ix || !workspace || !out) return SIVF_ERR_ARG;
    *out = nullptr;
    if (ix->broken) return SIVF_ERR_STATE;
    const RegLayout L = reg_layout(ix->cfg);
    if (ws_bytes < L.total || ((uintptr_t)workspace % ALIGN) != 0) return SIVF_ERR_ARG;
    sivf_registry *r = new (std::nothrow) sivf_registry();
    if (!r) return SIVF_ERR_STATE;
    char *w = (char *)workspace;
    r->ix = ix;
    r->R.keys = (int64_t *)(w + L.keys);
    r->R.vals = (int32_t *)(w + L.vals);
    r->R.ext_of = (int64_t *)(w + L.ext_of);
    r->R.free_ids = (int32_t *)(w + L.free_ids);
    r->R.cap = L.cap;
    r->R.id_cap = ix->cfg.id_capacity;
    r->ctl = (int32_t *)(w + L.ctl);
    r->slot = (int64_t *)(w + L.slot);
    r->fresh = (int32_t *)(w + L.fresh);
    r->internal = (int64_t *)(w + L.internal);
    hipStream_t st = as_stream(stream);
    ix->last = st;
    launch_fill_i32(st, r->ctl, REG_CTL_WORDS, 0);
    launch_fill_i64(st, r->R.ext_of, r->R.id_cap, REG_EMPTY);
    launch_reg_rebuild(st, r->R, r->ctl);          // an empty table
    launch_reg_free_stack(st, r->R, r->ctl);       // every internal id free
    if (!dev_ok(hipGetLastError())) {
        delete r;
        return SIVF_ERR_DEVICE;
    }
    *out = r;
    return SIVF_OK;
}

sivf_status sivf_registry_destroy(sivf_registry *r) {
    if (!r) return SIVF_ERR_ARG;
    delete r;
    return SIVF_OK;
}

sivf_status sivf_registry_add(sivf_registry *r, int64_t n, const float *x, const int64_t *ext_ids, void *stream) {
    if (!r) return SIVF_ERR_ARG;
    sivf_index *ix = r->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    if (n < 0 || n > ix->cfg.max_batch || (n > 0 && (!x || !ext_ids))) return SIVF_ERR_ARG;
    if (n == 0) return SIVF_OK;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    reg_maybe_rebuild(r, st, n);
    r->used_bound += n;
    launch_reg_add_pre(st, r->R, (int)n, ext_ids, r->slot, r->fresh, r->internal, r->ctl);
    if (!dev_ok(hipGetLastError())) return SIVF_ERR_DEVICE;
    sivf_status s = do_add(ix, n, x, r->internal, st);
    if (s != SIVF_OK) return s;
    launch_reg_add_post(st, r->R, ix->S, (int)n, r->slot, r->fresh, r->ctl);
    return launched(ix);
}

sivf_status sivf_registry_remove(sivf_registry *r, int64_t n, const int64_t *ext_ids, int64_t *n_removed,
                                 void *stream) {
    if (!r) return SIVF_ERR_ARG;
    sivf_index *ix = r->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    if (n < 0 || n > ix->cfg.max_batch || (n > 0 && !ext_ids)) return SIVF_ERR_ARG;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    if (n == 0) {
        if (n_removed) launch_fill_i64(st, n_removed, 1, 0);
        return launched(ix);
    }
    launch_reg_lookup(st, r->R, (int)n, ext_ids, r->slot, r->internal);
    // unmapped keys carry internal id -1, which the remove skips
    if (ix->S.bits) launch_remove_lazy(st, ix->S, (int)n, r->internal, n_removed, 2);
    else launch_remove(st, ix->S, (int)n, r->internal, n_removed, ix->B, 2);
    launch_call_end(st, ix->S);
    launch_reg_release(st, r->R, ix->S, (int)n, ext_ids, r->slot, r->ctl);
    return launched(ix);
}

sivf_status sivf_registry_search(sivf_registry *r, int64_t nq, const float *q, int32_t k, int32_t nprobe,
                                 float *dist, int64_t *labels, void *stream) {
    if (!r) return SIVF_ERR_ARG;
    sivf_index *ix = r->ix;
    if (ix->broken) return SIVF_ERR_STATE;
    hipStream_t st = as_stream(stream);
    ix->last = st;
    sivf_status s = do_search(ix, nq, q, k, nullptr, nprobe, nullptr, dist, labels, st);
    if (s != SIVF_OK || nq == 0) return s;
    launch_reg_labels(st, r->R, nq * k, labels);
    return launched(ix);
}

sivf_status sivf_registry_lookup(sivf_registry *r, int64_t n, const int64_t *ext_ids, int64_t *internal,
                                 void *stream) {
    if (!r || n < 0 || (n > 0 && (!ext_ids || !internal))) return SIVF_ERR_ARG;
    if (r->ix->broken) return SIVF_ERR_STATE;
    hipStream_t st = as_stream(stream);
    r->ix->last = st;
    if (n == 0) return SIVF_OK;
    launch_reg_lookup(st, r->R, (int)n, ext_ids, nullptr, internal);
    return launched(r->ix);
}

sivf_status sivf_registry_sync(sivf_registry *r, sivf_status *device_status) {
    if (!r) return SIVF_ERR_ARG;
    sivf_status ixs = SIVF_OK;
    sivf_status s = sivf_sync(r->ix, &ixs);
    if (s != SIVF_OK) return s;
    int32_t rs = 0, zero = 0;
    if (!dev_ok(hipMemcpy(&rs, r->ctl + REG_CTL_STATUS, 4, hipMemcpyDeviceToHost)) ||
        !dev_ok(hipMemcpy(r->ctl + REG_CTL_STATUS, &zero, 4, hipMemcpyHostToDevice)))
        return SIVF_ERR_DEVICE;
    if (device_status) *device_status = rs != 0 ? (sivf_status)rs : ixs;
    return SIVF_OK;
}

sivf_status sivf_registry_save(sivf_registry *r, const char *path) {
    if (!r || !path) return SIVF_ERR_ARG;
    if (!dev_ok(hipStreamSynchronize(r->ix->last))) return SIVF_ERR_DEVICE;
    std::vector<int64_t> ext((size_t)r->R.id_cap);
    if (!dev_ok(hipMemcpy(ext.data(), r->R.ext_of, ext.size() * 8, hipMemcpyDeviceToHost))) return SIVF_ERR_DEVICE;
    FILE *f = fopen(path, "wb");
    if (!f) return SIVF_ERR_ARG;
    FileCloser fc{f};
    const char magic[8] = {'S', 'I', 'V', 'F', 'R', 'E', 'G', '1'};
    const int64_t cap = r->R.id_cap;
    if (!write_all(f, magic, 8) || !write_all(f, &cap, 8) || !write_all(f, ext.data(), ext.size() * 8))
        return SIVF_ERR_ARG;
    return fflush(f) == 0 ? SIVF_OK : SIVF_ERR_ARG;
}

sivf_status sivf_registry_load(sivf_registry *r, const char *path, void *stream) {
    if (!r || !path) return SIVF_ERR_ARG;
    FILE *f = fopen(path, "rb");
    if (!f) return SIVF_ERR_ARG;
    FileCloser fc{f};
    char magic[8];
    int64_t cap = 0;
    if (!read_all(f, magic, 8) || memcmp(magic, "SIVFREG1", 8) != 0 || !read_all(f, &cap, 8) || cap < 1 ||
        cap > r->R.id_cap)
        return SIVF_ERR_ARG;
    std::vector<int64_t> ext((size_t)r->R.id_cap, REG_EMPTY);
    if (!read_all(f, ext.data(), (size_t)cap * 8)) return SIVF_ERR_ARG;
    hipStream_t st = as_stream(stream);
    r->ix->last = st;
    if (!dev_ok(hipMemcpyAsync(r->R.ext_of, ext.data(), ext.size() * 8, hipMemcpyHostToDevice, st)))
        return SIVF_ERR_DEVICE;
    launch_reg_rebuild(st, r->R, r->ctl);
    launch_reg_free_stack(st, r->R, r->ctl);
    r->used_bound = r->R.id_cap;
    if (!dev_ok(hipGetLastError()) || !dev_ok(hipStreamSynchronize(st))) return SIVF_ERR_DEVICE;
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
        case SIVF_ERR_TOO_LARGE: return "request larger than the fixed scratch of the no-allocation entry point";
    }
    return "unknown status";
}

}  // extern "C"
