/*
 * CPU reference oracle for the streaming IVF index (SIVF).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, sequential model of
 * what the GPU library computes.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the GPU library never links
 * or calls it, and the two share no code, headers or tables.
 *
 * The model is a *contiguous-array* inverted file: each list is a plain
 * dynamic array of (id, row) pairs, and an address table maps id -> (list,
 * position).  The paper claims its slab layout reaches exactly the same
 * result as a contiguous IVF (Sec. 5.3, "strict recall parity", and Sec. 5.8,
 * "zero recall loss"), so the contiguous form is the plain definition the GPU
 * path must match.
 *
 * Definitions written out here (the paper leaves precision, tie-breaks and
 * padding unstated; the readings taken are the ones listed in the design
 * notes of the repository):
 *   - coarse distance D(x,c): FP64, sequential fused multiply-add over the
 *     dimensions in ascending order; L2: sum (x_j - c_j)^2, IP: -(sum x_j c_j)
 *   - assignment l(x) = argmin_l D(x, c_l), ties -> smallest l  (the list
 *     assignment that Alg. 1 and Alg. 2 take as input)
 *   - probe set P(q) = first nprobe lists in (D(q,c_l), l) order (the probed
 *     list ids that Alg. 3 receives from the coarse quantizer)
 *   - fine distance (FP32 path): FP32, sequential fma over ascending
 *     dimensions; L2: t = q_j - x_j, r = fma(t,t,r); IP: r = fma(q_j,x_j,r)
 *   - result: first k live (dist, id) pairs of the probed lists, ordered by
 *     (dist asc, id asc) for L2 and (score desc, id asc) for IP; missing
 *     entries are id -1 with dist +inf (L2) or -inf (IP)   (Alg. 3)
 *   - mutation: operations applied one at a time in batch order; an add of a
 *     live id deletes it first ("delete-then-insert", Sec. 3, Data Model); a
 *     remove of an absent id is a no-op (idempotent delete, Alg. 4 and
 *     Theorem 3); removal swaps the list's last entry into the hole
 *   - space: a list of n entries occupies ceil(n / C) slabs of C slots
 *     (fixed-capacity slabs, Sec. 3.1); an add batch whose final state would
 *     need more slabs than the pool holds is rejected whole with NOSPACE and
 *     changes nothing (fail-fast on pool exhaustion, Sec. 3.2)
 *   - ids are dense in [0, id_capacity) (Sec. 3, Data Model); any id outside
 *     fails the whole call with ID_RANGE and changes nothing
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NOSPACE = -2, ORC_ERR_ID_RANGE = -3 };
enum { ORC_L2 = 0, ORC_IP = 1 };

/* ------------------------------------------------------------------ */
/* Distances                                                           */
/* ------------------------------------------------------------------ */

/* Coarse distance D(x, c) in FP64 (smaller is closer for both metrics). */
double orc_coarse_dist(const float *x, const float *c, int d, int metric)
{
    double r = 0.0;
    if (metric == ORC_L2) {
        for (int j = 0; j < d; j++) {
            double t = (double)x[j] - (double)c[j];
            r = fma(t, t, r);
        }
        return r;
    }
    for (int j = 0; j < d; j++)
        r = fma((double)x[j], (double)c[j], r);
    return -r;
}

/* Fine distance in FP32: squared L2 distance, or the inner product score. */
float orc_fine_dist(const float *q, const float *x, int d, int metric)
{
    float r = 0.0f;
    if (metric == ORC_L2) {
        for (int j = 0; j < d; j++) {
            float t = q[j] - x[j];
            r = fmaf(t, t, r);
        }
        return r;
    }
    for (int j = 0; j < d; j++)
        r = fmaf(q[j], x[j], r);
    return r;
}

/* ------------------------------------------------------------------ */
/* Coarse quantizer                                                    */
/* ------------------------------------------------------------------ */

/* Nearest centroid of each row; a tie keeps the smaller list id. */
void orc_assign(int64_t n, const float *x, int d, int nlist, const float *cent,
                int metric, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const float *xi = x + i * (int64_t)d;
        int best = 0;
        double bestd = orc_coarse_dist(xi, cent, d, metric);
        for (int l = 1; l < nlist; l++) {
            double dl = orc_coarse_dist(xi, cent + (int64_t)l * d, d, metric);
            if (dl < bestd) {
                bestd = dl;
                best = l;
            }
        }
        out[i] = best;
    }
}

typedef struct {
    double dist;
    int32_t list;
} coarse_pair;

static int cmp_coarse(const void *a, const void *b)
{
    const coarse_pair *u = (const coarse_pair *)a, *v = (const coarse_pair *)b;
    if (u->dist < v->dist) return -1;
    if (u->dist > v->dist) return 1;
    return (u->list > v->list) - (u->list < v->list);
}

/* The first m lists in (D, l) order, written in that order. */
static void probe_one(const float *q, int d, int nlist, const float *cent, int metric,
                      int m, int32_t *out, coarse_pair *tmp)
{
    for (int l = 0; l < nlist; l++) {
        tmp[l].dist = orc_coarse_dist(q, cent + (int64_t)l * d, d, metric);
        tmp[l].list = l;
    }
    qsort(tmp, (size_t)nlist, sizeof(coarse_pair), cmp_coarse);
    for (int p = 0; p < m; p++)
        out[p] = tmp[p].list;
}

/* Probe sets for nq queries; row i holds min(m, nlist) list ids, then -1. */
void orc_probe(int64_t nq, const float *q, int d, int nlist, const float *cent,
               int metric, int m, int32_t *out)
{
    int mm = m < nlist ? m : nlist;
#pragma omp parallel
    {
        coarse_pair *tmp = (coarse_pair *)malloc(sizeof(coarse_pair) * (size_t)nlist);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nq; i++) {
            int32_t *row = out + i * (int64_t)m;
            probe_one(q + i * (int64_t)d, d, nlist, cent, metric, mm, row, tmp);
            for (int p = mm; p < m; p++) row[p] = -1;
        }
        free(tmp);
    }
}

/* ------------------------------------------------------------------ */
/* Top-k bookkeeping: a sorted array of at most k (dist, id) entries    */
/* ------------------------------------------------------------------ */

/* Is (da, ia) ranked before (db, ib)?  L2: smaller distance first.  IP:
 * larger score first.  Equal values: smaller id first. */
static int ranks_before_f(float da, int64_t ia, float db, int64_t ib, int metric)
{
    if (metric == ORC_L2) {
        if (da < db) return 1;
        if (da > db) return 0;
    } else {
        if (da > db) return 1;
        if (da < db) return 0;
    }
    return ia < ib;
}

static int ranks_before_d(double da, int64_t ia, double db, int64_t ib, int metric)
{
    if (metric == ORC_L2) {
        if (da < db) return 1;
        if (da > db) return 0;
    } else {
        if (da > db) return 1;
        if (da < db) return 0;
    }
    return ia < ib;
}

static void topk_push_f(float *td, int64_t *ti, int *cnt, int k, float dv, int64_t iv, int metric)
{
    int n = *cnt;
    if (k <= 0) return;
    if (n == k && !ranks_before_f(dv, iv, td[n - 1], ti[n - 1], metric)) return;
    int p = n < k ? n : k - 1; /* slot that the new entry may take */
    while (p > 0 && ranks_before_f(dv, iv, td[p - 1], ti[p - 1], metric)) {
        td[p] = td[p - 1];
        ti[p] = ti[p - 1];
        p--;
    }
    td[p] = dv;
    ti[p] = iv;
    if (n < k) *cnt = n + 1;
}

static void topk_push_d(double *td, int64_t *ti, int *cnt, int k, double dv, int64_t iv, int metric)
{
    int n = *cnt;
    if (k <= 0) return;
    if (n == k && !ranks_before_d(dv, iv, td[n - 1], ti[n - 1], metric)) return;
    int p = n < k ? n : k - 1;
    while (p > 0 && ranks_before_d(dv, iv, td[p - 1], ti[p - 1], metric)) {
        td[p] = td[p - 1];
        ti[p] = ti[p - 1];
        p--;
    }
    td[p] = dv;
    ti[p] = iv;
    if (n < k) *cnt = n + 1;
}

/* ------------------------------------------------------------------ */
/* The contiguous-array inverted file                                  */
/* ------------------------------------------------------------------ */

typedef struct {
    int d, nlist, metric, C;
    int64_t num_slabs, id_capacity;
    float *cent;      /* nlist x d */
    int64_t *len;     /* entries per list */
    int64_t *cap;     /* allocated entries per list */
    int64_t **ids;    /* per list: ids */
    float **rows;     /* per list: rows, len x d */
    int32_t *att_list; /* id -> list, -1 when absent */
    int64_t *att_pos;  /* id -> position in its list */
} orc_index;

orc_index *orc_create(int d, int nlist, const float *cent, int metric, int C,
                      int64_t num_slabs, int64_t id_capacity)
{
    if (d <= 0 || nlist <= 0 || C <= 0 || num_slabs < 0 || id_capacity < 0) return NULL;
    if (metric != ORC_L2 && metric != ORC_IP) return NULL;
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    ix->d = d;
    ix->nlist = nlist;
    ix->metric = metric;
    ix->C = C;
    ix->num_slabs = num_slabs;
    ix->id_capacity = id_capacity;
    ix->cent = (float *)malloc(sizeof(float) * (size_t)nlist * (size_t)d);
    memcpy(ix->cent, cent, sizeof(float) * (size_t)nlist * (size_t)d);
    ix->len = (int64_t *)calloc((size_t)nlist, sizeof(int64_t));
    ix->cap = (int64_t *)calloc((size_t)nlist, sizeof(int64_t));
    ix->ids = (int64_t **)calloc((size_t)nlist, sizeof(int64_t *));
    ix->rows = (float **)calloc((size_t)nlist, sizeof(float *));
    ix->att_list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(id_capacity > 0 ? id_capacity : 1));
    ix->att_pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(id_capacity > 0 ? id_capacity : 1));
    for (int64_t u = 0; u < id_capacity; u++) {
        ix->att_list[u] = -1;
        ix->att_pos[u] = -1;
    }
    return ix;
}

void orc_destroy(orc_index *ix)
{
    if (!ix) return;
    for (int l = 0; l < ix->nlist; l++) {
        free(ix->ids[l]);
        free(ix->rows[l]);
    }
    free(ix->ids);
    free(ix->rows);
    free(ix->len);
    free(ix->cap);
    free(ix->cent);
    free(ix->att_list);
    free(ix->att_pos);
    free(ix);
}

static void list_append(orc_index *ix, int l, int64_t id, const float *row)
{
    int64_t n = ix->len[l];
    if (n == ix->cap[l]) {
        int64_t nc = ix->cap[l] ? 2 * ix->cap[l] : 16;
        ix->ids[l] = (int64_t *)realloc(ix->ids[l], sizeof(int64_t) * (size_t)nc);
        ix->rows[l] = (float *)realloc(ix->rows[l], sizeof(float) * (size_t)nc * (size_t)ix->d);
        ix->cap[l] = nc;
    }
    ix->ids[l][n] = id;
    memcpy(ix->rows[l] + n * ix->d, row, sizeof(float) * (size_t)ix->d);
    ix->len[l] = n + 1;
    ix->att_list[id] = l;
    ix->att_pos[id] = n;
}

/* Remove a live id: the list's last entry moves into the hole. */
static void list_swap_remove(orc_index *ix, int64_t id)
{
    int l = ix->att_list[id];
    int64_t pos = ix->att_pos[id];
    int64_t last = ix->len[l] - 1;
    if (pos != last) {
        int64_t moved = ix->ids[l][last];
        ix->ids[l][pos] = moved;
        memcpy(ix->rows[l] + pos * ix->d, ix->rows[l] + last * ix->d, sizeof(float) * (size_t)ix->d);
        ix->att_pos[moved] = pos;
    }
    ix->len[l] = last;
    ix->att_list[id] = -1;
    ix->att_pos[id] = -1;
}

static int64_t slabs_for(int64_t n, int C) { return (n + C - 1) / C; }

int64_t orc_used_slabs(const orc_index *ix)
{
    int64_t s = 0;
    for (int l = 0; l < ix->nlist; l++) s += slabs_for(ix->len[l], ix->C);
    return s;
}

int64_t orc_live(const orc_index *ix)
{
    int64_t s = 0;
    for (int l = 0; l < ix->nlist; l++) s += ix->len[l];
    return s;
}

int orc_add(orc_index *ix, int64_t n, const float *x, const int64_t *ids)
{
    if (n < 0) return ORC_ERR_ARG;
    for (int64_t i = 0; i < n; i++)
        if (ids[i] < 0 || ids[i] >= ix->id_capacity) return ORC_ERR_ID_RANGE;
    if (n == 0) return ORC_OK;

    int32_t *assign = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    orc_assign(n, x, ix->d, ix->nlist, ix->cent, ix->metric, assign);

    /* Dry run on the list lengths alone: apply the batch in order to a copy
     * of the lengths, then count the slabs the final state needs. */
    int64_t *len2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)ix->nlist);
    memcpy(len2, ix->len, sizeof(int64_t) * (size_t)ix->nlist);
    int32_t *saved = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        int64_t u = ids[i];
        saved[i] = ix->att_list[u];
        if (ix->att_list[u] >= 0) len2[ix->att_list[u]]--;
        len2[assign[i]]++;
        ix->att_list[u] = assign[i];
    }
    for (int64_t i = n - 1; i >= 0; i--) ix->att_list[ids[i]] = saved[i];
    int64_t need = 0;
    for (int l = 0; l < ix->nlist; l++) need += slabs_for(len2[l], ix->C);
    free(saved);
    free(len2);
    if (need > ix->num_slabs) {
        free(assign);
        return ORC_ERR_NOSPACE;
    }

    /* The real run, one operation at a time. */
    for (int64_t i = 0; i < n; i++) {
        int64_t u = ids[i];
        if (ix->att_list[u] >= 0) list_swap_remove(ix, u);
        list_append(ix, assign[i], u, x + i * (int64_t)ix->d);
    }
    free(assign);
    return ORC_OK;
}

int orc_remove(orc_index *ix, int64_t n, const int64_t *ids, int64_t *n_removed)
{
    if (n < 0) return ORC_ERR_ARG;
    for (int64_t i = 0; i < n; i++)
        if (ids[i] < 0 || ids[i] >= ix->id_capacity) return ORC_ERR_ID_RANGE;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; i++) {
        if (ix->att_list[ids[i]] >= 0) {
            list_swap_remove(ix, ids[i]);
            cnt++;
        }
    }
    if (n_removed) *n_removed = cnt;
    return ORC_OK;
}

/* Search.  k is the row stride of dist/labels; k_per_query (optional) gives
 * each query's own k <= k; nprobe_per_query (optional) each query's nprobe. */
int orc_search(const orc_index *ix, int64_t nq, const float *q, int k, const int32_t *k_per_query,
               int nprobe, const int32_t *nprobe_per_query, float *dist, int64_t *labels)
{
    if (nq < 0 || k < 0) return ORC_ERR_ARG;
    if (nprobe_per_query == NULL && nprobe <= 0) return ORC_ERR_ARG;
    for (int64_t i = 0; i < nq; i++) {
        if (k_per_query && (k_per_query[i] < 0 || k_per_query[i] > k)) return ORC_ERR_ARG;
        if (nprobe_per_query && nprobe_per_query[i] <= 0) return ORC_ERR_ARG;
    }
    const int d = ix->d, nlist = ix->nlist, metric = ix->metric;
    const float pad = metric == ORC_L2 ? INFINITY : -INFINITY;
#pragma omp parallel
    {
        coarse_pair *tmp = (coarse_pair *)malloc(sizeof(coarse_pair) * (size_t)nlist);
        int32_t *probes = (int32_t *)malloc(sizeof(int32_t) * (size_t)nlist);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < nq; i++) {
            const float *qi = q + i * (int64_t)d;
            int kq = k_per_query ? k_per_query[i] : k;
            int np = nprobe_per_query ? nprobe_per_query[i] : nprobe;
            if (np > nlist) np = nlist;
            float *td = dist + i * (int64_t)k;
            int64_t *ti = labels + i * (int64_t)k;
            int cnt = 0;
            probe_one(qi, d, nlist, ix->cent, metric, np, probes, tmp);
            for (int p = 0; p < np; p++) {
                int l = probes[p];
                for (int64_t e = 0; e < ix->len[l]; e++) {
                    float dv = orc_fine_dist(qi, ix->rows[l] + e * d, d, metric);
                    topk_push_f(td, ti, &cnt, kq, dv, ix->ids[l][e], metric);
                }
            }
            for (int j = cnt; j < k; j++) {
                td[j] = pad;
                ti[j] = -1;
            }
        }
        free(probes);
        free(tmp);
    }
    return ORC_OK;
}

/* Exact k nearest live entries by the FP64 coarse-distance definition, used
 * as recall ground truth.  dist holds the squared L2 distance (L2) or the
 * inner product (IP), as FP64. */
int orc_knn_live(const orc_index *ix, int64_t nq, const float *q, int k, double *dist, int64_t *labels)
{
    if (nq < 0 || k < 0) return ORC_ERR_ARG;
    const int d = ix->d, metric = ix->metric;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; i++) {
        const float *qi = q + i * (int64_t)d;
        double *td = dist + i * (int64_t)k;
        int64_t *ti = labels + i * (int64_t)k;
        int cnt = 0;
        for (int l = 0; l < ix->nlist; l++) {
            for (int64_t e = 0; e < ix->len[l]; e++) {
                double dv = orc_coarse_dist(qi, ix->rows[l] + e * d, d, metric);
                if (metric == ORC_IP) dv = -dv;
                topk_push_d(td, ti, &cnt, k, dv, ix->ids[l][e], metric);
            }
        }
        for (int j = cnt; j < k; j++) {
            td[j] = metric == ORC_L2 ? INFINITY : -INFINITY;
            ti[j] = -1;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* State inspection                                                    */
/* ------------------------------------------------------------------ */

void orc_list_len(const orc_index *ix, int64_t *out)
{
    for (int l = 0; l < ix->nlist; l++) out[l] = ix->len[l];
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    return (u > v) - (u < v);
}

/* Ids of every list, concatenated in list order, ascending within a list. */
void orc_ids_by_list(const orc_index *ix, int64_t *out)
{
    int64_t o = 0;
    for (int l = 0; l < ix->nlist; l++) {
        memcpy(out + o, ix->ids[l], sizeof(int64_t) * (size_t)ix->len[l]);
        qsort(out + o, (size_t)ix->len[l], sizeof(int64_t), cmp_i64);
        o += ix->len[l];
    }
}

/* List of a live id, or -1. */
int32_t orc_list_of(const orc_index *ix, int64_t id)
{
    if (id < 0 || id >= ix->id_capacity) return -1;
    return ix->att_list[id];
}

/* Copy of the stored row of a live id (returns 0), or -1 if absent. */
int orc_row_of(const orc_index *ix, int64_t id, float *out)
{
    if (id < 0 || id >= ix->id_capacity || ix->att_list[id] < 0) return -1;
    memcpy(out, ix->rows[ix->att_list[id]] + ix->att_pos[id] * ix->d, sizeof(float) * (size_t)ix->d);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
