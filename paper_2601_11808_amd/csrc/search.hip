// Search over the slab-resident lists (the paper's Sec. 3.3 / Alg. 3,
// re-designed for wave64 and query batches).
//
// The paper gives one warp to one query and walks each probed chain per
// query.  Here the (query, probed list) pairs of a whole batch are inverted
// to list-major work items: an item is one list and a tile of up to T queries
// that probe it.  One wave scans the list's slabs once per item (lane <->
// slot, 64 slots per step, coalesced 1 KiB loads), computing the canonical
// FP32 distance of every slot to all T queries of the tile, which sit in LDS.
// Each query keeps its best kcap (distance, id) keys sorted across the lanes
// of the wave; candidates below the current k-th key are inserted with
// ballots and lane shifts.  A final kernel merges the per-list partial
// results of each query.
//
//   k_inv_count   rank of each (query, probe) pair within its list (or
//                 k_inv_count_lds: block histograms, fewer global atomics)
//   k_inv_plan    per-list pair offsets; work items (list, tile)
//   k_inv_scatter pair ids grouped by list
//   k_scan        one wave per item: distances + per-query top-kcap
//   k_merge       one wave per query: kcap-way merge of its probe partials
#include "sivf_launch.h"

namespace sivf {

__device__ __forceinline__ int cdiv_s(int a, int b) { return (a + b - 1) / b; }

// Whether query qi belongs to the pass of class c.
__device__ __forceinline__ bool in_class(const KClass &c, int qi) {
    if (c.lo < 0 && c.hi == 0x7FFFFFFF) return true;
    int kq = c.kpq ? c.kpq[qi] : c.k;
    kq = kq < 0 ? 0 : (kq > c.k ? c.k : kq);
    return kq > c.lo && kq <= c.hi;
}

// List of pair p, or -1 when it probes nothing or its query is outside the pass.
__device__ __forceinline__ int pair_list(const int32_t *probes, int p, const KClass &c) {
    const int l = probes[p];
    return (l >= 0 && in_class(c, p / c.np_stride)) ? l : -1;
}

__global__ __launch_bounds__(256) void k_inv_count(Dev S, int npairs, const int32_t *__restrict__ probes,
                                                   int32_t *__restrict__ pair_rank, KClass cls) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool active = p < npairs;
    const int l = active ? pair_list(probes, p, cls) : -1;
    const bool act = l >= 0;
    const int r = act ? atomicAdd(&S.l_qc[l], 1) : 0;   // a wave's 64 pairs hit ~64 distinct lists
    if (active) pair_rank[p] = act ? r : -1;
}

// The same ranks with one device-scope atomic per (block, list) instead of
// one per pair: a block of 1024 threads takes INV_PB pairs, ranks them
// within the block by LDS atomics on a per-list histogram (nlist ints of
// dynamic LDS), reserves each list's block total with one atomic on l_qc,
// and adds that base.  Used when the histogram fits in 64 KiB.
constexpr int INV_PB = 8192;
__global__ __launch_bounds__(1024) void k_inv_count_lds(Dev S, int npairs, const int32_t *__restrict__ probes,
                                                        int32_t *__restrict__ pair_rank, KClass cls) {
    extern __shared__ int32_t hist[];
    const int tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * INV_PB;
    const int n = (int)min((int64_t)INV_PB, (int64_t)npairs - p0);
    for (int i = tid; i < S.nlist; i += 1024) hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += 1024) {
        const int l = pair_list(probes, (int)(p0 + i), cls);
        pair_rank[p0 + i] = l >= 0 ? atomicAdd(&hist[l], 1) : -1;
    }
    __syncthreads();
    for (int i = tid; i < S.nlist; i += 1024) {
        const int c = hist[i];
        if (c > 0) hist[i] = atomicAdd(&S.l_qc[i], c);
    }
    __syncthreads();
    for (int i = tid; i < n; i += 1024) {
        const int r = pair_rank[p0 + i];
        if (r >= 0) pair_rank[p0 + i] = r + hist[probes[p0 + i]];
    }
}

// Block sums of two int64 values (every thread gets both totals).
__device__ __forceinline__ void block_sum2(long long &a, long long &b, long long *sred) {
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane_id() == 0) {
        sred[w] = a;
        sred[16 + w] = b;
    }
    __syncthreads();
    a = 0;
    b = 0;
    for (int i = 0; i < nw; i++) {
        a += sred[i];
        b += sred[16 + i];
    }
}

__device__ __forceinline__ int list_chunks(int len, int sh) {
    return len > 0 ? (int)(((int64_t)len + (1ll << sh) - 1) >> sh) : 0;
}

// One block plans the whole search:
//  1. snapshot every list's length (the scan reads only these entries; a
//     second pass of the same search keeps the first pass's snapshot) and
//     lay out the (query, probe) pairs list by list;
//  2. split lists into chunks of 2^sh positions, with the smallest sh >= sh0
//     whose partial results (one per pair and chunk) and work items (one per
//     tile of T pairs and chunk) fit their buffers -- a long list is scanned
//     by many waves at once instead of one;
//  3. per-list offsets of partial slots and items; reset the work counters;
//  4. cut the items into 8 ranges, one per XCD, of equal scan cost (list
//     positions x query tiles) -- equal item counts leave XCDs idle while
//     others finish long lists -- each at most xcd_cap items (the blocks an
//     XCD receives in the dispatch schedule).
__global__ __launch_bounds__(1024) void k_inv_plan(Dev S, int T, int sh0, int64_t slot_cap, int64_t item_cap,
                                                   int xcd_cap, int snap, int32_t *__restrict__ heat) {
    __shared__ int sbuf[16];
    __shared__ long long sred[32];
    __shared__ long long scost[16];
    __shared__ int sxb[9];
    int carry_p = 0;
    for (int base = 0; base < S.nlist; base += 1024) {
        const int l = base + threadIdx.x;
        const bool valid = l < S.nlist;
        const int qc = valid ? S.l_qc[l] : 0;
        int tp;
        const int ep = block_excl_scan<1024>(qc, sbuf, &tp);
        if (valid) {
            if (snap) S.l_snap[l] = S.len[l];
            // probe count per list (host tier: the coldest lists are offloaded first), saturating
            if (heat && qc > 0) heat[l] = (int32_t)min((int64_t)heat[l] + qc, (int64_t)0x7FFFFFFF);
            S.l_qoff[l] = carry_p + ep;
            S.l_qcs[l] = qc;
            S.l_qc[l] = 0;
        }
        carry_p += tp;
    }
    // each thread re-reads only the lists it wrote above
    int sh = sh0;
    for (;;) {
        long long slots = 0, items = 0;
        for (int l = threadIdx.x; l < S.nlist; l += 1024) {
            const int qc = S.l_qcs[l];
            const int nc = qc > 0 ? list_chunks(S.l_snap[l], sh) : 0;
            slots += (long long)qc * nc;
            items += (long long)cdiv_s(qc, T) * nc;
        }
        block_sum2(slots, items, sred);
        if ((slots <= slot_cap && items <= item_cap) || sh >= 31) break;   // sh = 31: one chunk per list
        sh++;
    }
    // total scan cost first, so that each list can tell which XCD boundaries fall in it
    long long wsum = 0, wdummy = 0;
    for (int l = threadIdx.x; l < S.nlist; l += 1024) {
        const int qc = S.l_qcs[l];
        if (qc > 0) wsum += (long long)cdiv_s(qc, T) * S.l_snap[l];
    }
    block_sum2(wsum, wdummy, sred);
    if (threadIdx.x < 9) sxb[threadIdx.x] = -1;
    __syncthreads();
    int carry_s = 0, carry_i = 0;
    long long carry_w = 0;
    for (int base = 0; base < S.nlist; base += 1024) {
        const int l = base + threadIdx.x;
        const bool valid = l < S.nlist;
        const int qc = valid ? S.l_qcs[l] : 0;
        const int len = valid ? S.l_snap[l] : 0;
        const int nc = qc > 0 ? list_chunks(len, sh) : 0;
        const int ni = cdiv_s(qc, T) * nc;
        const long long wl = nc > 0 ? (long long)cdiv_s(qc, T) * len : 0;
        int ts, ti;
        long long tw;
        const int es = block_excl_scan<1024>(qc * nc, sbuf, &ts);
        const int ei = block_excl_scan<1024>(ni, sbuf, &ti);
        const long long ew = block_excl_scan64<1024>(wl, scost, &tw);
        if (valid) {
            S.l_pbase[l] = carry_s + es;
            S.l_ioff[l] = carry_i + ei;
            // XCD boundary x (1..7) at cost x * W / 8 falls in this list's [w0, w0 + wl)
            const long long w0 = carry_w + ew;
            for (int x = 1; x < 8 && wl > 0; x++) {
                const long long target = wsum * x / 8;
                if (target >= w0 && target < w0 + wl)
                    sxb[x] = carry_i + ei + (int)((double)(target - w0) / (double)wl * ni);
            }
        }
        carry_s += ts;
        carry_i += ti;
        carry_w += tw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n = carry_i;
        // boundaries not hit (zero-cost tail) follow the previous one; then cap every range
        int b = 0;
        S.ctl[CTL_XB] = 0;
        for (int x = 1; x < 8; x++) {
            int t = sxb[x] < 0 ? b : sxb[x];
            t = t < b ? b : t;
            t = t > b + xcd_cap ? b + xcd_cap : t;               // this range fits its XCD's blocks
            const int rest = n - (8 - x) * xcd_cap;               // the later ranges must fit too
            t = t < rest ? rest : t;
            t = t > n ? n : t;
            S.ctl[CTL_XB + x] = t;
            b = t;
        }
        S.ctl[CTL_XB + 8] = n;
        S.ctl[CTL_NITEMS] = n;
        S.ctl[CTL_CHUNK] = sh;
    }
    if (threadIdx.x < 8) S.ctl[CTL_WORK0 + CTL_WORK_STRIDE * threadIdx.x] = 0;
}

// Work items of each list, chunk-major (consecutive items read the same
// slabs for different query tiles).  One wave per list.
__global__ __launch_bounds__(256) void k_inv_items(Dev S, int T, int32_t *__restrict__ item_list,
                                                   int32_t *__restrict__ item_tile, int32_t *__restrict__ item_chunk) {
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6), lane = lane_id();
    if (l >= S.nlist) return;
    const int qc = S.l_qcs[l];
    if (qc == 0) return;
    const int nc = list_chunks(S.l_snap[l], S.ctl[CTL_CHUNK]);
    const int nt = cdiv_s(qc, T);
    const int base = S.l_ioff[l];
    for (int i = lane; i < nt * nc; i += 64) {
        item_list[base + i] = l;
        item_chunk[base + i] = i / nt;
        item_tile[base + i] = i % nt;
    }
}

__global__ __launch_bounds__(256) void k_inv_scatter(Dev S, int npairs, const int32_t *__restrict__ probes,
                                                     const int32_t *__restrict__ pair_rank,
                                                     int32_t *__restrict__ list_pairs) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npairs) return;
    const int r = pair_rank[p];
    if (r < 0) return;
    list_pairs[S.l_qoff[probes[p]] + r] = p;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const int lo = __shfl_xor((int)(uint32_t)v, m);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// ---------------------------------------------------------------- top-k
//
// Per query, the wave keeps its best keys sorted across the lanes (lane i
// holds the i-th best, lanes >= kcap hold ~0).  A key enters only if it beats
// the query's current k-th best (the threshold); such keys are appended to a
// 64-entry LDS buffer with one ballot.  When the buffer is full, and at the
// end of the list, the wave merges it into the sorted list: a bitonic sort of
// the buffer (descending), an element-wise min against the list (the 64
// smallest of both, as a bitonic sequence), and a bitonic merge.

// One compare-exchange step of a bitonic network over the 64 lanes: blocks
// of K lanes, partner distance J; `asc` is the direction of the final order.
template <int K, int J>
__device__ __forceinline__ uint64_t bitonic_step(uint64_t v, bool asc) {
    const int ln = lane_id();
    const uint64_t p = xor_lane_u64<J>(v);
    const bool up = ((ln & K) == 0) == asc;
    const bool keep_min = ((ln & J) == 0) == up;
    const uint64_t lo = p < v ? p : v, hi = p < v ? v : p;
    return keep_min ? lo : hi;
}

// Sort the wave's 64 keys across lanes, ascending or descending.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t v, bool asc) {
    v = bitonic_step<2, 1>(v, asc);
    v = bitonic_step<4, 2>(v, asc);
    v = bitonic_step<4, 1>(v, asc);
    v = bitonic_step<8, 4>(v, asc);
    v = bitonic_step<8, 2>(v, asc);
    v = bitonic_step<8, 1>(v, asc);
    v = bitonic_step<16, 8>(v, asc);
    v = bitonic_step<16, 4>(v, asc);
    v = bitonic_step<16, 2>(v, asc);
    v = bitonic_step<16, 1>(v, asc);
    v = bitonic_step<32, 16>(v, asc);
    v = bitonic_step<32, 8>(v, asc);
    v = bitonic_step<32, 4>(v, asc);
    v = bitonic_step<32, 2>(v, asc);
    v = bitonic_step<32, 1>(v, asc);
    v = bitonic_step<64, 32>(v, asc);
    v = bitonic_step<64, 16>(v, asc);
    v = bitonic_step<64, 8>(v, asc);
    v = bitonic_step<64, 4>(v, asc);
    v = bitonic_step<64, 2>(v, asc);
    v = bitonic_step<64, 1>(v, asc);
    return v;
}

// The 64 smallest keys of a (sorted ascending across lanes) and b (any
// order), sorted ascending: sort b descending; the element-wise min of a and
// b holds the 64 smallest as a bitonic sequence; half-cleaners sort it.
__device__ __forceinline__ uint64_t merge_sorted_with(uint64_t a, uint64_t b) {
    b = wave_sort64(b, false);
    uint64_t c = a < b ? a : b;
    c = bitonic_step<64, 32>(c, true);
    c = bitonic_step<64, 16>(c, true);
    c = bitonic_step<64, 8>(c, true);
    c = bitonic_step<64, 4>(c, true);
    c = bitonic_step<64, 2>(c, true);
    c = bitonic_step<64, 1>(c, true);
    return c;
}

// Half-cleaners: sort a bitonic sequence across the 64 lanes.
__device__ __forceinline__ uint64_t bitonic_clean(uint64_t v, bool asc) {
    v = bitonic_step<64, 32>(v, asc);
    v = bitonic_step<64, 16>(v, asc);
    v = bitonic_step<64, 8>(v, asc);
    v = bitonic_step<64, 4>(v, asc);
    v = bitonic_step<64, 2>(v, asc);
    v = bitonic_step<64, 1>(v, asc);
    return v;
}

// 128-key lists (k > 64): a holds ranks 0..63 and a2 ranks 64..127 (each
// sorted ascending across lanes).  Merge 64 unsorted keys b into them.  With
// b sorted descending, min(a, b) holds the 64 smallest of a and b and
// max(a, b) the rest; none of the former exceeds any key of a2, so the new
// ranks 64..127 are the 64 smallest of max(a, b) and a2.
__device__ __forceinline__ void merge128_with(uint64_t &a, uint64_t &a2, uint64_t b) {
    b = wave_sort64(b, false);
    const uint64_t lo = a < b ? a : b;
    const uint64_t hi = a < b ? b : a;
    a = bitonic_clean(lo, true);
    const uint64_t h = bitonic_clean(hi, false);
    a2 = bitonic_clean(a2 < h ? a2 : h, true);
}

// WIDE: kcap = 128 (two keys per lane).
template <int T, bool WIDE>
struct TopK {
    uint64_t top[T];              // sorted keys, per query (ranks 0..63)
    uint64_t top2[WIDE ? T : 1];  // ranks 64..127
    uint32_t thr[T];              // high word of the query's k-th best key (wave-uniform)
    int cnt[T];                   // keys waiting in the LDS buffer (wave-uniform)
};

// kq: LDS array with each query's k (0 = no results wanted).
template <int T, bool WIDE>
__device__ __forceinline__ void topk_init(TopK<T, WIDE> &K, const int *kq) {
#pragma unroll
    for (int t = 0; t < T; t++) {
        K.top[t] = ~0ull;
        if (WIDE) K.top2[t] = ~0ull;
        K.thr[t] = kq[t] > 0 ? 0xFFFFFFFFu : 0u;
        K.cnt[t] = 0;
    }
}

template <int T, bool WIDE>
__device__ __forceinline__ void topk_flush(TopK<T, WIDE> &K, int t, uint64_t *buf, const int *kq, int kcap) {
    __syncthreads();
    const int ln = lane_id();
    const uint64_t b = ln < K.cnt[t] ? buf[t * 64 + ln] : ~0ull;
    if (WIDE) {
        merge128_with(K.top[t], K.top2[t], b);
        K.top2[t] = ln + 64 < kcap ? K.top2[t] : ~0ull;
        const int r = kq[t] - 1;
        K.thr[t] = (uint32_t)((r < 64 ? readlane_u64(K.top[t], r) : readlane_u64(K.top2[t], r - 64)) >> 32);
    } else {
        uint64_t c = merge_sorted_with(K.top[t], b);
        c = ln < kcap ? c : ~0ull;
        K.top[t] = c;
        K.thr[t] = (uint32_t)(readlane_u64(c, kq[t] - 1) >> 32);
    }
    K.cnt[t] = 0;
    __syncthreads();
}

// Offer one candidate per lane to query t: hi is the high word of its key
// (ordered distance), id its low word.  Keys whose high word is at most the
// threshold's are buffered (a superset of those that beat the k-th key; the
// merge orders them exactly).
template <int T, bool WIDE>
__device__ __forceinline__ void topk_offer(TopK<T, WIDE> &K, int t, bool valid, uint32_t hi, uint32_t id,
                                           uint64_t *buf, const int *kq, int kcap) {
    bool pass = valid && hi <= K.thr[t];
    uint64_t mask = ballot(pass);
    if (mask) {
        int n = __builtin_popcountll(mask);
        if (K.cnt[t] + n > 64) {   // no room: merge first, then re-test against the new threshold
            topk_flush(K, t, buf, kq, kcap);
            pass = valid && hi <= K.thr[t];
            mask = ballot(pass);
            n = __builtin_popcountll(mask);
        }
        if (pass)
            buf[t * 64 + K.cnt[t] + (int)__builtin_popcountll(mask & lanemask_lt())] = ((uint64_t)hi << 32) | id;
        K.cnt[t] += n;
        if (K.cnt[t] == 64) topk_flush(K, t, buf, kq, kcap);
    }
}

// High word of a result key: L2 distances are never negative (the canonical
// sum starts at +0 and adds squares), so their order bits are bits | sign;
// an IP score of -0 ranks as +0.
template <int METRIC>
__device__ __forceinline__ uint32_t key_hi(float v) {
    return METRIC == 0 ? (__float_as_uint(v) | 0x80000000u) : ~ord_bits(zero_sign(v));
}

// Work items are cut into 8 contiguous ranges, one per XCD (blocks are
// dealt to the XCDs round robin): consecutive items share a list, so its
// slabs stay in that XCD's L2.  Two schedules (a template parameter: a loop
// around the scan body costs the hot loop scalar registers):
//  - dispatch (PERS = false): one wave per item; block b takes item b / 8
//    of XCD (b mod 8)'s range; the grid is the host's bound on the item
//    count rounded up to a multiple of 8, and the plan keeps every range
//    within grid / 8 items (surplus waves exit at once);
//  - persistent (PERS = true): a grid of resident waves pulls items from its
//    XCD's counter, then helps the other ranges; every wave ends once all 8
//    counters have passed their range.
#define SIVF_ITEM_LOOP_BEGIN                                                                     \
    for (int xs = 0; xs < (PERS ? 8 : 1); xs++) {                                                \
        const int xx = (int)((blockIdx.x + xs) & 7);                                             \
        const int lo = S.ctl[CTL_XB + xx], hi = S.ctl[CTL_XB + xx + 1];                          \
        for (int it = 0; PERS || it < 1; it++) {                                                 \
            int item;                                                                            \
            if (PERS) {                                                                          \
                item = 0;                                                                        \
                if (threadIdx.x == 0) item = atomicAdd(&S.ctl[CTL_WORK0 + CTL_WORK_STRIDE * xx], 1); \
                item = __builtin_amdgcn_readfirstlane(item) + lo; /* uniform: scalar addressing */ \
            } else {                                                                             \
                item = lo + (int)(blockIdx.x >> 3);                                              \
            }                                                                                    \
            if (item >= hi) break;
#define SIVF_ITEM_LOOP_END \
        }                  \
    }

// Decode a work item: list l, query tile, chunk of positions [p0, p1).
#define SIVF_ITEM_DECODE(TT)                                                                     \
    const int l = item_list[item], tile = item_tile[item];                                       \
    const int nt = min(TT, S.l_qcs[l] - tile * TT);                                              \
    const int len = S.l_snap[l];                                                                 \
    const int p0 = (int)((int64_t)item_chunk[item] << sh);                                       \
    const int p1 = (int)min((int64_t)len, (int64_t)p0 + (1ll << sh));                            \
    const int32_t *pairs = list_pairs + S.l_qoff[l] + tile * TT;

// Partial slot of query t of the item's tile: slot0 + t * nc.  Computed after
// the scan (re-reading the item) so that none of it holds a scalar register
// across the distance loop.
#define SIVF_ITEM_SLOT(TT)                                                                       \
    const int nc = list_chunks(len, S.ctl[CTL_CHUNK]);                                           \
    const int64_t slot0 = (int64_t)S.l_pbase[l] + (int64_t)tile * TT * nc + item_chunk[item];

// Distances of 64 consecutive list positions (lane <-> slot) to the T queries
// of a tile, in the canonical order (dimensions ascending, one fma each), then
// offered to each query's top-k.  QV(t, c) gives query t's dimension chunk c.
#define SIVF_SCAN_RANGE(QV)                                                                      \
    const int cs_ = __builtin_ctz(C), cm_ = C - 1; /* slab capacities are powers of two */       \
    const int nslab = (len + cm_) >> cs_;                                                        \
    int wbase = -(1 << 30), wslab = 0; /* lane j holds the slab of ordinal wbase + j */          \
    for (int base = p0; base < p1; base += 64) {                                                 \
        const int p = base + lane;                                                               \
        const bool valid = p < p1;                                                               \
        const int pc = valid ? p : p1 - 1;                                                       \
        const int last_ord = min(base + 63, p1 - 1) >> cs_;                                      \
        if (last_ord >= wbase + 64) {                                                            \
            wbase = base >> cs_;                                                                 \
            wslab = (wbase + lane < nslab) ? slab_of(S, l, wbase + lane) : 0;                    \
        }                                                                                        \
        const int slab = __shfl(wslab, (pc >> cs_) - wbase);                                     \
        const int slot = pc & cm_;                                                               \
        /* lazy deletes: a slot whose validity bit is clear holds no entry */                    \
        const bool live_ = valid && (!S.bits || ((valid_word(S, slab, slot) >> (slot & 63)) & 1ull)); \
        const float4 *xp = S.data + (int64_t)slab * dp4 * C + slot;                              \
        float acc[T];                                                                            \
        _Pragma("unroll") for (int t = 0; t < T; t++) acc[t] = 0.f;                              \
        _Pragma("unroll 2") for (int c = 0; c < dp4; c++) {                                      \
            const float4 xv = xp[(int64_t)c * C];                                                \
            _Pragma("unroll") for (int t = 0; t < T; t++) {                                      \
                const float4 qv = QV(t, c);                                                      \
                if (METRIC == 0) {                                                               \
                    float e;                                                                     \
                    e = qv.x - xv.x;                                                             \
                    acc[t] = __builtin_fmaf(e, e, acc[t]);                                       \
                    e = qv.y - xv.y;                                                             \
                    acc[t] = __builtin_fmaf(e, e, acc[t]);                                       \
                    e = qv.z - xv.z;                                                             \
                    acc[t] = __builtin_fmaf(e, e, acc[t]);                                       \
                    e = qv.w - xv.w;                                                             \
                    acc[t] = __builtin_fmaf(e, e, acc[t]);                                       \
                } else {                                                                         \
                    acc[t] = __builtin_fmaf(qv.x, xv.x, acc[t]);                                 \
                    acc[t] = __builtin_fmaf(qv.y, xv.y, acc[t]);                                 \
                    acc[t] = __builtin_fmaf(qv.z, xv.z, acc[t]);                                 \
                    acc[t] = __builtin_fmaf(qv.w, xv.w, acc[t]);                                 \
                }                                                                                \
            }                                                                                    \
        }                                                                                        \
        const uint32_t id = S.sids[(int64_t)slab * C + slot];                                    \
        _Pragma("unroll") for (int t = 0; t < T; t++) {                                          \
            if (t < nt) topk_offer(K, t, live_, key_hi<METRIC>(acc[t]), id, buf, skq, kcap);     \
        }                                                                                        \
    }                                                                                            \
    SIVF_ITEM_SLOT(T)                                                                            \
    _Pragma("unroll") for (int t = 0; t < T; t++) {                                              \
        if (t < nt) {                                                                            \
            if (K.cnt[t] > 0) topk_flush(K, t, buf, skq, kcap);                                  \
            uint64_t *dst = partials + (slot0 + (int64_t)t * nc) * kcap;                         \
            if (lane < kcap) dst[lane] = K.top[t];                                               \
            if (WIDE && lane + 64 < kcap) dst[64 + lane] = K.top2[WIDE ? t : 0];                 \
        }                                                                                        \
    }

__device__ __forceinline__ int query_k(const int32_t *kpq, int k, int qi) {
    int kq = kpq ? kpq[qi] : k;
    return kq < 0 ? 0 : (kq > k ? k : kq);
}

// Queries come straight from the caller's rows with wave-uniform addresses,
// so the compiler reads them through the scalar cache into SGPRs and every
// VALU op takes its query operand from an SGPR (no LDS traffic).  Needs
// d % 4 == 0 and 16-byte aligned rows.
template <int T, int METRIC, bool WIDE, bool PERS>
__global__ __launch_bounds__(64) void k_scan_sq(Dev S, const int32_t *__restrict__ item_list,
                                                const int32_t *__restrict__ item_tile,
                                                const int32_t *__restrict__ item_chunk,
                                                const int32_t *__restrict__ list_pairs,
                                                const float *__restrict__ q, int np_stride, int kcap, int k,
                                                const int32_t *__restrict__ kpq, uint64_t *__restrict__ partials) {
    __shared__ uint64_t buf[T * 64];
    __shared__ int skq[T];
    const int lane = threadIdx.x;
    const int dp4 = S.dp4, C = S.C, sh = S.ctl[CTL_CHUNK];
    SIVF_ITEM_LOOP_BEGIN
    SIVF_ITEM_DECODE(T)
    const float4 *qrow[T];
    TopK<T, WIDE> K;
#pragma unroll
    for (int t = 0; t < T; t++) {
        const int pr = pairs[t < nt ? t : 0];
        qrow[t] = reinterpret_cast<const float4 *>(q + (int64_t)(pr / np_stride) * S.d);
    }
    __syncthreads();
    if (lane < T) skq[lane] = lane < nt ? query_k(kpq, k, pairs[lane] / np_stride) : 0;
    __syncthreads();
    topk_init(K, skq);
#define SIVF_QV_SQ(t, c) qrow[t][c]
    SIVF_SCAN_RANGE(SIVF_QV_SQ)
#undef SIVF_QV_SQ
    SIVF_ITEM_LOOP_END
}

// General path: query rows of any alignment or dimension, staged in LDS.
template <int T, int METRIC, bool WIDE, bool PERS>
__global__ __launch_bounds__(64) void k_scan(Dev S, const int32_t *__restrict__ item_list,
                                             const int32_t *__restrict__ item_tile,
                                             const int32_t *__restrict__ item_chunk,
                                             const int32_t *__restrict__ list_pairs, const float *__restrict__ q,
                                             int np_stride, int kcap, int k, const int32_t *__restrict__ kpq,
                                             uint64_t *__restrict__ partials) {
    extern __shared__ float4 sq[];   // [T][dp4]
    __shared__ uint64_t buf[T * 64];
    __shared__ int skq[T];
    const int lane = threadIdx.x;
    const int dp4 = S.dp4, C = S.C, d = S.d, sh = S.ctl[CTL_CHUNK];
    SIVF_ITEM_LOOP_BEGIN
    SIVF_ITEM_DECODE(T)
    TopK<T, WIDE> K;
    __syncthreads();
    for (int t = 0; t < T; t++) {
        const int pr = t < nt ? pairs[t] : -1;
        const float *qr = q + (int64_t)(pr < 0 ? 0 : pr / np_stride) * d;
        for (int c = lane; c < dp4; c += 64) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pr >= 0) {
                const int j = 4 * c;
                v.x = j < d ? qr[j] : 0.f;
                v.y = j + 1 < d ? qr[j + 1] : 0.f;
                v.z = j + 2 < d ? qr[j + 2] : 0.f;
                v.w = j + 3 < d ? qr[j + 3] : 0.f;
            }
            sq[t * dp4 + c] = v;
        }
    }
    if (lane < T) skq[lane] = lane < nt ? query_k(kpq, k, pairs[lane] / np_stride) : 0;
    __syncthreads();
    topk_init(K, skq);
#define SIVF_QV_LDS(t, c) sq[(t) * dp4 + (c)]
    SIVF_SCAN_RANGE(SIVF_QV_LDS)
#undef SIVF_QV_LDS
    SIVF_ITEM_LOOP_END
}

#undef SIVF_SCAN_RANGE

// A pair whose list was split into chunks has one partial list per chunk:
// merge them into the first.  One thread per pair finds the split ones; the
// wave merges them one at a time.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_chunk_merge(Dev S, int npairs, const int32_t *__restrict__ probes,
                                                     const int32_t *__restrict__ pair_rank,
                                                     uint64_t *__restrict__ partials, int kcap) {
    const int p = blockIdx.x * 256 + threadIdx.x, lane = lane_id();
    const int sh = S.ctl[CTL_CHUNK];
    const int l = (p < npairs && pair_rank[p] >= 0) ? probes[p] : -1;   // pairs of this pass only
    const int nc = l >= 0 ? list_chunks(S.l_snap[l], sh) : 0;
    const int64_t slot = nc > 1 ? (int64_t)S.l_pbase[l] + (int64_t)pair_rank[p] * nc : 0;
    uint64_t mask = ballot(nc > 1);
    while (mask) {
        const int src = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int m = __shfl(nc, src);
        const int64_t s0 = ((int64_t)__shfl((int)(slot >> 32), src) << 32) | (uint32_t)__shfl((int)slot, src);
        uint64_t *dst = partials + s0 * kcap;
        uint64_t a = lane < kcap ? dst[lane] : ~0ull;
        uint64_t a2 = (WIDE && lane + 64 < kcap) ? dst[64 + lane] : ~0ull;
        for (int c = 1; c < m; c++) {
            const uint64_t *src_c = dst + (int64_t)c * kcap;
            const uint64_t b0 = lane < kcap ? src_c[lane] : ~0ull;
            if (WIDE) {
                merge128_with(a, a2, b0);
                const uint64_t b1 = lane + 64 < kcap ? src_c[64 + lane] : ~0ull;
                merge128_with(a, a2, b1);
            } else {
                a = merge_sorted_with(a, b0);
            }
        }
        if (lane < kcap) dst[lane] = a;
        if (WIDE && lane + 64 < kcap) dst[64 + lane] = a2;
    }
}

// One wave per query: repeatedly take the smallest head among the query's
// probe partial lists (each sorted, kcap long; a split list's chunks were
// merged into its first slot).  k: the call's k; each query keeps kmul * (its
// k) results, at most out_stride (the row stride of dist / labels, <= 128).
// prior (or NULL): one more sorted source per query, prior_stride keys (~0
// padded) -- the host tier's results; keys_out (or NULL): write the sorted
// keys there (stride out_stride, ~0 padded) instead of dist / labels.
__global__ __launch_bounds__(256) void k_merge(Dev S, int nq, int np_stride, const int32_t *__restrict__ probes,
                                               const int32_t *__restrict__ pair_rank,
                                               const uint64_t *__restrict__ partials, int kcap, int out_stride,
                                               int k, int kmul, const int32_t *__restrict__ kpq,
                                               float *__restrict__ dist, int64_t *__restrict__ labels, KClass cls,
                                               const uint64_t *__restrict__ prior, int prior_stride,
                                               uint64_t *__restrict__ keys_out) {
    __shared__ unsigned char heads[4][1024];
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int qi = blockIdx.x * 4 + w;
    if (qi >= nq || !in_class(cls, qi)) return;   // a query of another pass: its results come from that one
    const int sh = S.ctl[CTL_CHUNK];
    int kq = kpq ? kpq[qi] : k;
    kq = kq < 0 ? 0 : (kq > k ? k : kq);
    kq = min(kq * kmul, out_stride);
    const int32_t *prow = probes + (int64_t)qi * np_stride;
    const int32_t *rrow = pair_rank + (int64_t)qi * np_stride;
    auto head_key = [&](int p) -> uint64_t {
        const int l = prow[p];
        if (l < 0) return ~0ull;
        const int len = S.l_snap[l];
        if (len == 0) return ~0ull;
        const int h = heads[w][p];
        const int64_t slot = (int64_t)S.l_pbase[l] + (int64_t)rrow[p] * list_chunks(len, sh);
        return h < kcap ? partials[slot * kcap + h] : ~0ull;
    };
    uint64_t best = ~0ull;
    int bestp = -1;
    for (int p = lane; p < np_stride; p += 64) {
        heads[w][p] = 0;
        const uint64_t kk = head_key(p);
        if (kk < best) {
            best = kk;
            bestp = p;
        }
    }
    uint64_t res = ~0ull, res2 = ~0ull;   // result r sits in lane r (r < 64) or lane r - 64 of res2
    const uint64_t *prow_k = prior ? prior + (int64_t)qi * prior_stride : nullptr;
    int ph = 0;   // next key of the prior source (wave-uniform)
    uint64_t pv = prow_k ? prow_k[0] : ~0ull;
    for (int r = 0; r < kq; r++) {
        uint64_t m = best;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t u = shfl_xor_u64(m, o);
            m = u < m ? u : m;
        }
        if (pv < m) {   // the prior source's head is smallest (keys are distinct)
            if (lane == r) res = pv;
            if (lane + 64 == r) res2 = pv;
            ph++;
            pv = ph < prior_stride ? prow_k[ph] : ~0ull;
            continue;
        }
        if (m == ~0ull) break;
        if (lane == r) res = m;
        if (lane + 64 == r) res2 = m;
        if (best == m) {
            heads[w][bestp]++;
            best = ~0ull;
            bestp = -1;
            for (int p = lane; p < np_stride; p += 64) {
                const uint64_t kk = head_key(p);
                if (kk < best) {
                    best = kk;
                    bestp = p;
                }
            }
        }
    }
    for (int h = 0; h < 2; h++) {
        const int r = lane + 64 * h;
        if (r < out_stride) {
            const uint64_t key = h ? res2 : res;
            const int64_t o = (int64_t)qi * out_stride + r;
            if (keys_out) {
                keys_out[o] = r < kq ? key : ~0ull;
            } else if (r < kq && key != ~0ull) {
                dist[o] = key_value(key, S.metric);
                labels[o] = (int64_t)(uint32_t)key;
            } else {
                dist[o] = S.metric == 0 ? __int_as_float(0x7F800000) : __int_as_float((int)0xFF800000);
                labels[o] = -1;
            }
        }
    }
}

// Default queries per tile (the LDS path holds T * ceil(d/4) * 16 bytes,
// within 32 KiB).  Measured on the window workload: T=8 with two dimension
// chunks in flight beats T=16, whose query operands no longer fit the SGPR
// file.  The MFMA scan's tile is one 16-column operand.
int default_tile(int storage, int d, int C, int kcap) {
    if (storage != 0 || cert_ok(storage, d, C, kcap)) return 16;
    return d <= 1024 ? 8 : 4;
}

int search_tile(const Dev &S) { return S.tile; }

// ------------------------------------------------ reduced-precision scan
//
// Slabs in bf16 / fp16 ([slab][8-dim chunk][slot], 16 bytes per slot and
// chunk).  One wave scans a list for a tile of 16 queries with
// v_mfma_f32_16x16x32_{bf16,f16}: the A operand is 16 slots x 32 dims (lane l:
// slot l % 16, dims 8 (l / 16) .. +8 of the k-block), B the 16 queries
// rounded the same way, C the 16 x 16 fp32 scores (lane l: slots
// 4 (l / 16) .. +4, query l % 16).  Approximate distances:
// |x~|^2 + |q~|^2 - 2 x~.q~ (L2) or x~.q~ (IP), with FP32 accumulation.  Each
// query keeps its best kmul * k approximate candidates; the exact FP32
// re-rank over the shadow rows (k_rerank) decides the final order.

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <int DT>
__device__ __forceinline__ f32x4_t mfma_16x16x32(uint4 a, uint4 b, f32x4_t c) {
    if constexpr (DT == 1)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                      c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                     c, 0, 0, 0);
}

constexpr int MQ = 16;       // queries per MFMA tile
constexpr int MKB = 8;       // k-blocks of 32 dims: d <= 256
constexpr int MBUF = 96;     // candidate buffer per query (a step adds at most 64)

// Merge query t's buffered candidates into its sorted list (lane i = i-th
// best) and return the list's kq-th key's high word.
template <int NQ>
__device__ __forceinline__ uint32_t mfma_flush(uint64_t (&top)[NQ], int t, const uint64_t *buf, int cnt, int kq,
                                               int kcap) {
    const int lane = lane_id();
    const uint64_t b0 = lane < cnt ? buf[t * MBUF + lane] : ~0ull;
    uint64_t c = merge_sorted_with(top[t], b0);
    if (cnt > 64) {
        const uint64_t b1 = lane + 64 < cnt ? buf[t * MBUF + 64 + lane] : ~0ull;
        c = merge_sorted_with(c, b1);
    }
    c = lane < kcap ? c : ~0ull;
    top[t] = c;
    return kq > 0 ? (uint32_t)(readlane_u64(c, kq - 1) >> 32) : 0u;
}

template <int METRIC, int DT, int NKB, bool PERS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_scan_mfma(Dev S, const int32_t *__restrict__ item_list,
                                                  const int32_t *__restrict__ item_tile,
                                                  const int32_t *__restrict__ item_chunk,
                                                  const int32_t *__restrict__ list_pairs,
                                                  const float *__restrict__ q, int np_stride, int kcap, int k,
                                                  int kmul, const int32_t *__restrict__ kpq,
                                                  uint64_t *__restrict__ partials, uint32_t *__restrict__ gthr) {
    __shared__ uint64_t buf[MQ * MBUF];
    __shared__ int scnt[MQ], skq[MQ];
    const int lane = threadIdx.x, qcol = lane & 15, kgrp = lane >> 4;
    const int d = S.d, C = S.C, dp8 = S.dp8, sh = S.ctl[CTL_CHUNK];
    const int cs = __builtin_ctz(C), cm = C - 1;   // slab capacities are powers of two
    SIVF_ITEM_LOOP_BEGIN
    SIVF_ITEM_DECODE(MQ)
    __syncthreads();
    if (lane < MQ) {
        skq[lane] = lane < nt ? min(kmul * query_k(kpq, k, pairs[lane] / np_stride), kcap) : 0;
        scnt[lane] = 0;
    }
    // B operand: query qcol, dims 32 kb + 8 kgrp .. +8, rounded like the slabs
    const int qg = pairs[qcol < nt ? qcol : 0] / np_stride;   // query of column qcol
    const float *qr = q + (int64_t)qg * d;
    uint4 bq[NKB];
    float qn = 0.f;
#pragma unroll
    for (int kb = 0; kb < NKB; kb++) {
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int j = 32 * kb + 8 * kgrp + e;
            const float v = j < d ? qr[j] : 0.f;
            h[e] = DT == 1 ? to_bf16_bits(v) : to_f16_bits(v);
            const float r = DT == 1 ? bf16_bits_to_float(h[e]) : f16_bits_to_float(h[e]);
            qn = fmaf(r, r, qn);
        }
        bq[kb] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    }
    qn += __shfl_xor(qn, 16);
    qn += __shfl_xor(qn, 32);
    __syncthreads();
    uint32_t thr = skq[qcol] > 0 ? 0xFFFFFFFFu : 0u;   // threshold of query qcol (high word of its k-th key)
    // The same threshold as a float: a value passes when its key's high word is
    // at most thr, i.e. (L2) !(v > thr_f) or (IP) !(v < thr_f).  thr = ~0
    // (list not yet full) maps to NaN, which passes everything.
    const bool live = qcol < nt && skq[qcol] > 0;
    float thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
    uint64_t top[MQ];
#pragma unroll
    for (int t = 0; t < MQ; t++) top[t] = ~0ull;

    const int nslab = (len + cm) >> cs;
    int wbase = -(1 << 30), wslab = 0;
    const bool one_slab = cs >= 6 && !(p0 & 63);   // steps never straddle slabs
    for (int base = p0; base < p1; base += 64) {
        const int last_ord = min(base + 63, p1 - 1) >> cs;
        if (last_ord >= wbase + 64) {
            wbase = base >> cs;
            wslab = (wbase + lane < nslab) ? slab_of(S, l, wbase + lane) : 0;
        }
        // the 4 result rows of this lane in row group rg are positions
        // base + 16 rg + 4 kgrp .. +3: one slab (C >= 4), 16-byte aligned slots.
        // A operands of row group rg: slot 16 rg + qcol, 8-dim chunks 4 kb + kgrp;
        // two row groups in flight.  Chunks past the row repeat its last chunk
        // (their B lanes are zero); positions past the item read its last row
        // and are masked below.
        int64_t g4[4];
        const uint4 *hr[4];
        if (one_slab) {
            // the step's 64 positions lie in one slab: a scalar slab index
            const int64_t sb = __builtin_amdgcn_readlane(wslab, (base >> cs) - wbase);
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + 4 * kgrp, pr = base + 16 * rg + qcol;
                g4[rg] = sb * C + ((p < p1 ? p : ((p1 - 1) & ~3)) & cm);
                hr[rg] = S.hdata + sb * dp8 * C + ((pr < p1 ? pr : p1 - 1) & cm);
            }
        } else {
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + 4 * kgrp;
                const int pc = p < p1 ? p : ((p1 - 1) & ~3);
                g4[rg] = (int64_t)__shfl(wslab, (pc >> cs) - wbase) * C + (pc & cm);
            }
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + qcol;
                const int pc = p < p1 ? p : p1 - 1;
                const int slab = __shfl(wslab, (pc >> cs) - wbase);
                hr[rg] = S.hdata + (int64_t)slab * dp8 * C + (pc & cm);
            }
        }
        // the best R k-th key any work item has published for this query: a candidate behind it cannot
        // enter the query's final list (those R k keys are real candidates), so it tightens the filter
        const uint32_t pub = live ? __hip_atomic_load(gthr + qg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ~0u;
        float4 xn4[4] = {};
        if (METRIC == 0) {
#pragma unroll
            for (int rg = 0; rg < 4; rg++) xn4[rg] = *reinterpret_cast<const float4 *>(S.xnorm + g4[rg]);
        }
        f32x4_t acc[4];
        uint4 a0[NKB], a1[NKB];
        auto load_a = [&](uint4 (&a)[NKB], const uint4 *h) {
#pragma unroll
            for (int kb = 0; kb < NKB; kb++) a[kb] = h[(int64_t)min(4 * kb + kgrp, dp8 - 1) * C];
        };
        auto mma = [&](const uint4 (&a)[NKB]) {
            f32x4_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < NKB; kb++) c = mfma_16x16x32<DT>(a[kb], bq[kb], c);
            return c;
        };
        load_a(a0, hr[0]);
        load_a(a1, hr[1]);
        acc[0] = mma(a0);
        load_a(a0, hr[2]);
        acc[1] = mma(a1);
        load_a(a1, hr[3]);
        acc[2] = mma(a0);
        acc[3] = mma(a1);
        if (pub < thr) {
            thr = pub;
            thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
        }
        float vv[16];
        uint32_t pmask = 0;
#pragma unroll
        for (int rg = 0; rg < 4; rg++) {
            const float xs[4] = {xn4[rg].x, xn4[rg].y, xn4[rg].z, xn4[rg].w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float v = METRIC == 0 ? fmaf(-2.f, acc[rg][j], qn + xs[j]) : acc[rg][j];
                vv[4 * rg + j] = v;
                const bool pass = METRIC == 0 ? !(v > thr_f) : !(v < thr_f);
                pmask |= (pass ? 1u : 0u) << (4 * rg + j);
            }
        }
        if (!live) pmask = 0;
        // in range and (lazy deletes) live
        pmask &= lane_valid16(step_valid(S, base, p1, wslab, wbase, cs, cm), kgrp);
        if (ballot(pmask != 0)) {
            // offsets of this lane's candidates among the 4 lanes of its query
            const int np = __builtin_popcount(pmask);
            int incl = np;
            int u = __shfl_up(incl, 16);
            if (kgrp >= 1) incl += u;
            u = __shfl_up(incl, 32);
            if (kgrp >= 2) incl += u;
            int at = scnt[qcol] + incl - np;
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                if ((pmask >> (4 * rg)) & 0xFu) {
                    const uint4 id4 = *reinterpret_cast<const uint4 *>(S.sids + g4[rg]);
                    const uint32_t ids[4] = {id4.x, id4.y, id4.z, id4.w};
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        if ((pmask >> (4 * rg + j)) & 1u) {
                            const float v = vv[4 * rg + j];
                            const uint32_t hi = METRIC == 0 ? ord_bits(v) : ~ord_bits(zero_sign(v));
                            buf[qcol * MBUF + at] = ((uint64_t)hi << 32) | ids[j];
                            at++;
                        }
                    }
                }
            }
            __syncthreads();
            if (kgrp == 3) scnt[qcol] = at;   // the last lane of the query holds the new count
            __syncthreads();
            // merge buffers that could overflow on the next step, and fill a
            // query's list as soon as it has k candidates (sets its threshold)
            bool need = false;
            if (lane < MQ) {
                const int cnt = scnt[lane];
                need = cnt > MBUF - 64 || (thr == 0xFFFFFFFFu && cnt > 0 && cnt >= skq[lane]);
            }
            const uint64_t fm = ballot(need);
            if (fm) {
#pragma unroll
                for (int t = 0; t < MQ; t++) {
                    if ((fm >> t) & 1ull) {
                        const uint32_t nthr = mfma_flush<MQ>(top, t, buf, scnt[t], skq[t], kcap);
                        // publish a full list's R k-th key for the query's other work items (the query
                        // index is read while the whole wave is active)
                        const int qt = __builtin_amdgcn_readlane(qg, t);
                        if (lane == 0 && nthr != 0xFFFFFFFFu)
                            __hip_atomic_fetch_min(gthr + qt, nthr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (qcol == t) {
                            thr = nthr;
                            thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
                        }
                    }
                }
                __syncthreads();
                if (lane < MQ && ((fm >> lane) & 1ull)) scnt[lane] = 0;
                __syncthreads();
            }
        }
    }
    SIVF_ITEM_SLOT(MQ)
#pragma unroll
    for (int t = 0; t < MQ; t++) {
        if (t < nt) {
            const int cnt = scnt[t];
            if (cnt > 0) mfma_flush<MQ>(top, t, buf, cnt, skq[t], kcap);
            if (lane < kcap) partials[(slot0 + (int64_t)t * nc) * kcap + lane] = top[t];
        }
    }
    SIVF_ITEM_LOOP_END
}

// Insert key c into a list sorted ascending across lanes s0 .. s0 + KC - 1
// (lane s0 + i holds the i-th smallest); the largest key drops out and the
// other lanes keep their keys.  Keys are distinct.
template <int KC>
__device__ __forceinline__ uint64_t sorted_insert(uint64_t a, uint64_t c, int s0) {
    const int lane = lane_id();
    // previous lane's key: DPP wave_shr:1 (lane 0 keeps its own, unused)
    const uint32_t plo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)a, (int)(uint32_t)a, 0x138, 0xf, 0xf, false);
    const uint32_t phi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(a >> 32), (int)(uint32_t)(a >> 32), 0x138,
                                                                0xf, 0xf, false);
    const uint64_t prev = ((uint64_t)phi << 32) | plo;
    const uint64_t r = a < c ? a : ((lane == s0 || prev < c) ? c : prev);
    return (KC == 64 || (lane >= s0 && lane < s0 + KC)) ? r : a;
}

// Canonical FP32 value of one (row, query) pair, exactly as the VALU scan
// computes it (one fma per dimension, ascending, over the padded chunks);
// four chunks of loads in flight.  qv4: the query's zero-padded row in LDS.
template <int METRIC>
__device__ __forceinline__ void cert_chunk(float &r, float4 qv, float4 xv) {
    if (METRIC == 0) {
        float e;
        e = qv.x - xv.x;
        r = __builtin_fmaf(e, e, r);
        e = qv.y - xv.y;
        r = __builtin_fmaf(e, e, r);
        e = qv.z - xv.z;
        r = __builtin_fmaf(e, e, r);
        e = qv.w - xv.w;
        r = __builtin_fmaf(e, e, r);
    } else {
        r = __builtin_fmaf(qv.x, xv.x, r);
        r = __builtin_fmaf(qv.y, xv.y, r);
        r = __builtin_fmaf(qv.z, xv.z, r);
        r = __builtin_fmaf(qv.w, xv.w, r);
    }
}

template <int METRIC>
__device__ __forceinline__ float cert_exact(const float4 *__restrict__ xp, int C, int dp4, const float4 *qv4) {
    float r = 0.f;
    int c0 = 0;
    for (; c0 + 4 <= dp4; c0 += 4) {
        float4 xv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) xv[u] = xp[(int64_t)(c0 + u) * C];
#pragma unroll
        for (int u = 0; u < 4; u++) cert_chunk<METRIC>(r, qv4[c0 + u], xv[u]);
    }
    for (; c0 < dp4; c0++) cert_chunk<METRIC>(r, qv4[c0], xp[(int64_t)c0 * C]);
    return r;
}

template <int NB>
__device__ __forceinline__ void cert_load_a(float4 (&a)[NB], const float4 *__restrict__ xr, int C, int kgrp, int dp4) {
#pragma unroll
    for (int b = 0; b < NB; b++) a[b] = xr[(int64_t)min(4 * b + kgrp, dp4 - 1) * C];
}

// 16 slots x 16 queries over all dimensions; B operand (query l % 16, chunk
// 4 b + l / 16) read from the LDS query rows.
template <int NB>
__device__ __forceinline__ f32x4_t cert_mfma(const float4 (&a)[NB], const float4 *qrow, int kgrp, int dp4) {
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    // the next chunk's LDS read is in flight during this chunk's MFMAs
    float4 nb = kgrp < dp4 ? qrow[kgrp] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const float4 bv = nb;
        if (b + 1 < NB) {
            const int c = 4 * b + 4 + kgrp;
            nb = c < dp4 ? qrow[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].x, bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].y, bv.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].z, bv.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].w, bv.w, acc, 0, 0, 0);
    }
    return acc;
}

// ------------------------------------------------ certified FP32 MFMA scan
//
// FP32 slabs with results identical to the canonical scan.  For this contraction
// v_mfma_f32_16x16x4_f32 does four times the work per cycle of the sub + fma VALU
// form; it gives approximate values for 16 slots x 16 queries:
// Dt = |x|^2 + |q|^2 - 2 x.q (L2) or -x.q (IP, as a distance).  A slot can be
// among a query's k best only if Dt - e is at most the query's current k-th best
// canonical value; only those pairs get their canonical FP32 distance recomputed
// (sequential fma over ascending dimensions, exactly as the VALU scan computes it)
// and inserted into the query's exact sorted list.
//
// Half-width e.  With rounding error at most one unit 2^-24 per operation, the MFMA
// form (norms included) differs from the exact value by at most (2d + 4) 2^-24
// (|x| + |q|)^2 and the canonical sum by (d + 2) 2^-24 |q - x|^2; IP: 2d and d times
// 2^-24 |x||q|.  The kernel uses cf (|x| + |q|)^2 with cf = (5d + 32) 2^-24 (IP:
// (4d + 32) 2^-24 |x||q|), plus 2^-122 sqrt(d) (|x| + |q|) + 2^-120 d for underflow,
// relaxed to e = e1 (|x|^2 + |q|^2) + e0 so that no square root is needed (the
// margin covers the rounding of the fp32 norms and of e).  An overflowing value gives
// inf or NaN in the test, and both pass.
//
// Before a query has k exact values (the first step of a work item), its threshold
// is the k-th smallest upper bound Dt + e among the step's candidates, found by
// bisection: at least k candidates lie at or below it, so the k best do too.
//
// Layout.  A operand (lane l): slot l % 16 of the row group, the 4 dimensions of
// chunk 4 b + l / 16 (one float4), fed to 4 consecutive MFMAs one component each;
// the B operand holds the same dimensions of query l % 16 (read from the tile's
// query rows in LDS), so every MFMA pairs equal dimensions and the 4 x NB MFMAs of
// a row group cover all 16 NB dimensions.  C (lane l): slots 4 (l / 16) .. +3,
// query l % 16.  Passing pairs are queued in LDS and recomputed one per lane,
// in full rounds of 64 (the queue drains early when a query has no k-th value
// yet, before the slab window moves, and at the end of the item).
// Exact lists: KC keys per query sorted across KC lanes, 64 / KC queries per
// register (KC = 16 for kcap 16, else 64).  KC = 128 (k up to 128): ranks
// 0..63 stay in registers as for KC = 64; ranks 64..127 are kept only for
// queries whose k exceeds 64, in the upper half of the query's own partial
// slot (read and written back by the inserting lanes, each its own rank; an
// LDS copy would cost the kernel a third of its resident waves); a key that
// enters the low half pushes its largest key down into the high half.
template <int METRIC, int NB, bool PERS, int KC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_scan_cert(Dev S, const int32_t *__restrict__ item_list,
                                                  const int32_t *__restrict__ item_tile,
                                                  const int32_t *__restrict__ item_chunk,
                                                  const int32_t *__restrict__ list_pairs,
                                                  const float *__restrict__ q, int np_stride, int kcap, int k,
                                                  const int32_t *__restrict__ kpq,
                                                  uint64_t *__restrict__ partials, uint32_t *__restrict__ gthr) {
    extern __shared__ float4 sqr[];    // the tile's 16 query rows, zero-padded to dp4 chunks, stride dp4 + 1
    __shared__ uint32_t pq[64 * MQ + 64];   // queued passing pairs: window position << 4 | query
    __shared__ int skq[MQ];
    const int lane = threadIdx.x, qcol = lane & 15, kgrp = lane >> 4;
    const int d = S.d, C = S.C, dp4 = S.dp4, sh = S.ctl[CTL_CHUNK];
    const int qs = dp4 + 1;   // LDS row stride: rows start in different banks
    const int cs = __builtin_ctz(C), cm = C - 1;   // slab capacities are powers of two
    // half-width e = e1 (|x|^2 + |q|^2) + e0, from (|x| + |q|)^2 <= 2 (|x|^2 + |q|^2),
    // |x||q| <= (|x|^2 + |q|^2) / 2 and |x| + |q| <= 1 + (|x|^2 + |q|^2)
    const float cf = METRIC == 0 ? (5.0f * d + 32.0f) * 0x1p-24f : (4.0f * d + 32.0f) * 0x1p-24f;
    const float ca = sqrtf((float)d) * 0x1p-122f, cb = (float)d * 0x1p-120f;
    const float e1 = (METRIC == 0 ? 2.f * cf : 0.5f * cf) + ca, e0 = ca + cb;
    SIVF_ITEM_LOOP_BEGIN
    SIVF_ITEM_DECODE(MQ)
    __syncthreads();
    if (lane < MQ) {
        const int qi = pairs[lane < nt ? lane : 0] / np_stride;
        skq[lane] = lane < nt ? min(query_k(kpq, k, qi), kcap) : 0;
    }
    for (int i = lane; i < MQ * dp4; i += 64) {
        const int t = i / dp4, j = 4 * (i - t * dp4);
        const float *qr = q + (int64_t)(pairs[t < nt ? t : 0] / np_stride) * d;
        float4 v;
        v.x = j < d ? qr[j] : 0.f;
        v.y = j + 1 < d ? qr[j + 1] : 0.f;
        v.z = j + 2 < d ? qr[j + 2] : 0.f;
        v.w = j + 3 < d ? qr[j + 3] : 0.f;
        sqr[t * qs + (j >> 2)] = v;
    }
    __syncthreads();
    const int qg = pairs[qcol < nt ? qcol : 0] / np_stride;   // query of column qcol
    float qn2 = 0.f;   // |q|^2 of query qcol
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int c = 4 * b + kgrp;
        const float4 v = c < dp4 ? sqr[qcol * qs + c] : make_float4(0.f, 0.f, 0.f, 0.f);
        qn2 = fmaf(v.x, v.x, qn2);
        qn2 = fmaf(v.y, v.y, qn2);
        qn2 = fmaf(v.z, v.z, qn2);
        qn2 = fmaf(v.w, v.w, qn2);
    }
    qn2 += __shfl_xor(qn2, 16);
    qn2 += __shfl_xor(qn2, 32);
    __syncthreads();
    uint32_t thr = skq[qcol] > 0 ? 0xFFFFFFFFu : 0u;   // high word of query qcol's k-th exact key
    // the k-th exact value as a float (L2: distance, IP: score); ~0 maps to NaN, which passes all
    const bool live = qcol < nt && skq[qcol] > 0;
    float thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
    // sorted exact lists: query t in register t / QPR, lanes KC (t % QPR) .. +KC-1
    // (KC = 128: ranks 0..63 in register t, the rest in LDS)
    constexpr int QPR = KC == 128 ? 1 : 64 / KC, NR = MQ / QPR;
    uint64_t top[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) top[r] = ~0ull;
    uint32_t hset = 0;   // KC = 128: queries whose ranks 64..127 have been written to their slot

    const int nslab = (len + cm) >> cs;
    int wbase = -(1 << 30), wslab = 0;
    int qn = 0;   // queued pairs (fewer than 64 carry over to the next step)
    const bool one_slab = cs >= 6 && !(p0 & 63);   // steps never straddle slabs
    for (int base = p0; base < p1; base += 64) {
        const int last_ord = min(base + 63, p1 - 1) >> cs;
        if (last_ord >= wbase + 64) {
            wbase = base >> cs;
            wslab = (wbase + lane < nslab) ? slab_of(S, l, wbase + lane) : 0;
        }
        // the 4 result rows of this lane in row group rg: positions base + 16 rg + 4 kgrp .. +3
        // A operands of row group rg: slot 16 rg + qcol, chunks 4 b + kgrp; two
        // row groups in flight (the loads of the next overlap this one's MFMAs).
        // Chunks past the row repeat its last chunk (their B lanes are zero and
        // stored values are finite); positions past the item read its last row
        // and are masked below.
        int64_t g4[4];
        const float4 *xr[4];
        if (one_slab) {
            // the step's 64 positions lie in one slab: a scalar slab index
            const int64_t sb = __builtin_amdgcn_readlane(wslab, (base >> cs) - wbase);
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + 4 * kgrp, pr = base + 16 * rg + qcol;
                g4[rg] = sb * C + ((p < p1 ? p : ((p1 - 1) & ~3)) & cm);
                xr[rg] = S.data + sb * dp4 * C + ((pr < p1 ? pr : p1 - 1) & cm);
            }
        } else {
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + 4 * kgrp;
                const int pc = p < p1 ? p : ((p1 - 1) & ~3);
                g4[rg] = (int64_t)__shfl(wslab, (pc >> cs) - wbase) * C + (pc & cm);
            }
#pragma unroll
            for (int rg = 0; rg < 4; rg++) {
                const int p = base + 16 * rg + qcol;
                const int pc = p < p1 ? p : p1 - 1;
                const int slab = __shfl(wslab, (pc >> cs) - wbase);
                xr[rg] = S.data + (int64_t)slab * dp4 * C + (pc & cm);
            }
        }
        // the best k-th key value any work item has published for this query: a pair behind it cannot
        // enter the query's final k (those k keys are real candidates), so it serves as the threshold
        const uint32_t pub = live ? __hip_atomic_load(gthr + qg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ~0u;
        float4 xn4[4];
#pragma unroll
        for (int rg = 0; rg < 4; rg++) xn4[rg] = *reinterpret_cast<const float4 *>(S.xnorm + g4[rg]);
        f32x4_t acc[4];
        float4 a0[NB], a1[NB];
        cert_load_a<NB>(a0, xr[0], C, kgrp, dp4);
        cert_load_a<NB>(a1, xr[1], C, kgrp, dp4);
        acc[0] = cert_mfma<NB>(a0, sqr + qcol * qs, kgrp, dp4);
        cert_load_a<NB>(a0, xr[2], C, kgrp, dp4);
        acc[1] = cert_mfma<NB>(a1, sqr + qcol * qs, kgrp, dp4);
        cert_load_a<NB>(a1, xr[3], C, kgrp, dp4);
        acc[2] = cert_mfma<NB>(a0, sqr + qcol * qs, kgrp, dp4);
        acc[3] = cert_mfma<NB>(a1, sqr + qcol * qs, kgrp, dp4);
        // distance space (L2: the distance; IP: minus the score): value v and
        // certified half-width e of every (slot, query) pair of this lane
        float vv[16], ee[16];
        // bit 4 rg + j: position 16 rg + 4 kgrp + j in range and (lazy deletes) live
        const uint32_t vm = lane_valid16(step_valid(S, base, p1, wslab, wbase, cs, cm), kgrp);
#pragma unroll
        for (int rg = 0; rg < 4; rg++) {
            const float xs[4] = {xn4[rg].x, xn4[rg].y, xn4[rg].z, xn4[rg].w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float sq = qn2 + xs[j];
                vv[4 * rg + j] = METRIC == 0 ? fmaf(-2.f, acc[rg][j], sq) : -acc[rg][j];
                ee[4 * rg + j] = fmaf(e1, sq, e0);
            }
        }
        if (pub < thr) {
            thr = pub;
            thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
        }
        // the query's k-th best value so far in distance space (NaN: none yet, all pass)
        float thd = METRIC == 0 ? thr_f : -thr_f;
        const bool warm = live && thr == 0xFFFFFFFFu;
        if (ballot(warm)) {
            // No k-th value yet: bound it by the k-th smallest upper bound v + e
            // among this step's candidates of the query (lanes qcol + 16 i hold
            // them): at least k candidates lie at or below it, so the k best
            // do too.  Bisection keeps count(v + e <= hi) >= k.
            int nv = 0;
            float mn = __int_as_float(0x7F800000), mx = -__int_as_float(0x7F800000);
#pragma unroll
            for (int i = 0; i < 16; i++) {
                float u = vv[i] + ee[i];
                if (!(u <= __int_as_float(0x7F800000))) u = __int_as_float(0x7F800000);   // NaN: +inf
                if ((vm >> i) & 1u) {
                    nv++;
                    mn = fminf(mn, u);
                    mx = fmaxf(mx, u);
                }
            }
            nv += __shfl_xor(nv, 16);
            nv += __shfl_xor(nv, 32);
            mn = fminf(mn, __shfl_xor(mn, 16));
            mn = fminf(mn, __shfl_xor(mn, 32));
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            const int kq = skq[qcol];
            float lo = mn, hi = mx;
            for (int it = 0; it < 10; it++) {
                const float mid = lo + 0.5f * (hi - lo);
                int c = 0;
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    const float u = vv[i] + ee[i];
                    c += (((vm >> i) & 1u) && u <= mid) ? 1 : 0;
                }
                c += __shfl_xor(c, 16);
                c += __shfl_xor(c, 32);
                if (c >= kq) hi = mid;
                else lo = mid;
            }
            if (warm && nv >= kq) thd = hi;
        }
        uint32_t pmask = 0;
#pragma unroll
        for (int i = 0; i < 16; i++) pmask |= (!(vv[i] - ee[i] > thd) ? 1u : 0u) << i;
        if (!live) pmask = 0;
        pmask &= vm;
        if (ballot(pmask != 0)) {
            // queue the passing (position, query) pairs in lane order
            const int np = __builtin_popcount(pmask);
            const int incl = wave_incl_scan_dpp(np);
            int at = qn + incl - np;
            qn += __builtin_amdgcn_readlane(incl, 63);
            const int wpos = base - (wbase << cs);   // queued positions are relative to the slab window
            uint32_t m = pmask;
            while (m) {
                const int bit = __builtin_ctz(m);
                m &= m - 1;
                pq[at++] = ((uint32_t)(wpos + 16 * (bit >> 2) + 4 * kgrp + (bit & 3)) << 4) | (uint32_t)qcol;
            }
        }
        // Recompute full rounds of 64 pairs; everything when a query still waits
        // for its first k-th value, before the slab window moves, and at the end.
        const int nb = base + 64;
        const bool drain = ballot(live && thr == 0xFFFFFFFFu) != 0 || nb >= p1 ||
                           (min(nb + 63, p1 - 1) >> cs) >= wbase + 64;
        const int nproc = drain ? qn : (qn & ~63);
        if (nproc > 0) {
            __syncthreads();
            for (int r0 = 0; r0 < nproc; r0 += 64) {
                const bool act = r0 + lane < nproc;
                const uint32_t e = pq[act ? r0 + lane : r0];
                const int t = (int)(e & 15), pw = (int)(e >> 4);
                const int slab = __shfl(wslab, pw >> cs), slot = pw & cm;
                uint64_t key = ~0ull;
                if (act) {
                    const float r = cert_exact<METRIC>(S.data + (int64_t)slab * dp4 * C + slot, C, dp4, sqr + t * qs);
                    key = ((uint64_t)key_hi<METRIC>(r) << 32) | S.sids[(int64_t)slab * C + slot];
                }
                // insert the exact keys into their queries' sorted lists, one at a time
#pragma unroll
                for (int t2 = 0; t2 < MQ; t2++) {
                    uint64_t bm = ballot(act && t == t2);
                    if (bm) {
                        const int kq = __builtin_amdgcn_readfirstlane(skq[t2]);   // > 0: only live queries have pairs
                        uint64_t hi = ~0ull;      // KC = 128, k > 64: ranks 64..127
                        uint64_t *hdst = nullptr;
                        if constexpr (KC == 128) {
                            if (kq > 64) {
                                SIVF_ITEM_SLOT(MQ)
                                hdst = partials + (slot0 + (int64_t)t2 * nc) * kcap + 64;
                                if ((hset >> t2) & 1u) hi = hdst[lane];
                                hset |= 1u << t2;
                            }
                        }
                        // only keys below the query's current k-th key can change its k best
                        uint64_t kth;
                        if constexpr (KC == 128) kth = kq <= 64 ? readlane_u64(top[t2], kq - 1) : readlane_u64(hi, kq - 65);
                        else kth = readlane_u64(top[t2 / QPR], KC * (t2 % QPR) + kq - 1);
                        bm = ballot(act && t == t2 && key < kth);
                        while (bm) {
                            const int src = (int)__builtin_ctzll(bm);
                            bm &= bm - 1;
                            uint64_t c = readlane_u64(key, src);
                            if constexpr (KC == 128) {
                                // a key below the low half's largest enters it and pushes that one down
                                const uint64_t lmax = readlane_u64(top[t2], 63);
                                if (c < lmax) {
                                    top[t2] = sorted_insert<64>(top[t2], c, 0);
                                    c = lmax;
                                }
                                if (kq > 64) hi = sorted_insert<64>(hi, c, 0);
                            } else {
                                top[t2 / QPR] = sorted_insert<KC>(top[t2 / QPR], c, KC * (t2 % QPR));
                            }
                        }
                        uint32_t nthr = 0u;
                        if constexpr (KC == 128) {
                            if (kq > 64) hdst[lane] = hi;
                            nthr = (uint32_t)((kq <= 64 ? readlane_u64(top[t2], kq - 1) : readlane_u64(hi, kq - 65)) >> 32);
                        } else {
                            nthr = kq > 0 ? (uint32_t)(readlane_u64(top[t2 / QPR], KC * (t2 % QPR) + kq - 1) >> 32) : 0u;
                        }
                        // publish a full list's k-th key value for the query's other work items (the
                        // query index is read while the whole wave is active)
                        const int qt = __builtin_amdgcn_readlane(qg, t2);
                        if (lane == 0 && nthr != 0xFFFFFFFFu)
                            __hip_atomic_fetch_min(gthr + qt, nthr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (qcol == t2) {
                            thr = nthr;
                            thr_f = METRIC == 0 ? from_ord(thr) : from_ord(~thr);
                        }
                    }
                }
            }
            // move the unprocessed tail (< 64 pairs) to the front
            const int rest = qn - nproc;
            const uint32_t v = lane < rest ? pq[nproc + lane] : 0u;
            __syncthreads();
            if (lane < rest) pq[lane] = v;
            qn = rest;
        }
        __syncthreads();   // queue writes of this step before the next step's appends
    }
    SIVF_ITEM_SLOT(MQ)
    if constexpr (KC == 128) {
#pragma unroll
        for (int t = 0; t < MQ; t++) {
            if (t < nt) {
                uint64_t *dst = partials + (slot0 + (int64_t)t * nc) * kcap;
                dst[lane] = top[t];
                if (!((hset >> t) & 1u)) dst[64 + lane] = ~0ull;   // no rank 64..127 key yet
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < MQ; t++)
            if (t < nt && (lane >> (KC == 64 ? 6 : 4)) == (KC == 64 ? 0 : t % QPR) && (lane & (KC - 1)) < kcap)
                partials[(slot0 + (int64_t)t * nc) * kcap + (lane & (KC - 1))] = top[t / QPR];
    }
    SIVF_ITEM_LOOP_END
}

// Exact FP32 re-rank: one wave per query; lane i recomputes the canonical
// FP32 distance of candidate i from the fp32 shadow row, then the wave sorts
// the keys and keeps the query's k best.
__global__ __launch_bounds__(256) void k_rerank(Dev S, int nq, const float *__restrict__ q, int kc,
                                                const int64_t *__restrict__ cand, int k, int kmul,
                                                const int32_t *__restrict__ kpq, float *__restrict__ dist,
                                                int64_t *__restrict__ labels) {
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int qi = blockIdx.x * 4 + w;
    if (qi >= nq) return;
    const int kq = query_k(kpq, k, qi);
    const int nc = min(kq * kmul, kc);
    const int d = S.d, C = S.C;
    uint64_t key = ~0ull;
    if (lane < nc) {
        const int64_t id = cand[(int64_t)qi * kc + lane];
        const uint32_t g = id >= 0 ? S.att[id] : INVALID;
        if (g != INVALID) {
            const float4 *xp = S.data + (int64_t)(g / C) * S.dp4 * C + g % C;
            const float *qr = q + (int64_t)qi * d;
            float r = 0.f;
            for (int c = 0; c < S.dp4; c++) {
                const float4 xv = xp[(int64_t)c * C];
                const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
                for (int e = 0; e < 4; e++) {
                    const int j = 4 * c + e;
                    if (j < d) {
                        if (S.metric == 0) {
                            const float t = qr[j] - xs[e];
                            r = __builtin_fmaf(t, t, r);
                        } else {
                            r = __builtin_fmaf(qr[j], xs[e], r);
                        }
                    }
                }
            }
            key = make_key(r, (uint32_t)id, S.metric);
        }
    }
    key = wave_sort64(key, true);
    if (lane < k) {
        const int64_t o = (int64_t)qi * k + lane;
        if (lane < kq && key != ~0ull) {
            dist[o] = key_value(key, S.metric);
            labels[o] = (int64_t)(uint32_t)key;
        } else {
            dist[o] = S.metric == 0 ? __int_as_float(0x7F800000) : __int_as_float((int)0xFF800000);
            labels[o] = -1;
        }
    }
}

// Work items of a call without splitting: tiles of T pairs per list.  The
// plan may split long lists until the items reach twice this (or the
// buffer); the dispatch grid stays at this size.
static int64_t items_unsplit(const Dev &S, int npairs) {
    const int T = search_tile(S);
    return (npairs + T - 1) / T + (npairs < S.nlist ? npairs : S.nlist);
}

static int64_t item_limit(const Dev &S, const SearchBufs &W, int npairs) {
    const int64_t lim = 2 * items_unsplit(S, npairs);
    return lim < W.item_cap ? lim : W.item_cap;
}

// Grid of a scan launch: the call's item bound rounded up to a multiple of 8
// (dispatch), or the waves that fit on the chip at the kernel's occupancy
// (persistent).
template <typename K>
static unsigned scan_grid(K kernel, const Dev &S, const SearchBufs &W, int npairs, size_t smem) {
    if (!S.persistent) {
        const int64_t g = (item_limit(S, W, npairs) + 7) / 8 * 8;
        return (unsigned)(g < 8 ? 8 : g);
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, smem) != hipSuccess || per_cu < 1)
        per_cu = 8;
    static int cus = 0;   // compute units of the first device used (all GPUs of a node are one part)
    if (cus == 0) {
        int dev = 0, n = 0;
        cus = (hipGetDevice(&dev) == hipSuccess &&
               hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                  ? n
                  : 256;
    }
    return (unsigned)(per_cu * cus);
}

void launch_search_scan_mfma(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const float *q,
                             int np_stride, int kcap, int k, int kmul, const int32_t *k_per_query) {
    const int npairs = nq * np_stride;
    // k-blocks of 32 dimensions held as B operands: 2, 3, 4 or 8 (d <= 256)
    const int nkb = (S.d + 31) / 32;
    launch_fill_i32(st, reinterpret_cast<int32_t *>(W.gthr), nq, -1);   // no key published yet
#define SIVF_LAUNCH_MFMA_P(M, D, K, P)                                                                       \
    hipLaunchKernelGGL((k_scan_mfma<M, D, K, P>), dim3(scan_grid(k_scan_mfma<M, D, K, P>, S, W, npairs, 0)),    \
                       dim3(64), 0, st, S, W.item_list, W.item_tile, W.item_chunk, W.list_pairs, q, np_stride,  \
                       kcap, k, kmul, k_per_query, W.partials, W.gthr)
#define SIVF_LAUNCH_MFMA(M, D, K)                                                                            \
    do {                                                                                                     \
        if (S.persistent) SIVF_LAUNCH_MFMA_P(M, D, K, true);                                                 \
        else SIVF_LAUNCH_MFMA_P(M, D, K, false);                                                             \
    } while (0)
#define SIVF_LAUNCH_MFMA_K(M, D)                                                                             \
    do {                                                                                                     \
        if (nkb <= 2) SIVF_LAUNCH_MFMA(M, D, 2);                                                             \
        else if (nkb == 3) SIVF_LAUNCH_MFMA(M, D, 3);                                                        \
        else if (nkb == 4) SIVF_LAUNCH_MFMA(M, D, 4);                                                        \
        else SIVF_LAUNCH_MFMA(M, D, 8);                                                                      \
    } while (0)
    if (S.metric == 0 && S.storage == 1) SIVF_LAUNCH_MFMA_K(0, 1);
    else if (S.metric == 0) SIVF_LAUNCH_MFMA_K(0, 2);
    else if (S.storage == 1) SIVF_LAUNCH_MFMA_K(1, 1);
    else SIVF_LAUNCH_MFMA_K(1, 2);
#undef SIVF_LAUNCH_MFMA_K
#undef SIVF_LAUNCH_MFMA
#undef SIVF_LAUNCH_MFMA_P
}

void launch_rerank(hipStream_t st, const Dev &S, int nq, const float *q, int kc, const int64_t *cand, int k,
                   int kmul, const int32_t *k_per_query, float *dist, int64_t *labels) {
    hipLaunchKernelGGL(k_rerank, dim3((nq + 3) / 4), dim3(256), 0, st, S, nq, q, kc, cand, k, kmul, k_per_query,
                       dist, labels);
}

template <int T, bool WIDE, bool PERS>
static void launch_scan_p(hipStream_t st, const Dev &S, const SearchBufs &W, const float *q, int np_stride,
                          int kcap, int k, const int32_t *kpq, int npairs) {
    const bool sq = (S.d % 4 == 0) && (((uintptr_t)q & 15) == 0);
#define SIVF_LAUNCH_SCAN(KERN, SMEM)                                                                         \
    hipLaunchKernelGGL(KERN, dim3(scan_grid(KERN, S, W, npairs, SMEM)), dim3(64), SMEM, st, S, W.item_list,   \
                       W.item_tile, W.item_chunk, W.list_pairs, q, np_stride, kcap, k, kpq, W.partials)
    if (sq) {
        if (S.metric == 0) SIVF_LAUNCH_SCAN((k_scan_sq<T, 0, WIDE, PERS>), 0);
        else SIVF_LAUNCH_SCAN((k_scan_sq<T, 1, WIDE, PERS>), 0);
        return;
    }
    const size_t smem = (size_t)T * S.dp4 * sizeof(float4);
    if (S.metric == 0) SIVF_LAUNCH_SCAN((k_scan<T, 0, WIDE, PERS>), smem);
    else SIVF_LAUNCH_SCAN((k_scan<T, 1, WIDE, PERS>), smem);
#undef SIVF_LAUNCH_SCAN
}

template <int T, bool WIDE>
static void launch_scan_t(hipStream_t st, const Dev &S, const SearchBufs &W, const float *q, int np_stride,
                          int kcap, int k, const int32_t *kpq, int npairs) {
    if (S.persistent) launch_scan_p<T, WIDE, true>(st, S, W, q, np_stride, kcap, k, kpq, npairs);
    else launch_scan_p<T, WIDE, false>(st, S, W, q, np_stride, kcap, k, kpq, npairs);
}

void launch_search_plan(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const KClass &cls, int snap,
                        int32_t *heat) {
    const int np_stride = cls.np_stride;
    const int npairs = nq * np_stride;
    const unsigned pb = (unsigned)((npairs + 255) / 256);
    const int T = search_tile(S);
    if (S.nlist <= 16384)
        hipLaunchKernelGGL(k_inv_count_lds, dim3((unsigned)((npairs + INV_PB - 1) / INV_PB)), dim3(1024),
                           (size_t)S.nlist * 4, st, S, npairs, W.probes, W.pair_rank, cls);
    else
        hipLaunchKernelGGL(k_inv_count, dim3(pb), dim3(256), 0, st, S, npairs, W.probes, W.pair_rank, cls);
    const int64_t lim = item_limit(S, W, npairs);
    hipLaunchKernelGGL(k_inv_plan, dim3(1), dim3(1024), 0, st, S, T, S.chunk_shift, W.slot_cap, lim,
                       (int)((lim + 7) / 8), snap, heat);
    hipLaunchKernelGGL(k_inv_items, dim3((S.nlist + 3) / 4), dim3(256), 0, st, S, T, W.item_list, W.item_tile,
                       W.item_chunk);
    hipLaunchKernelGGL(k_inv_scatter, dim3(pb), dim3(256), 0, st, S, npairs, W.probes, W.pair_rank,
                       W.list_pairs);
}

bool cert_ok(int storage, int d, int C, int kcap) { return storage == 0 && d <= 256 && C >= 4 && kcap <= 128; }

template <int METRIC, int NB, int KC>
static void launch_cert_nb(hipStream_t st, const Dev &S, const SearchBufs &W, const float *q, int np_stride,
                           int kcap, int k, const int32_t *kpq, int npairs) {
    const size_t smem = (size_t)MQ * (S.dp4 + 1) * sizeof(float4);
#define SIVF_LAUNCH_CERT(P)                                                                                  \
    hipLaunchKernelGGL((k_scan_cert<METRIC, NB, P, KC>), dim3(scan_grid(k_scan_cert<METRIC, NB, P, KC>, S, W, npairs, smem)), \
                       dim3(64), smem, st, S, W.item_list, W.item_tile, W.item_chunk, W.list_pairs, q, np_stride, \
                       kcap, k, kpq, W.partials, W.gthr)
    if (S.persistent) SIVF_LAUNCH_CERT(true);
    else SIVF_LAUNCH_CERT(false);
#undef SIVF_LAUNCH_CERT
}

template <int METRIC>
static void launch_cert(hipStream_t st, const Dev &S, const SearchBufs &W, const float *q, int np_stride, int kcap,
                        int k, const int32_t *kpq, int npairs) {
    // blocks of 16 dimensions held as B operands (d <= 256)
    // sorted lists of 16 keys (kcap 16: four queries per register), 64 (kcap 32, 64) or
    // 128 (kcap 128: ranks 64..127 in the partial slot)
    const int nb = (S.d + 15) / 16;
    launch_fill_i32(st, reinterpret_cast<int32_t *>(W.gthr), npairs / np_stride, -1);   // no key published yet
#define SIVF_CERT_NB(KC)                                                                                     \
    do {                                                                                                     \
        if (nb <= 2) launch_cert_nb<METRIC, 2, KC>(st, S, W, q, np_stride, kcap, k, kpq, npairs);            \
        else if (nb <= 4) launch_cert_nb<METRIC, 4, KC>(st, S, W, q, np_stride, kcap, k, kpq, npairs);       \
        else if (nb <= 8) launch_cert_nb<METRIC, 8, KC>(st, S, W, q, np_stride, kcap, k, kpq, npairs);       \
        else launch_cert_nb<METRIC, 16, KC>(st, S, W, q, np_stride, kcap, k, kpq, npairs);                   \
    } while (0)
    if (kcap <= 16) SIVF_CERT_NB(16);
    else if (kcap <= 64) SIVF_CERT_NB(64);
    else SIVF_CERT_NB(128);
#undef SIVF_CERT_NB
}

void launch_search_scan(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const float *q, int np_stride,
                        int kcap, int k, const int32_t *k_per_query) {
    const int T = search_tile(S);
    const int npairs = nq * np_stride;
    if (T == 16) {   // the schedule setter admits tile 16 only where cert_ok holds
        if (S.metric == 0) launch_cert<0>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
        else launch_cert<1>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
        return;
    }
    if (kcap > 64) {
        if (T == 8) launch_scan_t<8, true>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
        else launch_scan_t<4, true>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
    } else {
        if (T == 8) launch_scan_t<8, false>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
        else launch_scan_t<4, false>(st, S, W, q, np_stride, kcap, k, k_per_query, npairs);
    }
}

void launch_search_merge(hipStream_t st, const Dev &S, const SearchBufs &W, int nq, const KClass &cls, int kcap,
                         int out_stride, int k, int kmul, const int32_t *k_per_query, float *dist,
                         int64_t *labels, const uint64_t *prior, int prior_stride, uint64_t *keys_out) {
    const int np_stride = cls.np_stride;
    const int npairs = nq * np_stride;
    const unsigned pb = (unsigned)((npairs + 255) / 256);
    if (kcap > 64)
        hipLaunchKernelGGL(k_chunk_merge<true>, dim3(pb), dim3(256), 0, st, S, npairs, W.probes, W.pair_rank,
                           W.partials, kcap);
    else
        hipLaunchKernelGGL(k_chunk_merge<false>, dim3(pb), dim3(256), 0, st, S, npairs, W.probes, W.pair_rank,
                           W.partials, kcap);
    hipLaunchKernelGGL(k_merge, dim3((nq + 3) / 4), dim3(256), 0, st, S, nq, np_stride, W.probes, W.pair_rank,
                       W.partials, kcap, out_stride, k, kmul, k_per_query, dist, labels, cls, prior, prior_stride,
                       keys_out);
}

}  // namespace sivf
