// In-place mutation of the slab-resident inverted lists.
//
// Insert (the paper's ingestion, Sec. 3.2 / Alg. 2, re-designed as a batch):
//   prepare  validate ids, elect the last occurrence of each id in the batch
//   count    per-list counts and ranks with wave-aggregated atomics (lanes of
//            a wave that target the same list share one atomic) -- every
//            vector gets a distinct position without a CAS retry loop
//   admit    whole-batch check that the final state fits in the pool; else
//            NOSPACE and no state change (fail-fast, Sec. 3.2)
//   [delete  live ids of the batch are deleted first: delete-then-insert, Sec. 3]
//   alloc    per list: slabs needed = ceil(new_len/C) - ceil(len/C); one
//            atomic per block of 256 lists pops them from the free stack
//            (the stack of Sec. 3.1 / Alg. 1), then the list tables are
//            extended in parallel
//   scatter  payload, id and address-table entry of every vector
//
// Delete (the paper's eviction, Sec. 3.4 / Alg. 4, with compaction instead of
// a validity bitmap): the address table gives each id's slot in O(1); the
// deleted set D of a list with n entries leaves n' = n - |D| entries; holes
// below n' are refilled with the surviving entries of the tail window
// [n', n), so the list stays dense, and the slabs past ceil(n'/C) return to
// the free stack.
//   mark      address-table exchange, tombstone, per-list deletion counts
//   plan      per-list offsets of the tail windows, new lengths
//   holes     deleted positions below n', numbered per list
//   move      tail-window positions in list order; survivors fill the holes
//   finalize  new lengths; emptied tail slabs and pages back to the stacks  An id is deleted by exactly one thread: the one whose
// atomic exchange on the address table sees it live (idempotent delete,
// Theorem 3).
#include "sivf_launch.h"

namespace sivf {

__device__ __forceinline__ int cdiv(int a, int b) { return (a + b - 1) / b; }

// Lazy deletes: make a written slot visible (the paper's Alg. 2): a release
// fence at agent scope orders the slot's payload, id and address-table writes
// before the atomic OR that sets its validity bit, so a reader that sees the
// bit (on any XCD) sees the entry.
__device__ __forceinline__ void publish_slot(const Dev &S, int slab, int slot) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_or(S.bits + (int64_t)slab * S.bw + (slot >> 6), 1ull << (slot & 63), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ insert

__global__ __launch_bounds__(256) void k_add_prepare(Dev S, int n, const int64_t *__restrict__ ids) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t u = ids[i];
    if (u < 0 || u >= S.id_capacity)
        fail_call(S.ctl, -3);
    else
        atomicMax(&S.mark[u], i);
}

// fresh_only: the call may not hold live ids (SIVF_ERR_LIVE_ID otherwise).
template <bool BLK>
__global__ __launch_bounds__(256) void k_add_count(Dev S, int n, const int64_t *__restrict__ ids,
                                                   const int32_t *__restrict__ assign, int32_t *__restrict__ rank,
                                                   int fresh_only) {
    extern __shared__ int32_t hist[];
    // no early return: this kernel may fail the call while other waves of the
    // block are still starting, and every thread must reach the block's
    // barriers; a failed call's counts are cleared by the admission kernel
    const bool failed = call_failed(S.ctl);
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool active = i < n && !failed;
    const int64_t u = active ? ids[i] : 0;
    bool win = active && S.mark[u] == i;
    int l = win ? assign[i] : 0;
    // a row with no valid list (non-finite input) fails the whole call
    const bool bad = win && (unsigned)l >= (unsigned)S.nlist;
    if (ballot(bad) && lane_id() == 0) fail_call(S.ctl, -1);
    if (bad) {
        win = false;
        l = 0;
    }
    const int r = list_agg_inc<BLK>(S.l_acnt, l, win, hist, S.nlist, true);
    if (active) rank[i] = win ? r : -1;
    const uint32_t g = win ? S.att[u] : INVALID;
    const bool live = g != INVALID;
    // with compacting deletes only (the host tier, whose positions index no
    // device slab, needs lazy deletes)
    const int lo = (live && !S.bits) ? S.sowner[g / (uint32_t)S.C] : 0;
    // an upsert frees a position only with compacting deletes (a lazy delete leaves a dead slot)
    list_agg_inc<BLK>(S.l_prem, lo, live && !S.bits, hist, S.nlist, false);
    if (ballot(live) && lane_id() == 0) {
        if (fresh_only)
            fail_call(S.ctl, -6);
        else
            atomicExch(&S.ctl[CTL_UPSERT], S.ctl[CTL_SEQ]);
    }
}

// One block: does the final state fit in the pool?  Also clears the per-list
// counts of a call that already failed (k_add_count may have counted part of
// the batch before the failure was raised).
__global__ __launch_bounds__(1024) void k_add_admit(Dev S) {
    __shared__ long long sred[16];
    const int tid = threadIdx.x;
    if (call_failed(S.ctl)) {
        for (int l = tid; l < S.nlist; l += 1024) {
            S.l_prem[l] = 0;
            S.l_acnt[l] = 0;
        }
        return;
    }
    long long need = 0;
    for (int l = tid; l < S.nlist; l += 1024) need += cdiv(S.len[l] - S.l_prem[l] + S.l_acnt[l], S.C);
    for (int o = 32; o > 0; o >>= 1) need += __shfl_xor(need, o);
    if (lane_id() == 0) sred[tid >> 6] = need;
    __syncthreads();
    long long tot = 0;
    for (int w = 0; w < 16; w++) tot += sred[w];
    const bool reject = tot > S.num_slabs;
    if (reject && tid == 0) fail_call(S.ctl, -2);
    if (tid == 0) S.ctl[CTL_EBASE] = 0;
    for (int l = tid; l < S.nlist; l += 1024) {
        S.l_prem[l] = 0;
        if (reject) S.l_acnt[l] = 0;
    }
}

// Find the entry i of a block-local exclusive scan es[0..255] whose range
// [es[i], es[i] + cnt[i]) holds s: the last index with es[i] <= s.
__device__ __forceinline__ int owner_of(const int *es, int s) {
    int lo = 0, hi = 255;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (es[mid] <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_add_alloc(Dev S) {
    __shared__ int s_es[256], s_nso[256], sbuf[4], s_base[3];
    if (call_failed(S.ctl)) return;
    const int tid = threadIdx.x;
    const int l = blockIdx.x * 256 + tid;
    const bool valid = l < S.nlist;
    const int cnt = valid ? S.l_acnt[l] : 0;
    const int oldlen = valid ? S.len[l] : 0;
    const int newlen = oldlen + cnt;
    const int nso = cdiv(oldlen, S.C), nsn = cdiv(newlen, S.C);
    const int pgo = cdiv(nso, PAGE), pgn = cdiv(nsn, PAGE);
    int tot_s, tot_p, tot_e;
    const int es = block_excl_scan<256>(nsn - nso, sbuf, &tot_s);
    const int ep = block_excl_scan<256>(pgn - pgo, sbuf, &tot_p);
    const int ee = block_excl_scan<256>(cnt, sbuf, &tot_e);
    if (tid == 0) {
        s_base[0] = tot_s ? atomicSub(&S.ctl[CTL_SLAB_TOP], tot_s) - tot_s : 0;
        s_base[1] = tot_p ? atomicSub(&S.ctl[CTL_PAGE_TOP], tot_p) - tot_p : 0;
        s_base[2] = tot_e ? atomicAdd(&S.ctl[CTL_EBASE], tot_e) : 0;   // this block's lists' new entries
    }
    s_es[tid] = es;
    s_nso[tid] = nso;
    __syncthreads();
    if (cnt > 0) {
        S.l_base[l] = oldlen;
        S.l_eoff[l] = s_base[2] + ee;
        S.len[l] = newlen;
        S.l_acnt[l] = 0;
        for (int j = 0; j < pgn - pgo; j++)
            S.dir[(int64_t)l * S.dir_cap + pgo + j] = S.free_pages[s_base[1] + ep + j];
    }
    __syncthreads();
    for (int s = tid; s < tot_s; s += 256) {
        const int i = owner_of(s_es, s);
        const int li = blockIdx.x * 256 + i;
        const int ord = s_nso[i] + (s - s_es[i]);
        const int slab = S.free_slabs[s_base[0] + s];
        const int page = S.dir[(int64_t)li * S.dir_cap + ord / PAGE];
        S.pages[(int64_t)page * PAGE + ord % PAGE] = slab;
        S.sowner[slab] = li;
        S.sord[slab] = ord;
    }
}

// Entry order of the new entries: entry l_eoff[l] + rank is list l's rank-th
// new position; inv[entry] = its source row.
__global__ __launch_bounds__(256) void k_add_inv(Dev S, int n, const int32_t *__restrict__ assign,
                                                 const int32_t *__restrict__ rank, int32_t *__restrict__ inv,
                                                 uint32_t *__restrict__ dstg) {
    if (call_failed(S.ctl)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int r = rank[i];
    if (r < 0) return;
    // the entry's destination slot, resolved here (many rows in flight) so
    // that the copy kernel starts from two independent loads
    const int l = assign[i];
    const int e = S.l_eoff[l] + r;
    const int pos = S.l_base[l] + r;
    inv[e] = i;
    dstg[e] = (uint32_t)slab_of(S, l, pos / S.C) * (uint32_t)S.C + (uint32_t)(pos % S.C);
}

// One lane per new entry, in entry order: consecutive lanes fill consecutive
// slots of a list, so each 16-byte dimension chunk of 64 entries is one
// contiguous KiB write; the lane reads its source row in order.
template <bool VEC>
__global__ __launch_bounds__(256) void k_add_scatter(Dev S, const float *__restrict__ x,
                                                     const int64_t *__restrict__ ids,
                                                     const int32_t *__restrict__ assign,
                                                     const int32_t *__restrict__ rank,
                                                     const int32_t *__restrict__ inv) {
    if (call_failed(S.ctl)) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= S.ctl[CTL_EBASE]) return;
    const int i = inv[e];
    const int l = assign[i];
    const int pos = S.l_base[l] + rank[i];
    const int slab = slab_of(S, l, pos / S.C);
    const int slot = pos % S.C;
    float4 *dst = S.data + (int64_t)slab * S.dp4 * S.C + slot;
    const float *xr = x + (int64_t)i * S.d;
    float n32 = 0.f;   // fp32 squared norm (fp32 storage)
    for (int c = 0; c < S.dp4; c++) {
        float4 v;
        if (VEC) {
            v = reinterpret_cast<const float4 *>(xr)[c];
        } else {
            const int j = 4 * c;
            v.x = j < S.d ? xr[j] : 0.f;
            v.y = j + 1 < S.d ? xr[j + 1] : 0.f;
            v.z = j + 2 < S.d ? xr[j + 2] : 0.f;
            v.w = j + 3 < S.d ? xr[j + 3] : 0.f;
        }
        dst[(int64_t)c * S.C] = v;
        n32 = fmaf(v.x, v.x, n32);
        n32 = fmaf(v.y, v.y, n32);
        n32 = fmaf(v.z, v.z, n32);
        n32 = fmaf(v.w, v.w, n32);
    }
    const uint32_t g = (uint32_t)slab * (uint32_t)S.C + (uint32_t)slot;
    if (S.storage == 0) S.xnorm[g] = n32;
    if (S.storage != 0) {
        // reduced-precision copy (round to nearest even), 8 dims per chunk,
        // and the fp32 squared norm of the rounded row (L2 scan epilogue)
        uint4 *hdst = S.hdata + (int64_t)slab * S.dp8 * S.C + slot;
        float nrm = 0.f;
        for (int c = 0; c < S.dp8; c++) {
            uint32_t h[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int j = 8 * c + q;
                const float v = j < S.d ? xr[j] : 0.f;
                h[q] = S.storage == 1 ? to_bf16_bits(v) : to_f16_bits(v);
                const float r = S.storage == 1 ? bf16_bits_to_float(h[q]) : f16_bits_to_float(h[q]);
                nrm = fmaf(r, r, nrm);
            }
            hdst[(int64_t)c * S.C] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                                h[6] | (h[7] << 16));
        }
        if (S.xnorm) S.xnorm[g] = nrm;
    }
    {
        const int64_t u = ids[i];
        S.sids[g] = (uint32_t)u;
        S.att[u] = g;
    }
    if (S.bits) publish_slot(S, slab, slot);
}

// LDS-staged form of the scatter (rows of at most 64 chunks, 16-byte aligned):
// one wave per SENT consecutive new entries.  The wave first reads the
// entries' source rows whole (consecutive lanes read consecutive chunks of a
// row) into LDS, then writes chunk c of every entry (consecutive lanes,
// consecutive slots), so reads and writes are both contiguous runs.  16
// entries per wave keep the staging area at 8.25 KiB (d = 128), so that many
// waves per CU have loads in flight.
constexpr int SENT = 16;

__global__ __launch_bounds__(64) void k_add_scatter_lds(Dev S, const float *__restrict__ x,
                                                         const int64_t *__restrict__ ids,
                                                         const int32_t *__restrict__ inv,
                                                         const uint32_t *__restrict__ dstg) {
    extern __shared__ __align__(16) float4 srow[];   // [SENT][dp4 + 1]
    if (call_failed(S.ctl)) return;
    const int lane = threadIdx.x;
    const int e0 = blockIdx.x * SENT;
    const int nent = S.ctl[CTL_EBASE];
    if (e0 >= nent) return;
    const int cnt = min(SENT, nent - e0);
    const int dp4 = S.dp4, ld = dp4 + 1;
    // entry lane (lane < cnt): source row, destination slab and slot
    int i = 0, slab = 0, slot = 0;
    if (lane < cnt) {
        i = inv[e0 + lane];
        const uint32_t g = dstg[e0 + lane];
        slab = (int)(g / (uint32_t)S.C);
        slot = (int)(g % (uint32_t)S.C);
    }
    // rows into LDS: 8 chunks per lane in flight (all of a 128-dim batch)
    const int tot = cnt * dp4;
    for (int f0 = 0; f0 < tot; f0 += 8 * WAVE) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int f = min(f0 + u * WAVE + lane, tot - 1);   // past the end: re-read the last chunk
            const int r = f / dp4;
            const int src = __shfl(i, r);
            v[u] = reinterpret_cast<const float4 *>(x + (int64_t)src * S.d)[f - r * dp4];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int f = f0 + u * WAVE + lane;
            const int r = f / dp4;
            if (f < tot) srow[r * ld + (f - r * dp4)] = v[u];
        }
    }
    __syncthreads();
    // chunk c of entry e: lanes e + SENT * h take chunks h, h + WAVE / SENT, ...
    {
        const int e = lane % SENT, h = lane / SENT;
        const int sl = __shfl(slab, e), so = __shfl(slot, e);
        if (e < cnt) {
            float4 *dst = S.data + (int64_t)sl * dp4 * S.C + so;
            for (int c = h; c < dp4; c += WAVE / SENT) dst[(int64_t)c * S.C] = srow[e * ld + c];
        }
    }
    if (lane < cnt) {
        const uint32_t g = (uint32_t)slab * (uint32_t)S.C + (uint32_t)slot;
        const float *row = reinterpret_cast<const float *>(srow + lane * ld);
        if (S.storage == 0) {
            float n32 = 0.f;   // fp32 squared norm, sequential over ascending dimensions
            for (int j = 0; j < 4 * dp4; j++) n32 = fmaf(row[j], row[j], n32);
            S.xnorm[g] = n32;
        } else {
            // reduced-precision copy (round to nearest even), 8 dims per chunk,
            // and the fp32 squared norm of the rounded row (L2 scan epilogue)
            uint4 *hdst = S.hdata + (int64_t)slab * S.dp8 * S.C + slot;
            float nrm = 0.f;
            for (int c = 0; c < S.dp8; c++) {
                uint32_t hb[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const int j = 8 * c + q;
                    const float v = j < S.d ? row[j] : 0.f;
                    hb[q] = S.storage == 1 ? to_bf16_bits(v) : to_f16_bits(v);
                    const float r = S.storage == 1 ? bf16_bits_to_float(hb[q]) : f16_bits_to_float(hb[q]);
                    nrm = fmaf(r, r, nrm);
                }
                hdst[(int64_t)c * S.C] = make_uint4(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16),
                                                    hb[4] | (hb[5] << 16), hb[6] | (hb[7] << 16));
            }
            if (S.xnorm) S.xnorm[g] = nrm;
        }
        const int64_t u = ids[i];
        S.sids[g] = (uint32_t)u;
        S.att[u] = g;
        if (S.bits) publish_slot(S, slab, slot);
    }
}

__global__ __launch_bounds__(256) void k_add_cleanup(Dev S, int n, const int64_t *__restrict__ ids) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t u = ids[i];
    if (u >= 0 && u < S.id_capacity) S.mark[u] = -1;
}

// ------------------------------------------------------------------ delete

__device__ __forceinline__ bool rm_skip(const Dev &S, int mode) {
    if (call_failed(S.ctl)) return true;
    return mode == 1 && S.ctl[CTL_UPSERT] != S.ctl[CTL_SEQ];
}

__global__ __launch_bounds__(256) void k_rm_validate(Dev S, int n, const int64_t *__restrict__ ids) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t u = ids[i];
    if (u < 0 || u >= S.id_capacity) fail_call(S.ctl, -3);
}

template <bool BLK>
__global__ __launch_bounds__(256) void k_rm_mark(Dev S, int n, const int64_t *__restrict__ ids,
                                                 uint32_t *__restrict__ rec, int mode) {
    extern __shared__ int32_t hist[];
    if (rm_skip(S, mode)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int64_t u = i < n ? ids[i] : -1;
    const bool active = u >= 0 && u < S.id_capacity;   // out-of-range ids: rejected before (mode 0) or skipped (mode 2)
    const uint32_t g = active ? atomicExch(&S.att[u], INVALID) : INVALID;
    const bool hit = g != INVALID;
    int l = 0;
    if (hit) {
        S.sids[g] = INVALID;   // tombstone: this slot no longer holds a live entry
        l = S.sowner[g / (uint32_t)S.C];
    }
    list_agg_inc<BLK>(S.l_m, l, hit, hist, S.nlist, false);
    if (i < n) rec[i] = g;
}

// One block: segment offsets of each list's survivor slots and new lengths.
__global__ __launch_bounds__(1024) void k_rm_plan(Dev S, int64_t *n_removed, int mode) {
    __shared__ int sbuf[16];
    if (rm_skip(S, mode)) {
        if (n_removed && threadIdx.x == 0) *n_removed = 0;
        return;
    }
    int carry = 0;
    for (int base = 0; base < S.nlist; base += 1024) {
        const int l = base + threadIdx.x;
        const int m = l < S.nlist ? S.l_m[l] : 0;
        int tot;
        const int ex = block_excl_scan<1024>(m, sbuf, &tot);
        if (l < S.nlist) {
            S.l_off[l] = carry + ex;
            S.l_newlen[l] = S.len[l] - m;
            S.l_q[l] = 0;
            S.l_s[l] = 0;
            S.l_h[l] = 0;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        S.ctl[CTL_RMTOT] = carry;
        if (n_removed) *n_removed = carry;
    }
}

// Holes: deleted positions below the new length n' of their list.  The h-th
// hole of list l (in any order) is stored at seg[l_off[l] + h].
template <bool BLK>
__global__ __launch_bounds__(256) void k_rm_holes(Dev S, int n, const uint32_t *__restrict__ rec,
                                                  int32_t *__restrict__ seg, int mode) {
    extern __shared__ int32_t hist[];
    if (rm_skip(S, mode)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const uint32_t g = i < n ? rec[i] : INVALID;
    const bool hit = g != INVALID;
    int l = 0;
    bool hole = false;
    if (hit) {
        const uint32_t slab = g / (uint32_t)S.C;
        l = S.sowner[slab];
        hole = S.sord[slab] * S.C + (int)(g % (uint32_t)S.C) < S.l_newlen[l];
    }
    const int h = list_agg_inc<BLK>(S.l_h, l, hole, hist, S.nlist, true);
    if (hole) seg[S.l_off[l] + h] = (int32_t)g;
}

// Tail-window entry -> list map for the move: entries l_off[l] .. +l_m[l]
// belong to list l.  One wave per list.
__global__ __launch_bounds__(256) void k_rm_expand(Dev S, int32_t *__restrict__ emap, int mode) {
    if (rm_skip(S, mode)) return;
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (l >= S.nlist) return;
    const int m = S.l_m[l], o = S.l_off[l];
    for (int j = lane_id(); j < m; j += 64) emap[o + j] = l;
}

// The tail windows [n', n) of all lists with deletions, list after list, one
// lane per position (the window of list l has l_m[l] positions and starts at
// entry l_off[l]).  A position that still holds a live entry is a survivor;
// the r-th survivor of a list moves into its r-th hole.  Consecutive lanes
// read consecutive slots, so each 16-byte dimension chunk of a wave's
// survivors is one contiguous read; the holes they fill are scattered.
template <bool HALF>
__global__ __launch_bounds__(256) void k_rm_move(Dev S, int n, const int32_t *__restrict__ seg,
                                                 const int32_t *__restrict__ emap, int mode) {
    if (rm_skip(S, mode)) return;
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int total = S.ctl[CTL_RMTOT];
    const bool active = e < total;
    const int l = active ? emap[e] : 0;
    uint32_t src = 0, id = INVALID;
    if (active) {
        const int tp = S.l_newlen[l] + (e - S.l_off[l]);
        src = (uint32_t)slab_of(S, l, tp / S.C) * (uint32_t)S.C + (uint32_t)(tp % S.C);
        id = S.sids[src];
        // compacting lazy deletes: the validity bit tells a dead slot (its id word is stale)
        if (S.bits && !((S.bits[(int64_t)(src / S.C) * S.bw + ((src % S.C) >> 6)] >> ((src % S.C) & 63)) & 1ull))
            id = INVALID;
    }
    const bool surv = id != INVALID;
    const int r = wave_agg_inc(S.l_s, l, surv);
    if (!surv) return;
    const uint32_t dst = (uint32_t)seg[S.l_off[l] + r];
    const int64_t ss = (int64_t)(src / S.C), sl = src % S.C, ds = (int64_t)(dst / S.C), dl = dst % S.C;
    const float4 *sp = S.data + ss * S.dp4 * S.C + sl;
    float4 *dp = S.data + ds * S.dp4 * S.C + dl;
    int c = 0;
    for (; c + 16 <= S.dp4; c += 16) {   // 16 chunks of the row in flight
        float4 v[16];
#pragma unroll
        for (int j = 0; j < 16; j++) v[j] = sp[(int64_t)(c + j) * S.C];
#pragma unroll
        for (int j = 0; j < 16; j++) dp[(int64_t)(c + j) * S.C] = v[j];
    }
    for (; c < S.dp4; c++) dp[(int64_t)c * S.C] = sp[(int64_t)c * S.C];
    if (HALF) {
        const uint4 *hs = S.hdata + ss * S.dp8 * S.C + sl;
        uint4 *hd = S.hdata + ds * S.dp8 * S.C + dl;
        for (int c8 = 0; c8 < S.dp8; c8++) hd[(int64_t)c8 * S.C] = hs[(int64_t)c8 * S.C];
    }
    if (S.xnorm) S.xnorm[dst] = S.xnorm[src];
    S.sids[dst] = id;
    S.att[id] = dst;
    if (S.bits)   // compaction of lazy deletes: the hole holds a live entry again
        atomicOr((unsigned long long *)(S.bits + ds * S.bw + (dl >> 6)), 1ull << (dl & 63));
}

// Per list: new length, and the tail slabs (and table pages) past the new
// end go back to the free stacks.
__global__ __launch_bounds__(256) void k_rm_finalize(Dev S, int mode) {
    __shared__ int s_es[256], s_nsn[256], sbuf[4], s_base[2];
    if (rm_skip(S, mode)) return;
    const int tid = threadIdx.x;
    const int l = blockIdx.x * 256 + tid;
    const bool valid = l < S.nlist;
    const int m = valid ? S.l_m[l] : 0;
    const int oldlen = valid ? S.len[l] : 0;
    const int nl = oldlen - m;
    const int nso = cdiv(oldlen, S.C), nsn = cdiv(nl, S.C);
    const int pgo = cdiv(nso, PAGE), pgn = cdiv(nsn, PAGE);
    int tot_s, tot_p;
    const int es = block_excl_scan<256>(nso - nsn, sbuf, &tot_s);
    const int ep = block_excl_scan<256>(pgo - pgn, sbuf, &tot_p);
    if (tid == 0) {
        s_base[0] = tot_s ? atomicAdd(&S.ctl[CTL_SLAB_TOP], tot_s) : 0;
        s_base[1] = tot_p ? atomicAdd(&S.ctl[CTL_PAGE_TOP], tot_p) : 0;
    }
    s_es[tid] = es;
    s_nsn[tid] = nsn;
    __syncthreads();
    for (int s = tid; s < tot_s; s += 256) {
        const int i = owner_of(s_es, s);
        const int li = blockIdx.x * 256 + i;
        const int ord = s_nsn[i] + (s - s_es[i]);
        const int slab = slab_of(S, li, ord);
        if (S.bits)   // validity words are reset before the slab goes back on the stack
            for (int w = 0; w < S.bw; w++) S.bits[(int64_t)slab * S.bw + w] = 0;
        S.free_slabs[s_base[0] + s] = slab;
        S.sowner[slab] = -1;
    }
    __syncthreads();
    if (m > 0) {
        if (S.bits && (nl % S.C) != 0) {
            // the last kept slab: slots past the new length hold no entry
            const int64_t slab = slab_of(S, l, nsn - 1);
            for (int s = nl % S.C; s < S.C; s++)
                S.bits[slab * S.bw + (s >> 6)] &= ~(1ull << (s & 63));
        }
        if (S.bits) S.l_dead[l] -= m;
        for (int j = 0; j < pgo - pgn; j++)
            S.free_pages[s_base[1] + ep + j] = S.dir[(int64_t)l * S.dir_cap + pgn + j];
        S.len[l] = nl;
        S.l_m[l] = 0;
    }
}

// ------------------------------------------------------------ lazy deletes

__global__ void k_rm_lazy_begin(int32_t *ctl) {
    if (threadIdx.x == 0) ctl[CTL_RMTOT] = 0;
}

// The paper's eviction (Alg. 4): the address-table exchange finds the slot in
// O(1) and makes exactly one thread own the id; the atomic AND clears its
// validity bit, and the old word shows the 1 -> 0 transition that counts the
// removal (Theorem 3).  Nothing moves; the slot stays dead until compaction.
// An entry in the host tier loses its bit in the device-resident cold bitmap
// the same way.
template <bool BLK>
__global__ __launch_bounds__(256) void k_rm_lazy(Dev S, int n, const int64_t *__restrict__ ids, int mode) {
    extern __shared__ int32_t hist[];
    if (rm_skip(S, mode == 1 ? 1 : 0)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int64_t u = i < n ? ids[i] : -1;
    const bool active = u >= 0 && u < S.id_capacity;
    const uint32_t g = active ? atomicExch(&S.att[u], INVALID) : INVALID;
    bool gone = false, cold = false;
    int l = 0;
    if (g != INVALID) {
        cold = (g & COLD_BIT) != 0;
        const uint32_t pos = g & ~COLD_BIT;
        const int64_t slab = pos / (uint32_t)S.C;
        const int slot = (int)(pos % (uint32_t)S.C);
        const uint64_t bit = 1ull << (slot & 63);
        const uint64_t old = __hip_atomic_fetch_and((cold ? S.cbits : S.bits) + slab * S.bw + (slot >> 6), ~bit,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        gone = (old & bit) != 0;
        l = cold ? S.csowner[slab] : S.sowner[slab];
    }
    list_agg_inc<BLK>(S.l_dead, l, gone && !cold, hist, S.nlist, false);
    if (gone && cold) atomicAdd(&S.cdead[l], 1);
    const uint64_t gm = ballot(gone);
    if (gm && lane_id() == __builtin_ctzll(gm)) atomicAdd(&S.ctl[CTL_RMTOT], (int)__builtin_popcountll(gm));
}

__global__ void k_rm_lazy_end(Dev S, int64_t *n_removed) {
    if (threadIdx.x == 0) *n_removed = call_failed(S.ctl) ? 0 : S.ctl[CTL_RMTOT];
}

// ------------------------------------------------------------ compaction

// One block.  List l is compacted when its dead slots are at least
// frac * len (and > 0); lists in order take dead slots out of the budget, the
// last one partly: m' of its dead slots are removed (n' = len - m'), the
// others stay dead.  Then as k_rm_plan: tail-window offsets, new lengths.
__global__ __launch_bounds__(1024) void k_cmp_plan(Dev S, float frac, int budget, int64_t *n_compacted) {
    __shared__ int sbuf[16];
    int carry = 0;
    for (int base = 0; base < S.nlist; base += 1024) {
        const int l = base + threadIdx.x;
        int want = 0;
        if (l < S.nlist) {
            const int dead = S.l_dead[l];
            want = (dead > 0 && (float)dead >= frac * (float)S.len[l]) ? dead : 0;
        }
        int tot;
        const int ex = block_excl_scan<1024>(want, sbuf, &tot);
        const int room = budget - carry - ex;
        const int m = want < room ? want : (room > 0 ? room : 0);
        int tot_m;
        const int exm = block_excl_scan<1024>(m, sbuf, &tot_m);
        if (l < S.nlist) {
            S.l_m[l] = m;
            S.l_off[l] = carry + exm;
            S.l_newlen[l] = S.len[l] - m;
            S.l_q[l] = 0;
            S.l_s[l] = 0;
            S.l_h[l] = 0;
        }
        carry += tot_m;
    }
    if (threadIdx.x == 0) {
        S.ctl[CTL_RMTOT] = carry;
        if (n_compacted) *n_compacted = carry;
    }
}

// Dead slots in each compacted list's tail window [n', len): l_q[l].
__global__ __launch_bounds__(256) void k_cmp_tail(Dev S, const int32_t *__restrict__ emap) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int total = S.ctl[CTL_RMTOT];
    const bool active = e < total;
    int l = 0;
    bool dead = false;
    if (active) {
        l = emap[e];
        const int tp = S.l_newlen[l] + (e - S.l_off[l]);
        const int slab = slab_of(S, l, tp / S.C), slot = tp % S.C;
        dead = !((S.bits[(int64_t)slab * S.bw + (slot >> 6)] >> (slot & 63)) & 1ull);
    }
    wave_agg_inc(S.l_q, l, dead);
}

// Holes: dead slots below n'.  A compacted list needs one per survivor of its
// tail window (m' - tail dead); any that many of its dead slots will do, the
// others stay dead.  One thread per slab.
__global__ __launch_bounds__(256) void k_cmp_holes(Dev S, int32_t *__restrict__ seg) {
    const int64_t slab = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slab >= S.num_slabs) return;
    const int l = S.sowner[slab];
    if (l < 0 || S.l_m[l] == 0) return;
    const int need = S.l_m[l] - S.l_q[l];
    const int nl = S.l_newlen[l];
    const int p0 = S.sord[slab] * S.C;
    for (int s = 0; s < S.C && p0 + s < nl; s++) {
        const uint32_t g = (uint32_t)slab * (uint32_t)S.C + (uint32_t)s;
        if ((S.bits[slab * S.bw + (s >> 6)] >> (s & 63)) & 1ull) continue;   // live
        const int h = atomicAdd(&S.l_h[l], 1);
        if (h >= need) break;
        seg[S.l_off[l] + h] = (int32_t)g;
    }
}


__global__ __launch_bounds__(256) void k_get_rows(Dev S, int n, const int64_t *__restrict__ ids,
                                                  float *__restrict__ rows) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int i = gid >> 4, sub = gid & 15;
    if (i >= n) return;
    const int64_t u = ids[i];
    const uint32_t g = (u >= 0 && u < S.id_capacity) ? S.att[u] : INVALID;
    float *out = rows + (int64_t)i * S.d;
    if (g == INVALID) {
        for (int j = sub; j < S.d; j += 16) out[j] = __int_as_float(0x7FC00000);
        return;
    }
    const uint32_t pos = g & ~COLD_BIT;   // a host-tier entry reads its row from host memory
    const float4 *src = ((g & COLD_BIT) ? S.cdata : S.data) + (int64_t)(pos / S.C) * S.dp4 * S.C + pos % S.C;
    for (int c = sub; c < S.dp4; c += 16) {
        const float4 v = src[(int64_t)c * S.C];
        const float e[4] = {v.x, v.y, v.z, v.w};
        for (int t = 0; t < 4; t++)
            if (4 * c + t < S.d) out[4 * c + t] = e[t];
    }
}

// Checkpoint packing: entries [e0, e0 + n) of all lists in list order (list
// l's entries are e in [off[l], off[l + 1]), positions ascending; with a host
// tier (tier = 1) its cold segment, viewed as Sc, follows its len[l] device
// positions) -> fp32 rows (d floats each) and ids.  One wave per entry.
__global__ __launch_bounds__(256) void k_pack(Dev S, Dev Sc, int tier, const int32_t *__restrict__ off, int64_t e0,
                                              int n, float *__restrict__ rows, uint32_t *__restrict__ ids) {
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (i >= n) return;
    const int64_t e = e0 + i;
    int lo = 0, hi = S.nlist - 1;
    while (lo < hi) {   // the last list whose entries start at or before e
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    int p = (int)(e - off[lo]);
    const bool cold = tier && p >= S.len[lo];
    if (cold) p -= S.len[lo];
    const int slab = cold ? slab_of(Sc, lo, p / S.C) : slab_of(S, lo, p / S.C), slot = p % S.C;
    const float4 *src = (cold ? Sc.data : S.data) + (int64_t)slab * S.dp4 * S.C + slot;
    const uint64_t *bits = cold ? Sc.bits : S.bits;
    const uint32_t *sids = cold ? Sc.sids : S.sids;
    float *out = rows + (int64_t)i * S.d;
    for (int c = lane_id(); c < S.dp4; c += 64) {
        const float4 v = src[(int64_t)c * S.C];
        const float ev[4] = {v.x, v.y, v.z, v.w};
        for (int t = 0; t < 4; t++)
            if (4 * c + t < S.d) out[4 * c + t] = ev[t];
    }
    if (lane_id() == 0) {
        const bool live = !bits || ((bits[(int64_t)slab * S.bw + (slot >> 6)] >> (slot & 63)) & 1ull);
        ids[i] = live ? sids[(int64_t)slab * S.C + slot] : INVALID;
    }
}

// ------------------------------------------------------------ host tier
//
// The cold pool is a second slab pool in the device pool's layout, held in
// pinned host memory (rows, ids) with its bookkeeping on the device; Sc is
// the device struct viewing it (its per-list scratch arrays are the device
// pool's).  Offloading a list moves every position of it to the end of the
// list's cold segment: the add allocator on Sc gives the cold slabs, a copy
// moves rows, ids and validity bits and points live ids' address-table
// entries at their cold positions, and the remove finalizer releases the
// list's device slabs.

// One block: per offloaded list, its positions as the cold allocation and as
// the device-pool release.
__global__ __launch_bounds__(1024) void k_tier_plan(Dev S, Dev Sc, const int32_t *__restrict__ olist, int n) {
    for (int i = threadIdx.x; i < n; i += 1024) {
        const int l = olist[i];
        const int cnt = S.len[l];
        S.l_acnt[l] = cnt;              // new cold positions (the add allocator on the cold view)
        S.l_m[l] = cnt;                 // every device position leaves (the remove finalizer)
        Sc.l_dead[l] += S.l_dead[l];    // dead slots move along, still dead
        S.l_dead[l] = cnt;              // the finalizer subtracts the positions it releases
    }
    if (threadIdx.x == 0) Sc.ctl[CTL_EBASE] = 0;
}

// Grid (ceil(longest / 256), lists): one thread per position of an offloaded
// list; position p goes to cold position l_base[l] + p (after the segment's
// earlier entries).  Runs before the device slabs are released.
__global__ __launch_bounds__(256) void k_tier_copy(Dev S, Dev Sc, const int32_t *__restrict__ olist) {
    const int l = olist[blockIdx.y];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= S.len[l]) return;
    const int C = S.C;
    const int hs = slab_of(S, l, p / C), hsl = p % C;
    const int cp = S.l_base[l] + p;
    const int cs = slab_of(Sc, l, cp / C), csl = cp % C;
    const float4 *src = S.data + (int64_t)hs * S.dp4 * C + hsl;
    float4 *dst = Sc.data + (int64_t)cs * S.dp4 * C + csl;
    for (int c = 0; c < S.dp4; c++) dst[(int64_t)c * C] = src[(int64_t)c * C];
    const uint32_t id = S.sids[(int64_t)hs * C + hsl];
    Sc.sids[(int64_t)cs * C + csl] = id;
    if ((S.bits[(int64_t)hs * S.bw + (hsl >> 6)] >> (hsl & 63)) & 1ull) {   // live: its id now lives in the tier
        atomicOr((unsigned long long *)(Sc.bits + (int64_t)cs * S.bw + (csl >> 6)), 1ull << (csl & 63));
        S.att[id] = COLD_BIT | ((uint32_t)cs * (uint32_t)C + (uint32_t)csl);
    }
}

// One block: cold segments with no live entry left leave whole (the remove
// finalizer on the cold view releases their slabs); the number of released
// positions goes to *n_out.
__global__ __launch_bounds__(1024) void k_tier_reclaim_plan(Dev Sc, int64_t *n_out) {
    __shared__ long long sred[16];
    long long tot = 0;
    for (int l = threadIdx.x; l < Sc.nlist; l += 1024) {
        const int n = Sc.len[l];
        const bool dead = n > 0 && Sc.l_dead[l] == n;
        Sc.l_m[l] = dead ? n : 0;
        tot += dead ? n : 0;
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if (lane_id() == 0) sred[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < 16; w++) t += sred[w];
        *n_out = t;
    }
}

// Last kernel of an add or remove call: the next call gets a new sequence number.
__global__ void k_call_end(int32_t *ctl) {
    if (threadIdx.x == 0) ctl[CTL_SEQ] = ctl[CTL_SEQ] + 1;
}

// ------------------------------------------------------------------ launch

static unsigned blocks(int64_t threads, int per = 256) { return (unsigned)((threads + per - 1) / per); }

// Per-list LDS histograms when nlist ints fit in 64 KiB.
static bool blk_hist(const Dev &S) { return S.nlist <= 16384; }
static size_t hist_bytes(const Dev &S) { return blk_hist(S) ? (size_t)S.nlist * 4 : 0; }
#define SIVF_LAUNCH_BLK(K, grid, st, S, ...)                                                                  \
    do {                                                                                                     \
        if (blk_hist(S))                                                                                     \
            hipLaunchKernelGGL(K<true>, dim3(grid), dim3(256), hist_bytes(S), st, S, __VA_ARGS__);          \
        else                                                                                                 \
            hipLaunchKernelGGL(K<false>, dim3(grid), dim3(256), 0, st, S, __VA_ARGS__);                     \
    } while (0)

void launch_add_prepare(hipStream_t st, const Dev &S, int n, const int64_t *ids) {
    hipLaunchKernelGGL(k_add_prepare, dim3(blocks(n)), dim3(256), 0, st, S, n, ids);
}

void launch_add_count(hipStream_t st, const Dev &S, int n, const int64_t *ids, const Batch &B, int fresh_only) {
    SIVF_LAUNCH_BLK(k_add_count, blocks(n), st, S, n, ids, B.assign, B.rank, fresh_only);
}

void launch_add_admit(hipStream_t st, const Dev &S) {
    hipLaunchKernelGGL(k_add_admit, dim3(1), dim3(1024), 0, st, S);
}

void launch_add_alloc(hipStream_t st, const Dev &S) {
    hipLaunchKernelGGL(k_add_alloc, dim3(blocks(S.nlist)), dim3(256), 0, st, S);
}

void launch_add_scatter(hipStream_t st, const Dev &S, int n, const float *x, const int64_t *ids, const Batch &B) {
    // B.rec (free during an add once its upsert deletes are done) takes each entry's destination slot
    hipLaunchKernelGGL(k_add_inv, dim3(blocks(n)), dim3(256), 0, st, S, n, B.assign, B.rank, B.inv, B.rec);
    const bool vec = (S.d % 4 == 0) && (((uintptr_t)x & 15) == 0);
    if (vec && S.dp4 <= 64)
        hipLaunchKernelGGL(k_add_scatter_lds, dim3(blocks(n, SENT)), dim3(64),
                           (size_t)SENT * (S.dp4 + 1) * sizeof(float4), st, S, x, ids, B.inv, B.rec);
    else if (vec)
        hipLaunchKernelGGL(k_add_scatter<true>, dim3(blocks(n)), dim3(256), 0, st, S, x, ids, B.assign, B.rank,
                           B.inv);
    else
        hipLaunchKernelGGL(k_add_scatter<false>, dim3(blocks(n)), dim3(256), 0, st, S, x, ids, B.assign, B.rank,
                           B.inv);
}

void launch_add_cleanup(hipStream_t st, const Dev &S, int n, const int64_t *ids) {
    hipLaunchKernelGGL(k_add_cleanup, dim3(blocks(n)), dim3(256), 0, st, S, n, ids);
}

void launch_remove(hipStream_t st, const Dev &S, int n, const int64_t *ids, int64_t *n_removed, const Batch &B, int mode) {
    if (mode == 0) hipLaunchKernelGGL(k_rm_validate, dim3(blocks(n)), dim3(256), 0, st, S, n, ids);
    SIVF_LAUNCH_BLK(k_rm_mark, blocks(n), st, S, n, ids, B.rec, mode);
    hipLaunchKernelGGL(k_rm_plan, dim3(1), dim3(1024), 0, st, S, n_removed, mode);
    SIVF_LAUNCH_BLK(k_rm_holes, blocks(n), st, S, n, B.rec, B.seg, mode);
    hipLaunchKernelGGL(k_rm_expand, dim3(blocks(S.nlist, 4)), dim3(256), 0, st, S, B.inv, mode);
    if (S.storage != 0)
        hipLaunchKernelGGL(k_rm_move<true>, dim3(blocks(n)), dim3(256), 0, st, S, n, B.seg, B.inv, mode);
    else
        hipLaunchKernelGGL(k_rm_move<false>, dim3(blocks(n)), dim3(256), 0, st, S, n, B.seg, B.inv, mode);
    hipLaunchKernelGGL(k_rm_finalize, dim3(blocks(S.nlist)), dim3(256), 0, st, S, mode);
}

void launch_remove_lazy(hipStream_t st, const Dev &S, int n, const int64_t *ids, int64_t *n_removed, int mode) {
    if (mode == 0) hipLaunchKernelGGL(k_rm_validate, dim3(blocks(n)), dim3(256), 0, st, S, n, ids);
    if (mode != 1) hipLaunchKernelGGL(k_rm_lazy_begin, dim3(1), dim3(64), 0, st, S.ctl);
    SIVF_LAUNCH_BLK(k_rm_lazy, blocks(n), st, S, n, ids, mode);
    if (mode != 1 && n_removed) hipLaunchKernelGGL(k_rm_lazy_end, dim3(1), dim3(64), 0, st, S, n_removed);
}

void launch_compact(hipStream_t st, const Dev &S, float min_dead_fraction, int budget, int64_t *n_compacted,
                    const Batch &B) {
    hipLaunchKernelGGL(k_cmp_plan, dim3(1), dim3(1024), 0, st, S, min_dead_fraction, budget, n_compacted);
    hipLaunchKernelGGL(k_rm_expand, dim3(blocks(S.nlist, 4)), dim3(256), 0, st, S, B.inv, 0);
    hipLaunchKernelGGL(k_cmp_tail, dim3(blocks(budget)), dim3(256), 0, st, S, B.inv);
    hipLaunchKernelGGL(k_cmp_holes, dim3(blocks(S.num_slabs)), dim3(256), 0, st, S, B.seg);
    if (S.storage != 0)
        hipLaunchKernelGGL(k_rm_move<true>, dim3(blocks(budget)), dim3(256), 0, st, S, budget, B.seg, B.inv, 0);
    else
        hipLaunchKernelGGL(k_rm_move<false>, dim3(blocks(budget)), dim3(256), 0, st, S, budget, B.seg, B.inv, 0);
    hipLaunchKernelGGL(k_rm_finalize, dim3(blocks(S.nlist)), dim3(256), 0, st, S, 0);
}

void launch_call_end(hipStream_t st, const Dev &S) {
    hipLaunchKernelGGL(k_call_end, dim3(1), dim3(64), 0, st, S.ctl);
}

void launch_pack(hipStream_t st, const Dev &S, const Dev *Sc, const int32_t *off, int64_t e0, int n, float *rows,
                 uint32_t *ids) {
    if (n > 0)
        hipLaunchKernelGGL(k_pack, dim3((n + 3) / 4), dim3(256), 0, st, S, Sc ? *Sc : S, Sc ? 1 : 0, off, e0, n,
                           rows, ids);
}

void launch_tier_offload(hipStream_t st, const Dev &S, const Dev &Sc, const int32_t *olist, int n, int longest) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tier_plan, dim3(1), dim3(1024), 0, st, S, Sc, olist, n);
    hipLaunchKernelGGL(k_add_alloc, dim3(blocks(S.nlist)), dim3(256), 0, st, Sc);
    if (longest > 0)
        hipLaunchKernelGGL(k_tier_copy, dim3(blocks(longest), (unsigned)n), dim3(256), 0, st, S, Sc, olist);
    hipLaunchKernelGGL(k_rm_finalize, dim3(blocks(S.nlist)), dim3(256), 0, st, S, 0);
}

void launch_tier_reclaim(hipStream_t st, const Dev &Sc, int64_t *n_out) {
    hipLaunchKernelGGL(k_tier_reclaim_plan, dim3(1), dim3(1024), 0, st, Sc, n_out);
    hipLaunchKernelGGL(k_rm_finalize, dim3(blocks(Sc.nlist)), dim3(256), 0, st, Sc, 0);
}

void launch_get_rows(hipStream_t st, const Dev &S, int n, const int64_t *ids, float *rows) {
    hipLaunchKernelGGL(k_get_rows, dim3(blocks((int64_t)n * 16)), dim3(256), 0, st, S, n, ids, rows);
}

}  // namespace sivf
