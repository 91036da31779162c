// Device-side definitions shared by the SIVF kernels (gfx950, wave64).
//
// Index state in the caller's workspace (all offsets 256-byte aligned):
//   slab pool     data   [num_slabs][dp4][C] float4   (dp4 = ceil(d / 4))
//                 sids   [num_slabs][C]      uint32   (id of each slot)
//                 sowner [num_slabs]         int32    (list holding the slab, -1 = free)
//                 sord   [num_slabs]         int32    (ordinal of the slab in its list)
//   free stacks   free_slabs[num_slabs], free_pages[num_pages]; tops in ctl[]
//   list tables   dir[nlist][dir_cap] -> page id; pages[num_pages][PAGE] -> slab id
//                 len[nlist]: entries of each list; a list of n entries holds
//                 ceil(n / C) slabs and its entries sit densely at positions 0..n-1
//   address table att[id_capacity] = slab * C + slot, or INVALID
//
// Within a slab, slot s keeps dimension chunk c (4 floats) at data[slab][c][s]:
// 64 lanes mapped to 64 consecutive slots load one contiguous KiB per chunk.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sivf {

constexpr uint32_t INVALID = 0xFFFFFFFFu;   // empty address-table entry / tombstoned slot
// Address-table flag of an entry in the host tier: the low 31 bits are its
// position (slab * C + slot) in the cold pool.
constexpr uint32_t COLD_BIT = 0x80000000u;
constexpr int PAGE = 256;                   // slab ids per page of a list table
constexpr int WAVE = 64;

// Slots of the control block (int32).
enum Ctl {
    CTL_SLAB_TOP = 0,   // entries on the free slab stack
    CTL_PAGE_TOP = 1,   // entries on the free page stack
    CTL_STATUS = 2,     // first data-dependent error since the last sync
    CTL_GATE = 3,       // sequence number of the call that failed (its later kernels skip)
    CTL_UPSERT = 4,     // sequence number of the add call that holds live ids
    CTL_NITEMS = 5,     // search: work items of the current call
    CTL_SEQ = 6,        // sequence number of the current add/remove call; its last kernel bumps it
    CTL_CHUNK = 7,      // search: log2 of the positions per work item (a list's chunk)
    CTL_EBASE = 8,      // add: new entries handed out so far (per-list entry offsets)
    CTL_RMTOT = 9,      // remove: entries deleted by the current call (positions of all tail windows)
    CTL_XB = 16,        // search: first item of each XCD's range (words 16..24; word 24 = item count)
    CTL_WORK0 = 64,     // search, persistent schedule: 8 work counters, one per XCD range of items,
    CTL_WORK_STRIDE = 32,  // each on its own 128-byte line (words 64, 96, .., 288)
    CTL_WORDS = 320
};

struct Dev {
    int d, dp4, nlist, C, metric;
    int storage;          // 0 = fp32 slabs; 1 = bf16, 2 = fp16 slabs with the fp32 pool as shadow
    int dp8;              // ceil(d / 8): 16-byte chunks of a reduced-precision row
    int tile;             // search schedule: queries per work item (fp32 scan: 4 or 8; MFMA scan: 16)
    int chunk_shift;      // search schedule: a work item covers at most 2^chunk_shift list positions
    int persistent;       // search schedule: 0 = one wave per work item; 1 = resident waves pull items
    int64_t num_slabs, num_pages, dir_cap, id_capacity;
    const float *cent;    // [nlist][dp4*4], zero padded
    const uint16_t *cent_h;  // [nlist][dp4*4] bf16 copy (reduced-precision indexes: coarse GEMM operand)
    const float *cn2;     // [nlist] fp32 squared norms
    const double *cnorm;  // [nlist] fp64 norms
    const double *cmax;   // [1] largest centroid norm
    float4 *data;         // fp32 rows (the stored vectors, or the exact shadow)
    uint4 *hdata;         // [num_slabs][dp8][C] 8 x 16-bit (reduced-precision storage only)
    float *xnorm;         // [num_slabs * C] squared norm of the stored row: the fp32 row (fp32 storage)
                          // or the rounded row (reduced precision, L2); NULL otherwise
    uint32_t *sids;
    int32_t *sowner, *sord;
    int32_t *free_slabs, *free_pages, *pages, *dir;
    int32_t *len;
    uint32_t *att;
    int32_t *mark;
    int32_t *ctl;
    // per-list scratch (nlist each)
    int32_t *l_acnt, *l_prem, *l_base, *l_eoff;      // add
    int32_t *l_m, *l_off, *l_newlen, *l_q, *l_s, *l_h; // remove
    int32_t *l_qc, *l_qcs, *l_qoff;                  // search
    int32_t *l_snap;   // search: list lengths when the search was planned (it scans only these)
    int32_t *l_pbase;  // search: first partial-result slot of the list's (pair, chunk) results
    int32_t *l_ioff;   // search: first work item of the list
    int32_t *l_dead;   // lazy deletes: dead slots of each list below its length
    // Lazy deletes (NULL with compacting deletes): validity bit of every slot,
    // bw = ceil(C / 64) words per slab; bit s % 64 of word s / 64 is slot s.
    uint64_t *bits;
    int bw;
    // Host tier (all NULL without one): rows of cold entries (pinned host
    // memory), their validity bits, the owning list of each cold slab, and
    // each list's dead cold slots.  Cold entries are deleted lazily.
    const float4 *cdata;
    uint64_t *cbits;
    int32_t *csowner, *cdead;
};

// Validity word of slot `slot` of `slab` (lazy deletes), read with an atomic
// load at agent scope: a delete running on another XCD at the same time is
// seen as soon as its atomic AND is, not from a stale cached line.
__device__ __forceinline__ uint64_t valid_word(const Dev &S, int64_t slab, int slot) {
    return __hip_atomic_load(S.bits + slab * S.bw + (slot >> 6), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Validity of the 64 positions base .. base + 63 of a scan step (bit j:
// position base + j is below p1 and, with lazy deletes, live).  wslab/wbase:
// lane j holds the slab of ordinal wbase + j.  Every lane must call it.
__device__ __forceinline__ uint64_t step_valid(const Dev &S, int base, int p1, int wslab, int wbase, int cs, int cm) {
    const int lim = p1 - base;
    const uint64_t inr = lim >= 64 ? ~0ull : ((1ull << (lim > 0 ? lim : 0)) - 1);
    if (!S.bits) return inr;
    const int p = base + (int)__lane_id();
    const int pc = p < p1 ? p : p1 - 1;
    const int slab = __shfl(wslab, (pc >> cs) - wbase);
    const int slot = pc & cm;
    const bool ok = p < p1 && ((valid_word(S, slab, slot) >> (slot & 63)) & 1ull);
    return __ballot(ok);
}

// The 16 bits of a step mask that a lane of the MFMA scans owns: bit 4 rg + j
// is position 16 rg + 4 kgrp + j of the step (row group rg, lane group kgrp).
__device__ __forceinline__ uint32_t lane_valid16(uint64_t vm, int kgrp) {
    const uint64_t s = vm >> (4 * kgrp);
    return (uint32_t)((s & 0xFull) | ((s >> 12) & 0xF0ull) | ((s >> 24) & 0xF00ull) | ((s >> 36) & 0xF000ull));
}

__device__ __forceinline__ int slab_of(const Dev &S, int l, int ord) {
    int page = S.dir[(int64_t)l * S.dir_cap + ord / PAGE];
    return S.pages[(int64_t)page * PAGE + ord % PAGE];
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Lane i receives lane (i ^ J)'s value.  Strides 1, 2, 4, 8 stay inside a
// 16-lane row and use DPP (quad_perm, row_shl/row_shr, row_ror); 16 uses a
// ds_swizzle xor pattern and 32 a ds_bpermute.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    const int x = (int)v;
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else if constexpr (J == 4) {
        const int up = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xF, 0xF, false);    // row_shl:4 (from i+4)
        const int dn = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);    // row_shr:4 (from i-4)
        return (uint32_t)((lane_id() & 4) ? dn : up);
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (J == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401F);                     // xor 16 within 32
    } else {
        return (uint32_t)__shfl_xor(x, J);
    }
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane_u64(uint64_t v) {
    const uint32_t lo = xor_lane<J>((uint32_t)v), hi = xor_lane<J>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}


__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    int lo = __shfl((int)(uint32_t)v, src);
    int hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// fp32 -> bf16 / fp16 bits, round to nearest even.
__device__ __forceinline__ uint32_t to_bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0u;   // NaN stays NaN
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ uint32_t to_f16_bits(float f) {
    const _Float16 h = (_Float16)f;   // v_cvt_f16_f32: round to nearest even
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_bits_to_float(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float f16_bits_to_float(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

// Order-preserving map float -> uint32 (larger float, larger code).
__device__ __forceinline__ uint32_t ord_bits(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float from_ord(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(b);
}

// -0 and +0 are the same score: both rank as +0 (an inner product of tiny
// values whose sum rounds to zero from below is -0), so equal scores tie on
// the id as for every other value.
__device__ __forceinline__ float zero_sign(float v) { return v == 0.f ? 0.f : v; }

// Result ranking key: smaller key = better result; ties broken by smaller id.
// L2 ranks by ascending distance, IP by descending score.
__device__ __forceinline__ uint64_t make_key(float v, uint32_t id, int metric) {
    uint32_t hi = metric == 0 ? ord_bits(v) : ~ord_bits(zero_sign(v));
    return ((uint64_t)hi << 32) | id;
}
__device__ __forceinline__ float key_value(uint64_t key, int metric) {
    uint32_t hi = (uint32_t)(key >> 32);
    return metric == 0 ? from_ord(hi) : from_ord(~hi);
}

// Wave-aggregated atomicAdd of 1 per active lane on counters[key]: lanes with
// equal keys share one atomic; each lane gets a distinct old value.  Every
// lane of the wave must call it (active may be false).
__device__ __forceinline__ int wave_agg_inc(int32_t *counters, int key, bool active) {
    uint64_t act = ballot(active);
    int result = 0;
    const uint64_t lt = lanemask_lt();
    while (act) {
        const int leader = __builtin_ctzll(act);
        const int lkey = readlane_i(key, leader);
        const uint64_t grp = ballot(active && key == lkey) & act;
        int base = 0;
        if (lane_id() == leader) base = atomicAdd(&counters[lkey], (int)__builtin_popcountll(grp));
        base = readlane_i(base, leader);
        if ((grp >> lane_id()) & 1ull) result = base + (int)__builtin_popcountll(grp & lt);
        act &= ~grp;
    }
    return result;
}

// Block-aggregated form of wave_agg_inc, one key per thread of a block of NT
// threads: the block counts in an LDS histogram (hist, nkeys entries) first,
// then each key present reserves its range with one device atomic, so a wave
// whose lanes hit many different keys does not wait on one returning atomic
// per key.  Returns each active thread's distinct old value (0 when
// want_rank is false: the counts are only added).  Every thread of the block
// must call it.
template <int NT>
__device__ __forceinline__ int block_agg_inc(int32_t *counters, int key, bool active, int32_t *hist, int nkeys,
                                             bool want_rank) {
    const int tid = threadIdx.x;
    __syncthreads();   // a previous call's readers are done with hist
    for (int k = tid; k < nkeys; k += NT) hist[k] = 0;
    __syncthreads();
    const int local = active ? atomicAdd(&hist[key], 1) : 0;
    __syncthreads();
    for (int k = tid; k < nkeys; k += NT) {
        const int c = hist[k];
        if (c > 0) {
            if (want_rank)
                hist[k] = atomicAdd(&counters[k], c);
            else
                atomicAdd(&counters[k], c);
        }
    }
    __syncthreads();
    return (active && want_rank) ? hist[key] + local : 0;
}

// Per-list counters of a mutation kernel: LDS histogram when it fits (BLK),
// else wave aggregation.
template <bool BLK>
__device__ __forceinline__ int list_agg_inc(int32_t *counters, int key, bool active, int32_t *hist, int nkeys,
                                            bool want_rank) {
    if (BLK) return block_agg_inc<256>(counters, key, active, hist, nkeys, want_rank);
    return wave_agg_inc(counters, key, active);
}

// Record the first data-dependent error of a call and stop its later kernels.
// The call's sequence number lives on the device, so a call replayed from a
// captured graph gets a fresh one each time.
__device__ __forceinline__ void fail_call(int32_t *ctl, int status) {
    atomicCAS(&ctl[CTL_STATUS], 0, status);
    atomicExch(&ctl[CTL_GATE], ctl[CTL_SEQ]);
}

__device__ __forceinline__ bool call_failed(const int32_t *ctl) { return ctl[CTL_GATE] == ctl[CTL_SEQ]; }

// Inclusive sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o);
        if (l >= o) v += u;
    }
    return v;
}

// The same inclusive sum without LDS permutes: DPP row shifts build the sum
// inside each row of 16 lanes, then each row adds the totals of the rows
// before it (lanes 15, 31 and 47, read as scalars).  Every lane must call it.
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1 (lane 0 of a row adds 0)
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    const int r = lane_id() >> 4;
    const int s0 = __builtin_amdgcn_readlane(v, 15), s1 = __builtin_amdgcn_readlane(v, 31),
              s2 = __builtin_amdgcn_readlane(v, 47);
    return v + (r >= 1 ? s0 : 0) + (r >= 2 ? s1 : 0) + (r >= 3 ? s2 : 0);
}

// Exclusive sum over a block of NT threads (NT multiple of 64, <= 1024);
// *total receives the block sum.  Uses sbuf[NT/64] of shared memory.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int *sbuf, int *total) {
    const int w = threadIdx.x / 64, l = lane_id();
    int incl = wave_incl_scan(v);
    if (l == 63) sbuf[w] = incl;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        int s = sbuf[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// Exclusive prefix sum of 64-bit values over a block of NT threads.
template <int NT>
__device__ __forceinline__ long long block_excl_scan64(long long v, long long *sbuf, long long *total) {
    const int w = threadIdx.x / 64, l = lane_id();
    long long incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(incl, o);
        if (l >= o) incl += u;
    }
    if (l == 63) sbuf[w] = incl;
    __syncthreads();
    long long before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        const long long s = sbuf[i];
        if (i < w) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

}  // namespace sivf
