// External id registry: arbitrary 64-bit external ids (e.g. UUID halves,
// hashes) mapped onto the index's dense internal id range [0, id_capacity).
// The paper keeps this map in a host-side registry in front of its dense
// identifier space (Sec. 3, Data Model); here it is device-resident, so a
// batch of external ids is resolved without a host round trip:
//   - an open-addressing hash table (linear probing, power-of-two size) of
//     key -> internal id; a removed key leaves a tombstone, and the table is
//     rebuilt from the live map before used slots could pass half the table;
//   - ext_of[internal id] = the external id it holds (the reverse map, used
//     to translate search results and to rebuild the table);
//   - a stack of free internal ids.
// Two key values are reserved as table markers (EMPTY and TOMB below) and
// cannot be used as external ids.
#include "sivf_launch.h"

namespace sivf {

__device__ __forceinline__ uint64_t mix64(uint64_t k) {   // a 64-bit finalizer (xor-shift-multiply)
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Find the slot of key (or -1).  Tombstones do not end the probe.
__device__ __forceinline__ int64_t reg_find(const RegDev &R, int64_t key) {
    uint64_t h = mix64((uint64_t)key) & (uint64_t)(R.cap - 1);
    for (int64_t step = 0; step < R.cap; step++) {
        const int64_t k = R.keys[h];
        if (k == key) return (int64_t)h;
        if (k == REG_EMPTY) return -1;
        h = (h + 1) & (uint64_t)(R.cap - 1);
    }
    return -1;
}

// Find key or claim an empty slot for it.  *fresh = 1 when this lane's CAS
// claimed the slot (a duplicate of the same key in the batch finds the slot
// the winner claimed).  Returns -1 only if the table is full.
__device__ __forceinline__ int64_t reg_claim(const RegDev &R, int64_t key, int *fresh) {
    *fresh = 0;
    uint64_t h = mix64((uint64_t)key) & (uint64_t)(R.cap - 1);
    for (int64_t step = 0; step < R.cap; step++) {
        int64_t k = R.keys[h];
        if (k == REG_EMPTY) {
            const unsigned long long old =
                atomicCAS((unsigned long long *)&R.keys[h], (unsigned long long)REG_EMPTY, (unsigned long long)key);
            if ((int64_t)old == REG_EMPTY) {
                *fresh = 1;
                return (int64_t)h;
            }
            k = (int64_t)old;
        }
        if (k == key) return (int64_t)h;
        h = (h + 1) & (uint64_t)(R.cap - 1);
    }
    return -1;
}

__device__ __forceinline__ bool reg_key_ok(int64_t key) { return key != REG_EMPTY && key != REG_TOMB; }

// add, step 1: claim or find each key's slot.
__global__ __launch_bounds__(256) void k_reg_claim(RegDev R, int n, const int64_t *__restrict__ ext,
                                                   int64_t *__restrict__ slot, int32_t *__restrict__ fresh,
                                                   int32_t *ctl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t key = ext[i];
    if (!reg_key_ok(key)) {
        atomicCAS(&ctl[REG_CTL_STATUS], 0, -1);   // SIVF_ERR_ARG
        slot[i] = -1;
        fresh[i] = 0;
        return;
    }
    int f = 0;
    const int64_t s = reg_claim(R, key, &f);
    if (s < 0) atomicCAS(&ctl[REG_CTL_STATUS], 0, -2);   // table full: SIVF_ERR_NOSPACE
    slot[i] = s;
    fresh[i] = f;
}

// add, step 2: each freshly claimed slot takes an internal id from the free
// stack (one atomic per wave); step 3 resolves every row to its internal id.
__global__ __launch_bounds__(256) void k_reg_alloc(RegDev R, int n, const int64_t *__restrict__ ext,
                                                   const int64_t *__restrict__ slot,
                                                   const int32_t *__restrict__ fresh, int32_t *ctl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool want = i < n && fresh[i] && slot[i] >= 0;
    const uint64_t m = ballot(want);
    int base = 0;
    if (m) {
        // The wave takes its ids off the top of the stack.  A wave that finds
        // fewer than it asked for returns the shortfall, so the count never
        // stays below zero: the stack ends empty and the ids handed out are
        // exactly those that were on it.
        const int cnt = (int)__builtin_popcountll(m);
        const int leader = __builtin_ctzll(m);
        if (lane_id() == leader) {
            base = atomicSub(&ctl[REG_CTL_TOP], cnt);
            if (base < cnt) atomicAdd(&ctl[REG_CTL_TOP], cnt - (base > 0 ? base : 0));
        }
        base = readlane_i(base, leader);
    }
    if (!want) return;
    const int t = base - 1 - (int)__builtin_popcountll(m & lanemask_lt());
    if (t < 0) {   // internal id space exhausted: the key maps to nothing
        atomicCAS(&ctl[REG_CTL_STATUS], 0, -2);
        R.vals[slot[i]] = -1;
        return;
    }
    const int32_t id = R.free_ids[t];
    R.vals[slot[i]] = id;
    R.ext_of[id] = ext[i];
}

__global__ __launch_bounds__(256) void k_reg_resolve(RegDev R, int n, const int64_t *__restrict__ slot,
                                                     int64_t *__restrict__ internal) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t s = slot[i];
    const int32_t v = s >= 0 ? R.vals[s] : -1;
    internal[i] = v;
}

// add, step 4 (after the index add): a freshly mapped key whose internal id
// is not live (the add was rejected) is unmapped again.  Only the lane that
// claimed the slot does it.
__global__ __launch_bounds__(256) void k_reg_rollback(RegDev R, Dev S, int n, const int64_t *__restrict__ slot,
                                                      const int32_t *__restrict__ fresh, int32_t *ctl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const bool f = i < n && fresh[i] && slot[i] >= 0;
    bool undo = false;
    int32_t id = -1;
    if (f) {
        id = R.vals[slot[i]];
        undo = id < 0 || S.att[id] == INVALID;
    }
    const bool push = undo && id >= 0;
    const uint64_t m = ballot(push);
    int base = 0;
    if (m) {
        if (lane_id() == __builtin_ctzll(m)) base = atomicAdd(&ctl[REG_CTL_TOP], (int)__builtin_popcountll(m));
        base = readlane_i(base, __builtin_ctzll(m));
    }
    if (!undo) return;
    if (push) {
        R.free_ids[base + (int)__builtin_popcountll(m & lanemask_lt())] = id;
        R.ext_of[id] = REG_EMPTY;
    }
    R.vals[slot[i]] = -1;
    R.keys[slot[i]] = REG_TOMB;
}

// lookup / remove, step 1: internal id of each key (-1 if unmapped).
__global__ __launch_bounds__(256) void k_reg_lookup(RegDev R, int n, const int64_t *__restrict__ ext,
                                                    int64_t *__restrict__ slot, int64_t *__restrict__ internal) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t key = ext[i];
    const int64_t s = reg_key_ok(key) ? reg_find(R, key) : -1;
    if (slot) slot[i] = s;
    internal[i] = s >= 0 ? (int64_t)R.vals[s] : -1;
}

// remove, step 2 (after the index remove): keys whose internal id is no
// longer live are unmapped; the CAS on the key makes that happen once per
// key even when the batch repeats it.
__global__ __launch_bounds__(256) void k_reg_release(RegDev R, Dev S, int n, const int64_t *__restrict__ ext,
                                                     const int64_t *__restrict__ slot, int32_t *ctl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    bool push = false;
    int32_t id = -1;
    if (i < n && slot[i] >= 0) {
        const int64_t s = slot[i];
        id = R.vals[s];
        if (id >= 0 && S.att[id] == INVALID) {
            const unsigned long long old = atomicCAS((unsigned long long *)&R.keys[s], (unsigned long long)ext[i],
                                                     (unsigned long long)REG_TOMB);
            push = (int64_t)old == ext[i];
        }
    }
    const uint64_t m = ballot(push);
    int base = 0;
    if (m) {
        if (lane_id() == __builtin_ctzll(m)) base = atomicAdd(&ctl[REG_CTL_TOP], (int)__builtin_popcountll(m));
        base = readlane_i(base, __builtin_ctzll(m));
    }
    if (!push) return;
    R.free_ids[base + (int)__builtin_popcountll(m & lanemask_lt())] = id;
    R.ext_of[id] = REG_EMPTY;
}

// search: internal labels -> external ids, in place (-1 stays -1).
__global__ __launch_bounds__(256) void k_reg_labels(RegDev R, int64_t n, int64_t *__restrict__ labels) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t v = labels[i];
    if (v >= 0) labels[i] = R.ext_of[v];
}

// rebuild: clear the table, then insert every live (external, internal) pair.
__global__ __launch_bounds__(256) void k_reg_clear(RegDev R) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < R.cap) {
        R.keys[i] = REG_EMPTY;
        R.vals[i] = -1;
    }
}

__global__ __launch_bounds__(256) void k_reg_reinsert(RegDev R, int32_t *ctl) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= R.id_cap) return;
    const int64_t key = R.ext_of[id];
    if (key == REG_EMPTY) return;
    int f = 0;
    const int64_t s = reg_claim(R, key, &f);
    if (s < 0) {
        atomicCAS(&ctl[REG_CTL_STATUS], 0, -2);
        return;
    }
    R.vals[s] = (int32_t)id;
}

// free stack = every internal id without an external id, ascending (one block).
__global__ __launch_bounds__(1024) void k_reg_free_stack(RegDev R, int32_t *ctl) {
    __shared__ int sbuf[16];
    int carry = 0;
    for (int64_t base = 0; base < R.id_cap; base += 1024) {
        const int64_t id = base + threadIdx.x;
        const int f = (id < R.id_cap && R.ext_of[id] == REG_EMPTY) ? 1 : 0;
        int tot;
        const int ex = block_excl_scan<1024>(f, sbuf, &tot);
        if (f) R.free_ids[carry + ex] = (int32_t)id;
        carry += tot;
    }
    if (threadIdx.x == 0) ctl[REG_CTL_TOP] = carry;
}

static unsigned rblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_reg_add_pre(hipStream_t st, const RegDev &R, int n, const int64_t *ext, int64_t *slot, int32_t *fresh,
                        int64_t *internal, int32_t *ctl) {
    hipLaunchKernelGGL(k_reg_claim, dim3(rblocks(n)), dim3(256), 0, st, R, n, ext, slot, fresh, ctl);
    hipLaunchKernelGGL(k_reg_alloc, dim3(rblocks(n)), dim3(256), 0, st, R, n, ext, slot, fresh, ctl);
    hipLaunchKernelGGL(k_reg_resolve, dim3(rblocks(n)), dim3(256), 0, st, R, n, slot, internal);
}

void launch_reg_add_post(hipStream_t st, const RegDev &R, const Dev &S, int n, const int64_t *slot,
                         const int32_t *fresh, int32_t *ctl) {
    hipLaunchKernelGGL(k_reg_rollback, dim3(rblocks(n)), dim3(256), 0, st, R, S, n, slot, fresh, ctl);
}

void launch_reg_lookup(hipStream_t st, const RegDev &R, int n, const int64_t *ext, int64_t *slot, int64_t *internal) {
    hipLaunchKernelGGL(k_reg_lookup, dim3(rblocks(n)), dim3(256), 0, st, R, n, ext, slot, internal);
}

void launch_reg_release(hipStream_t st, const RegDev &R, const Dev &S, int n, const int64_t *ext,
                        const int64_t *slot, int32_t *ctl) {
    hipLaunchKernelGGL(k_reg_release, dim3(rblocks(n)), dim3(256), 0, st, R, S, n, ext, slot, ctl);
}

void launch_reg_labels(hipStream_t st, const RegDev &R, int64_t n, int64_t *labels) {
    if (n > 0) hipLaunchKernelGGL(k_reg_labels, dim3(rblocks(n)), dim3(256), 0, st, R, n, labels);
}

void launch_reg_rebuild(hipStream_t st, const RegDev &R, int32_t *ctl) {
    hipLaunchKernelGGL(k_reg_clear, dim3(rblocks(R.cap)), dim3(256), 0, st, R);
    hipLaunchKernelGGL(k_reg_reinsert, dim3(rblocks(R.id_cap)), dim3(256), 0, st, R, ctl);
}

void launch_reg_free_stack(hipStream_t st, const RegDev &R, int32_t *ctl) {
    hipLaunchKernelGGL(k_reg_free_stack, dim3(1), dim3(1024), 0, st, R, ctl);
}

}  // namespace sivf
