// Index creation: the pre-allocated slab pool with every slab on the free
// stack (Sec. 3.1; the paper's SlabManager keeps a monolithic pool and a
// device free stack, Sec. 4.1), an empty address table, and the centroid copy
// with the norms used by the coarse quantizer's error bounds.
#include "sivf_launch.h"

namespace sivf {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_i32(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ void k_fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One block per centroid: zero-padded copy, fp32 squared norm, fp64 norm and
// the running maximum norm (non-negative doubles order like their bits).
__global__ __launch_bounds__(256) void k_init_cent(float *cent, float *cn2, double *cnorm, double *cmax,
                                                   uint16_t *cent_h, const float *src, int d, int dpad) {
    __shared__ float s32[4];
    __shared__ double s64[4];
    const int l = blockIdx.x, tid = threadIdx.x;
    float a = 0.f;
    double b = 0.0;
    for (int j = tid; j < dpad; j += 256) {
        const float v = j < d ? src[(int64_t)l * d + j] : 0.f;
        cent[(int64_t)l * dpad + j] = v;
        if (cent_h) cent_h[(int64_t)l * dpad + j] = (uint16_t)to_bf16_bits(v);
        a = fmaf(v, v, a);
        b = __fma_rn((double)v, (double)v, b);
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    if ((tid & 63) == 0) {
        s32[tid >> 6] = a;
        s64[tid >> 6] = b;
    }
    __syncthreads();
    if (tid == 0) {
        const float ta = s32[0] + s32[1] + s32[2] + s32[3];
        const double tb = s64[0] + s64[1] + s64[2] + s64[3];
        // the norm only enters the error bound: round it up by a relative 2^-50
        const double nrm = sqrt(tb) * (1.0 + 0x1p-50);
        cn2[l] = ta;
        cnorm[l] = nrm;
        atomicMax((unsigned long long *)cmax, (unsigned long long)__double_as_longlong(nrm));
    }
}

__global__ void k_init_ctl(int32_t *ctl, int64_t num_slabs, int64_t num_pages) {
    const int i = threadIdx.x;
    if (i < CTL_WORDS) ctl[i] = 0;
    if (i == CTL_GATE || i == CTL_UPSERT) ctl[i] = -1;
    if (i == CTL_SLAB_TOP) ctl[i] = (int32_t)num_slabs;
    if (i == CTL_PAGE_TOP) ctl[i] = (int32_t)num_pages;
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

static void fill(hipStream_t st, int32_t *p, int64_t n, int32_t v) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}

void launch_fill_i32(hipStream_t st, int32_t *p, int64_t n, int32_t v) { fill(st, p, n, v); }

void launch_fill_i64(hipStream_t st, int64_t *p, int64_t n, int64_t v) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i64_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
}

void launch_init_state(hipStream_t st, const Dev &S, const float *centroids) {
    const int dpad = S.dp4 * 4;
    launch_fill_i64(st, (int64_t *)S.cmax, 1, 0);
    hipLaunchKernelGGL(k_init_cent, dim3(S.nlist), dim3(256), 0, st, (float *)S.cent, (float *)S.cn2,
                       (double *)S.cnorm, (double *)S.cmax, (uint16_t *)S.cent_h, centroids, S.d, dpad);
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(S.num_slabs)), dim3(256), 0, st, S.free_slabs, S.num_slabs);
    hipLaunchKernelGGL(k_iota_i32, dim3(grid_for(S.num_pages)), dim3(256), 0, st, S.free_pages, S.num_pages);
    fill(st, S.sowner, S.num_slabs, -1);
    fill(st, S.sord, S.num_slabs, 0);
    fill(st, (int32_t *)S.att, S.id_capacity, -1);
    fill(st, S.mark, S.id_capacity, -1);
    fill(st, S.len, S.nlist, 0);
    int32_t *lists[] = {S.l_acnt, S.l_prem, S.l_base, S.l_eoff, S.l_m, S.l_off, S.l_newlen, S.l_q, S.l_s,
                        S.l_h, S.l_qc, S.l_qcs, S.l_qoff, S.l_snap, S.l_pbase, S.l_ioff, S.l_dead};
    for (int32_t *p : lists) fill(st, p, S.nlist, 0);
    if (S.bits) launch_fill_i64(st, (int64_t *)S.bits, S.num_slabs * S.bw, 0);   // no slot holds an entry
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(CTL_WORDS), 0, st, S.ctl, S.num_slabs, S.num_pages);
}

}  // namespace sivf
