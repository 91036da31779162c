// Continuous batching of the serving form (the paper's mixed workload,
// Sec. 5.5): searches that queue while the search stream is busy are
// coalesced into one search launch.  Two copy kernels bracket that launch:
// the gather packs the requests' query rows into one batch and writes each
// row's k and nprobe; the scatter copies each row's results back into its
// request's own output (row stride = that request's k).  A batch lists its
// requests as segments of consecutive rows, in submission order.
#include "sivf_launch.h"

namespace sivf {

// Segment holding batch row r: the last segment whose first row is <= r.
__device__ __forceinline__ int seg_of(const SrvSeg *__restrict__ segs, int nseg, int r) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].row0 <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One wave per batch row.
__global__ __launch_bounds__(256) void k_srv_gather(const SrvSeg *__restrict__ segs, int nseg, int nrows, int d,
                                                    float *__restrict__ q, int32_t *__restrict__ kq,
                                                    int32_t *__restrict__ npq) {
    const int r = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (r >= nrows) return;
    const int s = seg_of(segs, nseg, r);
    const SrvSeg g = segs[s];
    const float *src = g.q + (int64_t)(r - g.row0) * d;
    float *dst = q + (int64_t)r * d;
    for (int j = lane_id(); j < d; j += 64) dst[j] = src[j];
    if (lane_id() == 0) {
        kq[r] = g.k;
        npq[r] = g.nprobe;
    }
}

__global__ __launch_bounds__(256) void k_srv_scatter(const SrvSeg *__restrict__ segs, int nseg, int nrows,
                                                     int kstride, const float *__restrict__ dist,
                                                     const int64_t *__restrict__ labels) {
    const int r = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (r >= nrows) return;
    const int s = seg_of(segs, nseg, r);
    const SrvSeg g = segs[s];
    const int64_t o = (int64_t)(r - g.row0) * g.k;
    for (int j = lane_id(); j < g.k; j += 64) {
        g.dist[o + j] = dist[(int64_t)r * kstride + j];
        g.labels[o + j] = labels[(int64_t)r * kstride + j];
    }
}

void launch_srv_gather(hipStream_t st, const SrvSeg *segs, int nseg, int nrows, int d, float *q, int32_t *kq,
                       int32_t *npq) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_srv_gather, dim3((nrows + 3) / 4), dim3(256), 0, st, segs, nseg, nrows, d, q, kq, npq);
}

void launch_srv_scatter(hipStream_t st, const SrvSeg *segs, int nseg, int nrows, int kstride, const float *dist,
                        const int64_t *labels) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_srv_scatter, dim3((nrows + 3) / 4), dim3(256), 0, st, segs, nseg, nrows, kstride, dist,
                       labels);
}

}  // namespace sivf
