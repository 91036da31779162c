// Coarse quantizer: nearest centroid (insert) and nprobe nearest centroids
// (search), the list assignment taken as input by Alg. 1/Alg. 2 and the probed
// list ids read by Alg. 3 of the paper.
//
// Two kernels:
//  1. k_coarse_gemm: approximate distances Dt[r][l] = |x|^2 + |c|^2 - 2 x.c
//     (IP: -x.c) for a block of rows against all centroids, the dot products
//     on FP32 MFMA (v_mfma_f32_16x16x4_f32).
//  2. k_coarse_select: exact top-m lists by (D, l), where D is the canonical
//     FP64 distance (sequential fma over ascending dimensions).  With
//     tau = m-th smallest Dt and per-list error bounds E_l >= |Dt_l - D_l|,
//     every list with Dt_l - E_l <= tau + max E is re-evaluated exactly; this
//     set provably holds the true top-m, so the decision equals a plain
//     argmin/argsort over exact D for any input.
#include "sivf_dev.h"
#include "sivf_launch.h"

namespace sivf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int METRIC>
__global__ __launch_bounds__(256) void k_coarse_gemm(const float *__restrict__ X, int n, int d,
                                                     const float *__restrict__ cent, int dpad,
                                                     const float *__restrict__ cn2, int nlist,
                                                     float *__restrict__ out, const int32_t *ctl,
                                                     int gated) {
    constexpr int BM = 64, BN = 64, BK = 32;
    __shared__ float sA[BM][BK + 1];
    __shared__ float sB[BN][BK + 1];
    __shared__ float sqn[BM];
    if (gated && call_failed(ctl)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r0 = blockIdx.x * BM, c0 = blockIdx.y * BN;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float qn = 0.f;
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    const int ar = r0 + lr, bc = c0 + lr;
    for (int k0 = 0; k0 < dpad; k0 += BK) {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int kk = k0 + lk + e;
            float va = (ar < n && kk < d) ? X[(int64_t)ar * d + kk] : 0.f;
            float vb = (bc < nlist && kk < dpad) ? cent[(int64_t)bc * dpad + kk] : 0.f;
            sA[lr][lk + e] = va;
            sB[lr][lk + e] = vb;
            qn = fmaf(va, va, qn);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; i++) a[i] = sA[wr + 16 * i + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; j++) b[j] = sB[wc + 16 * j + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    qn += __shfl_xor(qn, 1);
    qn += __shfl_xor(qn, 2);
    if ((tid & 3) == 0) sqn[lr] = qn;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int row = wr + 16 * i + 4 * (lane >> 4) + rr;
                const int gr = r0 + row, gc = c0 + wc + 16 * j + (lane & 15);
                if (gr < n && gc < nlist) {
                    const float dot = acc[i][j][rr];
                    out[(int64_t)gr * nlist + gc] =
                        METRIC == 0 ? (sqn[row] + cn2[gc]) - 2.0f * dot : -dot;
                }
            }
}

__device__ __forceinline__ double canon_dist(const float *sx, const float *__restrict__ c, int d,
                                             int metric) {
    double r = 0.0;
    if (metric == 0) {
        for (int j = 0; j < d; j++) {
            const double t = (double)sx[j] - (double)c[j];
            r = __fma_rn(t, t, r);
        }
        return r;
    }
    for (int j = 0; j < d; j++) r = __fma_rn((double)sx[j], (double)c[j], r);
    return -r;
}

constexpr int SEL_CAP = 512;   // candidates buffered per exact re-check round

// One block of 256 threads per row.  Dynamic shared memory:
//   sx[dpad] float | kd[mmax] kl[mmax] nd[mmax] nl[mmax] | cd[SEL_CAP] cl[SEL_CAP]
__global__ __launch_bounds__(256) void k_coarse_select(
    const float *__restrict__ dt, const float *__restrict__ X, int n, int d, const float *__restrict__ cent,
    int dpad, const double *__restrict__ cnorm, const double *__restrict__ cmax, int nlist, int metric,
    int m_uniform, const int32_t *__restrict__ m_per_row, int mmax, int32_t *__restrict__ out,
    int out_stride, const int32_t *ctl, int gated) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int hist[256];
    __shared__ int sbuf[8];
    __shared__ double sred[4];
    __shared__ int sdig[2];
    if (gated && call_failed(ctl)) return;
    const int row = blockIdx.x;
    if (row >= n) return;
    const int tid = threadIdx.x;
    double *kd = (double *)smem;
    double *nd = kd + mmax;
    double *cd = nd + mmax;
    int *kl = (int *)(cd + SEL_CAP);
    int *nl = kl + mmax;
    int *cl = nl + mmax;
    float *sx = (float *)(cl + SEL_CAP);

    int m = m_per_row ? m_per_row[row] : m_uniform;
    m = m < nlist ? m : nlist;
    m = m < mmax ? m : mmax;
    m = m < 1 ? 1 : m;
    const float *xr = X + (int64_t)row * d;
    double q2 = 0.0;
    for (int j = tid; j < dpad; j += 256) {
        const float v = j < d ? xr[j] : 0.f;
        sx[j] = v;
        q2 = __fma_rn((double)v, (double)v, q2);
    }
    for (int o = 32; o > 0; o >>= 1) q2 += __shfl_xor(q2, o);
    if ((tid & 63) == 0) sred[tid >> 6] = q2;
    __syncthreads();
    const double qn = sqrt(sred[0] + sred[1] + sred[2] + sred[3]);
    const double coef = (4.0 * d + 16.0) * 0x1p-24;
    const double eabs = (double)d * 0x1p-120;
    const double cm = *cmax;
    const double emax = metric == 0 ? coef * (qn + cm) * (qn + cm) + eabs : coef * qn * cm + eabs;
    const float *drow = dt + (int64_t)row * nlist;

    // tau = m-th smallest approximate distance (radix select on ordered bits).
    uint32_t prefix = 0, pmask = 0;
    int rem = m;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        for (int l = tid; l < nlist; l += 256) {
            const uint32_t key = ord_bits(drow[l]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
        }
        __syncthreads();
        const int h = hist[tid];
        int tot;
        const int ex = block_excl_scan<256>(h, sbuf, &tot);
        if (ex < rem && rem <= ex + h) {
            sdig[0] = tid;
            sdig[1] = ex;
        }
        __syncthreads();
        prefix |= (uint32_t)sdig[0] << shift;
        pmask |= 0xFFu << shift;
        rem -= sdig[1];
        __syncthreads();
    }
    const double ub = (double)from_ord(prefix) + emax;

    int nk = 0, nb = 0;
    auto flush = [&]() {
        for (int e = tid; e < nb; e += 256) cd[e] = canon_dist(sx, cent + (int64_t)cl[e] * dpad, d, metric);
        __syncthreads();
        const int total = nk + nb;
        for (int e = tid; e < total; e += 256) {
            const double de = e < nk ? kd[e] : cd[e - nk];
            const int le = e < nk ? kl[e] : cl[e - nk];
            int rank = 0;
            for (int f = 0; f < total; f++) {
                const double df = f < nk ? kd[f] : cd[f - nk];
                const int lf = f < nk ? kl[f] : cl[f - nk];
                rank += (df < de) || (df == de && lf < le);
            }
            if (rank < m) {
                nd[rank] = de;
                nl[rank] = le;
            }
        }
        __syncthreads();
        nk = total < m ? total : m;
        for (int e = tid; e < nk; e += 256) {
            kd[e] = nd[e];
            kl[e] = nl[e];
        }
        nb = 0;
        __syncthreads();
    };
    for (int base = 0; base < nlist; base += 256) {
        const int l = base + tid;
        int isc = 0;
        if (l < nlist) {
            const double dv = (double)drow[l];
            const double cn = cnorm[l];
            const double el = metric == 0 ? coef * (qn + cn) * (qn + cn) + eabs : coef * qn * cn + eabs;
            isc = (dv - el <= ub) ? 1 : 0;
        }
        int tot;
        const int pos = block_excl_scan<256>(isc, sbuf, &tot);
        if (nb + tot > SEL_CAP) flush();
        if (isc) cl[nb + pos] = l;
        nb += tot;
        __syncthreads();
    }
    flush();
    int32_t *orow = out + (int64_t)row * out_stride;
    for (int p = tid; p < out_stride; p += 256) orow[p] = p < nk ? kl[p] : -1;
}

size_t coarse_select_smem(int dpad, int mmax) {
    return (size_t)(2 * mmax + SEL_CAP) * sizeof(double) + (size_t)(2 * mmax + SEL_CAP) * sizeof(int) +
           (size_t)dpad * sizeof(float) + 16;
}

void launch_coarse_gemm(hipStream_t st, const float *X, int n, int d, const float *cent, int dpad,
                        const float *cn2, int nlist, int metric, float *out, const int32_t *ctl,
                        int gated) {
    dim3 grid((n + 63) / 64, (nlist + 63) / 64);
    if (metric == 0)
        hipLaunchKernelGGL(k_coarse_gemm<0>, grid, dim3(256), 0, st, X, n, d, cent, dpad, cn2, nlist, out,
                           ctl, gated);
    else
        hipLaunchKernelGGL(k_coarse_gemm<1>, grid, dim3(256), 0, st, X, n, d, cent, dpad, cn2, nlist, out,
                           ctl, gated);
}

void launch_coarse_select(hipStream_t st, const float *dt, const float *X, int n, int d, const float *cent,
                          int dpad, const double *cnorm, const double *cmax, int nlist, int metric,
                          int m_uniform, const int32_t *m_per_row, int mmax, int32_t *out, int out_stride,
                          const int32_t *ctl, int gated) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_coarse_select, dim3(n), dim3(256), coarse_select_smem(dpad, mmax), st, dt, X, n, d,
                       cent, dpad, cnorm, cmax, nlist, metric, m_uniform, m_per_row, mmax, out, out_stride,
                       ctl, gated);
}

}  // namespace sivf
