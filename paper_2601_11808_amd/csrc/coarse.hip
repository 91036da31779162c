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
//     argmin/argsort over exact D for any input.  Rows or centroids large
//     enough for an fp32 square to overflow are re-checked against every
//     list, in both kernels.
#include "sivf_dev.h"
#include "sivf_launch.h"

namespace sivf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Block tile: 128 rows x 128 centroids, 256 threads; each wave owns a 64x64
// quarter as 4x4 accumulators of v_mfma_f32_16x16x4_f32.  K advances 32 per
// step: the next 32-wide slice of both operands is fetched into registers
// (float4 loads) while the current one, stored k-major in LDS, feeds the
// MFMAs.  The LDS row stride of 144 floats puts the two 16-lane k-groups of a
// half-wave read in disjoint banks.
constexpr int GM = 128, GN = 128, GK = 32, GLD = GM + 16;
constexpr int GROUP = 16;   // lists per group minimum (insert path)

// Smallest value m1 (at group position a) and second smallest m2 of a group
// of 16 lists.  A lane pushes its 4 values, then the lanes holding the other
// positions of the group (lane ^ 16, lane ^ 32) are merged in; both sides of an
// exchange end with the same triple.  A NaN counts as +inf.  Equal smallest
// values leave m2 == m1.
__device__ __forceinline__ void min2_push(float &m1, float &m2, int &a, float v, int idx) {
    if (v < m1) {
        m2 = m1;
        m1 = v;
        a = idx;
    } else if (v < m2) {
        m2 = v;
    }
}
__device__ __forceinline__ void min2_merge(float &m1, float &m2, int &a, float om1, float om2, int oa) {
    if (om1 < m1 || (om1 == m1 && oa < a)) {
        m2 = fminf(m1, om2);
        m1 = om1;
        a = oa;
    } else {
        m2 = fminf(m2, om1);
    }
}
template <int J>
__device__ __forceinline__ void min2_xor(float &m1, float &m2, int &a) {
    const float om1 = __shfl_xor(m1, J), om2 = __shfl_xor(m2, J);
    const int oa = __shfl_xor(a, J);
    min2_merge(m1, m2, a, om1, om2, oa);
}
// The second smallest value rounded down to a multiple of 2^SEG_BITS in the
// ordered key space (so it never grows: the relative change is below 2^-12),
// with the position of the smallest (< 2^SEG_BITS) in the freed low bits.
constexpr int SEG_BITS = 11;
constexpr uint32_t SEG_MASK = (1u << SEG_BITS) - 1;
__device__ __forceinline__ uint32_t min2_pack(float m2, int a) { return (ord_bits(m2) & ~SEG_MASK) | (uint32_t)a; }

constexpr int HLD = GK + 8;  // bf16 operands: row-major LDS rows of 32 + 8 halves (80 bytes)

typedef __bf16 cbf16x8 __attribute__((ext_vector_type(8)));

// GMIN = 0: write Dt[r][l] for every list (out row stride ldo = nlist).
// GMIN = 1: write only the minimum of each group of 16 consecutive lists,
//           out[r][l / 16] (ldo = ceil(nlist / 16)); a NaN counts as +inf;
//           out2[r][l / 16] = min2_pack(second smallest, position of the
//           smallest) of the same group (here a segment is one group).
// BF = 1: both operands rounded to bf16 (round to nearest even) and
//         multiplied on v_mfma_f32_16x16x32_bf16 (16 times the FP32 MFMA
//         rate); |x|^2 and |c|^2 stay fp32 from the exact values.  The
//         re-check bound then adds the operand rounding (coarse_err).
template <int METRIC, int GMIN, bool VEC, int BF>
__global__ __launch_bounds__(256) void k_coarse_gemm(const float *__restrict__ X, int n, int d,
                                                     const float *__restrict__ cent,
                                                     const uint16_t *__restrict__ cent_h, int dpad,
                                                     const float *__restrict__ cn2, int nlist,
                                                     float *__restrict__ out, uint32_t *__restrict__ out2, int ldo,
                                                     const int32_t *ctl, int gated, int xcd_map) {
    // fp32: k-major [GK][GLD] floats per operand; bf16: row-major [GM][HLD] halves per operand
    __shared__ __align__(16) float sbuf[2][BF ? (GM * HLD / 2) : (GK * GLD)];
    __shared__ float sqn[GM];
    float(*sA)[GLD] = reinterpret_cast<float(*)[GLD]>(sbuf[0]);
    float(*sB)[GLD] = reinterpret_cast<float(*)[GLD]>(sbuf[1]);
    uint16_t(*hA)[HLD] = reinterpret_cast<uint16_t(*)[HLD]>(sbuf[0]);
    uint16_t(*hB)[HLD] = reinterpret_cast<uint16_t(*)[HLD]>(sbuf[1]);
    if (gated && call_failed(ctl)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // Block -> (row block, centroid block).  With xcd_map each XCD (blocks are
    // dealt round robin) owns a contiguous range of centroid blocks and walks
    // every row block for one before the next, so a centroid tile is fetched
    // into one L2 and reused by all row blocks.
    const int nrb = (n + GM - 1) / GM, ncb = (nlist + GN - 1) / GN;
    int rb, cb;
    if (xcd_map) {
        const int per = (ncb + 7) >> 3, j = (int)(blockIdx.x >> 3);
        cb = (int)(blockIdx.x & 7) * per + j / nrb;
        rb = j % nrb;
        if (cb >= ncb || j / nrb >= per) return;
    } else {
        rb = (int)blockIdx.x % nrb;
        cb = (int)blockIdx.x / nrb;
    }
    const int r0 = rb * GM, c0 = cb * GN;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int lrow = tid >> 3, lk = (tid & 7) * 4;   // loader: 8 threads x float4 per row, 32 rows per pass
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float4 ra[4], rbf[4];
    uint2 rbh[4];   // bf16 centroid halves (BF)
    float qp[4] = {0.f, 0.f, 0.f, 0.f};
    const int kend = (dpad + GK - 1) / GK * GK;

    auto gload = [&](int k0) {
        const int kk = k0 + lk;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = r0 + lrow + 32 * i;
            if (VEC) {   // d % 4 == 0: kk < d covers all four
                ra[i] = (r < n && kk < d) ? *(const float4 *)(X + (int64_t)r * d + kk) : make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                const float *p = X + (int64_t)r * d;
                ra[i].x = (r < n && kk + 0 < d) ? p[kk + 0] : 0.f;
                ra[i].y = (r < n && kk + 1 < d) ? p[kk + 1] : 0.f;
                ra[i].z = (r < n && kk + 2 < d) ? p[kk + 2] : 0.f;
                ra[i].w = (r < n && kk + 3 < d) ? p[kk + 3] : 0.f;
            }
            const int c = c0 + lrow + 32 * i;   // centroid rows are zero-padded to dpad (a multiple of 4)
            if (BF)
                rbh[i] = (c < nlist && kk < dpad) ? *(const uint2 *)(cent_h + (int64_t)c * dpad + kk)
                                                  : make_uint2(0u, 0u);
            else
                rbf[i] = (c < nlist && kk < dpad) ? *(const float4 *)(cent + (int64_t)c * dpad + kk)
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int rr = lrow + 32 * i;
            qp[i] = fmaf(ra[i].x, ra[i].x, qp[i]);
            qp[i] = fmaf(ra[i].y, ra[i].y, qp[i]);
            qp[i] = fmaf(ra[i].z, ra[i].z, qp[i]);
            qp[i] = fmaf(ra[i].w, ra[i].w, qp[i]);
            if (BF) {
                *reinterpret_cast<uint2 *>(&hA[rr][lk]) =
                    make_uint2(to_bf16_bits(ra[i].x) | (to_bf16_bits(ra[i].y) << 16),
                               to_bf16_bits(ra[i].z) | (to_bf16_bits(ra[i].w) << 16));
                *reinterpret_cast<uint2 *>(&hB[rr][lk]) = rbh[i];
                continue;
            }
            sA[lk + 0][rr] = ra[i].x;
            sA[lk + 1][rr] = ra[i].y;
            sA[lk + 2][rr] = ra[i].z;
            sA[lk + 3][rr] = ra[i].w;
            sB[lk + 0][rr] = rbf[i].x;
            sB[lk + 1][rr] = rbf[i].y;
            sB[lk + 2][rr] = rbf[i].z;
            sB[lk + 3][rr] = rbf[i].w;
        }
    };
    gload(0);
    for (int k0 = 0; k0 < kend; k0 += GK) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (k0 + GK < kend) gload(k0 + GK);
        if (BF) {
            // lane l: row (or centroid) l % 16 of the block, halves 8 (l / 16) .. +8 of the step
            const int kg = (lane >> 4) * 8;
            uint4 av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; i++) av[i] = *reinterpret_cast<const uint4 *>(&hA[wr + 16 * i + (lane & 15)][kg]);
#pragma unroll
            for (int j = 0; j < 4; j++) bv[j] = *reinterpret_cast<const uint4 *>(&hB[wc + 16 * j + (lane & 15)][kg]);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cbf16x8, bv[j]),
                                                                       __builtin_bit_cast(cbf16x8, av[i]),
                                                                       acc[i][j], 0, 0, 0);
            continue;
        }
#pragma unroll
        for (int s = 0; s < GK / 4; s++) {
            const int kr = 4 * s + (lane >> 4);
            float av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; i++) av[i] = sA[kr][wr + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; j++) bv[j] = sB[kr][wc + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j], av[i], acc[i][j], 0, 0, 0);
        }
    }
    // |x|^2 of each row: the 8 loader threads of a row are adjacent lanes
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float v = qp[i];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if ((tid & 7) == 0) sqn[lrow + 32 * i] = v;
    }
    __syncthreads();
    // The MFMAs compute the transposed tile (centroids as rows): lane holds
    // the dot of row wr + 16 i + lane % 16 with the 4 consecutive centroids
    // wc + 16 j + 4 (lane / 16) .. +3, so a 16-list group minimum takes 3
    // in-register mins and 2 lane exchanges, and full rows store 4 floats.
    const bool vec4 = (ldo & 3) == 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int row = wr + 16 * i + (lane & 15);
        const int gr = r0 + row;
        const float sq = sqn[row];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int gc0 = c0 + wc + 16 * j;
            const int gcb = gc0 + 4 * (lane >> 4);
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int gc = gcb + r;
                const float c2 = (METRIC == 0 && gc < nlist) ? cn2[gc] : 0.f;
                const float dot = acc[i][j][r];
                v[r] = METRIC == 0 ? (sq + c2) - 2.0f * dot : -dot;
            }
            if (!GMIN) {
                if (gr < n) {
                    float *o = out + (int64_t)gr * ldo + gcb;
                    if (vec4 && gcb + 3 < nlist) {
                        *reinterpret_cast<float4 *>(o) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            if (gcb + r < nlist) o[r] = v[r];
                    }
                }
            } else {
                float m1 = __builtin_inff(), m2 = __builtin_inff();
                int a = 0;
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if (gcb + r < nlist) min2_push(m1, m2, a, v[r], 4 * (lane >> 4) + r);
                min2_xor<16>(m1, m2, a);
                min2_xor<32>(m1, m2, a);
                if ((lane >> 4) == 0 && gr < n && gc0 < nlist) {
                    out[(int64_t)gr * ldo + gc0 / GROUP] = m1;
                    out2[(int64_t)gr * ldo + gc0 / GROUP] = min2_pack(m2, a);
                }
            }
        }
    }
}

// Certified bound on |Dt - D| for a row of norm qn and a list of norm cn: the
// FP32 arithmetic of the GEMM ((4d+16) 2^-24 (|x|+|c|)^2, IP: |x||c|, plus
// an underflow term) and, with bf16 operands (bf = 1), their rounding:
// |x.c - x~.c~| <= (2u + u^2)|x||c| with u = 2^-8 (Cauchy-Schwarz), counted
// twice for L2's -2 x.c, plus the bf16 subnormal spacing.
__device__ __forceinline__ double coarse_err(int metric, int d, int bf, double qn, double cn) {
    const double coef = (4.0 * d + 16.0) * 0x1p-24;
    double e = metric == 0 ? coef * (qn + cn) * (qn + cn) : coef * qn * cn;
    if (bf) {
        const double u = 0x1p-8, m = metric == 0 ? 2.0 : 1.0;
        e += m * (2.0 * u + u * u) * 1.01 * qn * cn + m * 0x1p-132 * sqrt((double)d) * (qn + cn);
    }
    return e + (double)d * 0x1p-120;
}

// Group minima of the insert path on bf16 MFMA, row-stationary (padded rows
// of at most 128 dimensions): a block of 8 waves takes 256 rows -- rounded to
// bf16 once and held in registers, wave w owning rows 32 w .. 32 w + 31 as two
// 16-row operands per 32-dimension step -- and sweeps nct consecutive tiles of 128
// centroids, each streamed through LDS (double buffer: the next tile's loads
// are in flight while the current one feeds the MFMAs; one barrier per
// tile).  Per tile each row gets its 8 group minima, out[r][g] as
// k_coarse_gemm<., 1> writes them; |c|^2 comes from LDS (+inf past nlist),
// and Dt = |x|^2 + (|c|^2 - 2 x.c) takes one fma per list.  Each lane also
// keeps, over the segment's tiles, the smallest and second smallest Dt of its
// rows among its own lists and the position of the smallest; the 4 lanes of a
// row merge them at the end, and out2[r][segment] = min2_pack(second
// smallest, position in the segment).
//
// MODE GM_PLAIN (more than 16 tiles of lists, where the tracking costs more
// in this kernel than the re-checks it saves) writes only the group minima.
// GM_SEG writes out2 as above.  GM_DEC (one segment holds every list) writes
// no out2: a row whose second smallest Dt exceeds the smallest by more than
// twice the certified bound (coarse_err with an upper bound of the row's norm
// and the largest centroid norm) has its nearest list decided here, with the argmin
// kernel's test; the others get ASSIGN_UNDECIDED in assign[] and only their
// group minima for the argmin kernel's re-check.
constexpr int HK = 128, HBLD = HK + 8;   // halves of a padded row; LDS row stride (halves)
constexpr int HW = 8, HR = 32 * HW;      // waves per block, rows per block
constexpr int32_t ASSIGN_UNDECIDED = -2;
constexpr int GM_PLAIN = 0, GM_SEG = 1, GM_DEC = 2;
template <int METRIC, int MODE>
__global__ __launch_bounds__(64 * HW) void k_coarse_gmin_h(const float *__restrict__ X, int n, int d,
                                                       const uint16_t *__restrict__ cent_h, int dpad,
                                                       const float *__restrict__ cn2, int nlist,
                                                       float *__restrict__ out, uint32_t *__restrict__ out2, int ldo,
                                                       int nct, int xcd_map, const double *__restrict__ cmax,
                                                       int32_t *__restrict__ assign, int assign_stride,
                                                       const int32_t *ctl, int gated) {
    __shared__ __align__(16) uint16_t sB[2][GN * HBLD];
    __shared__ __align__(16) float sC[2][GN];
    if (gated && call_failed(ctl)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nrb = (n + HR - 1) / HR, ncb = (nlist + GN - 1) / GN, ncs = (ncb + nct - 1) / nct;
    int rb, sg;
    if (xcd_map) {   // each XCD owns a contiguous range of centroid segments (tiles stay in its L2)
        const int per = (ncs + 7) >> 3, j = (int)(blockIdx.x >> 3);
        sg = (int)(blockIdx.x & 7) * per + j / nrb;
        rb = j % nrb;
        if (sg >= ncs || j / nrb >= per) return;
    } else {
        rb = (int)blockIdx.x % nrb;
        sg = (int)blockIdx.x / nrb;
    }
    const int r0 = rb * HR, t0 = sg * nct, t1 = min(t0 + nct, ncb);
    constexpr bool DEC = MODE == GM_DEC, TRACK = MODE != GM_PLAIN;
    // this lane's rows (16 i + lane % 16 of the wave's 32) as bf16 operands, and their |x|^2
    uint4 a[2][4];
    float sq[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const int r = r0 + 32 * w + 16 * i + (lane & 15);
        float part = 0.f;
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            const int k = 32 * ks + 8 * (lane >> 4);
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; e++) v[e] = (r < n && k + e < d) ? X[(int64_t)r * d + k + e] : 0.f;
#pragma unroll
            for (int e = 0; e < 8; e++) part = fmaf(v[e], v[e], part);
            a[i][ks] = make_uint4(to_bf16_bits(v[0]) | (to_bf16_bits(v[1]) << 16),
                                  to_bf16_bits(v[2]) | (to_bf16_bits(v[3]) << 16),
                                  to_bf16_bits(v[4]) | (to_bf16_bits(v[5]) << 16),
                                  to_bf16_bits(v[6]) | (to_bf16_bits(v[7]) << 16));
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        sq[i] = part;
    }
    // tile loader: thread t fills quarter t & 3 of centroid row t >> 2 (32 halves: 4 x 16 bytes when
    // rows are 16-byte aligned, dpad % 8 == 0, else 8 x 8 bytes; dpad % 4 == 0, so a chunk is all in
    // or all out)
    const int lr = tid >> 2, lq = (tid & 3) * 32;
    const bool v16 = (dpad & 7) == 0;
    uint2 stg[8];
    float stc = 0.f;
    auto gload = [&](int t) {
        const int c = t * GN + lr;
        const uint16_t *src = cent_h + (int64_t)c * dpad + lq;
        if (v16) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint4 v = (c < nlist && lq + 8 * q < dpad) ? *reinterpret_cast<const uint4 *>(src + 8 * q)
                                                                 : make_uint4(0u, 0u, 0u, 0u);
                stg[2 * q] = make_uint2(v.x, v.y);
                stg[2 * q + 1] = make_uint2(v.z, v.w);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; q++)
                stg[q] = (c < nlist && lq + 4 * q < dpad) ? *reinterpret_cast<const uint2 *>(src + 4 * q)
                                                          : make_uint2(0u, 0u);
        }
        if (tid < GN) {
            const int cc = t * GN + tid;
            stc = cc < nlist ? (METRIC == 0 ? cn2[cc] : 0.f) : __builtin_inff();
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; q++)
            *reinterpret_cast<uint4 *>(&sB[buf][lr * HBLD + lq + 8 * q]) =
                make_uint4(stg[2 * q].x, stg[2 * q].y, stg[2 * q + 1].x, stg[2 * q + 1].y);
        if (tid < GN) sC[buf][tid] = stc;
    };
    gload(t0);
    lstore(0);
    __syncthreads();
    const bool vec = (ldo & 3) == 0;
    // per row i, this lane's smallest (b1, at segment position ba) and second smallest b2 of |c|^2 - 2 x.c
    float b1[2] = {__builtin_inff(), __builtin_inff()}, b2[2] = {__builtin_inff(), __builtin_inff()};
    int ba[2] = {0, 0};
    for (int t = t0; t < t1; t++) {
        const int cur = (t - t0) & 1;
        if (t + 1 < t1) gload(t + 1);
        floatx4 acc[2][8];
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 8; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint4 b = *reinterpret_cast<const uint4 *>(
                    &sB[cur][(16 * j + (lane & 15)) * HBLD + 32 * ks + 8 * (lane >> 4)]);
#pragma unroll
                for (int i = 0; i < 2; i++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cbf16x8, b),
                                                                       __builtin_bit_cast(cbf16x8, a[i][ks]),
                                                                       acc[i][j], 0, 0, 0);
            }
        }
        // lane: row 16 i + lane % 16, lists 16 j + 4 (lane / 16) .. +3 of the tile
#pragma unroll
        for (int i = 0; i < 2; i++) {
            float gm[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const float4 c2 = *reinterpret_cast<const float4 *>(&sC[cur][16 * j + 4 * (lane >> 4)]);
                const float cs[4] = {c2.x, c2.y, c2.z, c2.w};
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; r++)   // lists past nlist carry |c|^2 = +inf (IP: masked the same way)
                    v[r] = METRIC == 0 ? fmaf(-2.0f, acc[i][j][r], cs[r])
                                       : (cs[r] == 0.f ? -acc[i][j][r] : __builtin_inff());
                // smallest (at position qp) and second smallest of the 4 values by a min / max network;
                // fminf / fmaxf drop a NaN, so a NaN counts as +inf or duplicates a value (never a
                // smaller second value)
                const float lo01 = fminf(v[0], v[1]), lo23 = fminf(v[2], v[3]);
                float m1 = fminf(lo01, lo23);
                if (TRACK) {
                    const float hi01 = fmaxf(v[0], v[1]), hi23 = fmaxf(v[2], v[3]);
                    const bool c23 = lo23 < lo01;
                    const float qsec = fminf(fmaxf(lo01, lo23), fminf(hi01, hi23));
                    const int qp = c23 ? (v[3] < v[2] ? 3 : 2) : (v[1] < v[0] ? 1 : 0);
                    // merge into the running pair: the second smallest of {b1, b2, m1, qsec}
                    const float nb2 = fminf(fmaxf(b1[i], m1), fminf(b2[i], qsec));
                    if (m1 < b1[i]) ba[i] = (t - t0) * GN + 16 * j + 4 * (lane >> 4) + qp;
                    b1[i] = fminf(b1[i], m1);
                    b2[i] = nb2;
                }
                m1 = fminf(m1, __shfl_xor(m1, 16));
                m1 = fminf(m1, __shfl_xor(m1, 32));
                gm[j] = METRIC == 0 ? sq[i] + m1 : m1;
            }
            const int gr = r0 + 32 * w + 16 * i + (lane & 15);
            if ((lane >> 4) == 0 && gr < n) {
                float *o = out + (int64_t)gr * ldo + t * (GN / GROUP);
                if (vec && t * (GN / GROUP) + 8 <= ldo) {
                    *reinterpret_cast<float4 *>(o) = make_float4(gm[0], gm[1], gm[2], gm[3]);
                    *reinterpret_cast<float4 *>(o + 4) = make_float4(gm[4], gm[5], gm[6], gm[7]);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j++)
                        if (t * (GN / GROUP) + j < ldo) o[j] = gm[j];
                }
            }
        }
        if (t + 1 < t1) lstore(cur ^ 1);   // its last readers finished before the previous barrier
        __syncthreads();
    }
    if (MODE == GM_SEG) {
#pragma unroll
        for (int i = 0; i < 2; i++) {
            min2_xor<16>(b1[i], b2[i], ba[i]);
            min2_xor<32>(b1[i], b2[i], ba[i]);
            const int gr = r0 + 32 * w + 16 * i + (lane & 15);
            // adding |x|^2 is monotone: the order, and so the position, stay
            if ((lane >> 4) == 0 && gr < n)
                out2[(int64_t)gr * ncs + sg] = min2_pack(METRIC == 0 ? sq[i] + b2[i] : b2[i], ba[i]);
        }
    }
    if (DEC) {
        const double cm = *cmax;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            min2_xor<16>(b1[i], b2[i], ba[i]);
            min2_xor<32>(b1[i], b2[i], ba[i]);
            const int gr = r0 + 32 * w + 16 * i + (lane & 15);
            if ((lane >> 4) == 0 && gr < n) {
                // an upper bound on |x| from the fp32 sum of squares (d + 2 roundings of at most 2^-24
                // relative each; the additive term covers squares flushed to zero); a non-finite
                // coordinate makes it inf or NaN, and the row is left undecided
                const double qn = sqrt((double)sq[i] * (1.0 + (d + 4) * 0x1p-23)) * (1.0 + 0x1p-50) + 0x1p-56;
                const double e = coarse_err(METRIC, d, 1, qn, cm);
                const float d1 = METRIC == 0 ? sq[i] + b1[i] : b1[i], d2 = METRIC == 0 ? sq[i] + b2[i] : b2[i];
                const bool ok = qn + cm < 0x1p60 && (double)d2 - e > (double)d1 + e && ba[i] < nlist;
                assign[(int64_t)gr * assign_stride] = ok ? ba[i] : ASSIGN_UNDECIDED;
            }
        }
    }
}

// Canonical FP64 coarse distance (sequential fma over ascending dimensions;
// IP: minus the dot product) of row x to centroid c.  c is 16-byte aligned
// and zero-padded to a multiple of 4; x is read up to d (a padded x would add
// exact zeros).  Centroid values are fetched 32 at a time (8 float4) ahead of
// their fmas, so the loop is not one memory latency per dimension.
__device__ __forceinline__ double canon_dist(const float *x, const float *__restrict__ c, int d, int metric) {
    double r = 0.0;
    const float4 *c4 = reinterpret_cast<const float4 *>(c);
    int j = 0;
    for (; j + 32 <= d; j += 32) {
        float4 cv[8];
#pragma unroll
        for (int e = 0; e < 8; e++) cv[e] = c4[(j >> 2) + e];
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const float cs[4] = {cv[e].x, cv[e].y, cv[e].z, cv[e].w};
#pragma unroll
            for (int f = 0; f < 4; f++) {
                const double xv = (double)x[j + 4 * e + f];
                if (metric == 0) {
                    const double t = xv - (double)cs[f];
                    r = __fma_rn(t, t, r);
                } else {
                    r = __fma_rn(xv, (double)cs[f], r);
                }
            }
        }
    }
    for (; j < d; j++) {
        const double xv = (double)x[j];
        if (metric == 0) {
            const double t = xv - (double)c[j];
            r = __fma_rn(t, t, r);
        } else {
            r = __fma_rn(xv, (double)c[j], r);
        }
    }
    return metric == 0 ? r : -r;
}

constexpr int SEL_CAP = 512;   // candidates buffered per exact re-check round

// One block of 256 threads per row.  Dynamic shared memory:
//   sx[dpad] float | kd[mmax] kl[mmax] nd[mmax] nl[mmax] | cd[SEL_CAP] cl[SEL_CAP]
__global__ __launch_bounds__(256) void k_coarse_select(
    const float *__restrict__ dt, const float *__restrict__ X, int n, int d, const float *__restrict__ cent,
    int dpad, const double *__restrict__ cnorm, const double *__restrict__ cmax, int nlist, int metric,
    int m_uniform, const int32_t *__restrict__ m_per_row, int mmax, int32_t *__restrict__ out,
    int out_stride, const int32_t *ctl, int gated, int bf) {
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
    const double qn = sqrt(sred[0] + sred[1] + sred[2] + sred[3]) * (1.0 + 0x1p-50);
    const double cm = *cmax;
    const double emax = coarse_err(metric, d, bf, qn, cm);
    // Below 2^60 for |x| + max |c| no fp32 square, norm sum or dot product of
    // the GEMM can overflow, so every approximation is finite and the bound
    // holds; above it (or for a non-finite norm) every list is re-checked.
    const bool every = !(qn + cm < 0x1p60);
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
            const double el = coarse_err(metric, d, bf, qn, cn);
            // written as "not above" so that a NaN approximation (or a NaN
            // tau) keeps the list as a candidate
            isc = (every || !(dv - el > ub)) ? 1 : 0;
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

// The same selection for up to 2,048 lists and nprobe <= 64, one wave per
// row and no block barrier: the row's approximate distances sit in registers
// (lane l holds lists l + 64 i); tau, the m-th smallest, is found bit by bit
// on their ordered keys (the key the radix select above finds); candidates
// (the same test) are queued per wave in LDS and re-checked 64 at a time, each
// batch merged into the row's best m -- sorted across the lanes by (exact
// distance, list id) -- by a bitonic network.
constexpr int SW_MAXL = 2048, SW_MAXM = 64, SW_Q = 128;

__device__ __forceinline__ uint64_t ord64(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x + 0.0);   // -0 ranks as +0
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ bool lex_less(uint64_t ka, int la, uint64_t kb, int lb) {
    return ka < kb || (ka == kb && la < lb);
}

// One compare-exchange step over the 64 lanes (blocks of K lanes, partner
// distance J) on (key, list) pairs; asc: the final order.
template <int J>
__device__ __forceinline__ void sel_step(uint64_t &k, int &l, int K, bool asc) {
    const int lane = lane_id();
    const uint64_t pk = xor_lane_u64<J>(k);
    const int pl = (int)xor_lane<J>((uint32_t)l);
    const bool up = ((lane & K) == 0) == asc;
    const bool keep_min = ((lane & J) == 0) == up;
    const bool p_less = lex_less(pk, pl, k, l);
    if (keep_min == p_less) {   // take the partner's pair
        k = pk;
        l = pl;
    }
}

// Half-cleaners J = 32 .. 1 of blocks of K lanes.
__device__ __forceinline__ void sel_clean(uint64_t &k, int &l, int K, bool asc) {
    if (K > 32) sel_step<32>(k, l, K, asc);
    if (K > 16) sel_step<16>(k, l, K, asc);
    if (K > 8) sel_step<8>(k, l, K, asc);
    if (K > 4) sel_step<4>(k, l, K, asc);
    if (K > 2) sel_step<2>(k, l, K, asc);
    sel_step<1>(k, l, K, asc);
}

__device__ __forceinline__ void sel_sort64(uint64_t &k, int &l, bool asc) {
#pragma unroll
    for (int K = 2; K <= 64; K <<= 1) sel_clean(k, l, K, asc);
}

__global__ __launch_bounds__(256) void k_coarse_select_w(
    const float *__restrict__ dt, const float *__restrict__ X, int n, int d, const float *__restrict__ cent,
    int dpad, const double *__restrict__ cnorm, const double *__restrict__ cmax, int nlist, int metric,
    int m_uniform, const int32_t *__restrict__ m_per_row, int mmax, int32_t *__restrict__ out,
    int out_stride, const int32_t *ctl, int gated, int bf) {
    extern __shared__ __align__(16) unsigned char smem[];   // per wave: the row (dpad floats), then the queue
    if (gated && call_failed(ctl)) return;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int row = blockIdx.x * 4 + w;
    if (row >= n) return;   // whole waves only: this kernel has no block barrier
    float *sx = reinterpret_cast<float *>(smem) + w * dpad;
    int *qu = reinterpret_cast<int *>(reinterpret_cast<float *>(smem) + 4 * dpad) + w * SW_Q;
    int m = m_per_row ? m_per_row[row] : m_uniform;
    m = m < nlist ? m : nlist;
    m = m < mmax ? m : mmax;
    m = m < 1 ? 1 : m;
    const float *xr = X + (int64_t)row * d;
    double q2 = 0.0;
    for (int j = lane; j < dpad; j += 64) {
        const float v = j < d ? xr[j] : 0.f;
        sx[j] = v;
        q2 = __fma_rn((double)v, (double)v, q2);
    }
    for (int o = 32; o > 0; o >>= 1) q2 += __shfl_xor(q2, o);
    const double qn = sqrt(q2) * (1.0 + 0x1p-50);
    const double cm = *cmax;
    const double emax = coarse_err(metric, d, bf, qn, cm);
    const bool every = !(qn + cm < 0x1p60);
    const float *drow = dt + (int64_t)row * nlist;
    uint32_t key[SW_MAXL / 64];
#pragma unroll
    for (int i = 0; i < SW_MAXL / 64; i++) {
        const int l = 64 * i + lane;
        key[i] = l < nlist ? ord_bits(drow[l]) : 0xFFFFFFFFu;
    }
    // tau: the m-th smallest key, bit by bit (count(key < t) < m keeps bit b set); counts by ballot
    const int ni = (nlist + 63) >> 6;
    uint32_t t = 0;
    for (int b = 31; b >= 0; b--) {
        const uint32_t trial = t | (1u << b);
        int c = 0;
#pragma unroll
        for (int i = 0; i < SW_MAXL / 64; i++)
            if (i < ni) c += (int)__builtin_popcountll(ballot(key[i] < trial));
        if (c < m) t = trial;
    }
    const double ub = (double)from_ord(t) + emax;
    // the row's best m so far: rank r in lane r (empty: all ones)
    uint64_t bk = ~0ull;
    int bl = 0x7FFFFFFF;
    int qn_ = 0;
    auto batch = [&](int c) {   // re-check queue[0, c) (c <= 64) and merge it in
        const int lc = lane < c ? qu[lane] : -1;
        uint64_t k = ~0ull;
        int l = 0x7FFFFFFF;
        if (lc >= 0) {
            k = ord64(canon_dist(sx, cent + (int64_t)lc * dpad, d, metric));
            l = lc;
        }
        sel_sort64(k, l, false);   // descending: the element-wise minimum with bk is bitonic
        if (lex_less(k, l, bk, bl)) {
            bk = k;
            bl = l;
        }
        sel_clean(bk, bl, 64, true);
    };
    // candidate test of every list first (all norm loads in flight together), then the queue
    uint32_t cbits = 0;
#pragma unroll
    for (int i = 0; i < SW_MAXL / 64; i++) {
        const int l = 64 * i + lane;
        if (i < ni && l < nlist) {
            const double dv = (double)from_ord(key[i]);
            const double el = coarse_err(metric, d, bf, qn, cnorm[l]);
            cbits |= (every || !(dv - el > ub)) ? (1u << i) : 0u;   // "not above": a NaN keeps the list
        }
    }
    for (int i = 0; i < ni; i++) {
        const int l = 64 * i + lane;
        const bool isc = (cbits >> i) & 1u;
        const uint64_t bm = ballot(isc);
        if (bm) {
            if (isc) qu[qn_ + (int)__builtin_popcountll(bm & lanemask_lt())] = l;
            qn_ += (int)__builtin_popcountll(bm);
            __builtin_amdgcn_wave_barrier();
            if (qn_ >= 64) {
                batch(64);
                const int rest = qn_ - 64;
                const int v = lane < rest ? qu[64 + lane] : 0;
                __builtin_amdgcn_wave_barrier();
                if (lane < rest) qu[lane] = v;
                __builtin_amdgcn_wave_barrier();
                qn_ = rest;
            }
        }
    }
    if (qn_ > 0) batch(qn_);
    int32_t *orow = out + (int64_t)row * out_stride;
    for (int p = lane; p < out_stride; p += 64) orow[p] = (p < m && bl != 0x7FFFFFFF) ? bl : -1;
}

// Nearest list per row (m = 1) from the group minima of k_coarse_gemm<.., 1>.
// tau = the smallest approximate distance; every list whose certified
// interval can reach below the best one lies in a group whose minimum is at
// most tau + 2 max E, so those groups are re-checked exactly (canonical FP64
// distance, ties to the lower list).  When the second smallest approximate
// distance of the row (the other groups' minima and the best group's second
// value) exceeds tau + 2 max E, no other list can reach below the best one:
// its canonical distance is smaller than every other list's, and it is taken
// without a re-check.  Rows with a non-finite coordinate get -1 (the insert
// then fails); rows or centroids so large that fp32 squares could overflow
// are re-checked against every list.  One wave per row (row wave-uniform: its
// coordinates are read through the scalar cache).  Without gsec (rows the
// group-minima kernel left undecided) the separation test is skipped.
__device__ __forceinline__ void argmin_row(int row, const float *__restrict__ gmin,
                                           const uint32_t *__restrict__ gsec, int gps, int ldg,
                                           const float *__restrict__ X, int d,
                                           const float *__restrict__ cent, int dpad,
                                           const double *__restrict__ cmax, int nlist, int metric,
                                           int32_t *__restrict__ out, int out_stride, int bf) {
    const int lane = threadIdx.x & 63;
    const float *xr = X + (int64_t)row * d;
    double q2 = 0.0;
    bool fin = true;
    for (int j = lane; j < d; j += 64) {
        const float v = xr[j];
        fin = fin && __builtin_isfinite(v);
        q2 = __fma_rn((double)v, (double)v, q2);
    }
    if (ballot(!fin)) {
        if (lane == 0) out[(int64_t)row * out_stride] = -1;
        return;
    }
    for (int o = 32; o > 0; o >>= 1) q2 += __shfl_xor(q2, o);
    const double qn = sqrt(q2) * (1.0 + 0x1p-50);
    const double cm = *cmax;
    const double emax = coarse_err(metric, d, bf, qn, cm);
    const bool every = !(qn + cm < 0x1p60);
    const float *g = gmin + (int64_t)row * ldg;
    // the smallest group minimum t (group tg) and the second smallest t2
    float t = __builtin_inff(), t2 = __builtin_inff();
    int tg = 0x7fffffff;
    for (int gi = lane; gi < ldg; gi += 64) min2_push(t, t2, tg, g[gi], gi);
    min2_xor<32>(t, t2, tg);
    min2_xor<16>(t, t2, tg);
    min2_xor<8>(t, t2, tg);
    min2_xor<4>(t, t2, tg);
    min2_xor<2>(t, t2, tg);
    min2_xor<1>(t, t2, tg);
    if (gsec && !every && tg < ldg) {
        // segments of gps groups: the best group's segment gives the position of the smallest and
        // its second smallest; t2 covers the lists of every other group
        const int sg = tg / gps, nseg = (ldg + gps - 1) / gps;
        const uint32_t p = gsec[(int64_t)row * nseg + sg];
        const float sec = fminf(t2, from_ord(p & ~SEG_MASK));
        const int l = sg * gps * GROUP + (int)(p & SEG_MASK);
        if ((double)sec - emax > (double)t + emax && l < nlist) {
            if (lane == 0) out[(int64_t)row * out_stride] = l;
            return;
        }
    }
    const double ub = (double)t + 2.0 * emax;
    double best = __builtin_inf();
    int bestl = 0x7fffffff;
    for (int g0 = 0; g0 < ldg; g0 += 64) {
        const int gi = g0 + lane;
        uint64_t mask = ballot(gi < ldg && (every || (double)g[gi] <= ub));
        while (mask) {
            // up to 4 qualifying groups per pass, 16 lanes (lists) each
            int sel = -1;
            for (int s = 0; s < 4 && mask; s++) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1;
                if ((lane >> 4) == s) sel = g0 + b;
            }
            const int l = sel * GROUP + (lane & 15);
            if (sel >= 0 && l < nlist) {
                const double r = canon_dist(xr, cent + (int64_t)l * dpad, d, metric);
                if (r < best || (r == best && l < bestl)) {
                    best = r;
                    bestl = l;
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int ol = __shfl_xor(bestl, o);
        if (ob < best || (ob == best && ol < bestl)) {
            best = ob;
            bestl = ol;
        }
    }
    if (lane == 0) out[(int64_t)row * out_stride] = bestl < nlist ? bestl : -1;
}

// all_rows: one wave per row.  Otherwise every wave takes chunks of AM_CHUNK
// rows and re-checks only those marked ASSIGN_UNDECIDED (small chunks: the
// re-checks, a latency chain each, spread over many waves).
constexpr int AM_CHUNK = 16, AM_MAXB = 16384;
__global__ __launch_bounds__(256) void k_coarse_argmin(const float *__restrict__ gmin,
                                                       const uint32_t *__restrict__ gsec, int gps, int ldg,
                                                       const float *__restrict__ X, int n, int d,
                                                       const float *__restrict__ cent, int dpad,
                                                       const double *__restrict__ cmax, int nlist, int metric,
                                                       int32_t *__restrict__ out, int out_stride,
                                                       const int32_t *ctl, int gated, int bf, int all_rows) {
    if (gated && call_failed(ctl)) return;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (all_rows) {
        const int row = __builtin_amdgcn_readfirstlane(wid);
        if (row < n) argmin_row(row, gmin, gsec, gps, ldg, X, d, cent, dpad, cmax, nlist, metric, out, out_stride, bf);
        return;
    }
    const int nw = gridDim.x * 4, lane = threadIdx.x & 63;
    for (int c0 = wid * AM_CHUNK; c0 < n; c0 += nw * AM_CHUNK) {
        const int r = c0 + lane;
        uint64_t m = ballot(lane < AM_CHUNK && r < n && out[(int64_t)r * out_stride] == ASSIGN_UNDECIDED);
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            argmin_row(__builtin_amdgcn_readfirstlane(c0 + b), gmin, nullptr, 1, ldg, X, d, cent, dpad, cmax,
                       nlist, metric, out, out_stride, bf);
        }
    }
}

size_t coarse_select_smem(int dpad, int mmax) {
    return (size_t)(2 * mmax + SEL_CAP) * sizeof(double) + (size_t)(2 * mmax + SEL_CAP) * sizeof(int) +
           (size_t)dpad * sizeof(float) + 16;
}

template <int GMIN>
static void coarse_gemm_t(hipStream_t st, const float *X, int n, int d, const float *cent,
                          const uint16_t *cent_h, int dpad,
                          const float *cn2, int nlist, int metric, float *out, uint32_t *out2, int ldo,
                          const int32_t *ctl, int gated, int bf) {
    const int nrb = (n + GM - 1) / GM, ncb = (nlist + GN - 1) / GN;
    const int xcd_map = ncb >= 8 ? 1 : 0;   // fewer centroid blocks than XCDs: plain order
    const unsigned grid = xcd_map ? (unsigned)(8 * ((ncb + 7) / 8) * nrb) : (unsigned)(nrb * ncb);
    const bool vec = (d % 4 == 0) && (((uintptr_t)X & 15) == 0);
#define SIVF_GEMM(M, V, B)                                                                                      \
    hipLaunchKernelGGL((k_coarse_gemm<M, GMIN, V, B>), dim3(grid), dim3(256), 0, st, X, n, d, cent, cent_h, dpad, \
                       cn2, nlist, out, out2, ldo, ctl, gated, xcd_map)
#define SIVF_GEMM_B(M, V)                                                                                       \
    do {                                                                                                        \
        if (bf) SIVF_GEMM(M, V, 1); else SIVF_GEMM(M, V, 0);                                                    \
    } while (0)
    if (metric == 0) {
        if (vec) SIVF_GEMM_B(0, true); else SIVF_GEMM_B(0, false);
    } else {
        if (vec) SIVF_GEMM_B(1, true); else SIVF_GEMM_B(1, false);
    }
#undef SIVF_GEMM_B
#undef SIVF_GEMM
}

void launch_coarse_gemm(hipStream_t st, const float *X, int n, int d, const float *cent, const uint16_t *cent_h, int dpad,
                        const float *cn2, int nlist, int metric, float *out, const int32_t *ctl,
                        int gated, int bf) {
    if (n > 0) coarse_gemm_t<0>(st, X, n, d, cent, cent_h, dpad, cn2, nlist, metric, out, nullptr, nlist, ctl, gated, bf);
}

int coarse_groups(int nlist) { return (nlist + GROUP - 1) / GROUP; }

// Scratch words per (row, group) of the nearest-list path: the group minima,
// plus room for the second-minimum words except in the plain bf16 sweep (more
// than 16 tiles of lists).
int coarse_assign_words(int nlist, int dpad) {
    return (dpad <= HK && (nlist + GN - 1) / GN > 16) ? 1 : 2;
}

void launch_coarse_assign(hipStream_t st, float *scratch, const float *X, int n, int d, const float *cent,
                          const uint16_t *cent_h, int dpad, const float *cn2, const double *cmax, int nlist, int metric, int32_t *out,
                          int out_stride, const int32_t *ctl, int gated, int bf) {
    if (n <= 0) return;
    const int ldg = coarse_groups(nlist);
    // group minima (n ldg words), then the packed second values (at most n ldg words; none in the
    // plain sweep, see coarse_assign_words)
    uint32_t *gsec = reinterpret_cast<uint32_t *>(scratch + (int64_t)n * ldg);
    bool decided = false;
    int gps = 1;   // groups per segment of gsec
    if (bf && dpad <= HK) {
        // row-stationary bf16 sweep: segments of nct centroid tiles, enough blocks to fill the chip
        const int nrb = (n + HR - 1) / HR, ncb = (nlist + GN - 1) / GN;
        int nct = (int)(((int64_t)nrb * ncb) / 1024);
        nct = nct < 1 ? 1 : (nct > 16 ? 16 : nct);
        // a block per CU at least, and 16 tiles or fewer: one segment, so rows are decided in the sweep
        if (nrb >= 256 && ncb <= 16) nct = ncb;
        const int ncs = (ncb + nct - 1) / nct;
        const int xcd_map = ncs >= 8 ? 1 : 0;
        const unsigned grid = xcd_map ? (unsigned)(8 * ((ncs + 7) / 8) * nrb) : (unsigned)(nrb * ncs);
        decided = ncs == 1;   // one block sees every list of its rows
        const int mode = decided ? GM_DEC : (ncb <= 16 ? GM_SEG : GM_PLAIN);
        gps = nct * (GN / GROUP);
        if (mode == GM_PLAIN) gsec = nullptr;
#define SIVF_GMIN(M, MODE)                                                                                       \
    hipLaunchKernelGGL((k_coarse_gmin_h<M, MODE>), dim3(grid), dim3(64 * HW), 0, st, X, n, d, cent_h, dpad, cn2,  \
                       nlist, scratch, gsec, ldg, nct, xcd_map, cmax, out, out_stride, ctl, gated)
#define SIVF_GMIN_M(M)                                                                                           \
    do {                                                                                                         \
        if (mode == GM_DEC) SIVF_GMIN(M, GM_DEC);                                                                \
        else if (mode == GM_SEG) SIVF_GMIN(M, GM_SEG);                                                           \
        else SIVF_GMIN(M, GM_PLAIN);                                                                             \
    } while (0)
        if (metric == 0) SIVF_GMIN_M(0); else SIVF_GMIN_M(1);
#undef SIVF_GMIN_M
#undef SIVF_GMIN
    } else {
        coarse_gemm_t<1>(st, X, n, d, cent, cent_h, dpad, cn2, nlist, metric, scratch, gsec, ldg, ctl, gated, bf);
    }
    if (decided) {
        const int chunks = (n + AM_CHUNK - 1) / AM_CHUNK, nb = (chunks + 3) / 4;
        hipLaunchKernelGGL(k_coarse_argmin, dim3(nb < AM_MAXB ? nb : AM_MAXB), dim3(256), 0, st, scratch, nullptr, 1, ldg, X,
                           n, d, cent, dpad, cmax, nlist, metric, out, out_stride, ctl, gated, bf, 0);
    } else {
        hipLaunchKernelGGL(k_coarse_argmin, dim3((n + 3) / 4), dim3(256), 0, st, scratch, gsec, gps, ldg, X, n, d, cent,
                           dpad, cmax, nlist, metric, out, out_stride, ctl, gated, bf, 1);
    }
}

void launch_coarse_select(hipStream_t st, const float *dt, const float *X, int n, int d, const float *cent,
                          int dpad, const double *cnorm, const double *cmax, int nlist, int metric,
                          int m_uniform, const int32_t *m_per_row, int mmax, int32_t *out, int out_stride,
                          const int32_t *ctl, int gated, int bf) {
    if (n <= 0) return;
    if (nlist <= SW_MAXL && mmax <= SW_MAXM) {
        hipLaunchKernelGGL(k_coarse_select_w, dim3((n + 3) / 4), dim3(256),
                           (size_t)4 * dpad * sizeof(float) + (size_t)4 * SW_Q * sizeof(int), st, dt, X, n, d, cent,
                           dpad, cnorm, cmax, nlist, metric, m_uniform, m_per_row, mmax, out, out_stride, ctl, gated,
                           bf);
        return;
    }
    hipLaunchKernelGGL(k_coarse_select, dim3(n), dim3(256), coarse_select_smem(dpad, mmax), st, dt, X, n, d,
                       cent, dpad, cnorm, cmax, nlist, metric, m_uniform, m_per_row, mmax, out, out_stride,
                       ctl, gated, bf);
}

}  // namespace sivf
