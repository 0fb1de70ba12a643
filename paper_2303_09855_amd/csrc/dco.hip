// Explicit-candidate DCOs with a fixed threshold (Definition 2.1 decided by
// Algorithm 1, or by FDScanning / PDScanning), one lane per candidate; and the
// index-phase packing of rotated vectors into the blocked list layout.
#include "kernels.h"

namespace ads {

namespace {

template <int DT>
__global__ __launch_bounds__(ADS_WG) void dco_kernel(
    const void *__restrict__ data, const float *__restrict__ rows32, int source,
    const int64_t *__restrict__ list_off, const int32_t *__restrict__ list_of_pos,
    const int32_t *__restrict__ pos_of, int64_t n, int D, int dd, int b1, const float *__restrict__ q,
    const int64_t *__restrict__ cand, int64_t m, float r2, double eps0, int step, int method,
    uint8_t *__restrict__ mask, float *__restrict__ dist, int32_t *__restrict__ dims,
    unsigned long long *stats, IpArgs ipa) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_dco = 0, c_dims = 0, c_pos = 0;
    const bool ip = ipa.onorm != nullptr;
    float nn = 0.f;
    if (i < m && ip) {
        const int64_t id = cand[i];
        if (id >= 0 && id < n) {
            // <o,q> >= r  <=>  |o/|o| - q/|q||^2 <= 2 - 2 r / (|o||q|)   (Section 8, extension (1))
            nn = ipa.onorm[id] * (*ipa.qnorm);
            r2 = nn > 0.f ? 2.f - 2.f * ipa.r_ip / nn : (ipa.r_ip <= 0.f ? __builtin_inff() : -1.f);
        }
    }
    if (i < m) {
        const int64_t id = cand[i];
        if (id < 0 || id >= n) {
            mask[i] = 0;
            dist[i] = __builtin_nanf("");
            if (dims) dims[i] = -1;
        } else if (ip && (r2 < 0.f || nn == 0.f)) {
            // unreachable threshold, or a zero vector: decided without sampling
            const bool positive = nn == 0.f && ipa.r_ip <= 0.f;
            mask[i] = positive ? 1 : 0;
            dist[i] = positive ? 0.f : -__builtin_inff();
            if (dims) dims[i] = 0;
            c_dco = 1;
            c_pos = positive;
        } else {
            const int64_t p = pos_of[id];
            const int l = list_of_pos[p];
            const int64_t off = list_off[l];
            const int64_t nl = list_off[l + 1] - off;
            const int64_t v = p - off;
            // canonical order: partial sums of the layout's dd-wide blocks,
            // each from zero, added in block order (as in the scan kernel)
            float s_blocks = 0.f, pb = 0.f, s = 0.f;
            int next = step;
            int done = 0;
            int used = D;
            for (int t = 0; t < D; ++t) {
                float o;
                const int b = t / dd, k = t - b * dd;
                if (k == 0 && t > 0) {
                    s_blocks = s_blocks + pb;
                    pb = 0.f;
                }
                if (source) {
                    o = rows32[p * D + t];
                } else {
                    o = load_one<DT>(data, off * D + layout_offset(nl, v, b, dd, b1, D) + k);
                }
                float df = o - q[t];
                pb = __fmaf_rn(df, df, pb);
                s = s_blocks + pb;
                const int d = t + 1;
                if (d == next) {
                    next += step;
                    if (d < D && test_reject(s, test_coef(d, D, eps0, method), r2)) {
                        done = 1;
                        used = d;
                        break;
                    }
                }
            }
            const bool positive = !done && s <= r2;
            mask[i] = positive ? 1 : 0;
            if (ip) dist[i] = positive ? nn * (1.f - 0.5f * s) : -__builtin_inff();
            else dist[i] = positive ? __fsqrt_rn(s) : __builtin_inff();
            if (dims) dims[i] = used;
            c_dco = 1;
            c_dims = (unsigned long long)used;
            c_pos = positive;
        }
    }
    if (stats) {
        for (int o = 32; o > 0; o >>= 1) {
            c_dco += __shfl_down(c_dco, o);
            c_dims += __shfl_down(c_dims, o);
            c_pos += __shfl_down(c_pos, o);
        }
        if ((threadIdx.x & 63) == 0 && c_dco) {
            atomicAdd(stats + ADS_STAT_DCOS, c_dco);
            atomicAdd(stats + ADS_STAT_DIMS, c_dims);
            atomicAdd(stats + ADS_STAT_BYTES, c_dims * (unsigned long long)Elem<DT>::bytes);
            atomicAdd(stats + ADS_STAT_POSITIVES, c_pos);
        }
    }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)((b >> 16) | ((b & 0xffffu) ? 0x40u : 0u));
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// One thread per (stored position, group of 4 coordinates).
template <int DT>
__global__ __launch_bounds__(ADS_WG) void pack_kernel(
    const float *__restrict__ rot, const int32_t *__restrict__ ids,
    const int32_t *__restrict__ list_of_pos, const int64_t *__restrict__ list_off, int64_t n, int D,
    int dd, int b1, void *__restrict__ data, float *__restrict__ rows32) {
    const int G = D / 4;
    const int64_t tot = n * G;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / G;
        const int t = (int)(i - p * G) * 4;
        const int64_t id = ids[p];
        const float4 val = *reinterpret_cast<const float4 *>(rot + id * D + t);
        if (rows32) *reinterpret_cast<float4 *>(rows32 + p * D + t) = val;
        const int l = list_of_pos[p];
        const int64_t off = list_off[l];
        const int64_t nl = list_off[l + 1] - off;
        const int64_t v = p - off;
        const int b = t / dd, k = t - b * dd;
        const int64_t dst = off * D + layout_offset(nl, v, b, dd, b1, D) + k;
        const float vv[4] = {val.x, val.y, val.z, val.w};
        if constexpr (DT == ADS_F32) {
            *reinterpret_cast<float4 *>(reinterpret_cast<float *>(data) + dst) = val;
        } else {
            uint16_t *o = reinterpret_cast<uint16_t *>(data) + dst;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (DT == ADS_BF16) o[c] = f32_to_bf16_rne(vv[c]);
                else o[c] = __half_as_ushort(__float2half_rn(vv[c]));
            }
        }
    }
}

// out[r] = x[r] / |x[r]| (a zero row stays zero), norms[r] = |x[r]|.
__global__ __launch_bounds__(ADS_WG) void normalize_kernel(const float *x, int64_t n, int D, float *out,
                                                          float *norms) {
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    float acc = 0.f;
    for (int i = threadIdx.x; i < D; i += ADS_WG) acc = __fmaf_rn(x[r * D + i], x[r * D + i], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
    __shared__ float red[ADS_WG / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    const float nrm = __fsqrt_rn(red[0] + red[1] + red[2] + red[3]);
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    for (int i = threadIdx.x; i < D; i += ADS_WG) out[r * D + i] = x[r * D + i] * inv;
    if (threadIdx.x == 0 && norms) norms[r] = nrm;
}

__global__ __launch_bounds__(ADS_WG) void row_norms_kernel(const float *x, int64_t n, int D, float *out) {
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    float acc = 0.f;
    for (int i = threadIdx.x; i < D; i += ADS_WG) acc = __fmaf_rn(x[r * D + i], x[r * D + i], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
    __shared__ float red[ADS_WG / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace

hipError_t launch_dco(int dtype, const void *data, const float *rows32, int source,
                      const int64_t *list_off, const int32_t *list_of_pos, const int32_t *pos_of,
                      int64_t n, int D, int dd_layout, int b1, const float *q, const int64_t *cand,
                      int64_t m, float r2, double eps0, int step, int method, uint8_t *mask,
                      float *dist, int32_t *dims, unsigned long long *stats, const IpArgs *ip,
                      hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((m + ADS_WG - 1) / ADS_WG);
    const IpArgs ipa = ip ? *ip : IpArgs{nullptr, nullptr, 0.f};
    switch (dtype) {
        case ADS_F32:
            hipLaunchKernelGGL(dco_kernel<ADS_F32>, dim3(grid), dim3(ADS_WG), 0, s, data, rows32, source,
                               list_off, list_of_pos, pos_of, n, D, dd_layout, b1, q, cand, m, r2, eps0,
                               step, method, mask, dist, dims, stats, ipa);
            break;
        case ADS_BF16:
            hipLaunchKernelGGL(dco_kernel<ADS_BF16>, dim3(grid), dim3(ADS_WG), 0, s, data, rows32, source,
                               list_off, list_of_pos, pos_of, n, D, dd_layout, b1, q, cand, m, r2, eps0,
                               step, method, mask, dist, dims, stats, ipa);
            break;
        case ADS_F16:
            hipLaunchKernelGGL(dco_kernel<ADS_F16>, dim3(grid), dim3(ADS_WG), 0, s, data, rows32, source,
                               list_off, list_of_pos, pos_of, n, D, dd_layout, b1, q, cand, m, r2, eps0,
                               step, method, mask, dist, dims, stats, ipa);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack(int dtype, const float *rot, const int32_t *ids, const int32_t *list_of_pos,
                       const int64_t *list_off, int64_t n, int D, int dd, int b1, void *data,
                       float *rows32, hipStream_t s) {
    const int64_t tot = n * (D / 4);
    int64_t g = (tot + ADS_WG - 1) / ADS_WG;
    const unsigned grid = (unsigned)(g > 65536 * 4 ? 65536 * 4 : g);
    switch (dtype) {
        case ADS_F32:
            hipLaunchKernelGGL(pack_kernel<ADS_F32>, dim3(grid), dim3(ADS_WG), 0, s, rot, ids, list_of_pos,
                               list_off, n, D, dd, b1, data, rows32);
            break;
        case ADS_BF16:
            hipLaunchKernelGGL(pack_kernel<ADS_BF16>, dim3(grid), dim3(ADS_WG), 0, s, rot, ids, list_of_pos,
                               list_off, n, D, dd, b1, data, rows32);
            break;
        case ADS_F16:
            hipLaunchKernelGGL(pack_kernel<ADS_F16>, dim3(grid), dim3(ADS_WG), 0, s, rot, ids, list_of_pos,
                               list_off, n, D, dd, b1, data, rows32);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_normalize(const float *x, int64_t n, int D, float *out, float *norms, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)n), dim3(ADS_WG), 0, s, x, n, D, out, norms);
    return hipGetLastError();
}

hipError_t launch_row_norms(const float *x, int64_t n, int D, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)n), dim3(ADS_WG), 0, s, x, n, D, out);
    return hipGetLastError();
}

}  // namespace ads
