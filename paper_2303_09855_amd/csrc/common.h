// Internal helpers shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/ads.h"

#define ADS_WG 256          // threads per workgroup for every kernel here
#define ADS_WAVE 64

namespace ads {

// ---------------------------------------------------------------------------
// Keys: (squared distance, id) packed into one uint64 so that unsigned order is
// lexicographic order.  A non-negative float orders like its bit pattern.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t make_key(float s, uint32_t id) {
    return ((uint64_t)__float_as_uint(s) << 32) | (uint64_t)id;
}
__device__ __forceinline__ float key_dist2(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)k; }
constexpr uint64_t KEY_NONE = ~0ull;
// largest KNN-set capacity of a search (k_max, times 4 with the rerank)
constexpr int KCAP_LIMIT = 512;

// ---------------------------------------------------------------------------
// Stored layout of a list (IVF++, Section 5.2).  The first b1 blocks of dd
// coordinates of all the list's vectors are stored block by block
// ([block][vector][dd], the array A1 of the paper, read by the dense phase a
// tile at a time); the remaining D - b1 dd coordinates are stored vector by
// vector ([vector][D - b1 dd], the array A2, so the later blocks of one
// candidate are contiguous).  Element offset of block b of vector v within
// the list's slice of nl * D elements:
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t layout_offset(int64_t nl, int64_t v, int b, int dd, int b1, int D) {
    return b < b1 ? (int64_t)b * nl * dd + v * dd
                  : nl * (int64_t)b1 * dd + v * (int64_t)(D - b1 * dd) + (int64_t)(b - b1) * dd;
}

// ---------------------------------------------------------------------------
// Test coefficients.  For a DCO that has sampled d of D coordinates with
// partial sum S_d, ADSampling rejects dis <= r when
//     sqrt(D/d * S_d) > (1 + eps0/sqrt(d)) * r
// (Section 3.2), i.e. S_d > coef(d) * r^2 with coef(d) = (d/D)(1+eps0/sqrt(d))^2.
// PDScanning rejects when S_d > r^2 (coef = 1).  FDScanning never tests (+inf).
// Computed in double on the device by every kernel, so the scan and the
// explicit-candidate DCO use bit-identical thresholds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float test_coef(int d, int D, double eps0, int method) {
    if (method == ADS_METHOD_FDSCANNING) return __builtin_inff();
    if (method == ADS_METHOD_PDSCANNING) return 1.0f;
    if (__builtin_isinf(eps0)) return __builtin_inff();
    double g = 1.0 + eps0 / __builtin_sqrt((double)d);
    return (float)(((double)d / (double)D) * g * g);
}

// S > coef * r2 with the conventions: coef = +inf never rejects (also when
// r2 == 0, where inf * 0 would be NaN), r2 = +inf never rejects.
__device__ __forceinline__ bool test_reject(float s, float coef, float r2) {
    if (__builtin_isinf(coef)) return false;
    return s > coef * r2;
}

// ---------------------------------------------------------------------------
// Storage element loads (8 consecutive elements, converted to float).
// ---------------------------------------------------------------------------
template <int DT> struct Elem;
template <> struct Elem<ADS_F32> { typedef float T; static constexpr int bytes = 4; };
template <> struct Elem<ADS_BF16> { typedef uint16_t T; static constexpr int bytes = 2; };
template <> struct Elem<ADS_F16> { typedef uint16_t T; static constexpr int bytes = 2; };

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    return __half2float(__ushort_as_half((unsigned short)h));
}

// Loads N (multiple of 4 for f32, of 8 for 16-bit) contiguous elements starting
// at p (aligned to 16 bytes) into out[0..N).
template <int DT, int N>
__device__ __forceinline__ void load_elems(const void *p, float *out) {
    if constexpr (DT == ADS_F32) {
        const float4 *v = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
            float4 t = v[i];
            out[4 * i + 0] = t.x; out[4 * i + 1] = t.y; out[4 * i + 2] = t.z; out[4 * i + 3] = t.w;
        }
    } else {
        const uint4 *v = reinterpret_cast<const uint4 *>(p);
#pragma unroll
        for (int i = 0; i < N / 8; ++i) {
            uint4 t = v[i];
            uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (DT == ADS_BF16) {
                    out[8 * i + 2 * j + 0] = bf16_to_f32(w[j] & 0xffffu);
                    out[8 * i + 2 * j + 1] = bf16_to_f32(w[j] >> 16);
                } else {
                    out[8 * i + 2 * j + 0] = f16_to_f32(w[j] & 0xffffu);
                    out[8 * i + 2 * j + 1] = f16_to_f32(w[j] >> 16);
                }
            }
        }
    }
}

// One element of storage type DT at index i.
template <int DT>
__device__ __forceinline__ float load_one(const void *p, int64_t i) {
    if constexpr (DT == ADS_F32) return reinterpret_cast<const float *>(p)[i];
    else if constexpr (DT == ADS_BF16) return bf16_to_f32(reinterpret_cast<const uint16_t *>(p)[i]);
    else return f16_to_f32(reinterpret_cast<const uint16_t *>(p)[i]);
}

// ---------------------------------------------------------------------------
// Workgroup-wide bitonic sort of n (power of two) uint64 keys in LDS, ascending.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_bitonic_sort(uint64_t *buf, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t a = buf[i], b = buf[ixj];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) { buf[i] = b; buf[ixj] = a; }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wave (every lane active), by DPP:
// shifts by 1, 2, 4 and 8 lanes inside each 16-lane row, then the last lane of
// row 0 (row 2) added to row 1 (row 3) and lane 31 added to rows 2 and 3.  No
// LDS round trip; integer sums, so the result is exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

// ---------------------------------------------------------------------------
// Workgroup radix select: the k-th smallest (1-based) of n uint64 keys produced
// by get(i), passes of 8 bits from the most significant byte; it stops early
// once a single key carries the selected prefix.  The workgroup has 256
// threads (one histogram bin each).  hist: LDS [256] uint32; misc: LDS [8]
// uint32.  All threads return the key.  Requires 1 <= k <= n.
// ---------------------------------------------------------------------------
template <class Get>
__device__ uint64_t radix_kth(Get get, int n, int k, uint32_t *hist, uint32_t *misc) {
    __shared__ uint64_t found;
    uint64_t prefix = 0, pmask = 0;
    uint32_t kk = (uint32_t)k;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hist[t] = 0;
        __syncthreads();
        for (int i = t; i < n; i += blockDim.x) {
            uint64_t key = get(i);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        // inclusive prefix over the bins (within each wave, then across waves);
        // the bin holding the kk-th key is the one whose range covers kk
        const uint32_t h = hist[t];
        const uint32_t x = wave_incl_scan(h);
        if (lane == 63) misc[4 + wv] = x;
        __syncthreads();
        uint32_t base = 0;
        for (int w2 = 0; w2 < wv; ++w2) base += misc[4 + w2];
        const uint32_t incl = base + x, excl = incl - h;
        if (excl < kk && incl >= kk) {
            misc[0] = (uint32_t)t;
            misc[1] = kk - excl;
            misc[2] = h;
        }
        __syncthreads();
        const uint32_t sel = misc[0], cnt = misc[2];
        kk = misc[1];
        prefix |= (uint64_t)sel << shift;
        pmask |= (uint64_t)0xff << shift;
        __syncthreads();
        if (cnt == 1) {
            // one key carries the prefix: it is the k-th
            for (int i = t; i < n; i += blockDim.x) {
                uint64_t key = get(i);
                if ((key & pmask) == prefix) found = key;
            }
            __syncthreads();
            const uint64_t r = found;
            __syncthreads();
            return r;
        }
    }
    return prefix;
}

// ---------------------------------------------------------------------------
// k-th smallest (1-based) of n uint64 keys get(i), 1 <= k <= n, for a
// workgroup of NT threads (a multiple of 64, every thread calls it): radix
// select over bytes from the most significant one, stopping as soon as one key
// carries the selected prefix.  hist: LDS [256] uint32; misc: LDS [4] uint32;
// found: LDS uint64.  All threads return the key.
// ---------------------------------------------------------------------------
template <int NT, class Get>
__device__ uint64_t group_kth(Get get, int n, int k, uint32_t *hist, uint32_t *misc, uint64_t *found) {
    uint64_t prefix = 0, pmask = 0;
    uint32_t kk = (uint32_t)k;
    const int t = threadIdx.x;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = t; b < 256; b += NT) hist[b] = 0;
        __syncthreads();
        for (int i = t; i < n; i += NT) {
            const uint64_t key = get(i);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (t < 64) {
            // lane t owns bins 4t .. 4t+3; the bin whose cumulative range covers kk wins
            const uint32_t h0 = hist[4 * t], h1 = hist[4 * t + 1], h2 = hist[4 * t + 2], h3 = hist[4 * t + 3];
            const uint32_t sum = h0 + h1 + h2 + h3;
            const uint32_t x = wave_incl_scan(sum);
            const uint32_t c0 = x - sum, c1 = c0 + h0, c2 = c1 + h1, c3 = c2 + h2, c4 = c3 + h3;
            if (c0 < kk && kk <= c1) { misc[0] = 4 * t; misc[1] = kk - c0; misc[2] = h0; }
            if (c1 < kk && kk <= c2) { misc[0] = 4 * t + 1; misc[1] = kk - c1; misc[2] = h1; }
            if (c2 < kk && kk <= c3) { misc[0] = 4 * t + 2; misc[1] = kk - c2; misc[2] = h2; }
            if (c3 < kk && kk <= c4) { misc[0] = 4 * t + 3; misc[1] = kk - c3; misc[2] = h3; }
        }
        __syncthreads();
        const uint32_t sel = misc[0], cnt = misc[2];
        kk = misc[1];
        prefix |= (uint64_t)sel << shift;
        pmask |= (uint64_t)0xff << shift;
        __syncthreads();
        if (cnt == 1) {
            for (int i = t; i < n; i += NT) {
                const uint64_t key = get(i);
                if ((key & pmask) == prefix) *found = key;
            }
            __syncthreads();
            const uint64_t r = *found;
            __syncthreads();
            return r;
        }
    }
    return prefix;
}

// Exclusive prefix sum of one int per thread over a workgroup of W waves (every
// thread calls it); *total receives the sum.  wtot: LDS [W] ints.  Starts and
// ends with a workgroup barrier, so consecutive calls may share wtot.
template <int W>
__device__ int group_excl_scan(int v, int *wtot, int &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x = (int)wave_incl_scan((uint32_t)v);
    __syncthreads();
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
        const int t = wtot[ww];
        base += ww < w ? t : 0;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return base + x - v;
}

__host__ __device__ inline int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace ads
