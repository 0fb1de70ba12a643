// Lloyd's k-means for the IVF index phase (Section 2.2.2: the lists are the
// k-means clusters of the data; Section 6.1).  The host drives the iterations
// (api.hip: ads_kmeans); these are its kernels.
//
//   assignment: the inner products of a chunk of rows with every centre are
//   an FP32 GEMM on the matrix cores (gemm_nt_f32); argmin_kernel turns them
//   into |x|^2 + |c|^2 - 2 x.c and keeps the nearest centre, ties to the lower
//   centre id.
//   update: one wave per centre collects its members in ascending row order
//   and sums them in float64 in that order, so a centre depends only on its
//   member set (deterministic, independent of scheduling).
//   empty lists: farthest_kernel finds the member of a list farthest from its
//   centre (lower row on ties) with one 64-bit atomic maximum.
#include "kernels.h"

namespace ads {
namespace {

__global__ __launch_bounds__(ADS_WG) void gather_rows_kernel(const float *x, int D, const int32_t *rows,
                                                            int m, float *out) {
    const int j = blockIdx.x;
    if (j >= m) return;
    const int64_t r = rows[j];
    for (int i = threadIdx.x; i < D; i += ADS_WG) out[(int64_t)j * D + i] = x[r * D + i];
}

// One wave per row of the chunk: nearest centre by (squared distance, id).
__global__ __launch_bounds__(ADS_WG) void argmin_kernel(const float *dots, const float *xn, const float *cn,
                                                       int64_t m, int nlist, int32_t *assign, float *d2out) {
    const int64_t row = (int64_t)blockIdx.x * (ADS_WG / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const float *dr = dots + row * nlist;
    const float x2 = xn[row];
    float best = __builtin_inff();
    int bj = nlist;
    for (int j = lane; j < nlist; j += 64) {
        float d = x2 + cn[j] - 2.f * dr[j];
        d = d > 0.f ? d : 0.f;
        if (d < best) { best = d; bj = j; }        // j ascends per lane: the first minimum is kept
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float ob = __shfl_xor(best, o);
        const int oj = __shfl_xor(bj, o);
        if (ob < best || (ob == best && oj < bj)) { best = ob; bj = oj; }
    }
    if (lane == 0) {
        assign[row] = bj;
        d2out[row] = best;
    }
}

__global__ void count_kernel(const int32_t *assign, int64_t n, int32_t *counts) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&counts[assign[i]], 1);
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// The member of list l farthest from its centre: the largest (d2, -row) key.
__global__ void farthest_kernel(const int32_t *assign, const float *d2, int64_t n, int l,
                                unsigned long long *best) {
    unsigned long long mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (assign[i] != l) continue;
        const float d = d2[i] > 0.f ? d2[i] : 0.f;
        const unsigned long long key =
            ((unsigned long long)__float_as_uint(d) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)i);
        mine = key > mine ? key : mine;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(mine, o);
        mine = other > mine ? other : mine;
    }
    if ((threadIdx.x & 63) == 0 && mine) atomicMax(best, mine);
}

// One wave per centre: members in ascending row order, float64 sums in that
// order (LDS accumulators, D <= KM_DMAX), then the mean in float32.  A centre
// without members keeps its value.
constexpr int KM_DMAX = 4096;
constexpr int KM_BATCH = 512;

__global__ __launch_bounds__(64) void update_kernel(const float *x, int64_t n, int D, const int32_t *assign,
                                                    float *cent) {
    __shared__ double acc[KM_DMAX];
    __shared__ int32_t mem[KM_BATCH];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    for (int d = lane; d < D; d += 64) acc[d] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int64_t count = 0;
    int nb = 0;
    auto sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    auto flush = [&]() {
        sync();
        for (int t = 0; t < nb; ++t) {
            const float *xr = x + (int64_t)mem[t] * D;
            for (int d = lane; d < D; d += 64) acc[d] += (double)xr[d];
        }
        sync();
        nb = 0;
    };
    for (int64_t base = 0; base < n; base += 64) {
        const int64_t i = base + lane;
        const bool hit = i < n && assign[i] == j;
        const uint64_t m = __ballot(hit);
        if (!m) continue;
        const int c = __popcll(m);
        if (nb + c > KM_BATCH) flush();
        if (hit) mem[nb + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
        nb += c;
        count += c;
    }
    flush();
    if (count == 0) return;
    for (int d = lane; d < D; d += 64) cent[(int64_t)j * D + d] = (float)(acc[d] / (double)count);
}

}  // namespace

hipError_t launch_gather_rows(const float *x, int D, const int32_t *rows, int m, float *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)m), dim3(ADS_WG), 0, s, x, D, rows, m, out);
    return hipGetLastError();
}

hipError_t launch_argmin(const float *dots, const float *xn, const float *cn, int64_t m, int nlist,
                         int32_t *assign, float *d2, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t blocks = (m + ADS_WG / 64 - 1) / (ADS_WG / 64);
    hipLaunchKernelGGL(argmin_kernel, dim3((unsigned)blocks), dim3(ADS_WG), 0, s, dots, xn, cn, m, nlist, assign, d2);
    return hipGetLastError();
}

hipError_t launch_counts(const int32_t *assign, int64_t n, int nlist, int32_t *counts, hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(64), dim3(ADS_WG), 0, s, counts, (int64_t)nlist, 0);
    hipLaunchKernelGGL(count_kernel, dim3(1024), dim3(ADS_WG), 0, s, assign, n, counts);
    return hipGetLastError();
}

hipError_t launch_farthest(const int32_t *assign, const float *d2, int64_t n, int l, unsigned long long *best,
                           hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t *>(best), (int64_t)2, 0);
    hipLaunchKernelGGL(farthest_kernel, dim3(1024), dim3(ADS_WG), 0, s, assign, d2, n, l, best);
    return hipGetLastError();
}

hipError_t launch_update_centres(const float *x, int64_t n, int D, const int32_t *assign, int nlist, float *cent,
                                 hipStream_t s) {
    if (D > KM_DMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)nlist), dim3(64), 0, s, x, n, D, assign, cent);
    return hipGetLastError();
}

}  // namespace ads
