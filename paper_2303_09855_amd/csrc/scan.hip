// Kernels of an IVF+ / IVF++ search around the candidate scan (Sections
// 2.2.2 and 4): per-query setup, probe selection, grouping of (query, list)
// pairs by list, per-query merges after each sweep, the output and the float32
// rerank; and the dispatch of the scan kernel (scan_kernel.h) over its
// instantiations.
#include "kernels.h"

namespace ads {

template <int DT>
hipError_t launch_scan_d(const ScanArgs &a, int dd, int qw, int grid, bool pf, bool wide, hipStream_t s) {
    switch (dd) {
        case 8: return launch_scan_q<DT, 8>(a, qw, grid, pf, wide, s);
        case 16: return launch_scan_q<DT, 16>(a, qw, grid, pf, wide, s);
        case 32: return launch_scan_q<DT, 32>(a, qw, grid, pf, wide, s);
        case 64: return launch_scan_q<DT, 64>(a, qw, grid, pf, wide, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scan(const ScanArgs &a, int dtype, int dd, int qw, int grid, bool pf, bool wide, hipStream_t s) {
    switch (dtype) {
        case ADS_F32: return launch_scan_d<ADS_F32>(a, dd, qw, grid, pf, wide, s);
        case ADS_BF16: return launch_scan_d<ADS_BF16>(a, dd, qw, grid, pf, wide, s);
        case ADS_F16: return launch_scan_d<ADS_F16>(a, dd, qw, grid, pf, wide, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Sweep of a probe rank: [0,1) -> 0, [1,4) -> 1, [4,16) -> 2, ...
// ---------------------------------------------------------------------------
// With growth g = 2^lg: [0,1) -> 0, [1,g) -> 1, [g,g^2) -> 2, ...
__host__ __device__ inline int sweep_of(int rank, int lg) {
    if (rank <= 0) return 0;
    int l2 = 31 - __builtin_clz((unsigned)rank);
    return 1 + l2 / lg;
}

int num_sweeps(int nprobe_max, int lg) { return sweep_of(nprobe_max - 1, lg) + 1; }
int sweep_begin(int s, int lg) {
    if (s == 0) return 0;
    const int64_t v = (int64_t)1 << (lg * (s - 1));
    return v > (1 << 30) ? (1 << 30) : (int)v;
}

// ---------------------------------------------------------------------------
// Per-query setup: KNN-set size, probe count, thresholds and KNN sets.
// ---------------------------------------------------------------------------
__global__ void setup_kernel(const int32_t *K, const int32_t *nprobe, int nq, int k_max,
                             int nprobe_max, int kfactor, int kcap, int32_t *kq, int32_t *keff,
                             int32_t *npq, float *r2, uint64_t *tk) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) {
        int k = K ? K[q] : k_max;
        k = k < 0 ? 0 : (k > k_max ? k_max : k);
        int ke = k * kfactor;
        ke = ke > kcap ? kcap : ke;
        int np = nprobe ? nprobe[q] : nprobe_max;
        np = np < 0 ? 0 : (np > nprobe_max ? nprobe_max : np);
        kq[q] = k;
        keff[q] = ke;
        npq[q] = np;
        r2[q] = __builtin_inff();
    }
    int64_t tot = (int64_t)nq * kcap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x)
        tk[i] = KEY_NONE;
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------------------
// Probe selection (Section 2.2.2): the nprobe nearest centres per query,
// squared distance ||q'||^2 + ||c'||^2 - 2 q'.c' (clamped at 0), ascending by
// (distance, list id).
// ---------------------------------------------------------------------------
// The keys of one query stay in LDS for the selection passes when they fit
// beside the sorted output (at most 60 KB of keys in all).
__host__ __device__ inline bool probe_keys_cached(int nlist, int nprobe_max) {
    return next_pow2(nprobe_max) + nlist <= 7680;
}
size_t probe_select_smem(int nlist, int nprobe_max) {
    return sizeof(uint64_t) *
           ((size_t)next_pow2(nprobe_max) + (probe_keys_cached(nlist, nprobe_max) ? (size_t)nlist : 0));
}

__global__ __launch_bounds__(ADS_WG) void probe_select_kernel(
    const float *qrot, const float *dots, const float *cnorm, int D, int nlist, int nprobe_max,
    int32_t *probes) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = nprobe_max;
    const int P = next_pow2(k);
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem_raw);
    uint64_t *kc = buf + P;            // the keys, when probe_keys_cached
    __shared__ uint32_t hist[256];
    __shared__ uint32_t misc[8];
    __shared__ float red[ADS_WG / 64];
    const int q = blockIdx.x;
    const float *qr = qrot + (int64_t)q * D;
    float acc = 0.f;
    for (int i = threadIdx.x; i < D; i += ADS_WG) acc = __fmaf_rn(qr[i], qr[i], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    const float qn = red[0] + red[1] + red[2] + red[3];
    const float *dq = dots + (int64_t)q * nlist;
    auto key_of = [&](int i) -> uint64_t {
        float s = qn + cnorm[i] - 2.f * dq[i];
        s = s > 0.f ? s : 0.f;
        return make_key(s, (uint32_t)i);
    };
    const bool cached = probe_keys_cached(nlist, nprobe_max);
    if (cached) {
        for (int i = threadIdx.x; i < nlist; i += ADS_WG) kc[i] = key_of(i);
        __syncthreads();
    }
    auto get = [&](int i) -> uint64_t { return cached ? kc[i] : key_of(i); };
    uint64_t kth = KEY_NONE;
    if (k < nlist) kth = radix_kth(get, nlist, k, hist, misc);
    if (threadIdx.x == 0) misc[2] = 0;
    for (int i = threadIdx.x; i < P; i += ADS_WG) buf[i] = KEY_NONE;
    __syncthreads();
    for (int i = threadIdx.x; i < nlist; i += ADS_WG) {
        uint64_t key = get(i);
        if (key <= kth) {
            uint32_t p = atomicAdd(&misc[2], 1u);
            if (p < (uint32_t)k) buf[p] = key;
        }
    }
    __syncthreads();
    lds_bitonic_sort(buf, P);
    for (int i = threadIdx.x; i < k; i += ADS_WG) probes[(int64_t)q * nprobe_max + i] = (int32_t)key_id(buf[i]);
}

// ---------------------------------------------------------------------------
// Grouping of (query, rank) pairs by (sweep, list).
// ---------------------------------------------------------------------------
__global__ void group_count_kernel(const int32_t *probes, const int32_t *npq, const int32_t *keff,
                                   int nq, int nprobe_max, int nlist, int lg, int32_t *cnt) {
    int64_t tot = (int64_t)nq * nprobe_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / nprobe_max), rank = (int)(i % nprobe_max);
        if (rank >= npq[q] || keff[q] <= 0) continue;
        int l = probes[i];
        atomicAdd(&cnt[(int64_t)sweep_of(rank, lg) * nlist + l], 1);
    }
}

// Lists of one sweep -> XCDs.  The work of a list in a sweep is its query
// count times its length; XCD x owns the contiguous range of list ids whose
// work midpoints fall in the x-th eighth of the sweep's total work, so the
// eight XCDs (each with its own L2) get equal shares whatever the list sizes
// and query popularity.  Within its range an XCD takes the lists in
// decreasing work (ties by list id), so the longest units start first and do
// not form the tail of the launch.  Neither changes any result.
// Workgroup (sweep s, XCD x) writes order[s * nlist + i] for the positions i
// of its range and xb[s * 9 + x] = the range's first position (xb[s * 9 + 8]
// = nlist).
constexpr int ORDER_MAX = 4096;     // lists of one range sorted in LDS (larger ranges keep id order)

__global__ __launch_bounds__(512) void list_order_kernel(const int32_t *cnt, const int64_t *list_off, int nlist,
                                                         int32_t *order, int32_t *xb) {
    __shared__ uint64_t key[ORDER_MAX];
    __shared__ unsigned long long part[512];
    __shared__ int cnt_lo[512], cnt_hi[512];
    const int s = blockIdx.x >> 3, x = blockIdx.x & 7, t = threadIdx.x;
    const int32_t *c = cnt + (int64_t)s * nlist;
    auto work = [&](int l) -> unsigned long long {
        return (unsigned long long)c[l] * (unsigned long long)(list_off[l + 1] - list_off[l]);
    };
    // each thread takes a contiguous chunk of list ids; exclusive prefix of the chunk sums
    const int per = (nlist + 511) / 512;
    const int l0 = min(nlist, t * per), l1 = min(nlist, l0 + per);
    unsigned long long sum = 0;
    for (int l = l0; l < l1; ++l) sum += work(l);
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 512; o <<= 1) {
        const unsigned long long v = t >= o ? part[t - o] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const unsigned long long total = part[511];
    unsigned long long pre = part[t] - sum;
    // XCD of every list; the ranges are counted, so they partition the ids
    int lo = 0, hi = 0;
    for (int l = l0; l < l1; ++l) {
        const unsigned long long wl = work(l);
        int xl;
        if (total == 0) {
            xl = (int)((int64_t)l * 8 / nlist);
        } else {
            xl = (int)(8.0 * ((double)pre + 0.5 * (double)wl) / (double)total);
            xl = xl > 7 ? 7 : xl;
        }
        lo += xl < x;
        hi += xl <= x;
        pre += wl;
    }
    cnt_lo[t] = lo;
    cnt_hi[t] = hi;
    __syncthreads();
    for (int o = 256; o > 0; o >>= 1) {
        if (t < o) {
            cnt_lo[t] += cnt_lo[t + o];
            cnt_hi[t] += cnt_hi[t + o];
        }
        __syncthreads();
    }
    const int start = cnt_lo[0], n = cnt_hi[0] - cnt_lo[0];
    if (t == 0) {
        xb[s * 9 + x] = start;
        if (x == 7) xb[s * 9 + 8] = nlist;
    }
    int32_t *ord = order + (int64_t)s * nlist + start;
    if (n > ORDER_MAX) {
        for (int j = t; j < n; j += blockDim.x) ord[j] = start + j;
        return;
    }
    const int np2 = next_pow2(n > 0 ? n : 1);
    const uint64_t cap = (1ull << 40) - 1;
    for (int j = t; j < np2; j += blockDim.x) {
        uint64_t k = ~0ull;
        if (j < n) {
            uint64_t wl = work(start + j);
            wl = wl > cap ? cap : wl;
            k = ((cap - wl) << 24) | (uint64_t)j;
        }
        key[j] = k;
    }
    __syncthreads();
    lds_bitonic_sort(key, np2);
    for (int j = t; j < n; j += blockDim.x) ord[j] = start + (int)(key[j] & 0xffffffu);
}

// One workgroup of 1024 threads per sweep: exclusive prefix of cnt over
// lists (entry offsets into qent, continuing across sweeps: the workgroup
// first counts the entries of the earlier sweeps) and the unit offsets of
// every list in the XCD-major order of list_order_kernel (ceil(cnt / qw)
// units per list), with the first unit and the unit count of every XCD.
__global__ __launch_bounds__(1024) void group_scan_kernel(const int32_t *cnt, const int32_t *order, const int32_t *xb,
                                                          int nsweep, int nlist, int qw, int32_t *beg, int32_t *uoff,
                                                          int32_t *xoff, int32_t *xcnt) {
    __shared__ int32_t sa[1024];
    __shared__ int32_t carry;
    __shared__ int32_t xfirst[9];
    const int s = blockIdx.x;
    if (s >= nsweep) return;
    {
        int c = 0;
        for (int64_t i = threadIdx.x; i < (int64_t)s * nlist; i += 1024) c += cnt[i];
        sa[threadIdx.x] = c;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if (threadIdx.x < o) sa[threadIdx.x] += sa[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) carry = sa[0];
        __syncthreads();
    }
    {
        // entry offsets in natural list order
        for (int l0 = 0; l0 < nlist; l0 += 1024) {
            const int l = l0 + threadIdx.x;
            const int c = l < nlist ? cnt[(int64_t)s * nlist + l] : 0;
            sa[threadIdx.x] = c;
            __syncthreads();
            for (int o = 1; o < 1024; o <<= 1) {
                const int xa = threadIdx.x >= o ? sa[threadIdx.x - o] : 0;
                __syncthreads();
                sa[threadIdx.x] += xa;
                __syncthreads();
            }
            if (l < nlist) beg[(int64_t)s * nlist + l] = carry + sa[threadIdx.x] - c;
            __syncthreads();
            if (threadIdx.x == 1023) carry += sa[1023];
            __syncthreads();
        }
        // unit offsets in XCD-major order; xfirst[x] = first unit of XCD x
        __shared__ int32_t ucarry;
        if (threadIdx.x == 0) ucarry = 0;
        if (threadIdx.x < 9) xfirst[threadIdx.x] = -1;
        __syncthreads();
        const int32_t *xbs = xb + s * 9;
        for (int i0 = 0; i0 < nlist; i0 += 1024) {
            const int i = i0 + threadIdx.x;
            const int l = i < nlist ? order[(int64_t)s * nlist + i] : -1;
            const int c = l >= 0 ? cnt[(int64_t)s * nlist + l] : 0;
            const int ng = (c + qw - 1) / qw;
            sa[threadIdx.x] = ng;
            __syncthreads();
            for (int o = 1; o < 1024; o <<= 1) {
                const int xa = threadIdx.x >= o ? sa[threadIdx.x - o] : 0;
                __syncthreads();
                sa[threadIdx.x] += xa;
                __syncthreads();
            }
            const int ex = ucarry + sa[threadIdx.x] - ng;
            if (l >= 0) {
                uoff[(int64_t)s * nlist + l] = ex;
                for (int x = 0; x < 8; ++x)
                    if (xbs[x] == i) xfirst[x] = ex;
            }
            __syncthreads();
            if (threadIdx.x == 1023) ucarry += sa[1023];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            // empty ranges at the end start at the total
            int first[9];
            for (int x = 0; x < 8; ++x) first[x] = xfirst[x] >= 0 ? xfirst[x] : ucarry;
            first[8] = ucarry;
            for (int x = 0; x < 8; ++x) {
                xoff[s * 8 + x] = first[x];
                xcnt[s * 8 + x] = first[x + 1] - first[x];
            }
        }
        __syncthreads();
    }
}

// Writes the units of every (sweep, list): (list, first entry, query count).
__global__ void unit_expand_kernel(const int32_t *cnt, const int32_t *beg, const int32_t *uoff, int nsweep,
                                   int nlist, int qw, int64_t ucap, int4 *units) {
    const int64_t tot = (int64_t)nsweep * nlist;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = cnt[i];
        if (c <= 0) continue;
        const int s = (int)(i / nlist), l = (int)(i % nlist);
        const int b0 = beg[i];
        int4 *u = units + (int64_t)s * ucap + uoff[i];
        for (int g = 0; g * qw < c; ++g) u[g] = make_int4(l, b0 + g * qw, min(qw, c - g * qw), 0);
    }
}

__global__ void group_scatter_kernel(const int32_t *probes, const int32_t *npq, const int32_t *keff,
                                     int nq, int nprobe_max, int nlist, int lg, const int32_t *beg,
                                     int32_t *cursor, int2 *qent) {
    int64_t tot = (int64_t)nq * nprobe_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / nprobe_max), rank = (int)(i % nprobe_max);
        if (rank >= npq[q] || keff[q] <= 0) continue;
        int l = probes[i];
        int64_t slot = (int64_t)sweep_of(rank, lg) * nlist + l;
        int p = beg[slot] + atomicAdd(&cursor[slot], 1);
        qent[p] = make_int2(q, rank);
    }
}

// ---------------------------------------------------------------------------
// Merge after a sweep: the KNN set of query q becomes the keff[q] smallest
// keys among its previous set and the sweep's per-list sets.
// ---------------------------------------------------------------------------
constexpr int MERGE_LDS = 2048;   // keys a merge sorts in LDS

__global__ __launch_bounds__(ADS_WG) void merge_kernel(const uint64_t *slots, const int32_t *keff,
                                                      const int32_t *npq, int nprobe_max, int kcap,
                                                      int rank_a, int rank_b, uint64_t *tk,
                                                      float *r2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem_raw);
    __shared__ uint32_t hist[256];
    __shared__ uint32_t misc[8];
    const int q = blockIdx.x;
    const int K = keff[q];
    const int hi = min(rank_b, npq[q]);
    if (K <= 0 || hi <= rank_a) return;
    uint64_t *mytk = tk + (int64_t)q * kcap;
    const uint64_t *ms = slots + ((int64_t)q * nprobe_max + rank_a) * kcap;
    const int n = kcap + (hi - rank_a) * kcap;
    auto get = [&](int i) -> uint64_t { return i < kcap ? mytk[i] : ms[i - kcap]; };
    // Most slots are empty (a unit publishes only its positives): gather the
    // keys that are present into LDS in one pass and sort them there; fall
    // back to a radix select over the slots when they do not fit.
    __shared__ uint64_t cmp[MERGE_LDS];
    if (threadIdx.x == 0) misc[3] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += ADS_WG) {
        const uint64_t key = get(i);
        if (key != KEY_NONE) {
            const uint32_t p = atomicAdd(&misc[3], 1u);
            if (p < (uint32_t)MERGE_LDS) cmp[p] = key;
        }
    }
    __syncthreads();
    const int nv = (int)misc[3];
    if (nv <= MERGE_LDS) {
        const int P2 = next_pow2(nv > 0 ? nv : 1);
        for (int i = nv + threadIdx.x; i < P2; i += ADS_WG) cmp[i] = KEY_NONE;
        __syncthreads();
        lds_bitonic_sort(cmp, P2);
        for (int i = threadIdx.x; i < kcap; i += ADS_WG) mytk[i] = i < K && i < nv ? cmp[i] : KEY_NONE;
        if (threadIdx.x == 0) r2[q] = nv >= K ? key_dist2(cmp[K - 1]) : __builtin_inff();
        return;
    }
    uint64_t kth = KEY_NONE;
    if (nv > K) kth = radix_kth(get, n, K, hist, misc);
    const int P = next_pow2(kcap);
    if (threadIdx.x == 0) misc[2] = 0;
    for (int i = threadIdx.x; i < P; i += ADS_WG) buf[i] = KEY_NONE;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += ADS_WG) {
        uint64_t key = get(i);
        if (key != KEY_NONE && key <= kth) {
            uint32_t p = atomicAdd(&misc[2], 1u);
            if (p < (uint32_t)K) buf[p] = key;
        }
    }
    __syncthreads();
    lds_bitonic_sort(buf, P);
    for (int i = threadIdx.x; i < kcap; i += ADS_WG) mytk[i] = i < K ? buf[i] : KEY_NONE;
    if (threadIdx.x == 0) r2[q] = nv >= K ? key_dist2(buf[K - 1]) : __builtin_inff();
}

// ---------------------------------------------------------------------------
// Output: ids / distances of the first K entries of each KNN set.
// ---------------------------------------------------------------------------
__global__ void output_kernel(const uint64_t *tk, const int32_t *kq, int nq, int k_max, int kcap,
                              int64_t *ids, float *dist) {
    int64_t tot = (int64_t)nq * k_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / k_max), k = (int)(i % k_max);
        uint64_t key = k < kq[q] ? tk[(int64_t)q * kcap + k] : KEY_NONE;
        if (key == KEY_NONE) {
            ids[i] = -1;
            dist[i] = __builtin_inff();
        } else {
            ids[i] = (int64_t)key_id(key);
            dist[i] = __fsqrt_rn(key_dist2(key));
        }
    }
}

// Low-precision mode: recompute the keff candidates' distances from the
// float32 rows and keep the best K.  The sum is the scan's canonical one
// (per-block partials of dd coordinates, each from zero with fused
// multiply-adds in coordinate order, added in block order), so a reranked
// distance equals the float32 scan's distance of the same pair bit for bit.
__global__ __launch_bounds__(ADS_WG) void rerank_kernel(const uint64_t *tk, const int32_t *kq,
                                                       const int32_t *keff, const float *rows32,
                                                       const int32_t *pos_of, const float *qrot,
                                                       int D, int dd, int kcap, int k_max, int64_t *ids,
                                                       float *dist) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem_raw);
    const int q = blockIdx.x;
    const int P = next_pow2(kcap);
    const int ke = keff[q];
    const float *qr = qrot + (int64_t)q * D;
    for (int i = threadIdx.x; i < P; i += ADS_WG) {
        uint64_t key = KEY_NONE;
        if (i < ke) {
            uint64_t c = tk[(int64_t)q * kcap + i];
            if (c != KEY_NONE) {
                uint32_t id = key_id(c);
                const float *row = rows32 + (int64_t)pos_of[id] * D;
                float s = 0.f;
                for (int b0 = 0; b0 < D; b0 += dd) {
                    float pb = 0.f;
                    for (int t = b0; t < b0 + dd; ++t) {
                        float df = row[t] - qr[t];
                        pb = __fmaf_rn(df, df, pb);
                    }
                    s += pb;
                }
                key = make_key(s, id);
            }
        }
        buf[i] = key;
    }
    __syncthreads();
    lds_bitonic_sort(buf, P);
    const int K = kq[q];
    for (int k = threadIdx.x; k < k_max; k += ADS_WG) {
        uint64_t key = k < K ? buf[k] : KEY_NONE;
        int64_t o = (int64_t)q * k_max + k;
        if (key == KEY_NONE) {
            ids[o] = -1;
            dist[o] = __builtin_inff();
        } else {
            ids[o] = (int64_t)key_id(key);
            dist[o] = __fsqrt_rn(key_dist2(key));
        }
    }
}

__global__ void probes_out_kernel(const int32_t *probes, const int32_t *npq, int nq, int nprobe_max,
                                  int32_t *out) {
    int64_t tot = (int64_t)nq * nprobe_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / nprobe_max), r = (int)(i % nprobe_max);
        out[i] = r < npq[q] ? probes[i] : -1;
    }
}

}  // namespace ads
