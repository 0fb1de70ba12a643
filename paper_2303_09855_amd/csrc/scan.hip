// The IVF+ / IVF++ candidate scan with ADSampling DCOs (Sections 2.2.2, 3.3,
// 4 and 5.2), and the kernels around it: probe selection, grouping of
// (query, list) pairs by list, per-query merges and the final output.
//
// Schedule.  The probe ranks of every query are cut into sweeps
// [0,1), [1,4), [4,16), [16,64), ...  Each sweep is one list-major launch: a
// workgroup takes one list and every (query, rank) pair of the sweep that
// probes it, so the list's vectors are read from HBM once per sweep and
// reused for all those queries.  Inside a sweep a query's threshold r is the
// K-th distance of its KNN set after the previous sweeps (+inf before the
// first merge), lowered further by the K-th distance of the positives the
// workgroup has found for that query in the current list.  Every threshold
// used is therefore the exact K-th distance of a set of evaluated candidates
// (or +inf), which is what the failure analysis of Lemma 3.2 and Corollary 4.2
// needs.  A per-query merge after each sweep rebuilds the KNN set.  A query's
// result depends only on that query, never on the rest of the batch.
//
// Per workgroup: 64 vectors x QT queries form a tile of DCOs.  Coordinates are
// taken DD at a time from the blocked layout [block][vector][DD] (Section 5.2
// generalised).  While many pairs of the tile are alive, each lane owns one
// vector, keeps its DD coordinates in registers and walks the wave's queries
// (query coordinates broadcast from LDS).  Once at most 512 pairs survive,
// they are compacted into an LDS list and processed one pair per thread.
#include "kernels.h"

namespace ads {

constexpr int VT = 64;          // vectors per tile
constexpr int LIST_CAP = 512;   // compacted pair list capacity (2 per thread)


template <int DD, int QT>
struct ScanSmem {
    static constexpr int QPAD = DD + 4;
    float qs[QT][QPAD];
    uint64_t list[LIST_CAP];
    uint64_t pos[QT][VT];
    float r2s[QT];
    int qidx[QT], qrank[QT], qk[QT], pcnt[QT], tkcnt[QT], tkmax[QT];
    int alive_cnt, list_cnt, list_cnt2;
    // followed by float coef[nb] and uint64 tk[QT][kcap]
};

template <int DT, int DD, int QT>
__global__ __launch_bounds__(ADS_WG) void scan_kernel(ScanArgs a) {
    constexpr int QPW = QT / 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ScanSmem<DD, QT> &sm = *reinterpret_cast<ScanSmem<DD, QT> *>(smem_raw);
    float *coef = reinterpret_cast<float *>(smem_raw + sizeof(ScanSmem<DD, QT>));
    uint64_t *tk = reinterpret_cast<uint64_t *>(
        smem_raw + ((sizeof(ScanSmem<DD, QT>) + sizeof(float) * a.nb + 15) & ~(size_t)15));

    const int u = blockIdx.x;
    if (u >= *a.n_units) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int D = a.D, nb = a.nb, kcap = a.kcap;
    const int l = a.unit_list[u];
    const int beg = a.unit_beg[u], cnt = a.unit_cnt[u];
    const int64_t off = a.list_off[l];
    const int nl = (int)(a.list_off[l + 1] - off);
    constexpr int EB = Elem<DT>::bytes;
    const unsigned char *lbase = reinterpret_cast<const unsigned char *>(a.data) + off * (int64_t)D * EB;

    for (int b = tid; b < nb; b += ADS_WG) {
        int d = (b + 1) * DD;
        coef[b] = d < D ? test_coef(d, D, a.eps0, a.method) : 0.f;
    }

    unsigned long long my_dims = 0, my_pos = 0, my_dcos = 0;

    for (int c0 = 0; c0 < cnt; c0 += QT) {
        const int qc = min(QT, cnt - c0);
        if (tid < QT) {
            int k = 0;
            if (tid < qc) {
                int2 e = a.qent[beg + c0 + tid];
                sm.qidx[tid] = e.x;
                sm.qrank[tid] = e.y;
                k = a.keff[e.x];
                sm.r2s[tid] = a.r2_in[e.x];
            }
            sm.qk[tid] = k;
            sm.tkcnt[tid] = 0;
            sm.tkmax[tid] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            int act = 0;
            for (int j = 0; j < qc; ++j) act += sm.qk[j] > 0;
            my_dcos += (unsigned long long)act * (unsigned long long)nl;
        }

        for (int vc = 0; vc < nl; vc += VT) {
            if (tid < QT) sm.pcnt[tid] = 0;
            if (tid == 0) { sm.alive_cnt = 0; sm.list_cnt = 0; }
            const int v = vc + lane;
            const bool vvalid = v < nl;
            float S[QPW];
            uint32_t alive = 0;
#pragma unroll
            for (int jj = 0; jj < QPW; ++jj) {
                S[jj] = 0.f;
                int j = wave * QPW + jj;
                if (vvalid && j < qc && sm.qk[j] > 0) alive |= 1u << jj;
            }
            bool dense = true;
            __syncthreads();
            for (int b = 0; b < nb; ++b) {
                // stage the chunk's query coordinates of block b
                for (int i = tid; i < QT * (DD / 4); i += ADS_WG) {
                    int j = i / (DD / 4), k4 = (i % (DD / 4)) * 4;
                    if (j < qc) {
                        float4 t = *reinterpret_cast<const float4 *>(a.qrot + (int64_t)sm.qidx[j] * D + b * DD + k4);
                        sm.qs[j][k4 + 0] = t.x; sm.qs[j][k4 + 1] = t.y;
                        sm.qs[j][k4 + 2] = t.z; sm.qs[j][k4 + 3] = t.w;
                    }
                }
                __syncthreads();
                const int d = (b + 1) * DD;
                const float cf = coef[b];
                if (dense) {
                    if (alive) {
                        float o[DD];
                        load_elems<DT, DD>(lbase + ((int64_t)b * nl * DD + (int64_t)v * DD) * EB, o);
#pragma unroll
                        for (int jj = 0; jj < QPW; ++jj) {
                            if (!((alive >> jj) & 1u)) continue;
                            const int j = wave * QPW + jj;
                            float s = S[jj];
#pragma unroll
                            for (int k = 0; k < DD; ++k) {
                                float df = o[k] - sm.qs[j][k];
                                s = __fmaf_rn(df, df, s);
                            }
                            S[jj] = s;
                            if (d < D) {
                                if (test_reject(s, cf, sm.r2s[j])) {
                                    alive &= ~(1u << jj);
                                    my_dims += d;
                                }
                            } else {
                                alive &= ~(1u << jj);
                                my_dims += D;
                                if (s <= sm.r2s[j]) {
                                    int p = atomicAdd(&sm.pcnt[j], 1);
                                    sm.pos[j][p] = make_key(s, (uint32_t)a.ids[off + v]);
                                    ++my_pos;
                                }
                            }
                        }
                    }
                    if (d >= D) break;
                    int na = __popc(alive);
                    if (na) atomicAdd(&sm.alive_cnt, na);
                    __syncthreads();
                    const int n_alive = sm.alive_cnt;
                    if (n_alive == 0) break;
                    if (n_alive <= LIST_CAP) {
                        // switch to the compacted pair list
#pragma unroll
                        for (int jj = 0; jj < QPW; ++jj) {
                            if ((alive >> jj) & 1u) {
                                int p = atomicAdd(&sm.list_cnt, 1);
                                uint32_t tag = (uint32_t)((wave * QPW + jj) << 6 | lane);
                                sm.list[p] = ((uint64_t)__float_as_uint(S[jj]) << 32) | tag;
                            }
                        }
                        alive = 0;
                        dense = false;
                    }
                    __syncthreads();
                    if (tid == 0) sm.alive_cnt = 0;
                } else {
                    const int m = sm.list_cnt;
                    uint64_t e0 = KEY_NONE, e1 = KEY_NONE;
                    if (tid < m) e0 = sm.list[tid];
                    if (tid + ADS_WG < m) e1 = sm.list[tid + ADS_WG];
                    __syncthreads();
                    if (tid == 0) sm.list_cnt = 0;
                    __syncthreads();
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        uint64_t e = t == 0 ? e0 : e1;
                        if (e == KEY_NONE) continue;
                        const uint32_t tag = (uint32_t)e;
                        const int vl = tag & 63, j = (int)(tag >> 6);
                        const int vv = vc + vl;
                        float s = __uint_as_float((uint32_t)(e >> 32));
                        float o[DD];
                        load_elems<DT, DD>(lbase + ((int64_t)b * nl * DD + (int64_t)vv * DD) * EB, o);
#pragma unroll
                        for (int k = 0; k < DD; ++k) {
                            float df = o[k] - sm.qs[j][k];
                            s = __fmaf_rn(df, df, s);
                        }
                        if (d < D) {
                            if (test_reject(s, cf, sm.r2s[j])) {
                                my_dims += d;
                            } else {
                                int p = atomicAdd(&sm.list_cnt, 1);
                                sm.list[p] = ((uint64_t)__float_as_uint(s) << 32) | tag;
                            }
                        } else {
                            my_dims += D;
                            if (s <= sm.r2s[j]) {
                                int p = atomicAdd(&sm.pcnt[j], 1);
                                sm.pos[j][p] = make_key(s, (uint32_t)a.ids[off + vv]);
                                ++my_pos;
                            }
                        }
                    }
                    __syncthreads();
                    if (d >= D || sm.list_cnt == 0) break;
                }
            }
            __syncthreads();
            // fold this tile's positives into each query's local KNN set
            if (tid < qc) {
                const int j = tid;
                const int K = sm.qk[j];
                if (K > 0) {
                    uint64_t *mytk = tk + (int64_t)j * kcap;
                    int c = sm.tkcnt[j], mx = sm.tkmax[j];
                    const int np = sm.pcnt[j];
                    for (int p = 0; p < np; ++p) {
                        uint64_t key = sm.pos[j][p];
                        if (c < K) {
                            mytk[c++] = key;
                            if (c == K) {
                                mx = 0;
                                for (int t = 1; t < K; ++t) if (mytk[t] > mytk[mx]) mx = t;
                            }
                        } else if (key < mytk[mx]) {
                            mytk[mx] = key;
                            mx = 0;
                            for (int t = 1; t < K; ++t) if (mytk[t] > mytk[mx]) mx = t;
                        }
                    }
                    sm.tkcnt[j] = c;
                    sm.tkmax[j] = mx;
                    if (c == K) {
                        float kth = key_dist2(mytk[mx]);
                        if (kth < sm.r2s[j]) sm.r2s[j] = kth;
                    }
                }
            }
            __syncthreads();
        }
        // publish the local KNN sets of this chunk
        for (int i = tid; i < qc * kcap; i += ADS_WG) {
            const int j = i / kcap, t = i % kcap;
            uint64_t key = (sm.qk[j] > 0 && t < sm.tkcnt[j]) ? tk[(int64_t)j * kcap + t] : KEY_NONE;
            a.slots[((int64_t)sm.qidx[j] * a.nprobe_max + sm.qrank[j]) * kcap + t] = key;
        }
        __syncthreads();
    }

    if (a.stats) {
        // wave reductions, then one atomic per wave
        for (int o = 32; o > 0; o >>= 1) {
            my_dims += __shfl_down(my_dims, o);
            my_pos += __shfl_down(my_pos, o);
        }
        if (lane == 0) {
            atomicAdd(a.stats + ADS_STAT_DIMS, my_dims);
            atomicAdd(a.stats + ADS_STAT_BYTES, my_dims * (unsigned long long)EB);
            atomicAdd(a.stats + ADS_STAT_POSITIVES, my_pos);
            if (tid == 0) atomicAdd(a.stats + ADS_STAT_DCOS, my_dcos);
        }
    }
}

template <int DD, int QT>
size_t scan_smem_bytes(int nb, int kcap) {
    size_t s = sizeof(ScanSmem<DD, QT>) + sizeof(float) * nb;
    s = (s + 15) & ~(size_t)15;
    return s + sizeof(uint64_t) * (size_t)QT * kcap;
}

template <int DT, int DD, int QT>
hipError_t launch_scan_t(const ScanArgs &a, int grid, hipStream_t s) {
    size_t sh = scan_smem_bytes<DD, QT>(a.nb, a.kcap);
    if (sh > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((scan_kernel<DT, DD, QT>), dim3(grid), dim3(ADS_WG), sh, s, a);
    return hipGetLastError();
}

template <int DT, int DD>
hipError_t launch_scan_q(const ScanArgs &a, int qt, int grid, hipStream_t s) {
    switch (qt) {
        case 32: return launch_scan_t<DT, DD, 32>(a, grid, s);
        case 16: return launch_scan_t<DT, DD, 16>(a, grid, s);
        case 8: return launch_scan_t<DT, DD, 8>(a, grid, s);
        case 4: return launch_scan_t<DT, DD, 4>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

template <int DT>
hipError_t launch_scan_d(const ScanArgs &a, int dd, int qt, int grid, hipStream_t s) {
    switch (dd) {
        case 8: return launch_scan_q<DT, 8>(a, qt, grid, s);
        case 16: return launch_scan_q<DT, 16>(a, qt, grid, s);
        case 32: return launch_scan_q<DT, 32>(a, qt, grid, s);
        case 64: return launch_scan_q<DT, 64>(a, qt, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scan(const ScanArgs &a, int dtype, int dd, int qt, int grid, hipStream_t s) {
    switch (dtype) {
        case ADS_F32: return launch_scan_d<ADS_F32>(a, dd, qt, grid, s);
        case ADS_BF16: return launch_scan_d<ADS_BF16>(a, dd, qt, grid, s);
        case ADS_F16: return launch_scan_d<ADS_F16>(a, dd, qt, grid, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Sweep of a probe rank: [0,1) -> 0, [1,4) -> 1, [4,16) -> 2, ...
// ---------------------------------------------------------------------------
__host__ __device__ inline int sweep_of(int rank) {
    if (rank <= 0) return 0;
    int lg = 31 - __builtin_clz((unsigned)rank);
    return 1 + (lg >> 1);
}

int num_sweeps(int nprobe_max) { return sweep_of(nprobe_max - 1) + 1; }
int sweep_begin(int s) { return s == 0 ? 0 : 1 << (2 * (s - 1)); }

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
__global__ __launch_bounds__(ADS_WG) void probe_select_kernel(
    const float *qrot, const float *dots, const float *cnorm, int D, int nlist, int nprobe_max,
    int32_t *probes) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem_raw);
    __shared__ uint32_t hist[256];
    __shared__ uint32_t misc[4];
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
    auto get = [&](int i) -> uint64_t {
        float s = qn + cnorm[i] - 2.f * dq[i];
        s = s > 0.f ? s : 0.f;
        return make_key(s, (uint32_t)i);
    };
    const int k = nprobe_max;
    const int P = next_pow2(k);
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
                                   int nq, int nprobe_max, int nlist, int32_t *cnt) {
    int64_t tot = (int64_t)nq * nprobe_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / nprobe_max), rank = (int)(i % nprobe_max);
        if (rank >= npq[q] || keff[q] <= 0) continue;
        int l = probes[i];
        atomicAdd(&cnt[(int64_t)sweep_of(rank) * nlist + l], 1);
    }
}

// One workgroup of 1024 threads: exclusive prefix of cnt over (sweep, list)
// (entry offsets) and, per sweep, the compacted list of non-empty lists.
__global__ __launch_bounds__(1024) void group_scan_kernel(const int32_t *cnt, int nsweep, int nlist,
                                                          int32_t *beg, int32_t *unit_list,
                                                          int32_t *unit_beg, int32_t *unit_cnt,
                                                          int32_t *n_units) {
    __shared__ int32_t sa[1024], sb[1024];
    __shared__ int32_t carry_a, carry_b;
    if (threadIdx.x == 0) carry_a = 0;
    __syncthreads();
    for (int s = 0; s < nsweep; ++s) {
        if (threadIdx.x == 0) carry_b = 0;
        __syncthreads();
        for (int l0 = 0; l0 < nlist; l0 += 1024) {
            int l = l0 + threadIdx.x;
            int c = l < nlist ? cnt[(int64_t)s * nlist + l] : 0;
            sa[threadIdx.x] = c;
            sb[threadIdx.x] = c > 0;
            __syncthreads();
            for (int o = 1; o < 1024; o <<= 1) {
                int xa = threadIdx.x >= o ? sa[threadIdx.x - o] : 0;
                int xb = threadIdx.x >= o ? sb[threadIdx.x - o] : 0;
                __syncthreads();
                sa[threadIdx.x] += xa;
                sb[threadIdx.x] += xb;
                __syncthreads();
            }
            int ea = carry_a + sa[threadIdx.x] - c;       // exclusive
            int eb = carry_b + sb[threadIdx.x] - (c > 0);
            if (l < nlist) {
                beg[(int64_t)s * nlist + l] = ea;
                if (c > 0) {
                    unit_list[(int64_t)s * nlist + eb] = l;
                    unit_beg[(int64_t)s * nlist + eb] = ea;
                    unit_cnt[(int64_t)s * nlist + eb] = c;
                }
            }
            __syncthreads();
            if (threadIdx.x == 1023) {
                carry_a += sa[1023];
                carry_b += sb[1023];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) n_units[s] = carry_b;
        __syncthreads();
    }
}

__global__ void group_scatter_kernel(const int32_t *probes, const int32_t *npq, const int32_t *keff,
                                     int nq, int nprobe_max, int nlist, const int32_t *beg,
                                     int32_t *cursor, int2 *qent) {
    int64_t tot = (int64_t)nq * nprobe_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int q = (int)(i / nprobe_max), rank = (int)(i % nprobe_max);
        if (rank >= npq[q] || keff[q] <= 0) continue;
        int l = probes[i];
        int64_t slot = (int64_t)sweep_of(rank) * nlist + l;
        int p = beg[slot] + atomicAdd(&cursor[slot], 1);
        qent[p] = make_int2(q, rank);
    }
}

// ---------------------------------------------------------------------------
// Merge after a sweep: the KNN set of query q becomes the keff[q] smallest
// keys among its previous set and the sweep's per-list sets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ADS_WG) void merge_kernel(const uint64_t *slots, const int32_t *keff,
                                                      const int32_t *npq, int nprobe_max, int kcap,
                                                      int rank_a, int rank_b, uint64_t *tk,
                                                      float *r2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem_raw);
    __shared__ uint32_t hist[256];
    __shared__ uint32_t misc[4];
    const int q = blockIdx.x;
    const int K = keff[q];
    const int hi = min(rank_b, npq[q]);
    if (K <= 0 || hi <= rank_a) return;
    uint64_t *mytk = tk + (int64_t)q * kcap;
    const uint64_t *ms = slots + ((int64_t)q * nprobe_max + rank_a) * kcap;
    const int n = kcap + (hi - rank_a) * kcap;
    auto get = [&](int i) -> uint64_t { return i < kcap ? mytk[i] : ms[i - kcap]; };
    if (threadIdx.x == 0) misc[3] = 0;
    __syncthreads();
    uint32_t nv_local = 0;
    for (int i = threadIdx.x; i < n; i += ADS_WG) nv_local += get(i) != KEY_NONE;
    if (nv_local) atomicAdd(&misc[3], nv_local);
    __syncthreads();
    const int nv = (int)misc[3];
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
// float32 rows (same summation order as the float32 scan) and keep the best K.
__global__ __launch_bounds__(ADS_WG) void rerank_kernel(const uint64_t *tk, const int32_t *kq,
                                                       const int32_t *keff, const float *rows32,
                                                       const int32_t *pos_of, const float *qrot,
                                                       int D, int kcap, int k_max, int64_t *ids,
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
                for (int t = 0; t < D; ++t) {
                    float df = row[t] - qr[t];
                    s = __fmaf_rn(df, df, s);
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
