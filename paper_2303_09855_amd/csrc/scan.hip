// The IVF+ / IVF++ candidate scan with ADSampling DCOs (Sections 2.2.2, 3.3,
// 4 and 5.2), and the kernels around it: probe selection, grouping of
// (query, list) pairs by list, per-query merges and the final output.
//
// Schedule.  The probe ranks of every query are cut into sweeps
// [0,1), [1,g), [g,g^2), ... (g = 2^sweep_log2, 16 by default).  Each sweep
// is one list-major launch:
// the (query, rank) pairs of the sweep are grouped by list, and a unit of work
// is one list with up to QW of the queries that probe it, so a list's vectors
// are fetched from HBM about once per sweep and reused by all its queries.
// Inside a sweep a query's threshold r is the K-th distance of its KNN set
// after the previous sweeps (+inf before the first merge), lowered further by
// the K-th distance of the positives the unit has found for that query in the
// current list.  Every threshold used is therefore the exact K-th distance of
// a set of evaluated candidates (or +inf), which is what the failure analysis
// of Lemma 3.2 and Corollary 4.2 needs.  A per-query merge after each sweep
// rebuilds the KNN set.  A query's result depends only on that query, never
// on the rest of the batch.
//
// Execution.  A unit runs on one wave.  Units are laid out XCD-major:
// workgroup w serves the units of XCD (w mod 8), so every unit of a list lands
// on the same XCD and shares that XCD's L2; each XCD owns a range of lists of
// equal work (list_order_kernel).  The list is cut into 64-vector
// tiles.  In a tile a lane owns one vector: while more than dense_frac of the
// tile's (vector, query) pairs are alive, the lane keeps the vector's DD
// coordinates of the current block in registers and walks the unit's queries
// (query coordinates broadcast from LDS).  Then the surviving pairs are
// compacted into an LDS list and finish in the pair-list phase
// (scan_sparse.h).  The tile's positives are folded into each query's local
// KNN set and lower its threshold before the next tile.
//
// This is the register-dense variant; scan_mfma.hip evaluates the dense phase
// on the matrix cores and takes the same decisions.
#include "scan_sparse.h"

namespace ads {

// W waves per workgroup: each takes one 64-vector tile per round, and the
// round's positives lower the thresholds before the next round.
template <int DD, int QW, int W, int NQB>
struct ScanSmem {
    static constexpr int LCAP = 16 * QW;   // pairs alive when the dense phase hands over (<= 1/4)
    // wave-private
    float qs[W][NQB][QW][DD + 4];   // query block (double-buffered when prefetching)
    uint64_t list[W][2][LCAP];
    uint64_t pos[W][QW][64];
    int pcnt[W][QW];
    float thr[W][QW];               // rejection thresholds of the current block
    // shared by the unit
    float r2s[QW];
    int qidx[QW], qrank[QW], qk[QW], tkcnt[QW], tkmax[QW];
    // followed by float coef[nb] and uint64 tk[QW][kcap]
};

// PF: fetch the next block of the dense phase while the current one is
// evaluated (more registers; for sweeps with fewer units than wave slots).
template <int DT, int DD, int QW, bool PF, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(PF ? 2 : 4))) void scan_kernel(ScanArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using Smem = ScanSmem<DD, QW, W, PF ? 2 : 1>;
    // dense phase: read the next query block ahead (registers allow it for one
    // wave per workgroup, blocks of up to 16 coordinates and up to 8 queries)
    constexpr bool QPIPE = W == 1 && DD <= 16 && QW <= 8;
    Smem &sm = *reinterpret_cast<Smem *>(smem_raw);
    float *coef = reinterpret_cast<float *>(smem_raw + sizeof(Smem));
    uint64_t *tk = reinterpret_cast<uint64_t *>(smem_raw + ((sizeof(Smem) + sizeof(float) * a.nb + 15) & ~(size_t)15));

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int x = blockIdx.x & 7;
    const int P = gridDim.x >> 3;
    const int cntx = a.xcnt[x], basex = a.xoff[x];
    if ((int)(blockIdx.x >> 3) >= cntx) return;
    const int D = a.D, nb = a.nb, kcap = a.kcap;
    constexpr int EB = Elem<DT>::bytes;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    int *pcnt = sm.pcnt[w];

    for (int b = tid; b < nb; b += 64 * W) {
        int d = (b + 1) * DD;
        coef[b] = d < D ? test_coef(d, D, a.eps0, a.method) : 0.f;
    }
    unsigned long long my_dims = 0, my_pos = 0, my_dcos = 0;

    for (int k = blockIdx.x >> 3; k < cntx; k += P) {
        const int4 un = a.units[basex + k];
        const int l = un.x, qbeg = un.y, qc = un.z;
        const int64_t off = a.list_off[l];
        const int nl = (int)(a.list_off[l + 1] - off);
        const unsigned char *lbase = reinterpret_cast<const unsigned char *>(a.data) + off * (int64_t)D * EB;
        if (tid < QW) {
            int kq = 0;
            if (tid < qc) {
                const int2 e = a.qent[qbeg + tid];
                sm.qidx[tid] = e.x;
                sm.qrank[tid] = e.y;
                kq = a.keff[e.x];
                sm.r2s[tid] = a.r2_in[e.x];
            }
            sm.qk[tid] = kq;
            sm.tkcnt[tid] = 0;
            sm.tkmax[tid] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            int act = 0;
            for (int j = 0; j < qc; ++j) act += sm.qk[j] > 0;
            my_dcos += (unsigned long long)act * (unsigned long long)nl;
        }

        for (int r0 = 0; r0 < nl; r0 += 64 * W) {
            // thresholds change only at the end of a round of round_tiles tiles
            const bool round_end = ((r0 / 64 + W) % a.round_tiles) == 0 || r0 + 64 * W >= nl;
            // ---- this wave's slice: vectors [vc, vc + 64) ----
            const int vc = r0 + w * 64;
            if (lane < QW) pcnt[lane] = 0;
            const int v = vc + lane;
            const bool vvalid = v < nl;
            // am[jj]: lanes whose pair (the lane's vector, query jj) is
            // undecided, as a wave-uniform lane mask, so that liveness tests and
            // updates are scalar operations
            float S[QW];
            uint64_t am[QW];
            uint64_t amany = 0;
            int tile_pairs = 0;
#pragma unroll
            for (int jj = 0; jj < QW; ++jj) {
                S[jj] = 0.f;
                am[jj] = __ballot(vvalid && jj < qc && sm.qk[jj] > 0);
                amany |= am[jj];
                tile_pairs += __popcll(am[jj]);
            }
            // sampled dimensions of the pairs decided in the dense phase,
            // counted per wave: each pair decided in block b samples (b+1) DD
            unsigned long long wdims = 0;
            int na_prev = tile_pairs;
            int b = 0, m = 0;
            bool sparse = false;
            wave_sync();
            // dense phase: lane = vector, the unit's queries in turn
            constexpr int QPL = (QW * (DD / 4) + 63) / 64;    // query float4 per lane per block
            auto fetch_q = [&](int bb, float4 *qv) {
#pragma unroll
                for (int u = 0; u < QPL; ++u) {
                    const int i = lane + 64 * u;
                    const int jj = i / (DD / 4), k4 = (i % (DD / 4)) * 4;
                    if (i < QW * (DD / 4) && jj < qc)
                        qv[u] = *reinterpret_cast<const float4 *>(a.qrot + (int64_t)sm.qidx[jj] * D + bb * DD + k4);
                }
            };
            auto store_q = [&](const float4 *qv, float (*qd)[DD + 4]) {
#pragma unroll
                for (int u = 0; u < QPL; ++u) {
                    const int i = lane + 64 * u;
                    const int jj = i / (DD / 4), k4 = (i % (DD / 4)) * 4;
                    if (i < QW * (DD / 4) && jj < qc) {
                        qd[jj][k4 + 0] = qv[u].x; qd[jj][k4 + 1] = qv[u].y;
                        qd[jj][k4 + 2] = qv[u].z; qd[jj][k4 + 3] = qv[u].w;
                    }
                }
            };
            float o[DD];
            int qb = 0;                       // qs buffer of the current block
            if (PF && tile_pairs > 0) {
                float4 qv[QPL];
                fetch_q(0, qv);
                if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + ((int64_t)v * DD) * EB, o);
                store_q(qv, sm.qs[w][0]);
            }
            for (; tile_pairs > 0 && b < nb; ++b) {
                float o1[DD];
                float4 qv1[QPL];
                if constexpr (PF) {
                    const int bn = b + 1 < nb ? b + 1 : b;
                    fetch_q(bn, qv1);
                    if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + ((int64_t)bn * nl * DD + (int64_t)v * DD) * EB, o1);
                } else {
                    if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + ((int64_t)b * nl * DD + (int64_t)v * DD) * EB, o);
                    fetch_q(b, qv1);
                    store_q(qv1, sm.qs[w][0]);
                }
                float(*qs)[DD + 4] = sm.qs[w][qb];
                const int d = (b + 1) * DD;
                // rejection thresholds of the block: S > coef(d) r^2 (an infinite
                // coefficient gives +inf or NaN, and neither rejects)
                if (lane < QW) sm.thr[w][lane] = coef[b] * sm.r2s[lane];
                wave_sync();
                // canonical order: the block's partial from zero, then S += partial.
                // A query with no undecided pair in the tile is skipped by the
                // whole wave; lanes of decided pairs compute along, without effect.
                auto advance = [&](int jj, const float *qv) {
                    float pb = 0.f;
#pragma unroll
                    for (int kk = 0; kk < DD; ++kk) {
                        float df = o[kk] - qv[kk];
                        pb = __fmaf_rn(df, df, pb);
                    }
                    return S[jj] + pb;
                };
                if (d < D && QPIPE) {
                    // the next query's block is read from LDS while the
                    // current one is evaluated
                    float qa[DD], qn[DD];
                    float ta, tn = sm.thr[w][0];
#pragma unroll
                    for (int kk = 0; kk < DD; kk += 4)
                        *reinterpret_cast<float4 *>(qn + kk) = *reinterpret_cast<const float4 *>(&qs[0][kk]);
#pragma unroll
                    for (int jj = 0; jj < QW; ++jj) {
#pragma unroll
                        for (int kk = 0; kk < DD; ++kk) qa[kk] = qn[kk];
                        ta = tn;
                        if (jj + 1 < QW) {
                            constexpr int one = 1;
                            const int jn = jj + one < QW ? jj + one : jj;
                            tn = sm.thr[w][jn];
#pragma unroll
                            for (int kk = 0; kk < DD; kk += 4)
                                *reinterpret_cast<float4 *>(qn + kk) = *reinterpret_cast<const float4 *>(&qs[jn][kk]);
                        }
                        if (am[jj] == 0) continue;
                        const float s = advance(jj, qa);
                        S[jj] = s;
                        am[jj] &= ~__ballot(s > ta);
                    }
                } else if (d < D) {
#pragma unroll
                    for (int jj = 0; jj < QW; ++jj) {
                        if (am[jj] == 0) continue;
                        const float s = advance(jj, qs[jj]);
                        S[jj] = s;
                        am[jj] &= ~__ballot(s > sm.thr[w][jj]);
                    }
                } else {
#pragma unroll
                    for (int jj = 0; jj < QW; ++jj) {
                        if (am[jj] == 0) continue;
                        const float s = advance(jj, qs[jj]);
                        if (((am[jj] >> lane) & 1ull) && s <= sm.r2s[jj]) {
                            const int p = atomicAdd(&pcnt[jj], 1);
                            sm.pos[w][jj][p] = make_key(s, (uint32_t)a.ids[off + v]);
                            ++my_pos;
                        }
                        am[jj] = 0;
                    }
                }
                if constexpr (PF) {
                    store_q(qv1, sm.qs[w][qb ^ 1]);
                    qb ^= 1;
#pragma unroll
                    for (int k = 0; k < DD; ++k) o[k] = o1[k];
                }
                wave_sync();
                if (d >= D) {
                    wdims += (unsigned long long)na_prev * (unsigned long long)D;
                    break;
                }
                int na = 0;
                amany = 0;
#pragma unroll
                for (int jj = 0; jj < QW; ++jj) {
                    na += __popcll(am[jj]);
                    amany |= am[jj];
                }
                wdims += (unsigned long long)(na_prev - na) * (unsigned long long)d;
                na_prev = na;
                if (na == 0) break;
                if ((float)na <= a.dense_frac * (float)tile_pairs) {
                    uint64_t *list = sm.list[w][0];
                    int base = 0;
#pragma unroll
                    for (int jj = 0; jj < QW; ++jj) {
                        const bool bit = (am[jj] >> lane) & 1ull;
                        const uint64_t msk = __ballot(bit);
                        if (bit) {
                            const int p = base + __popcll(msk & lanemask_lt);
                            list[p] = ((uint64_t)__float_as_uint(S[jj]) << 32) | (uint32_t)(jj << 6 | lane);
                        }
                        base += __popcll(msk);
                    }
                    m = base;
                    sparse = true;
                    ++b;
                    break;
                }
            }
            if (lane == 0) my_dims += wdims;
            // the surviving pairs run to their decisions in the pair-list phase
            if (sparse) {
                SparseCtx ctx;
                ctx.lbase = lbase;
                ctx.nl = nl;
                ctx.vc = vc;
                ctx.qrot = a.qrot;
                ctx.qidx = sm.qidx;
                ctx.r2s = sm.r2s;
                ctx.coef = coef;
                ctx.D = D;
                ctx.nb = nb;
                ctx.vmarg = nullptr;
                ctx.qmarg = nullptr;
                ctx.exq = nullptr;
                const int32_t *tids = a.ids + off + vc;
                uint64_t(*pos)[64] = sm.pos[w];
                auto sink = [=](int jj, float s, int vv) {
                    const int p = atomicAdd(&pcnt[jj], 1);
                    pos[jj][p] = make_key(s, (uint32_t)tids[vv]);
                };
                const SparseOut so = sparse_run<DT, DD, false>(ctx, sm.list[w][0], sm.list[w][1], m, b, 0, sink);
                my_dims += so.dims;
                my_pos += so.pos;
            }
            __syncthreads();
            // fold the round's positives into each query's local KNN set
            if (tid < qc && sm.qk[tid] > 0) {
                const int j = tid, K = sm.qk[j];
                uint64_t *mytk = tk + (int64_t)j * kcap;
                int c = sm.tkcnt[j], mx = sm.tkmax[j];
                for (int ww = 0; ww < W; ++ww) {
                    const int np = sm.pcnt[ww][j];
                    for (int p = 0; p < np; ++p) {
                        const uint64_t key = sm.pos[ww][j][p];
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
                }
                sm.tkcnt[j] = c;
                sm.tkmax[j] = mx;
                if (round_end && c == K) {
                    const float kth = key_dist2(mytk[mx]);
                    if (kth < sm.r2s[j]) sm.r2s[j] = kth;
                }
            }
            __syncthreads();
        }
        // publish the unit's per-query KNN sets for the merge
        for (int i = tid; i < qc * kcap; i += 64 * W) {
            const int j = i / kcap, t = i % kcap;
            const uint64_t key = (sm.qk[j] > 0 && t < sm.tkcnt[j]) ? tk[(int64_t)j * kcap + t] : KEY_NONE;
            a.slots[((int64_t)sm.qidx[j] * a.nprobe_max + sm.qrank[j]) * kcap + t] = key;
        }
        __syncthreads();
    }

    if (a.stats) {
        for (int o = 32; o > 0; o >>= 1) {
            my_dims += __shfl_down(my_dims, o);
            my_pos += __shfl_down(my_pos, o);
            my_dcos += __shfl_down(my_dcos, o);
        }
        if (lane == 0) {
            atomicAdd(a.stats + ADS_STAT_DIMS, my_dims);
            atomicAdd(a.stats + ADS_STAT_BYTES, my_dims * (unsigned long long)EB);
            atomicAdd(a.stats + ADS_STAT_POSITIVES, my_pos);
            atomicAdd(a.stats + ADS_STAT_DCOS, my_dcos);
        }
    }
}

template <int DD, int QW, int W, bool PF>
size_t scan_smem_bytes(int nb, int kcap) {
    size_t s = sizeof(ScanSmem<DD, QW, W, PF ? 2 : 1>) + sizeof(float) * nb;
    s = (s + 15) & ~(size_t)15;
    return s + sizeof(uint64_t) * (size_t)QW * kcap;
}

// Three forms: one wave per unit (plain or prefetching) and four waves per
// unit (rounds of four tiles).
template <int DT, int DD, int QW>
hipError_t launch_scan_t(const ScanArgs &a, int grid, bool pf, bool wide, hipStream_t s) {
    // rounds of four tiles on four waves when the LDS fits, else on one wave
    // (same thresholds, same results)
    if (wide && a.round_tiles == 4) {
        const size_t sh = scan_smem_bytes<DD, QW, 4, false>(a.nb, a.kcap);
        if (sh <= 64 * 1024) {
            hipLaunchKernelGGL((scan_kernel<DT, DD, QW, false, 4>), dim3(grid), dim3(256), sh, s, a);
            return hipGetLastError();
        }
    }
    const size_t sh = pf ? scan_smem_bytes<DD, QW, 1, true>(a.nb, a.kcap) : scan_smem_bytes<DD, QW, 1, false>(a.nb, a.kcap);
    if (sh > 64 * 1024) return hipErrorInvalidValue;
    if (pf)
        hipLaunchKernelGGL((scan_kernel<DT, DD, QW, true, 1>), dim3(grid), dim3(64), sh, s, a);
    else
        hipLaunchKernelGGL((scan_kernel<DT, DD, QW, false, 1>), dim3(grid), dim3(64), sh, s, a);
    return hipGetLastError();
}

template <int DT, int DD>
hipError_t launch_scan_q(const ScanArgs &a, int qw, int grid, bool pf, bool wide, hipStream_t s) {
    switch (qw) {
        case 16: return launch_scan_t<DT, DD, 16>(a, grid, pf, wide, s);
        case 8: return launch_scan_t<DT, DD, 8>(a, grid, pf, wide, s);
        case 4: return launch_scan_t<DT, DD, 4>(a, grid, pf, wide, s);
        case 2: return launch_scan_t<DT, DD, 2>(a, grid, pf, wide, s);
        case 1: return launch_scan_t<DT, DD, 1>(a, grid, pf, wide, s);
    }
    return hipErrorInvalidValue;
}

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
