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

#pragma once
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
    int qidx[QW], qrank[QW], qk[QW], tkcnt[QW];
    uint64_t tkkth[QW];             // the K-th key of a full local KNN set
    uint64_t found;
    uint32_t misc[4];
    uint32_t hist[256];             // radix-select histogram of the fold
    // followed by float coef[nb] and uint64 tk[QW][kcap]
};

// Folds a round's positives into each query's local KNN set: the set becomes
// the K smallest keys of the set and the new positives, selected by the whole
// workgroup (radix select of the K-th key over the union, then the kept new
// keys fill the holes).  At the end of a round of tiles a full set lowers its
// query's threshold to the K-th distance.  Kept out of line: it runs once per
// round, and inlined it would add register pressure to the scan loop.
template <int W, class Smem>
__device__ __attribute__((noinline)) void fold_round(Smem &sm, uint64_t *tk, int kcap, int qc, bool round_end) {
    const int tid = threadIdx.x;
    for (int j = 0; j < qc; ++j) {
        const int K = sm.qk[j];
        if (K <= 0) continue;
        int m = 0;
        for (int ww = 0; ww < W; ++ww) m += sm.pcnt[ww][j];
        uint64_t *mytk = tk + (int64_t)j * kcap;
        const int c = sm.tkcnt[j];
        if (m > 0) {
            auto newkey = [&](int i) -> uint64_t {
                int ww = 0;
                while (i >= sm.pcnt[ww][j]) i -= sm.pcnt[ww][j], ++ww;
                return sm.pos[ww][j][i];
            };
            auto get = [&](int i) -> uint64_t { return i < c ? mytk[i] : newkey(i - c); };
            const int n = c + m;
            // the K-th key of the union, once the set will be full
            const uint64_t kth = n >= K ? group_kth<64 * W>(get, n, K, sm.hist, sm.misc, &sm.found) : KEY_NONE;
            // keys are distinct (distinct ids), so exactly min(n, K) keys are
            // <= kth.  The kept new keys (at most one per thread: m <= 64 W)
            // fill the holes of the set: slots >= c, and old keys > kth.
            const uint64_t nk = tid < m ? newkey(tid) : KEY_NONE;
            const bool keepnew = tid < m && nk <= kth;
            const int kn = n < K ? n : K;
            int nh = 0;
            for (int sl = tid; sl < kn; sl += 64 * W) nh += (sl >= c || mytk[sl] > kth);
            int htot, ntot;
            const int hbase = group_excl_scan<W>(nh, reinterpret_cast<int *>(sm.misc), htot);
            const int nrank = group_excl_scan<W>(keepnew ? 1 : 0, reinterpret_cast<int *>(sm.misc), ntot);
            // hole positions by rank, in the (consumed) positive buffers
            int *holes = reinterpret_cast<int *>(&sm.pos[0][0][0]);
            int hr = hbase;
            for (int sl = tid; sl < kn; sl += 64 * W)
                if (sl >= c || mytk[sl] > kth) holes[hr++] = sl;
            __syncthreads();
            if (keepnew) mytk[holes[nrank]] = nk;
            if (tid == 0) {
                sm.tkcnt[j] = kn;
                sm.tkkth[j] = kth;
            }
            __syncthreads();
        }
        if (tid == 0 && round_end && sm.tkcnt[j] == K) {
            const float kth = key_dist2(sm.tkkth[j]);
            if (kth < sm.r2s[j]) sm.r2s[j] = kth;
        }
    }
    __syncthreads();
}

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
            sm.tkkth[tid] = KEY_NONE;
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
                if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + layout_offset(nl, v, 0, DD, a.b1, D) * EB, o);
                store_q(qv, sm.qs[w][0]);
            }
            for (; tile_pairs > 0 && b < nb; ++b) {
                float o1[DD];
                float4 qv1[QPL];
                if constexpr (PF) {
                    const int bn = b + 1 < nb ? b + 1 : b;
                    fetch_q(bn, qv1);
                    if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + layout_offset(nl, v, bn, DD, a.b1, D) * EB, o1);
                } else {
                    if ((amany >> lane) & 1ull) load_elems<DT, DD>(lbase + layout_offset(nl, v, b, DD, a.b1, D) * EB, o);
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
                ctx.b1 = a.b1;
                const int32_t *tids = a.ids + off + vc;
                uint64_t(*pos)[64] = sm.pos[w];
                auto sink = [=](int jj, float s, int vv) {
                    const int p = atomicAdd(&pcnt[jj], 1);
                    pos[jj][p] = make_key(s, (uint32_t)tids[vv]);
                };
                const SparseOut so = sparse_run<DT, DD>(ctx, sm.list[w][0], sm.list[w][1], m, b, sink);
                my_dims += so.dims;
                my_pos += so.pos;
            }
            __syncthreads();
            fold_round<W>(sm, tk, kcap, qc, round_end);
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
}  // namespace ads
