// Candidate scan with the dense phase on the matrix cores.
//
// Same schedule, units, tiles, thresholds and outputs as the register-dense
// scan (scan.hip); only the way the first blocks of a tile are evaluated
// differs, and every decision is the one the canonical computation takes.
//
// Dense phase.  For a 64-vector tile and the unit's query slots, the block
// partial of every (vector, query) pair is taken in the dot-product form
//     ||o_b||^2 + ||q_b||^2 - 2 <o_b, q_b>
// with one v_mfma_f32_16x16x4_f32 chain per 16-vector slice: the A operand is
// -2 q (16 query slots x Delta_d), the B operand the slice's vectors, and one
// extra k-step adds the two block norms (query norm x 1, 1 x vector norm).
// Lane l then holds the pairs (query 4*(l/16) + i, vector 16*t + l%16).
//
// This S is not the canonical S (differences squared, summed in coordinate
// order), but it differs from it by at most m = kappa * (||o||^2 + ||q||^2),
// kappa a worst-case rounding bound times a safety factor (computed by the
// host from Delta_d and D / Delta_d).  A decision is taken only when it holds
// for every value within m: reject when S - coef(d) r^2 > m, keep when
// S - coef(d) r^2 <= -m.  A pair inside the band, and every pair that reaches
// d = D without being certainly non-positive, goes to the exact queue, which
// is re-evaluated from block 0 in the canonical form.  Hence rejections,
// their dimension counts, positives and distances all equal those of the
// canonical scan.
//
// After the dense phase the surviving pairs continue in the pair-list phase
// with the same margin, then the exact queue runs in chunks through the
// canonical pair-list phase; positives are folded into the unit's KNN sets
// after each chunk and the thresholds are lowered once per tile.
#include "scan_sparse.h"

namespace ads {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int QW>
struct MfmaSmem {
    static constexpr int LCAP = 16 * QW;   // pairs at the hand-off (<= 1/4 of the tile) and per exact chunk
    uint64_t list[2][LCAP];
    uint64_t posk[LCAP];
    uint16_t exq[64 * QW];
    uint8_t posq[LCAP];
    float vmarg[64];
    float r2s[QW], qmarg[QW];
    int qidx[QW], qrank[QW], qk[QW], tkcnt[QW], tkmax[QW];
    int npos;
    // followed by float coef[nb] and uint64 tk[QW][kcap]
};

// N consecutive storage elements (N = Delta_d / 4) converted to float.
template <int DT, int N>
__device__ __forceinline__ void load_run(const unsigned char *p, float *out) {
    if constexpr (DT == ADS_F32) {
        if constexpr (N % 4 == 0) {
#pragma unroll
            for (int i = 0; i < N / 4; ++i) {
                const float4 t = reinterpret_cast<const float4 *>(p)[i];
                out[4 * i] = t.x; out[4 * i + 1] = t.y; out[4 * i + 2] = t.z; out[4 * i + 3] = t.w;
            }
        } else {
            const float2 t = *reinterpret_cast<const float2 *>(p);
            out[0] = t.x; out[1] = t.y;
        }
    } else {
        uint32_t w[N / 2];
        if constexpr (N % 8 == 0) {
#pragma unroll
            for (int i = 0; i < N / 8; ++i) {
                const uint4 t = reinterpret_cast<const uint4 *>(p)[i];
                w[4 * i] = t.x; w[4 * i + 1] = t.y; w[4 * i + 2] = t.z; w[4 * i + 3] = t.w;
            }
        } else if constexpr (N == 4) {
            const uint2 t = *reinterpret_cast<const uint2 *>(p);
            w[0] = t.x; w[1] = t.y;
        } else {
            w[0] = *reinterpret_cast<const uint32_t *>(p);
        }
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            if constexpr (DT == ADS_BF16) {
                out[2 * i] = bf16_to_f32(w[i] & 0xffffu);
                out[2 * i + 1] = bf16_to_f32(w[i] >> 16);
            } else {
                out[2 * i] = f16_to_f32(w[i] & 0xffffu);
                out[2 * i + 1] = f16_to_f32(w[i] >> 16);
            }
        }
    }
}

// Number of set bits of a 16-bit per-lane mask summed over the wave, with
// ballots (no cross-lane data movement through LDS).
__device__ __forceinline__ int wave_count16(uint32_t bits) {
    int n = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) n += __popcll(__ballot((bits >> k) & 1u));
    return n;
}

template <int DT, int DD, int QW>
__global__ __launch_bounds__(64) void scan_mfma_kernel(ScanArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MfmaSmem<QW> &sm = *reinterpret_cast<MfmaSmem<QW> *>(smem_raw);
    float *coef = reinterpret_cast<float *>(smem_raw + sizeof(MfmaSmem<QW>));
    uint64_t *tk = reinterpret_cast<uint64_t *>(
        smem_raw + ((sizeof(MfmaSmem<QW>) + sizeof(float) * a.nb + 15) & ~(size_t)15));
    constexpr int LCAP = MfmaSmem<QW>::LCAP;
    constexpr int KS = DD / 4;             // k-steps per block = elements per lane per vector
    constexpr int EB = Elem<DT>::bytes;

    const int lane = threadIdx.x, n16 = lane & 15, g = lane >> 4;
    const int x = blockIdx.x & 7;
    const int P = gridDim.x >> 3;
    const int cntx = a.xcnt[x], basex = a.xoff[x];
    if ((int)(blockIdx.x >> 3) >= cntx) return;
    const int D = a.D, nb = a.nb, kcap = a.kcap, nb1 = nb + 1;

    for (int b = lane; b < nb; b += 64) {
        int d = (b + 1) * DD;
        coef[b] = d < D ? test_coef(d, D, a.eps0, a.method) : 0.f;
    }
    unsigned long long my_dims = 0, my_pos = 0, my_dcos = 0;   // per lane

    for (int k = blockIdx.x >> 3; k < cntx; k += P) {
        const int4 un = a.units[basex + k];
        const int l = un.x, qbeg = un.y, qc = un.z;
        const int64_t off = a.list_off[l];
        const int nl = (int)(a.list_off[l + 1] - off);
        const unsigned char *lbase = reinterpret_cast<const unsigned char *>(a.data) + off * (int64_t)D * EB;
        const float *bnl = a.blk_norm + off * (int64_t)nb;      // this list's block norms [nb][nl]
        if (lane < QW) {
            int kq = 0;
            if (lane < qc) {
                const int2 e = a.qent[qbeg + lane];
                sm.qidx[lane] = e.x;
                sm.qrank[lane] = e.y;
                kq = a.keff[e.x];
                sm.r2s[lane] = a.r2_in[e.x];
                sm.qmarg[lane] = a.kappa * a.qbn[(int64_t)e.x * nb1 + nb] + 1e-30f;
            }
            sm.qk[lane] = kq;
            sm.tkcnt[lane] = 0;
            sm.tkmax[lane] = 0;
        }
        wave_sync();
        if (lane == 0) {
            int act = 0;
            for (int j = 0; j < qc; ++j) act += sm.qk[j] > 0;
            my_dcos += (unsigned long long)act * (unsigned long long)nl;
        }
        // the C rows of this lane: query slots 4g + i
        bool qok[4];
        float qm[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int jq = 4 * g + i;
            qok[i] = jq < qc && sm.qk[jq] > 0;
            qm[i] = qok[i] ? sm.qmarg[jq] : 0.f;
        }
        // the A row of this lane: query slot n16
        const int64_t qrow = sm.qidx[n16 < qc ? n16 : 0];
        const float *qr = a.qrot + qrow * D + g * KS;
        const float *qb = a.qbn + qrow * nb1;

        SparseCtx ctx;
        ctx.lbase = lbase;
        ctx.nl = nl;
        ctx.qrot = a.qrot;
        ctx.qidx = sm.qidx;
        ctx.r2s = sm.r2s;
        ctx.coef = coef;
        ctx.D = D;
        ctx.nb = nb;
        ctx.vmarg = sm.vmarg;
        ctx.qmarg = sm.qmarg;
        ctx.exq = sm.exq;

        for (int vc = 0; vc < nl; vc += 64) {
            ctx.vc = vc;
            // thresholds change only at the end of a round of round_tiles tiles
            const bool round_end = ((vc >> 6) + 1) % a.round_tiles == 0 || vc + 64 >= nl;
            {
                const int v = vc + lane;
                sm.vmarg[lane] = v < nl ? a.kappa * a.vec_norm[off + v] : 0.f;
            }
            wave_sync();
            float r2v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) r2v[i] = qok[i] ? sm.r2s[4 * g + i] : 0.f;
            float S[4][4];
            uint32_t alive = 0;         // bit 4t+i: pair (vector 16t + n16, query slot 4g + i)
            uint32_t nothr = 0;         // pairs of slots without a threshold yet (r = +inf)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool vok = vc + 16 * t + n16 < nl;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    S[t][i] = 0.f;
                    if (vok && qok[i]) alive |= 1u << (4 * t + i);
                    if (__builtin_isinf(r2v[i])) nothr |= 1u << (4 * t + i);
                }
            }
            const int tile_pairs = wave_count16(alive);
            int nexq = 0, m = 0, b = 0;
            bool handoff = false;
            // Operands of one block.  Loads are unconditional: a slot past qc
            // reads slot 0's row and a vector past the list end reads the
            // list's last vector; their C rows / columns belong to pairs that
            // are never alive.  The next block's operands are fetched before
            // the current block is evaluated (the tile almost always needs it).
            float av[KS], bo[4][KS], on[4], qbv;
            auto fetch = [&](int bb, float *av_, float (*bo_)[KS], float *on_, float &qbv_) {
                load_run<ADS_F32, KS>(reinterpret_cast<const unsigned char *>(qr + bb * DD), av_);
                qbv_ = qb[bb];
                // wave-uniform bases, 32-bit lane offsets
                const unsigned char *bblk = lbase + (int64_t)bb * nl * (DD * EB);
                const float *bnb = bnl + (int64_t)bb * nl;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int vr = min(vc + 16 * t + n16, nl - 1);     // clamped list row
                    load_run<DT, KS>(bblk + (uint32_t)(vr * (DD * EB) + g * (KS * EB)), bo_[t]);
                    on_[t] = bnb[(uint32_t)vr];
                }
            };
            if (tile_pairs > 0) fetch(0, av, bo, on, qbv);
            for (; tile_pairs > 0 && b < nb; ++b) {
                float av1[KS], bo1[4][KS], on1[4], qbv1;
                fetch(b + 1 < nb ? b + 1 : b, av1, bo1, on1, qbv1);
                // the norm step: k-slot 0 carries (||q_b||^2, 1), k-slot 1 (1, ||o_b||^2)
                const float ax = g == 0 ? qbv : (g == 1 ? 1.f : 0.f);
                const int d = (b + 1) * DD;
                const bool last = d >= D;
                // at d < D: reject above coef(d) r^2, keep at or below it; at
                // d = D: certainly not a positive above r^2, and nothing is kept
                const float cf = last ? 1.f : coef[b];
                float thr[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) thr[i] = cf * r2v[i];
                uint32_t rb = 0, kb = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float bx = g == 0 ? 1.f : (g == 1 ? on[t] : 0.f);
                    v4f c = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int j = 0; j < KS; ++j)
                        c = __builtin_amdgcn_mfma_f32_16x16x4f32(-2.f * av[j], bo[t][j], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(ax, bx, c, 0, 0, 0);
                    const float vmt = sm.vmarg[16 * t + n16];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float s = S[t][i] + c[i];
                        S[t][i] = s;
                        const float mg = vmt + qm[i];
                        const float dl = s - thr[i];
                        rb |= (dl > mg ? 1u : 0u) << (4 * t + i);
                        kb |= (dl <= -mg ? 1u : 0u) << (4 * t + i);
                    }
                }
                // nothing is kept at d = D; a query without a threshold accepts
                // every candidate, so its pairs go to the exact queue at once
                if (last) kb = 0u;
                kb &= ~nothr;
                uint32_t ub = ~(rb | kb);
                rb &= alive;
                ub &= alive;
                alive &= ~(rb | ub);
                my_dims += (unsigned long long)__popc(rb) * (unsigned long long)d;
                if (__ballot(ub != 0)) {
                    const int ln = opaque(lane);
                    int tot;
                    int p = nexq + wave_excl_scan(__popc(ub), tot);
                    while (ub) {
                        const int bit = __ffs(ub) - 1;
                        ub &= ub - 1;
                        sm.exq[p++] = (uint16_t)((4 * (ln >> 4) + (bit & 3)) << 6 | (16 * (bit >> 2) + (ln & 15)));
                    }
                    nexq += tot;
                }
                const int na = wave_count16(alive);
                if (na == 0 || last) break;
                if ((float)na <= a.dense_frac * (float)tile_pairs) {
                    const int ln = opaque(lane);
                    int p = wave_excl_scan(__popc(alive), m);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if ((alive >> (4 * t + i)) & 1u)
                                sm.list[0][p++] = pair_entry(S[t][i], 4 * (ln >> 4) + i, 16 * t + (ln & 15));
                    }
                    handoff = true;
                    ++b;
                    break;
                }
#pragma unroll
                for (int j = 0; j < KS; ++j) av[j] = av1[j];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    on[t] = on1[t];
#pragma unroll
                    for (int j = 0; j < KS; ++j) bo[t][j] = bo1[t][j];
                }
                qbv = qbv1;
            }
            wave_sync();
            auto no_sink = [](int, float, int) {};
            if (handoff) {
                const SparseOut so = sparse_run<DT, DD, true>(ctx, sm.list[0], sm.list[1], m, b, nexq, no_sink);
                my_dims += so.dims;
                nexq = so.nexq;
            }
            // the exact queue, canonical from block 0, in chunks of LCAP pairs
            const int32_t *tids = a.ids + off + vc;
            MfmaSmem<QW> *smp = &sm;
            auto sink = [=](int jj, float s, int vv) {
                const int p = atomicAdd(&smp->npos, 1);
                smp->posk[p] = make_key(s, (uint32_t)tids[vv]);
                smp->posq[p] = (uint8_t)jj;
            };
            for (int c0 = 0; c0 < nexq; c0 += LCAP) {
                const int cnt = nexq - c0 < LCAP ? nexq - c0 : LCAP;
                wave_sync();
                for (int i = lane; i < cnt; i += 64) sm.list[0][i] = (uint64_t)sm.exq[c0 + i];
                if (lane == 0) sm.npos = 0;
                wave_sync();
                const SparseOut so = sparse_run<DT, DD, false>(ctx, sm.list[0], sm.list[1], cnt, 0, 0, sink);
                my_dims += so.dims;
                my_pos += so.pos;
                wave_sync();
                if (lane < qc && sm.qk[lane] > 0) {
                    const int j = lane, K = sm.qk[j], np = sm.npos;
                    uint64_t *mytk = tk + (int64_t)j * kcap;
                    int cc = sm.tkcnt[j], mx = sm.tkmax[j];
                    for (int p = 0; p < np; ++p) {
                        if (sm.posq[p] != j) continue;
                        const uint64_t key = sm.posk[p];
                        if (cc < K) {
                            mytk[cc++] = key;
                            if (cc == K) {
                                mx = 0;
                                for (int t = 1; t < K; ++t) if (mytk[t] > mytk[mx]) mx = t;
                            }
                        } else if (key < mytk[mx]) {
                            mytk[mx] = key;
                            mx = 0;
                            for (int t = 1; t < K; ++t) if (mytk[t] > mytk[mx]) mx = t;
                        }
                    }
                    sm.tkcnt[j] = cc;
                    sm.tkmax[j] = mx;
                }
            }
            wave_sync();
            // the round's positives lower the thresholds for the next round
            if (round_end && lane < qc && sm.qk[lane] > 0 && sm.tkcnt[lane] == sm.qk[lane]) {
                const float kth = key_dist2(tk[(int64_t)lane * kcap + sm.tkmax[lane]]);
                if (kth < sm.r2s[lane]) sm.r2s[lane] = kth;
            }
            wave_sync();
        }
        // publish the unit's per-query KNN sets for the merge
        for (int i = lane; i < qc * kcap; i += 64) {
            const int j = i / kcap, t = i % kcap;
            const uint64_t key = (sm.qk[j] > 0 && t < sm.tkcnt[j]) ? tk[(int64_t)j * kcap + t] : KEY_NONE;
            a.slots[((int64_t)sm.qidx[j] * a.nprobe_max + sm.qrank[j]) * kcap + t] = key;
        }
        wave_sync();
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

template <int DD, int QW>
size_t mfma_smem_bytes(int nb, int kcap) {
    size_t s = sizeof(MfmaSmem<QW>) + sizeof(float) * nb;
    s = (s + 15) & ~(size_t)15;
    return s + sizeof(uint64_t) * (size_t)QW * kcap;
}

template <int DT, int DD, int QW>
hipError_t launch_t(const ScanArgs &a, int grid, hipStream_t s) {
    const size_t sh = mfma_smem_bytes<DD, QW>(a.nb, a.kcap);
    if (sh > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((scan_mfma_kernel<DT, DD, QW>), dim3(grid), dim3(64), sh, s, a);
    return hipGetLastError();
}

template <int DT, int DD>
hipError_t launch_q(const ScanArgs &a, int qw, int grid, hipStream_t s) {
    switch (qw) {
        case 16: return launch_t<DT, DD, 16>(a, grid, s);
        case 8: return launch_t<DT, DD, 8>(a, grid, s);
        case 4: return launch_t<DT, DD, 4>(a, grid, s);
        case 2: return launch_t<DT, DD, 2>(a, grid, s);
        case 1: return launch_t<DT, DD, 1>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

template <int DT>
hipError_t launch_d(const ScanArgs &a, int dd, int qw, int grid, hipStream_t s) {
    switch (dd) {
        case 8: return launch_q<DT, 8>(a, qw, grid, s);
        case 16: return launch_q<DT, 16>(a, qw, grid, s);
        case 32: return launch_q<DT, 32>(a, qw, grid, s);
        case 64: return launch_q<DT, 64>(a, qw, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

namespace {

// One thread per stored vector: the squared norm of each of its blocks (fused
// multiply-adds in coordinate order) and their sum in block order.
template <int DT>
__global__ __launch_bounds__(ADS_WG) void block_norms_kernel(const void *data, const int32_t *list_of_pos,
                                                             const int64_t *list_off, int64_t n, int D, int dd,
                                                             float *blk_norm, float *vec_norm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int l = list_of_pos[p];
    const int64_t off = list_off[l];
    const int64_t nl = list_off[l + 1] - off;
    const int64_t v = p - off;
    const int nb = D / dd;
    float tot = 0.f;
    for (int b = 0; b < nb; ++b) {
        const int64_t e0 = off * D + ((int64_t)b * nl + v) * dd;
        float s = 0.f;
        for (int k = 0; k < dd; ++k) {
            const float o = load_one<DT>(data, e0 + k);
            s = __fmaf_rn(o, o, s);
        }
        blk_norm[off * nb + (int64_t)b * nl + v] = s;
        tot += s;
    }
    vec_norm[p] = tot;
}

// One wave per row: lane b takes blocks b, b+64, ...; lane 0 adds them up.
__global__ __launch_bounds__(64) void query_block_norms_kernel(const float *x, int64_t n, int D, int dd,
                                                               float *out) {
    extern __shared__ float bn[];
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    const int nb = D / dd;
    const float *row = x + r * D;
    for (int b = threadIdx.x; b < nb; b += 64) {
        float s = 0.f;
        for (int k = 0; k < dd; ++k) s = __fmaf_rn(row[b * dd + k], row[b * dd + k], s);
        bn[b] = s;
        out[r * (nb + 1) + b] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
        for (int b = 0; b < nb; ++b) tot += bn[b];
        out[r * (nb + 1) + nb] = tot;
    }
}

}  // namespace

hipError_t launch_block_norms(int dtype, const void *data, const int32_t *list_of_pos, const int64_t *list_off,
                              int64_t n, int D, int dd, float *blk_norm, float *vec_norm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((n + ADS_WG - 1) / ADS_WG);
    switch (dtype) {
        case ADS_F32:
            hipLaunchKernelGGL(block_norms_kernel<ADS_F32>, dim3(grid), dim3(ADS_WG), 0, s, data, list_of_pos,
                               list_off, n, D, dd, blk_norm, vec_norm);
            break;
        case ADS_BF16:
            hipLaunchKernelGGL(block_norms_kernel<ADS_BF16>, dim3(grid), dim3(ADS_WG), 0, s, data, list_of_pos,
                               list_off, n, D, dd, blk_norm, vec_norm);
            break;
        case ADS_F16:
            hipLaunchKernelGGL(block_norms_kernel<ADS_F16>, dim3(grid), dim3(ADS_WG), 0, s, data, list_of_pos,
                               list_off, n, D, dd, blk_norm, vec_norm);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_query_block_norms(const float *x, int64_t n, int D, int dd, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t sh = sizeof(float) * (size_t)(D / dd);
    for (int64_t r0 = 0; r0 < n; r0 += 1 << 30) {
        const int64_t rows = n - r0 < (1 << 30) ? n - r0 : (1 << 30);
        hipLaunchKernelGGL(query_block_norms_kernel, dim3((unsigned)rows), dim3(64), sh, s, x + r0 * D, rows, D, dd,
                           out + r0 * (D / dd + 1));
    }
    return hipGetLastError();
}

hipError_t launch_scan_mfma(const ScanArgs &a, int dtype, int dd, int qw, int grid, hipStream_t s) {
    switch (dtype) {
        case ADS_F32: return launch_d<ADS_F32>(a, dd, qw, grid, s);
        case ADS_BF16: return launch_d<ADS_BF16>(a, dd, qw, grid, s);
        case ADS_F16: return launch_d<ADS_F16>(a, dd, qw, grid, s);
    }
    return hipErrorInvalidValue;
}

float scan_margin_kappa(int dd, int nb) {
    // worst-case |S(dot form) - S(canonical)| / (||o||^2 + ||q||^2) is below
    // (5.5 dd + 8 nb + 14) u to first order (u = 2^-24); four times a rounder bound
    return 4.0f * (float)(6 * dd + 8 * nb + 16) * 0x1p-24f;
}

}  // namespace ads
