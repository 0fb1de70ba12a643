// Graph search with ADSampling DCOs: HNSW (Section 2.2.1, FDScanning DCOs),
// HNSW+ (Section 4, Algorithm 1 as the DCO against the largest distance of the
// result set R) and HNSW++ (Section 5.1: R1 of K exact distances supplies the
// DCO threshold and the answer; R2 of N_ef observed distances drives the beam).
//
// One workgroup of four waves per query.  The search is a chain of dependent
// steps, run by wave 0, so the parallelism inside a query is the neighbour
// list of the vertex being expanded: its not-yet-visited neighbours (up to 32)
// are DCO'd together by the four waves (8 neighbours each, 8 lanes per
// neighbour), against the threshold that holds when the expansion starts, and
// the partial sum after every block of delta_d coordinates is kept in LDS.  The sequential semantics
// (the threshold may shrink after each insertion) are then replayed neighbour
// by neighbour from those partial sums: a smaller threshold can only move a
// rejection to an earlier block (the test compares S_d with coef(d) r^2), so
// the stored sums always reach the block where the sequential DCO stops.  The
// outcome, the sampled dimensions and the observed distance are exactly those
// of the one-at-a-time loop over the same floating-point sums.
//
// Sets hold (squared distance, id) keys in LDS (lexicographic order, so no two
// keys tie).  S is the set of R's (R2's) members not expanded yet: with these
// keys an evicted member can never be expanded later, because R's largest key
// only shrinks once R is full, so popping the smallest unexpanded member of R
// and stopping when none is left expands exactly what the two-heap loop
// expands.  R is unsorted (pops and the largest key by wave reductions over
// per-lane lists of its stripes), R1 is a sorted array.  The threshold is +inf
// until the set is full.
#include "kernels.h"

namespace ads {

namespace {

constexpr int HN_LANES = 8;        // lanes per neighbour: 8 x float4 = 32 coordinates a step
constexpr int HN_GROUPS = ADS_WAVE / HN_LANES;
constexpr int HN_WAVES = 4;        // waves per query: wave 0 searches, every wave DCOs 8 neighbours
constexpr int HN_UNROLL = 8;       // steps of 32 coordinates loaded at once
constexpr int HN_TOP = 4;          // largest keys of its stripe of R kept by each lane
constexpr int HN_BOT = 4;          // smallest unexpanded keys of its stripe of R kept by each lane
constexpr int HN_BATCH = 4;        // set entries per lane read at once by the scans of R
constexpr int HN_REPLAY = 8;       // stored block sums per lane read at once by the replay
static_assert(HN_GROUPS * HN_WAVES == HN_MAXDEG, "one neighbour per lane group and wave");

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

struct Smem {
    float *q;          // [D] rotated query
    float *coef;       // [nb] test coefficients
    uint64_t *rk;      // [nef] R (HNSW, HNSW+) or R2 (HNSW++), ascending
    uint8_t *rx;       // [nef] expanded flags of rk
    uint64_t *r1k;     // [K] R1 (HNSW++)
    int *nbr;          // [HN_MAXDEG] neighbours being DCO'd
    int *tb;           // [HN_MAXDEG] block where the DCO stopped at the expansion's threshold
    float *cm;         // [HN_MAXDEG] max over tested blocks of S_b / coef_b (DCOs that reached d = D)
    float *rcoef;      // [nb] 1 / coef (0 where no test)
    float *psum;       // [HN_MAXDEG][nb] partial sums after each block
    int *job;          // [3] the DCO phase wave 0 hands to the other waves: m, r2 bits, stop flag
};

// Exchanges inside a group of 8 lanes (DPP, no LDS round trip): the value of
// lane gl ^ 1, gl ^ 2 (quad permutations) and gl ^ 4 (a row shift by four
// lanes in either direction; both neighbours of an 8-lane group lie in the
// same 16-lane row).
__device__ __forceinline__ float dpp_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_xor2(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_xor4(float x, bool upper) {
    const int up = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, false);   // lane - 4
    const int dn = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x104, 0xf, 0xf, false);   // lane + 4
    return __int_as_float(upper ? up : dn);
}

// Parallel DCOs of nbr[0..m) against r2 (squared threshold): wave `slot`
// takes neighbours 8 slot .. 8 slot + 7, one per group of 8 lanes.
// psum[j][b] receives the sum after block b up to the block where the DCO
// stops (rejection or the last block); tb[j] that block.  A lane holds 4
// coordinates of a step of 32; the block sums are reduced over the block's
// lanes (a fixed pairwise tree, the same value in every lane of the group) and
// added to S in block order.
template <int DD>
__device__ __forceinline__ void dco_phase(const HnswArgs &a, const Smem &sm, int m, float r2, int lane, int slot) {
    constexpr int BPS = 32 / DD;        // blocks per step
    const int gl = lane & (HN_LANES - 1);
    const int j = lane / HN_LANES + HN_GROUPS * slot;
    const bool upper = (gl & 4) != 0;
    const int steps = a.D >> 5;
    const int nb = a.nb;
    bool act = j < m;
    if (__ballot(act) == 0) return;
    float S = 0.f, cmx = 0.f;
    int term = nb - 1;
    const float *row = a.data + (act ? (int64_t)sm.nbr[j] * a.D : 0) + gl * 4;
    for (int s = 0; s < steps; s += HN_UNROLL) {
        if (__ballot(act) == 0) break;
        // every load is issued, from a valid address (the row's first step
        // where the group is idle or past the end), so that they all go out
        // together before the first is used
        float4 v[HN_UNROLL];
#pragma unroll
        for (int u = 0; u < HN_UNROLL; ++u) {
            const int su = act && s + u < steps ? s + u : 0;
            v[u] = *reinterpret_cast<const float4 *>(row + su * 32);
        }
#pragma unroll
        for (int u = 0; u < HN_UNROLL; ++u) {
            if (s + u >= steps) break;
            const float4 qv = *reinterpret_cast<const float4 *>(sm.q + (s + u) * 32 + gl * 4);
            // the step's test coefficients
            float cf[BPS], rc[BPS];
#pragma unroll
            for (int k = 0; k < BPS; ++k) {
                cf[k] = sm.coef[(s + u) * BPS + k];
                rc[k] = sm.rcoef[(s + u) * BPS + k];
            }
            if (!act) continue;
            const float y0 = v[u].x - qv.x, y1 = v[u].y - qv.y;
            const float y2 = v[u].z - qv.z, y3 = v[u].w - qv.w;
            float p = (y0 * y0 + y1 * y1) + (y2 * y2 + y3 * y3);
            // bsum[k]: the sum over the lanes of block k
            float bsum[BPS];
            if constexpr (DD == 8) {
                p += dpp_xor1(p);                 // pairs: block gl >> 1
                const float o2 = dpp_xor2(p);
                // the even and odd block of this lane's quad, then of the other quad
                const bool odd = (gl & 2) != 0;
                const float lo = odd ? o2 : p, hi = odd ? p : o2;
                const float lo4 = dpp_xor4(lo, upper), hi4 = dpp_xor4(hi, upper);
                bsum[0] = upper ? lo4 : lo;
                bsum[1] = upper ? hi4 : hi;
                bsum[BPS > 2 ? 2 : 0] = upper ? lo : lo4;
                bsum[BPS > 3 ? 3 : 0] = upper ? hi : hi4;
            } else if constexpr (DD == 16) {
                p += dpp_xor1(p);
                p += dpp_xor2(p);                 // quads: block gl >> 2
                const float o = dpp_xor4(p, upper);
                bsum[0] = upper ? o : p;
                bsum[BPS - 1] = upper ? p : o;
            } else {
                p += dpp_xor1(p);
                p += dpp_xor2(p);
                p += dpp_xor4(p, upper);
                bsum[0] = p;
            }
#pragma unroll
            for (int k = 0; k < BPS; ++k) {
                const int bi = (s + u) * BPS + k;
                S += bsum[k];
                if (gl == 0) sm.psum[j * nb + bi] = S;
                if (bi < nb - 1) {
                    if (test_reject(S, cf[k], r2)) {
                        term = bi;
                        act = false;
                        break;
                    }
                    cmx = fmaxf(cmx, S * rc[k]);
                }
            }
        }
    }
    if (j < m && gl == 0) {
        sm.tb[j] = term;
        sm.cm[j] = cmx;
    }
}

// A DCO that reached d = D at its phase's threshold rejects at no block for a
// threshold r2 above max_b S_b / coef_b: then coef_b r2 exceeds every S_b by
// far more than the rounding of the product and of the stored quotient (a
// margin of 1e-5), so test_reject is false at every block without evaluating
// them.  Closer thresholds are decided block by block.
__device__ __forceinline__ bool no_test_below(const Smem &sm, int j, int t0, int nb, float r2) {
    return t0 == nb - 1 && r2 > sm.cm[j] * 1.00001f;
}

// The sequential DCO of neighbour j at squared threshold r2 (<= the threshold
// of its dco_phase), replayed from the stored sums.  Returns the block where
// it stops; *pos / *s receive the positive flag and the sum there.
__device__ int replay(const HnswArgs &a, const Smem &sm, int j, float r2, float r2_phase, bool *pos,
                      float *s, int lane) {
    const int nb = a.nb;
    const int t0 = sm.tb[j];
    int stop = t0;
    if (r2 != r2_phase && !no_test_below(sm, j, t0, nb, r2)) {
        const int lim = t0 < nb - 1 ? t0 : nb - 2;     // blocks that carry a test
        stop = nb - 1;
        for (int b0 = 0; b0 <= lim; b0 += ADS_WAVE) {
            const int b = b0 + lane;
            const bool rej = b <= lim && test_reject(sm.psum[j * nb + b], sm.coef[b], r2);
            const uint64_t mask = wave_ballot(rej);
            if (mask) {
                stop = b0 + __ffsll((long long)mask) - 1;
                break;
            }
        }
    }
    *s = sm.psum[j * nb + stop];
    *pos = stop == nb - 1 && *s <= r2;
    return stop;
}

// Inserts key into the ascending array k[0..n) of capacity cap (<= 4096; the
// caller has checked that it belongs there); the largest key falls off a full
// array.  Returns the position.  The position comes from two ballots (every
// ceil(n/64)-th key, then the keys of the bracketing stretch); the move is done
// from the top down in stretches of 256 entries, four per lane, each stretch
// read completely before it is written one place higher.
__device__ int sorted_insert(uint64_t *k, uint8_t *x, int &n, int cap, uint64_t key, int lane) {
    int p = 0;
    if (n > 0) {
        const int S = (n + ADS_WAVE - 1) / ADS_WAVE;
        const int i1 = lane * S;
        const int b = __popcll(wave_ballot(i1 < n && k[i1] < key));
        if (b > 0) {
            const int base = (b - 1) * S + 1;
            const int i2 = base + lane;
            const bool lt = lane < S - 1 && i2 < n && k[i2] < key;
            p = base + __popcll(wave_ballot(lt));
        }
    }
    const int last = n < cap ? n : cap - 1;          // entries p..last-1 move up by one
    for (int hi = last; hi > p; hi -= 4 * ADS_WAVE) {
        const int lo = hi - 4 * ADS_WAVE > p ? hi - 4 * ADS_WAVE : p;
        uint64_t tk[4];
        uint8_t tx[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = lo + lane + c * ADS_WAVE;
            tk[c] = 0;
            tx[c] = 0;
            if (i < hi) {
                tk[c] = k[i];
                if (x) tx[c] = x[i];
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = lo + lane + c * ADS_WAVE;
            if (i < hi) {
                k[i + 1] = tk[c];
                if (x) x[i + 1] = tx[c];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        k[p] = key;
        if (x) x[p] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    if (n < cap) ++n;
    return p;
}

// Wave-wide reductions without LDS round trips: DPP exchanges inside each
// 16-lane row (lane ^ 1, lane ^ 2, then rotations by 4 and 8, after which every
// lane of a row holds the row's result), then the four rows' results read
// with readlane and combined; every lane returns the same value.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xf, 0xf, false);
}

// (key, index) pairs: keeps the pair for which better(new, new index, old,
// old index) holds.
template <int CTRL, class Better>
__device__ __forceinline__ void best_step(uint64_t &k, int &i, Better better) {
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)k), hi = dpp_u32<CTRL>((uint32_t)(k >> 32));
    const int oi = (int)dpp_u32<CTRL>((uint32_t)i);
    const uint64_t ok = ((uint64_t)hi << 32) | lo;
    if (better(ok, oi, k, i)) {
        k = ok;
        i = oi;
    }
}

template <class Better>
__device__ __forceinline__ void wave_best(uint64_t &k, int &i, Better better) {
    best_step<0xB1>(k, i, better);      // quad_perm 1,0,3,2
    best_step<0x4E>(k, i, better);      // quad_perm 2,3,0,1
    best_step<0x124>(k, i, better);     // row_ror:4
    best_step<0x128>(k, i, better);     // row_ror:8
    uint64_t bk = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(k >> 32), 0) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 16; r < ADS_WAVE; r += 16) {
        const uint64_t rk = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(k >> 32), r) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, r);
        const int ri = __builtin_amdgcn_readlane(i, r);
        if (better(rk, ri, bk, bi)) {
            bk = rk;
            bi = ri;
        }
    }
    k = bk;
    i = bi;
}

// Smallest key among the entries of k[0..n) whose flag equals want, and its
// index (-1 when there is none); every lane returns the same pair.  Keys are
// distinct, so the minimum is unique.
__device__ int argmin_flag(const uint64_t *k, const uint8_t *x, int n, uint8_t want, int lane, uint64_t *kout) {
    uint64_t best = KEY_NONE;
    int bi = -1;
    // HN_BATCH entries per lane are read before any is compared
    for (int i0 = lane; i0 < n; i0 += HN_BATCH * ADS_WAVE) {
        uint64_t v[HN_BATCH];
        bool ok[HN_BATCH];
#pragma unroll
        for (int c = 0; c < HN_BATCH; ++c) {
            const int i = i0 + c * ADS_WAVE;
            ok[c] = i < n;
            v[c] = ok[c] ? k[i] : KEY_NONE;
            ok[c] = ok[c] && x[i] == want;
        }
#pragma unroll
        for (int c = 0; c < HN_BATCH; ++c)
            if (ok[c] && v[c] < best) {
                best = v[c];
                bi = i0 + c * ADS_WAVE;
            }
    }
    wave_best(best, bi, [](uint64_t ok, int, uint64_t k, int) { return ok < k; });
    *kout = best;
    return bi;
}

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_sum(int v) {
    v += (int)dpp_u32<0xB1>((uint32_t)v);
    v += (int)dpp_u32<0x4E>((uint32_t)v);
    v += (int)dpp_u32<0x124>((uint32_t)v);
    v += (int)dpp_u32<0x128>((uint32_t)v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}

// x of lane k (k the same on every lane).
__device__ __forceinline__ int lane_value(int x, int k) { return __builtin_amdgcn_readlane(x, k); }
__device__ __forceinline__ float lane_value(float x, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
}

// replay() evaluated by one lane for its own neighbour j.
__device__ __forceinline__ int outcome_lane(const HnswArgs &a, const Smem &sm, int j, float r2, float r2_phase,
                                            bool *pos, float *s) {
    const int nb = a.nb;
    const int t0 = sm.tb[j];
    int stop = t0;
    if (r2 != r2_phase && !no_test_below(sm, j, t0, nb, r2)) {
        const int lim = t0 < nb - 1 ? t0 : nb - 2;     // blocks that carry a test
        stop = nb - 1;
        // HN_REPLAY blocks are read before any is tested
        for (int b0 = 0; b0 <= lim; b0 += HN_REPLAY) {
            float ps[HN_REPLAY], cf[HN_REPLAY];
#pragma unroll
            for (int c = 0; c < HN_REPLAY; ++c) {
                const int b = b0 + c <= lim ? b0 + c : lim;
                ps[c] = sm.psum[j * nb + b];
                cf[c] = sm.coef[b];
            }
            int hit = -1;
#pragma unroll
            for (int c = HN_REPLAY - 1; c >= 0; --c)
                if (b0 + c <= lim && test_reject(ps[c], cf[c], r2)) hit = b0 + c;
            if (hit >= 0) {
                stop = hit;
                break;
            }
        }
    }
    *s = sm.psum[j * nb + stop];
    *pos = stop == nb - 1 && *s <= r2;
    return stop;
}

}  // namespace

template <int DD>
__global__ __launch_bounds__(HN_WAVES * ADS_WAVE) void hnsw_search_kernel(HnswArgs a) {
    extern __shared__ __align__(16) unsigned char hn_smem[];
    const int lane = threadIdx.x & (ADS_WAVE - 1);
    // the wave index, as a scalar: the two roles below are wave-uniform
    // branches, so no wave ever meets the other role's barriers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / ADS_WAVE);
    const int qi = blockIdx.x;
    const int D = a.D, nb = a.nb;
    Smem sm;
    {
        unsigned char *p = hn_smem;
        sm.q = reinterpret_cast<float *>(p); p += (size_t)D * 4;
        sm.psum = reinterpret_cast<float *>(p); p += (size_t)HN_MAXDEG * nb * 4;
        sm.coef = reinterpret_cast<float *>(p); p += ((size_t)nb * 4 + 7) & ~(size_t)7;
        sm.rk = reinterpret_cast<uint64_t *>(p); p += (size_t)a.nef * 8;
        sm.r1k = reinterpret_cast<uint64_t *>(p); p += (size_t)a.K * 8;
        sm.nbr = reinterpret_cast<int *>(p); p += HN_MAXDEG * 4;
        sm.tb = reinterpret_cast<int *>(p); p += HN_MAXDEG * 4;
        sm.cm = reinterpret_cast<float *>(p); p += HN_MAXDEG * 4;
        sm.rcoef = reinterpret_cast<float *>(p); p += ((size_t)nb * 4 + 7) & ~(size_t)7;
        sm.job = reinterpret_cast<int *>(p); p += 16;
        sm.rx = p;
    }
    if (wv != 0) {
        // Waves 1..3 take their share of every DCO phase of wave 0: between
        // two workgroup barriers wave 0 publishes a phase (or the stop flag),
        // then all waves evaluate it and meet at a second barrier.
        for (;;) {
            __syncthreads();
            const int stop = __builtin_amdgcn_readfirstlane(sm.job[2]);
            if (stop) break;
            const int m = __builtin_amdgcn_readfirstlane(sm.job[0]);
            const float r2 = __int_as_float(__builtin_amdgcn_readfirstlane(sm.job[1]));
            dco_phase<DD>(a, sm, m, r2, lane, wv);
            __syncthreads();
        }
        return;
    }
    // wave 0: the search.  Every parallel DCO phase goes through run_dco.
    auto run_dco = [&](int m, float r2) {
        if (lane == 0) {
            sm.job[0] = m;
            sm.job[1] = __float_as_int(r2);
            sm.job[2] = 0;
        }
        __syncthreads();
        dco_phase<DD>(a, sm, m, r2, lane, 0);
        __syncthreads();
    };
    const float *qg = a.qrot + (int64_t)qi * D;
    for (int i = lane; i < D; i += ADS_WAVE) sm.q[i] = qg[i];
    for (int i = lane; i < nb; i += ADS_WAVE) {
        const float c = a.coef[i];
        sm.coef[i] = c;
        sm.rcoef[i] = __builtin_isinf(c) ? 0.f : 1.0f / c;
    }
    lds_sync();

    int64_t dcos = 0, dims = 0, hops = 0;
    constexpr int dd = DD;

    // entry vertex: a DCO with threshold +inf
    int cur = a.entry;
    if (lane == 0) sm.nbr[0] = cur;
    lds_sync();
    run_dco(1, __builtin_inff());
    float dcur = sm.psum[nb - 1];
    dcos += 1;
    dims += D;

    // upper layers: greedy descent with the current distance as threshold
    for (int l = a.max_level; l >= 1; --l) {
        for (;;) {
            const int32_t *rowp = a.up_adj + (a.up_off[cur] + (l - 1)) * (int64_t)a.M;
            int v = lane < a.M ? rowp[lane] : -1;
            const uint64_t valid = wave_ballot(v >= 0);
            const int m = __popcll(valid);          // rows are -1 padded at the end
            if (lane < m) sm.nbr[lane] = v;
            lds_sync();
            const float r0 = dcur;
            run_dco(m, r0);
            bool changed = false;
            for (int j = 0; j < m; ++j) {
                bool pos;
                float s;
                const int stop = replay(a, sm, j, dcur, r0, &pos, &s, lane);
                dcos += 1;
                dims += (int64_t)(stop + 1) * dd;
                const int u = sm.nbr[j];
                if (pos && make_key(s, (uint32_t)u) < make_key(dcur, (uint32_t)cur)) {
                    cur = u;
                    dcur = s;
                    changed = true;
                }
            }
            lds_sync();
            if (!__builtin_amdgcn_readfirstlane(changed ? 1 : 0)) break;
        }
    }

    // layer 0: beam search
    uint32_t *vis = a.visited + (int64_t)qi * a.vis_words;
    if (lane == 0) atomicOr(vis + (cur >> 5), 1u << (cur & 31));
    // R (R2 for HNSW++) is kept unsorted: a pop takes the smallest key not yet
    // expanded (one pass over the set and a wave reduction), and a full set
    // keeps its largest key (the threshold and the entry an insertion
    // replaces) in rmaxk / rmaxi.  For the largest key, lane l keeps in
    // registers the HN_TOP largest keys of its stripe (entries i = l mod 64),
    // or fewer: tn of them, always the tn largest of the stripe.  The largest
    // key of R is then a wave reduction over the stripes' first keys.  An
    // insertion replaces the largest key in place, so only that stripe
    // changes: its first key leaves the list and the new key enters it when it
    // is above the list's last one.  A stripe whose list runs empty makes every
    // lane re-read its stripe.  R1 (K entries) stays sorted.
    int nr = 0, nr1 = 0;
    uint64_t rmaxk = KEY_NONE;
    int rmaxi = -1;
    const bool pp = a.variant == ADS_HNSW_PP;
    uint64_t tl[HN_TOP];
    int ti[HN_TOP];
    int tn = 0;
    // the list's last (smallest) key; 0 when empty
    auto tl_last = [&]() {
        uint64_t k = 0;
#pragma unroll
        for (int c = 0; c < HN_TOP; ++c)
            if (c == tn - 1) k = tl[c];
        return k;
    };
    // key (at slot idx of R) enters this lane's list: appended when there is
    // room, else in place of the last key when above it; then moved up to its
    // place (descending order)
    auto tl_add = [&](uint64_t key, int idx) {
        if (tn == HN_TOP) {
            if (key <= tl[HN_TOP - 1]) return;
            tl[HN_TOP - 1] = key;
            ti[HN_TOP - 1] = idx;
        } else {
#pragma unroll
            for (int c = 0; c < HN_TOP; ++c)
                if (c == tn) {
                    tl[c] = key;
                    ti[c] = idx;
                }
            ++tn;
        }
#pragma unroll
        for (int c = HN_TOP - 1; c >= 1; --c)
            if (c < tn && tl[c] > tl[c - 1]) {
                const uint64_t tk = tl[c];
                tl[c] = tl[c - 1];
                tl[c - 1] = tk;
                const int tx = ti[c];
                ti[c] = ti[c - 1];
                ti[c - 1] = tx;
            }
    };
    // Likewise for pops: lane l keeps the bn smallest unexpanded keys of its
    // stripe (bn <= HN_BOT, ascending) and the count ucnt of unexpanded
    // entries there; the pop is a wave reduction over the lists' first keys.
    uint64_t bl[HN_BOT];
    int bx[HN_BOT];
    int bn = 0, ucnt = 0;
    auto bl_last = [&]() {
        uint64_t k = KEY_NONE;
#pragma unroll
        for (int c = 0; c < HN_BOT; ++c)
            if (c == bn - 1) k = bl[c];
        return k;
    };
    // key (at slot idx) enters this lane's list: appended when there is
    // room, else in place of the last key when below it; then moved down to
    // its place (ascending order)
    auto bl_add = [&](uint64_t key, int idx) {
        if (bn == HN_BOT) {
            if (key >= bl[HN_BOT - 1]) return;
            bl[HN_BOT - 1] = key;
            bx[HN_BOT - 1] = idx;
        } else {
#pragma unroll
            for (int c = 0; c < HN_BOT; ++c)
                if (c == bn) {
                    bl[c] = key;
                    bx[c] = idx;
                }
            ++bn;
        }
#pragma unroll
        for (int c = HN_BOT - 1; c >= 1; --c)
            if (c < bn && bl[c] < bl[c - 1]) {
                const uint64_t tk = bl[c];
                bl[c] = bl[c - 1];
                bl[c - 1] = tk;
                const int tx = bx[c];
                bx[c] = bx[c - 1];
                bx[c - 1] = tx;
            }
    };
    // removes entry c (< bn) of this lane's list
    auto bl_drop = [&](int c0) {
#pragma unroll
        for (int c = 0; c + 1 < HN_BOT; ++c)
            if (c >= c0) {
                bl[c] = bl[c + 1];
                bx[c] = bx[c + 1];
            }
        --bn;
    };
    auto unexpanded_reread = [&]() {
        bn = 0;
        ucnt = 0;
        for (int i0 = lane; i0 < nr; i0 += HN_BATCH * ADS_WAVE) {
            uint64_t v[HN_BATCH];
            bool u[HN_BATCH];
#pragma unroll
            for (int c = 0; c < HN_BATCH; ++c) {
                const int i = i0 + c * ADS_WAVE;
                u[c] = i < nr;
                v[c] = u[c] ? sm.rk[i] : KEY_NONE;
                u[c] = u[c] && sm.rx[i] == 0;
            }
#pragma unroll
            for (int c = 0; c < HN_BATCH; ++c)
                if (u[c]) {
                    ++ucnt;
                    bl_add(v[c], i0 + c * ADS_WAVE);
                }
        }
    };
    // a stripe with unexpanded entries and an empty list: re-read every stripe
    auto unexpanded_check = [&]() {
        if (__ballot(bn == 0 && ucnt > 0)) unexpanded_reread();
    };
    auto stripes_reread = [&]() {
        tn = 0;
        for (int i0 = lane; i0 < nr; i0 += HN_BATCH * ADS_WAVE) {
            uint64_t v[HN_BATCH];
#pragma unroll
            for (int c = 0; c < HN_BATCH; ++c) {
                const int i = i0 + c * ADS_WAVE;
                v[c] = i < nr ? sm.rk[i] : 0;
            }
#pragma unroll
            for (int c = 0; c < HN_BATCH; ++c)
                if (i0 + c * ADS_WAVE < nr) tl_add(v[c], i0 + c * ADS_WAVE);
        }
    };
    auto max_of_stripes = [&]() {
        uint64_t k = tn > 0 ? tl[0] : 0;
        int i = tn > 0 ? ti[0] : -1;
        wave_best(k, i, [](uint64_t ok, int oi, uint64_t kk, int ii) { return oi >= 0 && (ii < 0 || ok > kk); });
        rmaxk = k;
        rmaxi = i;
    };
    auto r_insert = [&](uint64_t key) {
        const int at = nr < a.nef ? nr : rmaxi;
        const bool owner = lane == (at & (ADS_WAVE - 1));
        if (nr >= a.nef && owner && sm.rx[at] == 0) {
            // the entry replaced was not expanded yet
            --ucnt;
            int f = -1;
#pragma unroll
            for (int c = 0; c < HN_BOT; ++c)
                if (c < bn && bx[c] == at) f = c;
            if (f >= 0) bl_drop(f);
        }
        if (owner) {
            // the new key joins the list when the list holds every unexpanded
            // entry of the stripe, or when it is below the list's last key
            const bool complete = bn == ucnt;
            ++ucnt;
            if (complete || (bn > 0 && key < bl_last())) bl_add(key, at);
        }
        lds_sync();
        if (lane == 0) {
            sm.rk[at] = key;
            sm.rx[at] = 0;
        }
        lds_sync();
        if (nr < a.nef) {
            ++nr;
            if (nr == a.nef) {
                stripes_reread();
                max_of_stripes();
            }
        } else {
            if (lane == (at & (ADS_WAVE - 1))) {
                // the stripe's first key was R's largest, at slot at
#pragma unroll
                for (int c = 0; c + 1 < HN_TOP; ++c) {
                    tl[c] = tl[c + 1];
                    ti[c] = ti[c + 1];
                }
                --tn;
                // the new key belongs to the list only when it is above the
                // list's last key: below it, keys of the stripe outside the
                // list may be larger
                if (tn > 0 && key > tl_last()) tl_add(key, at);
            }
            // a stripe with entries and an empty list: re-read every stripe
            const bool has = lane < nr;
            if (__ballot(has && tn == 0)) stripes_reread();
            max_of_stripes();
        }
        unexpanded_check();
    };
    r_insert(make_key(dcur, (uint32_t)cur));
    if (pp) sorted_insert(sm.r1k, nullptr, nr1, a.K, make_key(dcur, (uint32_t)cur), lane);
    lds_sync();
    for (;;) {
        // pop: the nearest member of R not expanded yet
        uint64_t pkey = bn > 0 ? bl[0] : KEY_NONE;
        int p = bn > 0 ? bx[0] : -1;
        wave_best(pkey, p, [](uint64_t ok, int, uint64_t k, int) { return ok < k; });
        if (p < 0) break;
        if (lane == (p & (ADS_WAVE - 1))) {
            bl_drop(0);
            --ucnt;
        }
        lds_sync();
        if (lane == 0) sm.rx[p] = 1;
        lds_sync();
        unexpanded_check();
        hops += 1;
        const int u = key_id(pkey);
        // neighbours not visited yet, in stored order
        const int32_t *rowp = a.adj0 + (int64_t)u * a.M0;
        int v = lane < a.M0 ? rowp[lane] : -1;
        bool fresh = false;
        if (v >= 0) {
            const uint32_t bit = 1u << (v & 31);
            fresh = (atomicOr(vis + (v >> 5), bit) & bit) == 0;
        }
        const uint64_t fm = wave_ballot(fresh);
        const int m = __popcll(fm);
        if (fresh) sm.nbr[__popcll(fm & ((1ull << lane) - 1))] = v;
        lds_sync();
        if (m == 0) continue;
        auto threshold = [&]() -> float {
            if (pp) return nr1 < a.K ? __builtin_inff() : key_dist2(sm.r1k[nr1 - 1]);
            return nr < a.nef ? __builtin_inff() : key_dist2(rmaxk);
        };
        const float r0 = threshold();
        run_dco(m, r0);
        // Replay of the sequential loop: all remaining neighbours are
        // evaluated at the current threshold at once (lane = neighbour); the
        // first one whose outcome changes a set ("hot") is then applied, the
        // threshold re-read, and the evaluation repeats after it.  Neighbours
        // before the hot one change nothing, so their outcomes at this
        // threshold are the sequential ones.
        // A lane's outcome depends only on its neighbour and the threshold, so
        // it is evaluated again only when the threshold has changed (HNSW++'s
        // threshold comes from R1, which R2's insertions leave alone).
        int j = 0;
        int stop = 0;
        bool pos = false;
        float sv = 0.f, obs = 0.f;
        uint32_t w_lane = 0;
        float r2_eval = __builtin_nanf("");
        while (j < m) {
            const float r2 = threshold();
            const bool full = nr >= a.nef, full1 = nr1 >= a.K;
            const uint64_t rmax = full ? rmaxk : KEY_NONE;
            const uint64_t r1max = pp && full1 ? sm.r1k[nr1 - 1] : KEY_NONE;
            if (!(r2 == r2_eval)) {
                if (lane >= j && lane < m) {
                    stop = outcome_lane(a, sm, lane, r2, r0, &pos, &sv);
                    w_lane = (uint32_t)sm.nbr[lane];
                    const int d = (stop + 1) * dd;
                    obs = d == D ? sv : (float)((double)sv * (double)D / (double)d);
                }
                r2_eval = r2;
            }
            bool hot = false;
            if (lane >= j && lane < m) {
                if (!pp)
                    hot = pos && make_key(sv, w_lane) < rmax;
                else
                    hot = (pos && make_key(sv, w_lane) < r1max) || make_key(obs, w_lane) < rmax;
            }
            const uint64_t hm = wave_ballot(hot);
            const int k = hm ? __ffsll((long long)hm) - 1 : m;
            dims += wave_sum(lane >= j && lane < k ? (stop + 1) * dd : 0);
            dcos += k - j;
            if (k == m) break;
            const int sk = lane_value(stop, k);
            const float s = lane_value(sv, k);
            const bool pk = lane_value(pos ? 1 : 0, k) != 0;
            const int d = (sk + 1) * dd;
            dcos += 1;
            dims += d;
            const uint32_t w = (uint32_t)sm.nbr[k];
            if (!pp) {
                r_insert(make_key(s, w));
            } else {
                if (pk) {
                    const uint64_t key = make_key(s, w);
                    if (key < r1max) sorted_insert(sm.r1k, nullptr, nr1, a.K, key, lane);
                }
                const uint64_t key2 = make_key(lane_value(obs, k), w);
                if (key2 < rmax) r_insert(key2);
            }
            lds_sync();
            j = k + 1;
        }
    }

    // release the other waves
    if (lane == 0) sm.job[2] = 1;
    __syncthreads();

    // answer: the K nearest of R (HNSW, HNSW+; every member is expanded now,
    // flag 1, and is taken out in ascending order) or R1 (HNSW++, sorted)
    for (int k = 0; k < a.K; ++k) {
        uint64_t key = KEY_NONE;
        if (pp) {
            if (k < nr1) key = sm.r1k[k];
        } else {
            const int i = argmin_flag(sm.rk, sm.rx, nr, 1, lane, &key);
            if (i >= 0 && lane == 0) sm.rx[i] = 2;
            lds_sync();
        }
        if (lane == 0) {
            const int64_t o = (int64_t)qi * a.K + k;
            if (key != KEY_NONE) {
                a.ids[o] = key_id(key);
                a.dist[o] = __builtin_sqrtf(key_dist2(key));
            } else {
                a.ids[o] = -1;
                a.dist[o] = __builtin_inff();
            }
        }
    }
    if (lane == 0) {
        if (a.qstats) {
            a.qstats[3 * (int64_t)qi + 0] = dcos;
            a.qstats[3 * (int64_t)qi + 1] = dims;
            a.qstats[3 * (int64_t)qi + 2] = hops;
        }
        if (a.stats) {
            atomicAdd(a.stats + 0, (unsigned long long)dcos);
            atomicAdd(a.stats + 1, (unsigned long long)dims);
            atomicAdd(a.stats + 2, (unsigned long long)hops);
        }
    }
}

__global__ void hnsw_setup_kernel(float *coef, int nb, int dd, int D, double eps0, int method,
                                  uint32_t *visited, int64_t words) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < nb) coef[tid] = tid == nb - 1 ? 1.0f : test_coef((int)(tid + 1) * dd, D, eps0, method);
    for (int64_t i = tid; i < words; i += (int64_t)gridDim.x * blockDim.x) visited[i] = 0u;
}

size_t hnsw_smem_bytes(int D, int nb, int nef, int K) {
    size_t b = (size_t)D * 4 + (size_t)HN_MAXDEG * nb * 4 + 2 * (((size_t)nb * 4 + 7) & ~(size_t)7) +
               (size_t)nef * 8 + (size_t)K * 8 + 3 * HN_MAXDEG * 4 + 16 + (size_t)nef;
    return (b + 15) & ~(size_t)15;
}

hipError_t launch_hnsw_setup(float *coef, int nb, int dd, int D, double eps0, int method,
                             uint32_t *visited, int64_t words, hipStream_t s) {
    int64_t g = (words + ADS_WG - 1) / ADS_WG;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(hnsw_setup_kernel, dim3((unsigned)g), dim3(ADS_WG), 0, s, coef, nb, dd, D, eps0,
                       method, visited, words);
    return hipGetLastError();
}

hipError_t launch_hnsw_search(const HnswArgs &a, int nq, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const size_t smem = hnsw_smem_bytes(a.D, a.nb, a.nef, a.K);
    switch (a.dd) {
        case 8: hipLaunchKernelGGL(hnsw_search_kernel<8>, dim3((unsigned)nq), dim3(HN_WAVES * ADS_WAVE), smem, s, a); break;
        case 16: hipLaunchKernelGGL(hnsw_search_kernel<16>, dim3((unsigned)nq), dim3(HN_WAVES * ADS_WAVE), smem, s, a); break;
        case 32: hipLaunchKernelGGL(hnsw_search_kernel<32>, dim3((unsigned)nq), dim3(HN_WAVES * ADS_WAVE), smem, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ads
