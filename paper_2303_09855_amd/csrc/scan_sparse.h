// The pair-list ("sparse") phase of the candidate scan.
//
// A list holds (vector of the current 64-vector tile, query of the unit)
// pairs that all stand at the same next block bcur, each with its partial
// squared distance S over blocks [0, bcur).  With n pairs left, each pair
// takes G = min(16, 64 / n) lanes (a power of two) that evaluate blocks
// bcur .. bcur+G-1 at once; an in-group scan gives S at every block boundary
// and the first deciding block is found with a ballot, so the decisions are
// those of testing block by block (Algorithm 1, one hypothesis test per
// Delta_d sampled coordinates).  Survivors advance by G blocks together and
// are compacted into the other list.
//
// Every block partial is computed in the canonical order (differences squared
// and summed from zero in coordinate order) and S is the sum of the partials
// in block order, so a pair's S at every block is bit-identical to the
// explicit-candidate DCO, whatever G is and whenever the pair entered a list.
//
// Decisions: reject iff S > coef(d) r^2 at d < D, positive iff S <= r^2 at
// d = D.
#pragma once
#include "kernels.h"

namespace ads {

// Orders this wave's LDS accesses (lanes of one wave run in lockstep).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Canonical block partial: s + sum_k (o_k - q_k)^2 over DD coordinates, fused
// multiply-adds in coordinate order.
template <int DT, int DD>
__device__ __forceinline__ float block_partial(const unsigned char *op, const float *qp, float s) {
#pragma unroll
    for (int k0 = 0; k0 < DD; k0 += 8) {
        float o[8];
        load_elems<DT, 8>(op + k0 * Elem<DT>::bytes, o);
        const float4 q0 = *reinterpret_cast<const float4 *>(qp + k0);
        const float4 q1 = *reinterpret_cast<const float4 *>(qp + k0 + 4);
        const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float df = o[k] - qv[k];
            s = __fmaf_rn(df, df, s);
        }
    }
    return s;
}

// x of the previous lane within each row of 16 lanes (DPP row_shr:1); the
// first lane of a row gets 0.
__device__ __forceinline__ float row_shr1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, true));
}

// List entry: S bits (high word) | query slot << 6 | vector of the tile.
__device__ __forceinline__ uint64_t pair_entry(float s, int jj, int vv) {
    return ((uint64_t)__float_as_uint(s) << 32) | (uint32_t)(jj << 6 | vv);
}

struct SparseCtx {
    const unsigned char *lbase;   // the list's blocked data
    int nl, vc;                   // list length, first vector of the tile
    const float *qrot;
    const int *qidx;              // [QW] query rows of the unit's slots (LDS)
    const float *r2s;             // [QW] thresholds (LDS)
    const float *coef;            // [nb] test coefficients (LDS)
    int D, nb, b1;
};

struct SparseOut {
    unsigned long long dims;      // this lane's sampled dimensions
    unsigned long long pos;       // this lane's positives
};

// Runs the pairs of list0[0..n) (all at block bcur) to their decisions, with
// list0 / list1 as ping-pong buffers.  A positive calls sink(jj, s, vv) on the
// pair's leader lane.
template <int DT, int DD, class Sink>
__device__ __forceinline__ SparseOut sparse_run(const SparseCtx &c, uint64_t *list0, uint64_t *list1, int n,
                                                int bcur, Sink sink) {
    uint32_t my_dims = 0, my_pos = 0;      // per lane and call: at most 64 pairs x D
    constexpr int EB = Elem<DT>::bytes;
    const int lane = threadIdx.x & 63;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    const int D = c.D, nb = c.nb;
    int cur = 0;
    while (n > 0 && bcur < nb) {
        wave_sync();
        // lanes per pair: a power of two up to 16, so that a group never
        // crosses a DPP row
        int G = 1;
        while (G < 16 && G * 2 * n <= 64 && G * 2 <= nb - bcur) G *= 2;
        const int ppr = 64 / G;                 // pairs per round
        const int gi = lane & (G - 1);
        const uint64_t *src = cur ? list1 : list0;
        uint64_t *dst = cur ? list0 : list1;
        int nout = 0;
        for (int r0p = 0; r0p < n; r0p += ppr) {
            const int pi = r0p + lane / G;
            const bool pv = pi < n;
            const uint64_t en = pv ? src[pi] : 0ull;
            const float s0 = __uint_as_float((uint32_t)(en >> 32));
            const int jj = (int)(((uint32_t)en >> 6) & 31u), vv = (int)(en & 63u);
            const int blk = bcur + gi;
            const bool bv = pv && blk < nb;
            float part = 0.f;
            if (bv) {
                const unsigned char *op = c.lbase + layout_offset(c.nl, c.vc + vv, blk, DD, c.b1, D) * EB;
                part = block_partial<DT, DD>(op, c.qrot + (int64_t)c.qidx[jj] * D + blk * DD, 0.f);
            }
            // S after each block, added in block order (the canonical order,
            // independent of G): after step t the first t + 1 lanes of every
            // group hold S_prev + p_0 + ... + p_gi, each lane adding its own
            // partial to its left neighbour's sum; the group's first lane keeps
            // s0 + p_0
            const bool g0 = gi == 0;
            float sb = g0 ? s0 + part : part;
#pragma unroll
            for (int t = 1; t < 16; ++t) {
                if (t >= G) break;
                const float y = row_shr1(sb) + part;
                sb = g0 ? sb : y;
            }
            const int d = (blk + 1) * DD;
            const float r2 = pv ? c.r2s[jj] : 0.f;
            const bool ev = bv && d < D && test_reject(sb, c.coef[bv ? blk : 0], r2);
            const uint64_t rm = __ballot(ev);
            const uint64_t gmask = ((1ull << G) - 1ull) << (lane & ~(G - 1));
            const uint64_t grm = rm & gmask;
            // the group's last block and the value of S there; the lane that
            // evaluated it decides for the group
            const int glast = min(G, nb - bcur) - 1;
            const float slast = sb;
            bool keep = false;
            if (pv && gi == glast) {
                if (grm) {
                    const int first = __ffsll((long long)grm) - 1;       // lane index of the event
                    my_dims += (uint32_t)(bcur + first - (lane & ~(G - 1)) + 1) * DD;
                } else if (bcur + glast + 1 >= nb) {
                    my_dims += D;
                    if (slast <= r2) {
                        sink(jj, slast, vv);
                        ++my_pos;
                    }
                } else {
                    keep = true;
                }
            }
            const uint64_t km = __ballot(keep);
            if (keep) {
                const int p = nout + __popcll(km & lanemask_lt);
                dst[p] = ((uint64_t)__float_as_uint(slast) << 32) | (uint32_t)(en & 0xffffffffu);
            }
            nout += __popcll(km);
        }
        n = nout;
        cur ^= 1;
        bcur += G;
    }
    return SparseOut{my_dims, my_pos};
}

}  // namespace ads
