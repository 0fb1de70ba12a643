// Launchers and kernels shared between the library's HIP sources.
#pragma once
#include "common.h"

namespace ads {

hipError_t gemm_nt_f32(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                       int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s);

struct ScanArgs {
    const void *data;
    const int64_t *list_off;
    const int32_t *ids;
    const float *qrot;
    const int32_t *keff;
    const float *r2_in;
    const int4 *units;      // this sweep's units, XCD-major: (list, first qent entry, queries, 0)
    const int32_t *xoff;    // [8] first unit of each XCD's range
    const int32_t *xcnt;    // [8] number of units of each XCD
    const int2 *qent;
    uint64_t *slots;
    unsigned long long *stats;
    double eps0;
    int method;
    int nprobe_max, kcap, D, nb;
    int b1;                 // blocks of the list-major region of the layout (layout_offset)
    float dense_frac;       // pairs alive at or below this fraction (<= 0.25) switch to the pair list
    int round_tiles;        // 64-vector tiles per threshold update (4 in the first sweeps, else 1)
};

hipError_t launch_scan(const ScanArgs &a, int dtype, int dd, int qw, int grid, bool prefetch, bool wide,
                       hipStream_t s);
// One (storage type, block width) slice of the scan instantiations, defined in
// scan_kernel.h and instantiated by scan_inst.hip (one object per slice).
template <int DT, int DD>
hipError_t launch_scan_q(const ScanArgs &a, int qw, int grid, bool pf, bool wide, hipStream_t s);

int num_sweeps(int nprobe_max, int lg);
int sweep_begin(int s, int lg);

// Inner-product mode of the explicit-candidate DCO (all NULL / 0 for L2).
struct IpArgs {
    const float *onorm;     // [n] raw norm of each base vector, by id
    const float *qnorm;     // device scalar: raw norm of the query
    float r_ip;             // inner-product threshold
};

hipError_t launch_dco(int dtype, const void *data, const float *rows32, int source,
                      const int64_t *list_off, const int32_t *list_of_pos, const int32_t *pos_of,
                      int64_t n, int D, int dd_layout, int b1, const float *q, const int64_t *cand,
                      int64_t m, float r2, double eps0, int step, int method, uint8_t *mask,
                      float *dist, int32_t *dims, unsigned long long *stats, const IpArgs *ip,
                      hipStream_t s);

hipError_t launch_normalize(const float *x, int64_t n, int D, float *out, float *norms, hipStream_t s);

hipError_t launch_pack(int dtype, const float *rot, const int32_t *ids, const int32_t *list_of_pos,
                       const int64_t *list_off, int64_t n, int D, int dd, int b1, void *data,
                       float *rows32, hipStream_t s);

hipError_t launch_row_norms(const float *x, int64_t n, int D, float *out, hipStream_t s);

// k-means (kmeans.hip)
hipError_t launch_gather_rows(const float *x, int D, const int32_t *rows, int m, float *out, hipStream_t s);
hipError_t launch_argmin(const float *dots, const float *xn, const float *cn, int64_t m, int nlist,
                         int32_t *assign, float *d2, hipStream_t s);
hipError_t launch_counts(const int32_t *assign, int64_t n, int nlist, int32_t *counts, hipStream_t s);
hipError_t launch_farthest(const int32_t *assign, const float *d2, int64_t n, int l, unsigned long long *best,
                           hipStream_t s);
hipError_t launch_update_centres(const float *x, int64_t n, int D, const int32_t *assign, int nlist, float *cent,
                                 hipStream_t s);

// Graph search (hnsw.hip)
constexpr int HN_MAXDEG = 32;       // largest neighbour row (M0 on layer 0, M above)
constexpr int HN_MAXBLOCKS = 128;   // largest D / delta_d
struct HnswArgs {
    const float *data;       // [n][D] transformed vectors, row-major
    const int32_t *adj0;     // [n][M0] layer-0 neighbours, -1 padded
    const int64_t *up_off;   // [n] first upper row of each vertex (-1 on layer 0 only)
    const int32_t *up_adj;   // [rows][M] upper-layer neighbours, -1 padded
    const float *qrot;       // [nq][D] transformed queries
    const float *coef;       // [nb] test coefficients (1 for the last block)
    uint32_t *visited;       // [nq][vis_words] bitmaps, zeroed before the launch
    int64_t vis_words;
    int64_t *ids;            // [nq][K]
    float *dist;             // [nq][K]
    int64_t *qstats;         // [nq][3] DCOs, sampled dims, expansions (or NULL)
    unsigned long long *stats;  // [3] accumulators (or NULL)
    int D, nb, dd, M0, M, entry, max_level, K, nef, variant;
};
size_t hnsw_smem_bytes(int D, int nb, int nef, int K);
hipError_t launch_hnsw_setup(float *coef, int nb, int dd, int D, double eps0, int method,
                             uint32_t *visited, int64_t words, hipStream_t s);
hipError_t launch_hnsw_search(const HnswArgs &a, int nq, hipStream_t s);

}  // namespace ads
