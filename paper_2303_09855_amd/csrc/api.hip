// Host side of the C ABI declared in include/ads.h: argument validation,
// index construction, workspace layout and the launch sequence of a search.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace ads {
__global__ void setup_kernel(const int32_t *K, const int32_t *nprobe, int nq, int k_max,
                             int nprobe_max, int kfactor, int kcap, int32_t *kq, int32_t *keff,
                             int32_t *npq, float *r2, uint64_t *tk);
__global__ void zero_i32_kernel(int32_t *p, int64_t n);
size_t probe_select_smem(int nlist, int nprobe_max);
__global__ void probe_select_kernel(const float *qrot, const float *dots, const float *cnorm, int D,
                                    int nlist, int nprobe_max, int32_t *probes);
__global__ void group_count_kernel(const int32_t *probes, const int32_t *npq, const int32_t *keff,
                                   int nq, int nprobe_max, int nlist, int lg, int32_t *cnt);
__global__ void list_order_kernel(const int32_t *cnt, const int64_t *list_off, int nlist, int32_t *order,
                                  int32_t *xb);
__global__ void group_scan_kernel(const int32_t *cnt, const int32_t *order, const int32_t *xb, int nsweep,
                                  int nlist, int qw, int32_t *beg, int32_t *uoff, int32_t *xoff, int32_t *xcnt);
__global__ void unit_expand_kernel(const int32_t *cnt, const int32_t *beg, const int32_t *uoff, int nsweep,
                                   int nlist, int qw, int64_t ucap, int4 *units);
__global__ void group_scatter_kernel(const int32_t *probes, const int32_t *npq, const int32_t *keff,
                                     int nq, int nprobe_max, int nlist, int lg, const int32_t *beg,
                                     int32_t *cursor, int2 *qent);
__global__ void merge_kernel(const uint64_t *slots, const int32_t *keff, const int32_t *npq,
                             int nprobe_max, int kcap, int rank_a, int rank_b, uint64_t *tk,
                             float *r2);
__global__ void output_kernel(const uint64_t *tk, const int32_t *kq, int nq, int k_max, int kcap,
                              int64_t *ids, float *dist);
__global__ void rerank_kernel(const uint64_t *tk, const int32_t *kq, const int32_t *keff,
                              const float *rows32, const int32_t *pos_of, const float *qrot, int D,
                              int dd, int kcap, int k_max, int64_t *ids, float *dist);
__global__ void probes_out_kernel(const int32_t *probes, const int32_t *npq, int nq, int nprobe_max,
                                  int32_t *out);
}  // namespace ads

using namespace ads;

struct ads_index {
    int64_t n = 0;
    int D = 0, nlist = 0, dd = 0, nb = 0, storage = 0, keep_fp32 = 0, max_list = 0, metric = 0;
    int b1 = 0;                  // blocks of the list-major region of the layout (layout_offset)
    float *norms = nullptr;      // [n] raw norms by id (cosine indexes)
    float *P = nullptr;          // [D][D]; NULL for an index of unrotated vectors
    float *cent_rot = nullptr;   // [nlist][D]
    float *cent_norm = nullptr;  // [nlist]
    int64_t *list_off = nullptr; // [nlist + 1]
    int32_t *ids = nullptr;      // [n] stored position -> id
    int32_t *pos_of = nullptr;   // [n] id -> stored position
    int32_t *list_of_pos = nullptr;  // [n]
    void *data = nullptr;        // blocked layout
    float *rows32 = nullptr;     // [n][D] float32 rows in stored order (optional)
    int64_t bytes = 0;
};

namespace {

thread_local std::string g_err;
thread_local ads_tuning g_tune = {0.f, 0, 4, 0, 0};

// Per-thread event profiler (ads_profile_enable / ads_profile_collect).
struct Profiler {
    bool on = false;
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Profiler() {
        for (auto &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
thread_local Profiler g_prof;

// Brackets one phase's launches with events when profiling is on.
struct PhaseTimer {
    hipStream_t s;
    int phase;
    hipEvent_t a = nullptr;
    PhaseTimer(int ph, hipStream_t st) : s(st), phase(ph) {
        if (!g_prof.on) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        if ((a = g_prof.get())) (void)hipEventRecord(a, s);
    }
    ~PhaseTimer() {
        if (!a) return;
        hipEvent_t b = g_prof.get();
        if (!b) { g_prof.pool.push_back(a); return; }
        (void)hipEventRecord(b, s);
        g_prof.recs.push_back({phase, a, b});
    }
};

ads_status fail(ads_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ads_status fail(ads_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

ads_status hip_fail(hipError_t e, const char *what) {
    return fail(ADS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int elem_bytes(int dt) { return dt == ADS_F32 ? 4 : 2; }

bool valid_dd(int dd) { return dd == 8 || dd == 16 || dd == 32 || dd == 64; }

void free_index(ads_index *ix) {
    if (!ix) return;
    void *ptrs[] = {ix->P, ix->cent_rot, ix->cent_norm, ix->list_off, ix->ids, ix->pos_of,
                    ix->list_of_pos, ix->data, ix->rows32, ix->norms};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete ix;
}

template <class T>
hipError_t dmalloc(T **p, size_t count, int64_t *acc) {
    *p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes);
    if (e == hipSuccess && acc) *acc += (int64_t)bytes;
    return e;
}

unsigned grid_for(int64_t n, int64_t cap = 65536) {
    int64_t g = (n + ADS_WG - 1) / ADS_WG;
    if (g < 1) g = 1;
    return (unsigned)(g > cap ? cap : g);
}

// Queries per scan unit for a KNN-set capacity (local KNN sets <= 4 KB of LDS),
// or the tuned value when it fits.
int qw_for(int kcap) {
    int auto_qw = 1;
    for (int qw = 8; qw > 1; qw >>= 1)
        if (qw * kcap <= 512) { auto_qw = qw; break; }
    const int t = g_tune.queries_per_unit;
    if (t > 0 && t * kcap <= 4096) return t;
    return auto_qw;
}

constexpr int KCAP_MAX = KCAP_LIMIT;
// Coordinates of every vector stored in the list-major region of the layout
// (IVF++'s array A1): the dense phase of the scan reads these a tile at a
// time; the rest is stored vector by vector for the pair-list phase.
#ifndef ADS_A1_DIMS
#define ADS_A1_DIMS 128
#endif
constexpr int A1_DIMS = ADS_A1_DIMS;
// Default of the prefetch_units knob: sweeps with fewer work units than this
// run the prefetching scan instantiation.
constexpr int64_t PREFETCH_UNITS = 8192;
// The first sweeps update thresholds once per round of four tiles (the
// register scan runs them with four waves per unit): more parallel work in
// the sweeps that have few units.
#ifndef ADS_WIDE_SWEEPS
#define ADS_WIDE_SWEEPS 2
#endif
constexpr int WIDE_SWEEPS = ADS_WIDE_SWEEPS;
// probe selection sorts the nprobe_max nearest centre keys in LDS (32 KB at 4096)
constexpr int NPROBE_MAX_LIMIT = 4096;

struct SearchLayout {
    size_t off_qrot, off_qunit, off_order, off_xb, off_dots, off_probes, off_kq, off_keff, off_npq, off_r2, off_tk, off_cnt,
        off_beg, off_cursor, off_uoff, off_xoff, off_xcnt, off_units, off_qent, off_slots, total;
    int nsweep, kcap, qw, lg;
    int64_t ucap;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

SearchLayout layout_for(const ads_index *ix, int nq, int k_max, int nprobe_max, int rerank) {
    SearchLayout L{};
    L.kcap = k_max * (rerank ? 4 : 1);
    L.qw = qw_for(L.kcap);
    L.lg = g_tune.sweep_log2;
    L.nsweep = num_sweeps(nprobe_max, L.lg);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + (bytes ? bytes : 1)); return at; };
    const size_t nqs = (size_t)(nq > 0 ? nq : 1);
    L.off_qrot = take(nqs * ix->D * sizeof(float));
    L.off_qunit = take(ix->metric == ADS_METRIC_COSINE ? nqs * ix->D * sizeof(float) : 0);
    L.off_dots = take(nqs * ix->nlist * sizeof(float));
    L.off_probes = take(nqs * nprobe_max * sizeof(int32_t));
    L.off_kq = take(nqs * sizeof(int32_t));
    L.off_keff = take(nqs * sizeof(int32_t));
    L.off_npq = take(nqs * sizeof(int32_t));
    L.off_r2 = take(nqs * sizeof(float));
    L.off_tk = take(nqs * L.kcap * sizeof(uint64_t));
    const size_t sl = (size_t)L.nsweep * ix->nlist;
    L.off_cnt = take(sl * sizeof(int32_t));
    L.off_cursor = take(sl * sizeof(int32_t));
    L.off_beg = take(sl * sizeof(int32_t));
    L.off_uoff = take(sl * sizeof(int32_t));
    L.off_order = take(sl * sizeof(int32_t));
    L.off_xb = take((size_t)L.nsweep * 9 * sizeof(int32_t));
    L.off_xoff = take((size_t)L.nsweep * 8 * sizeof(int32_t));
    L.off_xcnt = take((size_t)L.nsweep * 8 * sizeof(int32_t));
    L.ucap = ((int64_t)nqs * nprobe_max + L.qw - 1) / L.qw + ix->nlist;
    L.off_units = take((size_t)L.nsweep * L.ucap * sizeof(int4));
    L.off_qent = take(nqs * nprobe_max * sizeof(int2));
    L.off_slots = take(nqs * nprobe_max * (size_t)L.kcap * sizeof(uint64_t));
    L.total = o;
    return L;
}

ads_status check_search_args(const ads_index *ix, int32_t nq, int32_t k_max, int32_t nprobe_max,
                             int32_t rerank) {
    if (!ix) return fail(ADS_EINVAL, "index is NULL");
    if (nq < 0) return fail(ADS_EINVAL, "nq must be >= 0 (got %d)", nq);
    if (k_max < 1) return fail(ADS_EINVAL, "k_max must be >= 1 (got %d)", k_max);
    if (nprobe_max < 1 || nprobe_max > ix->nlist)
        return fail(ADS_EINVAL, "nprobe_max must be in [1, nlist=%d] (got %d)", ix->nlist, nprobe_max);
    if (nprobe_max > NPROBE_MAX_LIMIT)
        return fail(ADS_EUNSUPPORTED, "nprobe_max above %d is not supported", NPROBE_MAX_LIMIT);
    if (rerank != 0 && rerank != 1) return fail(ADS_EINVAL, "rerank must be 0 or 1");
    if (rerank && !ix->rows32)
        return fail(ADS_EINVAL, "rerank needs an index built with keep_fp32 = 1");
    const int kcap = k_max * (rerank ? 4 : 1);
    if (kcap > KCAP_MAX)
        return fail(ADS_EUNSUPPORTED, "k_max%s above %d is not supported", rerank ? " * 4" : "", KCAP_MAX);
    if ((int64_t)nq * nprobe_max >= (int64_t)1 << 31)
        return fail(ADS_EUNSUPPORTED, "nq * nprobe_max must be below 2^31");
    return ADS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Rotation
// ---------------------------------------------------------------------------

extern "C" ads_status ads_make_rotation(const double *gaussian, int32_t D, float *P_out, double *P64_out) {
    if (!gaussian || !P_out) return fail(ADS_EINVAL, "gaussian and P_out must not be NULL");
    if (D < 1) return fail(ADS_EINVAL, "D must be >= 1 (got %d)", D);
    const size_t N = (size_t)D;
    std::vector<double> a, v, rdiag, q;
    try {
        a.resize(N * N);
        v.resize(N * N);
        rdiag.resize(N);
        q.assign(N * N, 0.0);
    } catch (...) {
        return fail(ADS_ENOMEM, "host allocation failed");
    }
    // column-major working copy: a[j*D + i] = G[i][j]
    for (size_t i = 0; i < N; ++i)
        for (size_t j = 0; j < N; ++j) a[j * N + i] = gaussian[i * N + j];
    // Householder QR: H_k zeroes column k below the diagonal.
    for (size_t k = 0; k < N; ++k) {
        double *col = &a[k * N];
        double nrm = 0.0;
        for (size_t i = k; i < N; ++i) nrm += col[i] * col[i];
        nrm = std::sqrt(nrm);
        double *vk = &v[k * N];
        for (size_t i = 0; i < N; ++i) vk[i] = 0.0;
        if (nrm == 0.0) {
            rdiag[k] = 0.0;
            continue;
        }
        const double alpha = col[k] >= 0.0 ? -nrm : nrm;
        for (size_t i = k; i < N; ++i) vk[i] = col[i];
        vk[k] -= alpha;
        double vn = 0.0;
        for (size_t i = k; i < N; ++i) vn += vk[i] * vk[i];
        vn = std::sqrt(vn);
        if (vn == 0.0) {
            rdiag[k] = col[k];
            continue;
        }
        for (size_t i = k; i < N; ++i) vk[i] /= vn;
        for (size_t j = k; j < N; ++j) {
            double *cj = &a[j * N];
            double dot = 0.0;
            for (size_t i = k; i < N; ++i) dot += vk[i] * cj[i];
            dot *= 2.0;
            for (size_t i = k; i < N; ++i) cj[i] -= dot * vk[i];
        }
        rdiag[k] = a[k * N + k];
    }
    // Q = H_0 H_1 ... H_{D-1} applied to the identity (column-major q).
    for (size_t j = 0; j < N; ++j) q[j * N + j] = 1.0;
    for (size_t kk = N; kk-- > 0;) {
        const double *vk = &v[kk * N];
        for (size_t j = 0; j < N; ++j) {
            double *qj = &q[j * N];
            double dot = 0.0;
            for (size_t i = kk; i < N; ++i) dot += vk[i] * qj[i];
            if (dot == 0.0) continue;
            dot *= 2.0;
            for (size_t i = kk; i < N; ++i) qj[i] -= dot * vk[i];
        }
    }
    // Haar sign fix: Q <- Q diag(sign(diag R)).
    for (size_t j = 0; j < N; ++j) {
        const double sgn = rdiag[j] < 0.0 ? -1.0 : 1.0;
        for (size_t i = 0; i < N; ++i) {
            const double val = sgn * q[j * N + i];
            P_out[i * N + j] = (float)val;
            if (P64_out) P64_out[i * N + j] = val;
        }
    }
    return ADS_OK;
}

extern "C" ads_status ads_rotate(const float *P, int32_t D, const float *X, int64_t n, float *Y,
                                 hipStream_t stream) {
    if (n < 0) return fail(ADS_EINVAL, "n must be >= 0");
    if (n == 0) return ADS_OK;
    if (!P || !X || !Y) return fail(ADS_EINVAL, "P, X and Y must not be NULL");
    if (D < 1 || D % 4 != 0) return fail(ADS_EINVAL, "D must be a positive multiple of 4 (got %d)", D);
    if (X == Y) return fail(ADS_EINVAL, "X and Y must not alias");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    HIP_TRY(gemm_nt_f32(X, D, P, D, Y, D, n, D, D, stream), "rotate");
    return ADS_OK;
}

// ---------------------------------------------------------------------------
// Index
// ---------------------------------------------------------------------------

extern "C" ads_status ads_ivf_build(const float *base, int64_t n, int32_t D, const float *P,
                                    const float *centroids, int32_t nlist, const int32_t *assign,
                                    int32_t delta_d, int32_t storage, int32_t keep_fp32, int32_t metric,
                                    hipStream_t stream, ads_index **out) {
    if (!out) return fail(ADS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!base || !centroids || !assign)
        return fail(ADS_EINVAL, "base, centroids and assign must not be NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(ADS_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (D < 1 || D % 4 != 0) return fail(ADS_EINVAL, "D must be a positive multiple of 4 (got %d)", D);
    if (nlist < 1) return fail(ADS_EINVAL, "nlist must be >= 1 (got %d)", nlist);
    if (storage != ADS_F32 && storage != ADS_BF16 && storage != ADS_F16)
        return fail(ADS_EINVAL, "unknown storage type %d", storage);
    if (!valid_dd(delta_d))
        return fail(ADS_EUNSUPPORTED, "delta_d must be one of 8, 16, 32, 64 (got %d)", delta_d);
    if (D % delta_d != 0) return fail(ADS_EINVAL, "delta_d=%d must divide D=%d", delta_d, D);
    if (storage != ADS_F32 && D % 8 != 0) return fail(ADS_EINVAL, "16-bit storage needs D %% 8 == 0");
    if (keep_fp32 != 0 && keep_fp32 != 1) return fail(ADS_EINVAL, "keep_fp32 must be 0 or 1");
    if (metric != ADS_METRIC_L2 && metric != ADS_METRIC_COSINE) return fail(ADS_EINVAL, "unknown metric %d", metric);
    HIP_TRY(hipGetLastError(), "pending HIP error");

    std::vector<int32_t> h_assign;
    try {
        h_assign.resize((size_t)n);
    } catch (...) {
        return fail(ADS_ENOMEM, "host allocation failed");
    }
    HIP_TRY(hipMemcpyAsync(h_assign.data(), assign, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream),
            "copy assign");
    HIP_TRY(hipStreamSynchronize(stream), "synchronize");
    std::vector<int64_t> off((size_t)nlist + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        int32_t l = h_assign[(size_t)i];
        if (l < 0 || l >= nlist) return fail(ADS_EINVAL, "assign[%lld] = %d is outside [0, %d)", (long long)i, l, nlist);
        off[(size_t)l + 1]++;
    }
    int max_list = 0;
    for (int l = 0; l < nlist; ++l) {
        if (off[(size_t)l + 1] > max_list) max_list = (int)off[(size_t)l + 1];
        off[(size_t)l + 1] += off[(size_t)l];
    }
    // stable counting sort: ascending id inside every list
    std::vector<int32_t> ids((size_t)n), pos_of((size_t)n), lop((size_t)n);
    {
        std::vector<int64_t> cur(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            int32_t l = h_assign[(size_t)i];
            int64_t p = cur[(size_t)l]++;
            ids[(size_t)p] = (int32_t)i;
            pos_of[(size_t)i] = (int32_t)p;
            lop[(size_t)p] = l;
        }
    }

    ads_index *ix = new (std::nothrow) ads_index();
    if (!ix) return fail(ADS_ENOMEM, "host allocation failed");
    ix->n = n;
    ix->D = D;
    ix->nlist = nlist;
    ix->dd = delta_d;
    ix->nb = D / delta_d;
    // the list-major region (A1) holds the first A1_DIMS coordinates
    ix->b1 = A1_DIMS / delta_d < 1 ? 1 : A1_DIMS / delta_d;
    if (ix->b1 > ix->nb) ix->b1 = ix->nb;
    ix->storage = storage;
    ix->keep_fp32 = keep_fp32;
    ix->max_list = max_list;
    ix->metric = metric;
    float *rot = nullptr, *unit = nullptr;
    hipError_t e = hipSuccess;
#define BUILD_TRY(expr, what)          \
    do {                               \
        e = (expr);                    \
        if (e != hipSuccess) {         \
            ads_status st = hip_fail(e, what); \
            if (rot) (void)hipFree(rot); \
            if (unit) (void)hipFree(unit); \
            (void)hipStreamSynchronize(stream); \
            free_index(ix);            \
            if (e == hipErrorOutOfMemory) st = fail(ADS_ENOMEM, "%s: out of device memory", what); \
            return st;                 \
        }                              \
    } while (0)
    if (P) BUILD_TRY(dmalloc(&ix->P, (size_t)D * D, &ix->bytes), "alloc P");
    BUILD_TRY(dmalloc(&ix->cent_rot, (size_t)nlist * D, &ix->bytes), "alloc centroids");
    BUILD_TRY(dmalloc(&ix->cent_norm, (size_t)nlist, &ix->bytes), "alloc centroid norms");
    BUILD_TRY(dmalloc(&ix->list_off, (size_t)nlist + 1, &ix->bytes), "alloc offsets");
    BUILD_TRY(dmalloc(&ix->ids, (size_t)n, &ix->bytes), "alloc ids");
    BUILD_TRY(dmalloc(&ix->pos_of, (size_t)n, &ix->bytes), "alloc positions");
    BUILD_TRY(dmalloc(&ix->list_of_pos, (size_t)n, &ix->bytes), "alloc list of position");
    {
        const size_t data_bytes = (size_t)n * D * elem_bytes(storage);
        e = hipMalloc(&ix->data, data_bytes);
        if (e == hipSuccess) ix->bytes += (int64_t)data_bytes;
        BUILD_TRY(e, "alloc blocked layout");
    }
    if (keep_fp32) BUILD_TRY(dmalloc(&ix->rows32, (size_t)n * D, &ix->bytes), "alloc float32 rows");
    if (P) BUILD_TRY(hipMalloc(&rot, sizeof(float) * (size_t)n * D), "alloc rotation scratch");
    if (metric == ADS_METRIC_COSINE) {
        BUILD_TRY(dmalloc(&ix->norms, (size_t)n, &ix->bytes), "alloc norms");
        const size_t rows = (size_t)(n > nlist ? n : nlist);
        BUILD_TRY(hipMalloc(&unit, sizeof(float) * rows * D), "alloc normalisation scratch");
    }

    if (P) BUILD_TRY(hipMemcpyAsync(ix->P, P, sizeof(float) * D * D, hipMemcpyDeviceToDevice, stream), "copy P");
    BUILD_TRY(hipMemcpyAsync(ix->list_off, off.data(), sizeof(int64_t) * (nlist + 1), hipMemcpyHostToDevice, stream), "upload offsets");
    BUILD_TRY(hipMemcpyAsync(ix->ids, ids.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream), "upload ids");
    BUILD_TRY(hipMemcpyAsync(ix->pos_of, pos_of.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream), "upload positions");
    BUILD_TRY(hipMemcpyAsync(ix->list_of_pos, lop.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream), "upload list ids");
    // rotate every base vector (index phase, Section 6.1) and pack the lists
    const float *src = base;
    if (metric == ADS_METRIC_COSINE) {
        BUILD_TRY(launch_normalize(base, n, D, unit, ix->norms, stream), "normalise base");
        src = unit;
    }
    // without P the index stores the vectors as given (IVF* / IVF**, Section 6.1)
    if (P) BUILD_TRY(gemm_nt_f32(src, D, ix->P, D, rot, D, n, D, D, stream), "rotate base");
    BUILD_TRY(launch_pack(storage, P ? rot : src, ix->ids, ix->list_of_pos, ix->list_off, n, D, delta_d, ix->b1, ix->data,
                          ix->rows32, stream), "pack lists");
    const float *csrc = centroids;
    if (metric == ADS_METRIC_COSINE) {
        BUILD_TRY(hipStreamSynchronize(stream), "synchronize");   // unit is reused below
        BUILD_TRY(launch_normalize(centroids, nlist, D, unit, nullptr, stream), "normalise centroids");
        csrc = unit;
    }
    if (P)
        BUILD_TRY(gemm_nt_f32(csrc, D, ix->P, D, ix->cent_rot, D, nlist, D, D, stream), "rotate centroids");
    else
        BUILD_TRY(hipMemcpyAsync(ix->cent_rot, csrc, sizeof(float) * (size_t)nlist * D, hipMemcpyDeviceToDevice,
                                 stream), "copy centroids");
    BUILD_TRY(launch_row_norms(ix->cent_rot, nlist, D, ix->cent_norm, stream), "centroid norms");
    BUILD_TRY(hipStreamSynchronize(stream), "synchronize build");
    (void)hipFree(rot);
    rot = nullptr;
    if (unit) (void)hipFree(unit);
    unit = nullptr;
#undef BUILD_TRY
    *out = ix;
    return ADS_OK;
}

// ---------------------------------------------------------------------------
// k-means clustering of the index phase (Section 2.2.2)
// ---------------------------------------------------------------------------

namespace {

uint64_t splitmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Rows that seed the lists: the nlist rows whose SplitMix64 draws (counter
// seed + (i + 1) * golden gamma) are smallest, in ascending draw order.
std::vector<int32_t> kmeans_init_rows(int64_t n, int nlist, uint64_t seed) {
    std::vector<std::pair<uint64_t, int32_t>> k((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        k[(size_t)i] = {splitmix64(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull), (int32_t)i};
    std::partial_sort(k.begin(), k.begin() + nlist, k.end());
    std::vector<int32_t> rows((size_t)nlist);
    for (int j = 0; j < nlist; ++j) rows[(size_t)j] = k[(size_t)j].second;
    return rows;
}

}  // namespace

extern "C" ads_status ads_kmeans(const float *x, int64_t n, int32_t D, int32_t nlist, int32_t iters, uint64_t seed,
                                 float *centroids, int32_t *assign, hipStream_t stream) {
    if (!x || !centroids || !assign) return fail(ADS_EINVAL, "x, centroids and assign must not be NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(ADS_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (D < 1 || D > 4096) return fail(ADS_EINVAL, "D must be in [1, 4096] (got %d)", D);
    if (nlist < 1 || nlist > n) return fail(ADS_EINVAL, "nlist must be in [1, n] (got %d)", nlist);
    if (iters < 0) return fail(ADS_EINVAL, "iters must be >= 0 (got %d)", iters);
    HIP_TRY(hipGetLastError(), "pending HIP error");
    std::vector<int32_t> init;
    try {
        init = kmeans_init_rows(n, nlist, seed);
    } catch (...) {
        return fail(ADS_ENOMEM, "host allocation failed");
    }
    // chunk of rows whose centre products fit in 256 MB
    int64_t chunk = ((int64_t)64 << 20) / nlist;
    if (chunk < 1) chunk = 1;
    if (chunk > n) chunk = n;
    int32_t *rows = nullptr, *counts = nullptr;
    float *xn = nullptr, *cn = nullptr, *dots = nullptr, *d2 = nullptr;
    unsigned long long *best = nullptr;
    hipError_t e = hipSuccess;
    auto release = [&]() {
        void *ptrs[] = {rows, counts, xn, cn, dots, d2, best};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    };
#define KM_TRY(expr, what)                              \
    do {                                                \
        e = (expr);                                     \
        if (e != hipSuccess) {                          \
            (void)hipStreamSynchronize(stream);         \
            release();                                  \
            return e == hipErrorOutOfMemory ? fail(ADS_ENOMEM, "%s: out of device memory", what) \
                                            : hip_fail(e, what); \
        }                                               \
    } while (0)
    KM_TRY(hipMalloc(&rows, sizeof(int32_t) * nlist), "alloc init rows");
    KM_TRY(hipMalloc(&counts, sizeof(int32_t) * nlist), "alloc counts");
    KM_TRY(hipMalloc(&xn, sizeof(float) * n), "alloc row norms");
    KM_TRY(hipMalloc(&cn, sizeof(float) * nlist), "alloc centre norms");
    KM_TRY(hipMalloc(&dots, sizeof(float) * (size_t)chunk * nlist), "alloc centre products");
    KM_TRY(hipMalloc(&d2, sizeof(float) * n), "alloc distances");
    KM_TRY(hipMalloc(&best, sizeof(unsigned long long)), "alloc farthest key");
    KM_TRY(hipMemcpyAsync(rows, init.data(), sizeof(int32_t) * nlist, hipMemcpyHostToDevice, stream), "upload rows");
    KM_TRY(launch_gather_rows(x, D, rows, nlist, centroids, stream), "initial centres");
    KM_TRY(launch_row_norms(x, n, D, xn, stream), "row norms");
    std::vector<int32_t> hc((size_t)nlist);
    for (int it = 0; it <= iters; ++it) {
        // assignment to the nearest centre (ties to the lower id)
        KM_TRY(launch_row_norms(centroids, nlist, D, cn, stream), "centre norms");
        for (int64_t r0 = 0; r0 < n; r0 += chunk) {
            const int64_t m = n - r0 < chunk ? n - r0 : chunk;
            KM_TRY(gemm_nt_f32(x + r0 * D, D, centroids, D, dots, nlist, m, nlist, D, stream), "centre products");
            KM_TRY(launch_argmin(dots, xn + r0, cn, m, nlist, assign + r0, d2 + r0, stream), "nearest centre");
        }
        if (it == iters) break;     // the final assignment gives the lists
        // empty lists, in ascending id order, take the farthest member of the
        // largest list (lower id, then lower row on ties)
        KM_TRY(launch_counts(assign, n, nlist, counts, stream), "list sizes");
        KM_TRY(hipMemcpyAsync(hc.data(), counts, sizeof(int32_t) * nlist, hipMemcpyDeviceToHost, stream), "sizes");
        KM_TRY(hipStreamSynchronize(stream), "synchronize");
        for (int j = 0; j < nlist; ++j) {
            if (hc[(size_t)j] > 0) continue;
            int big = 0;
            for (int l = 1; l < nlist; ++l)
                if (hc[(size_t)l] > hc[(size_t)big]) big = l;
            if (hc[(size_t)big] < 2) break;     // nothing to move
            unsigned long long key = 0;
            KM_TRY(launch_farthest(assign, d2, n, big, best, stream), "farthest member");
            KM_TRY(hipMemcpyAsync(&key, best, sizeof key, hipMemcpyDeviceToHost, stream), "farthest key");
            KM_TRY(hipStreamSynchronize(stream), "synchronize");
            const int32_t row = (int32_t)(0xffffffffu - (uint32_t)(key & 0xffffffffu));
            KM_TRY(hipMemcpy(assign + row, &j, sizeof(int32_t), hipMemcpyHostToDevice), "move row");
            hc[(size_t)big] -= 1;
            hc[(size_t)j] = 1;
        }
        // every centre moves to the mean of its members
        KM_TRY(launch_update_centres(x, n, D, assign, nlist, centroids, stream), "centre update");
    }
    KM_TRY(hipStreamSynchronize(stream), "synchronize k-means");
#undef KM_TRY
    release();
    return ADS_OK;
}

extern "C" ads_status ads_build_ivf(const float *base, int64_t n, int32_t D, const float *P, int32_t nlist,
                                    int32_t iters, uint64_t seed, int32_t delta_d, int32_t storage,
                                    int32_t keep_fp32, int32_t metric, float *centroids_out, int32_t *assign_out,
                                    hipStream_t stream, ads_index **out) {
    if (!out) return fail(ADS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!base) return fail(ADS_EINVAL, "base must not be NULL");
    if (metric != ADS_METRIC_L2 && metric != ADS_METRIC_COSINE) return fail(ADS_EINVAL, "unknown metric %d", metric);
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(ADS_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (nlist < 1 || nlist > n) return fail(ADS_EINVAL, "nlist must be in [1, n] (got %d)", nlist);
    if (D < 1 || D > 4096 || D % 4 != 0) return fail(ADS_EINVAL, "D must be a multiple of 4 in [4, 4096] (got %d)", D);
    if (storage != ADS_F32 && storage != ADS_BF16 && storage != ADS_F16)
        return fail(ADS_EINVAL, "unknown storage type %d", storage);
    if (!valid_dd(delta_d)) return fail(ADS_EUNSUPPORTED, "delta_d must be one of 8, 16, 32, 64 (got %d)", delta_d);
    if (D % delta_d != 0) return fail(ADS_EINVAL, "delta_d=%d must divide D=%d", delta_d, D);
    if (iters < 0) return fail(ADS_EINVAL, "iters must be >= 0 (got %d)", iters);
    float *cent = centroids_out, *unit = nullptr;
    int32_t *asg = assign_out;
    bool own_c = false, own_a = false;
    auto release = [&]() {
        if (own_c && cent) (void)hipFree(cent);
        if (own_a && asg) (void)hipFree(asg);
        if (unit) (void)hipFree(unit);
    };
    hipError_t e = hipSuccess;
    if (!cent) {
        e = hipMalloc(&cent, sizeof(float) * (size_t)nlist * D);
        own_c = true;
    }
    if (e == hipSuccess && !asg) {
        e = hipMalloc(&asg, sizeof(int32_t) * (size_t)n);
        own_a = true;
    }
    // cosine: the lists are k-means clusters of the normalised vectors
    const float *kx = base;
    if (e == hipSuccess && metric == ADS_METRIC_COSINE) {
        e = hipMalloc(&unit, sizeof(float) * (size_t)n * D);
        if (e == hipSuccess) e = launch_normalize(base, n, D, unit, nullptr, stream);
        kx = unit;
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        release();
        return e == hipErrorOutOfMemory ? fail(ADS_ENOMEM, "k-means buffers: out of device memory")
                                        : hip_fail(e, "k-means buffers");
    }
    ads_status st = ads_kmeans(kx, n, D, nlist, iters, seed, cent, asg, stream);
    if (st == ADS_OK)
        st = ads_ivf_build(base, n, D, P, cent, nlist, asg, delta_d, storage, keep_fp32, metric, stream, out);
    (void)hipStreamSynchronize(stream);
    release();
    return st;
}

extern "C" ads_status ads_index_info(const ads_index *ix, ads_index_desc *info) {
    if (!ix || !info) return fail(ADS_EINVAL, "index and info must not be NULL");
    info->n = ix->n;
    info->D = ix->D;
    info->nlist = ix->nlist;
    info->delta_d = ix->dd;
    info->storage = ix->storage;
    info->has_fp32_copy = ix->rows32 != nullptr;
    info->rotated = ix->P != nullptr;
    info->a1_dims = ix->b1 * ix->dd;
    info->max_list = ix->max_list;
    info->metric = ix->metric;
    info->device_bytes = ix->bytes;
    return ADS_OK;
}

namespace {
__global__ void ids_to_i64_kernel(const int32_t *in, int64_t n, int64_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}
}  // namespace

extern "C" ads_status ads_index_lists(const ads_index *ix, int64_t *offsets, int64_t *ids,
                                      float *rot_centroids, hipStream_t stream) {
    if (!ix) return fail(ADS_EINVAL, "index is NULL");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    if (offsets)
        HIP_TRY(hipMemcpyAsync(offsets, ix->list_off, sizeof(int64_t) * (ix->nlist + 1), hipMemcpyDeviceToDevice, stream),
                "copy offsets");
    if (ids) {
        hipLaunchKernelGGL(ids_to_i64_kernel, dim3(grid_for(ix->n)), dim3(ADS_WG), 0, stream, ix->ids, ix->n, ids);
        HIP_TRY(hipGetLastError(), "copy ids");
    }
    if (rot_centroids)
        HIP_TRY(hipMemcpyAsync(rot_centroids, ix->cent_rot, sizeof(float) * ix->nlist * ix->D, hipMemcpyDeviceToDevice, stream),
                "copy centroids");
    return ADS_OK;
}

extern "C" ads_status ads_index_free(ads_index *ix) {
    if (!ix) return ADS_OK;
    (void)hipDeviceSynchronize();
    free_index(ix);
    return ADS_OK;
}

// ---------------------------------------------------------------------------
// Query phase
// ---------------------------------------------------------------------------

extern "C" ads_status ads_dco_batch(const ads_index *ix, const float *q_rot, const int64_t *cand, int64_t m,
                                    float r, float eps0, int32_t delta_d, int32_t method, int32_t source,
                                    uint8_t *pos_mask, float *dist, int32_t *dims, int64_t *stats,
                                    hipStream_t stream) {
    if (!ix) return fail(ADS_EINVAL, "index is NULL");
    if (m < 0) return fail(ADS_EINVAL, "m must be >= 0");
    if (m == 0) return ADS_OK;
    if (!q_rot || !cand || !pos_mask || !dist) return fail(ADS_EINVAL, "q_rot, cand, pos_mask and dist must not be NULL");
    if (!(r >= 0.f)) return fail(ADS_EINVAL, "r must be >= 0 (got %g)", (double)r);
    if (!(eps0 >= 0.f)) return fail(ADS_EINVAL, "eps0 must be >= 0 (got %g)", (double)eps0);
    if (delta_d < 1 || delta_d > ix->D) return fail(ADS_EINVAL, "delta_d must be in [1, D=%d] (got %d)", ix->D, delta_d);
    if (method < 0 || method > 2) return fail(ADS_EINVAL, "unknown method %d", method);
    if (source != 0 && source != 1) return fail(ADS_EINVAL, "source must be 0 or 1");
    if (source == 1 && !ix->rows32) return fail(ADS_EINVAL, "source 1 needs an index built with keep_fp32 = 1");
    if (!ix->P && method == ADS_METHOD_ADSAMPLING && !std::isinf(eps0))
        return fail(ADS_EINVAL, "ADSampling needs a rotated index (built with P); this one stores unrotated vectors");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    const float r2 = r * r;
    HIP_TRY(launch_dco(ix->storage, ix->data, ix->rows32, source, ix->list_off, ix->list_of_pos, ix->pos_of,
                       ix->n, ix->D, ix->dd, ix->b1, q_rot, cand, m, r2, (double)eps0, delta_d, method, pos_mask,
                       dist, dims, reinterpret_cast<unsigned long long *>(stats), nullptr, stream),
            "dco_batch");
    return ADS_OK;
}

extern "C" ads_status ads_dco_batch_ip(const ads_index *ix, const float *q, const int64_t *cand, int64_t m,
                                       float r, float eps0, int32_t delta_d, int32_t method, uint8_t *pos_mask,
                                       float *ip, int32_t *dims, int64_t *stats, hipStream_t stream) {
    if (!ix) return fail(ADS_EINVAL, "index is NULL");
    if (ix->metric != ADS_METRIC_COSINE) return fail(ADS_EINVAL, "inner-product DCOs need a cosine index");
    if (m < 0) return fail(ADS_EINVAL, "m must be >= 0");
    if (m == 0) return ADS_OK;
    if (!q || !cand || !pos_mask || !ip) return fail(ADS_EINVAL, "q, cand, pos_mask and ip must not be NULL");
    if (!std::isfinite(r)) return fail(ADS_EINVAL, "r must be finite");
    if (!(eps0 >= 0.f)) return fail(ADS_EINVAL, "eps0 must be >= 0 (got %g)", (double)eps0);
    if (delta_d < 1 || delta_d > ix->D) return fail(ADS_EINVAL, "delta_d must be in [1, D=%d] (got %d)", ix->D, delta_d);
    if (method < 0 || method > 2) return fail(ADS_EINVAL, "unknown method %d", method);
    if (!ix->P && method == ADS_METHOD_ADSAMPLING && !std::isinf(eps0))
        return fail(ADS_EINVAL, "ADSampling needs a rotated index (built with P); this one stores unrotated vectors");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    const int D = ix->D;
    float *scr = nullptr;
    HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&scr), sizeof(float) * (2 * (size_t)D + 64), stream), "scratch");
    float *qn = scr, *qr = scr + D, *qnorm = scr + 2 * D;
    hipError_t e = launch_normalize(q, 1, D, qn, qnorm, stream);
    if (e == hipSuccess) {
        if (ix->P) e = gemm_nt_f32(qn, D, ix->P, D, qr, D, 1, D, D, stream);
        else e = hipMemcpyAsync(qr, qn, sizeof(float) * D, hipMemcpyDeviceToDevice, stream);
    }
    IpArgs ipa{ix->norms, qnorm, r};
    if (e == hipSuccess)
        e = launch_dco(ix->storage, ix->data, ix->rows32, 0, ix->list_off, ix->list_of_pos, ix->pos_of, ix->n, D,
                       ix->dd, ix->b1, qr, cand, m, 0.f, (double)eps0, delta_d, method, pos_mask, ip, dims,
                       reinterpret_cast<unsigned long long *>(stats), &ipa, stream);
    (void)hipFreeAsync(scr, stream);
    if (e != hipSuccess) return hip_fail(e, "dco_batch_ip");
    return ADS_OK;
}

extern "C" uint64_t ads_search_workspace_size(const ads_index *ix, int32_t nq, int32_t k_max,
                                              int32_t nprobe_max, int32_t rerank) {
    if (check_search_args(ix, nq, k_max, nprobe_max, rerank) != ADS_OK) return 0;
    return (uint64_t)layout_for(ix, nq, k_max, nprobe_max, rerank).total;
}

extern "C" ads_status ads_search(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                                 const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                                 int32_t method, int32_t rerank, int64_t *ids, float *dist,
                                 int32_t *probes_out, int64_t *stats, void *workspace, hipStream_t stream) {
    ads_status st = check_search_args(ix, nq, k_max, nprobe_max, rerank);
    if (st != ADS_OK) return st;
    if (nq == 0) return ADS_OK;
    if (!q || !ids || !dist) return fail(ADS_EINVAL, "q, ids and dist must not be NULL");
    if (!(eps0 >= 0.f)) return fail(ADS_EINVAL, "eps0 must be >= 0 (got %g)", (double)eps0);
    if (method < 0 || method > 2) return fail(ADS_EINVAL, "unknown method %d", method);
    if (!ix->P && method == ADS_METHOD_ADSAMPLING && !std::isinf(eps0))
        return fail(ADS_EINVAL, "ADSampling needs a rotated index (built with P); this one stores unrotated vectors");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(ADS_EINVAL, "workspace must be 256-byte aligned");
    HIP_TRY(hipGetLastError(), "pending HIP error");

    const int eff_method = std::isinf(eps0) && method == ADS_METHOD_ADSAMPLING ? ADS_METHOD_FDSCANNING : method;
    const SearchLayout L = layout_for(ix, nq, k_max, nprobe_max, rerank);
    const int qw = L.qw;
    const int D = ix->D, nlist = ix->nlist;
    unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
    bool own = false;
    if (!ws) {
        hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&ws), L.total, stream);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ADS_ENOMEM, "workspace: out of device memory")
                                                             : hip_fail(e, "workspace allocation");
        own = true;
    }
    float *qrot = reinterpret_cast<float *>(ws + L.off_qrot);
    float *dots = reinterpret_cast<float *>(ws + L.off_dots);
    int32_t *probes = reinterpret_cast<int32_t *>(ws + L.off_probes);
    int32_t *kq = reinterpret_cast<int32_t *>(ws + L.off_kq);
    int32_t *keff = reinterpret_cast<int32_t *>(ws + L.off_keff);
    int32_t *npq = reinterpret_cast<int32_t *>(ws + L.off_npq);
    float *r2 = reinterpret_cast<float *>(ws + L.off_r2);
    uint64_t *tk = reinterpret_cast<uint64_t *>(ws + L.off_tk);
    int32_t *cnt = reinterpret_cast<int32_t *>(ws + L.off_cnt);
    int32_t *cursor = reinterpret_cast<int32_t *>(ws + L.off_cursor);
    int32_t *beg = reinterpret_cast<int32_t *>(ws + L.off_beg);
    int32_t *uoff = reinterpret_cast<int32_t *>(ws + L.off_uoff);
    int32_t *xoff = reinterpret_cast<int32_t *>(ws + L.off_xoff);
    int32_t *xcnt = reinterpret_cast<int32_t *>(ws + L.off_xcnt);
    int4 *units = reinterpret_cast<int4 *>(ws + L.off_units);
    int2 *qent = reinterpret_cast<int2 *>(ws + L.off_qent);
    uint64_t *slots = reinterpret_cast<uint64_t *>(ws + L.off_slots);

    hipError_t e = hipSuccess;
    auto done = [&](hipError_t err, const char *what) -> ads_status {
        if (own) (void)hipFreeAsync(ws, stream);
        return err == hipSuccess ? ADS_OK : hip_fail(err, what);
    };
#define SEARCH_TRY(expr, what)               \
    do {                                     \
        e = (expr);                          \
        if (e != hipSuccess) return done(e, what); \
    } while (0)

    const int sl = L.nsweep * nlist;
    {
        PhaseTimer t(ADS_PHASE_GROUP, stream);
        hipLaunchKernelGGL(setup_kernel, dim3(grid_for((int64_t)nq * L.kcap)), dim3(ADS_WG), 0, stream, K, nprobe,
                           nq, k_max, nprobe_max, rerank ? 4 : 1, L.kcap, kq, keff, npq, r2, tk);
        SEARCH_TRY(hipGetLastError(), "setup");
        hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(sl)), dim3(ADS_WG), 0, stream, cnt, (int64_t)sl);
        hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(sl)), dim3(ADS_WG), 0, stream, cursor, (int64_t)sl);
        SEARCH_TRY(hipGetLastError(), "zero counters");
    }
    // 1. query rotation (Section 3.1) and centre inner products (MFMA)
    {
        PhaseTimer t(ADS_PHASE_ROTATE, stream);
        const float *qsrc = q;
        if (ix->metric == ADS_METRIC_COSINE) {
            float *qunit = reinterpret_cast<float *>(ws + L.off_qunit);
            SEARCH_TRY(launch_normalize(q, nq, D, qunit, nullptr, stream), "normalise queries");
            qsrc = qunit;
        }
        if (ix->P) SEARCH_TRY(gemm_nt_f32(qsrc, D, ix->P, D, qrot, D, nq, D, D, stream), "rotate queries");
        else SEARCH_TRY(hipMemcpyAsync(qrot, qsrc, sizeof(float) * (size_t)nq * D, hipMemcpyDeviceToDevice,
                                       stream), "copy queries");
    }
    // 2. probe selection
    {
        PhaseTimer t(ADS_PHASE_PROBE, stream);
        SEARCH_TRY(gemm_nt_f32(qrot, D, ix->cent_rot, D, dots, nlist, nq, nlist, D, stream), "centre products");
        const size_t sh = probe_select_smem(nlist, nprobe_max);
        hipLaunchKernelGGL(probe_select_kernel, dim3(nq), dim3(ADS_WG), sh, stream, qrot, dots, ix->cent_norm, D,
                           nlist, nprobe_max, probes);
        SEARCH_TRY(hipGetLastError(), "probe selection");
    }
    // 3. group (query, rank) pairs by (sweep, list)
    {
        PhaseTimer t(ADS_PHASE_GROUP, stream);
        hipLaunchKernelGGL(group_count_kernel, dim3(grid_for((int64_t)nq * nprobe_max)), dim3(ADS_WG), 0, stream,
                           probes, npq, keff, nq, nprobe_max, nlist, L.lg, cnt);
        int32_t *order = reinterpret_cast<int32_t *>(ws + L.off_order);
        int32_t *xb = reinterpret_cast<int32_t *>(ws + L.off_xb);
        hipLaunchKernelGGL(list_order_kernel, dim3(8 * L.nsweep), dim3(512), 0, stream, cnt, ix->list_off, nlist,
                           order, xb);
        hipLaunchKernelGGL(group_scan_kernel, dim3(L.nsweep), dim3(1024), 0, stream, cnt, order, xb, L.nsweep, nlist, qw,
                           beg, uoff, xoff, xcnt);
        hipLaunchKernelGGL(group_scatter_kernel, dim3(grid_for((int64_t)nq * nprobe_max)), dim3(ADS_WG), 0, stream,
                           probes, npq, keff, nq, nprobe_max, nlist, L.lg, beg, cursor, qent);
        hipLaunchKernelGGL(unit_expand_kernel, dim3(grid_for(sl)), dim3(ADS_WG), 0, stream, cnt, beg, uoff,
                           L.nsweep, nlist, qw, L.ucap, units);
        SEARCH_TRY(hipGetLastError(), "grouping");
    }
    // 4. sweeps: list-major scan, then per-query merge
    for (int s = 0; s < L.nsweep; ++s) {
        const int ra = sweep_begin(s, L.lg);
        int rb = s + 1 < L.nsweep ? sweep_begin(s + 1, L.lg) : nprobe_max;
        if (rb > nprobe_max) rb = nprobe_max;
        ScanArgs a;
        a.data = ix->data;
        a.list_off = ix->list_off;
        a.ids = ix->ids;
        a.qrot = qrot;
        a.keff = keff;
        a.r2_in = r2;
        a.units = units + (size_t)s * L.ucap;
        a.xoff = xoff + s * 8;
        a.xcnt = xcnt + s * 8;
        a.qent = qent;
        a.slots = slots;
        a.stats = reinterpret_cast<unsigned long long *>(stats);
        a.eps0 = (double)eps0;
        a.method = eff_method;
        a.nprobe_max = nprobe_max;
        a.kcap = L.kcap;
        a.D = D;
        a.nb = ix->nb;
        a.b1 = ix->b1;
        // automatic: hand over at 1/8 of the tile's pairs alive (measured best on
        // the D = 960 workload with the IVF++ layout, for block widths 16 and 32)
        a.dense_frac = g_tune.dense_frac > 0.f ? g_tune.dense_frac : 0.125f;
        a.round_tiles = s < WIDE_SWEEPS ? 4 : 1;
        // persistent grid: 8 XCD lanes x P workgroups, P bounded by the units of the sweep
        const int64_t pairs = (int64_t)nq * (rb - ra);
        const int64_t units_bound = (pairs + qw - 1) / qw + (pairs < nlist ? pairs : nlist);
        int64_t P = (units_bound + 7) / 8;
        if (P > 4096) P = 4096;
        if (g_tune.grid_per_xcd > 0 && P > g_tune.grid_per_xcd) P = g_tune.grid_per_xcd;
        if (P < 1) P = 1;
        {
            PhaseTimer t(ADS_PHASE_SCAN, stream);
            const int64_t pf_units = g_tune.prefetch_units > 0 ? g_tune.prefetch_units : PREFETCH_UNITS;
            SEARCH_TRY(launch_scan(a, ix->storage, ix->dd, qw, (int)(8 * P), units_bound < pf_units,
                                   a.round_tiles == 4, stream), "scan");
        }
        const size_t sh = sizeof(uint64_t) * (size_t)next_pow2(L.kcap);
        PhaseTimer tm(ADS_PHASE_MERGE, stream);
        hipLaunchKernelGGL(merge_kernel, dim3(nq), dim3(ADS_WG), sh, stream, slots, keff, npq, nprobe_max, L.kcap,
                           ra, rb, tk, r2);
        SEARCH_TRY(hipGetLastError(), "merge");
    }
    // 5. output (or float32 rerank of the 4K survivors)
    {
        PhaseTimer t(ADS_PHASE_OUTPUT, stream);
        if (rerank) {
            const size_t sh = sizeof(uint64_t) * (size_t)next_pow2(L.kcap);
            hipLaunchKernelGGL(rerank_kernel, dim3(nq), dim3(ADS_WG), sh, stream, tk, kq, keff, ix->rows32,
                               ix->pos_of, qrot, D, ix->dd, L.kcap, k_max, ids, dist);
        } else {
            hipLaunchKernelGGL(output_kernel, dim3(grid_for((int64_t)nq * k_max)), dim3(ADS_WG), 0, stream, tk, kq,
                               nq, k_max, L.kcap, ids, dist);
        }
        SEARCH_TRY(hipGetLastError(), "output");
    }
    if (probes_out) {
        hipLaunchKernelGGL(probes_out_kernel, dim3(grid_for((int64_t)nq * nprobe_max)), dim3(ADS_WG), 0, stream,
                           probes, npq, nq, nprobe_max, probes_out);
        SEARCH_TRY(hipGetLastError(), "probes output");
    }
#undef SEARCH_TRY
    return done(hipSuccess, "");
}

// ---------------------------------------------------------------------------
// Allocation-free searches: the workspace is a file-scope device array.
// ---------------------------------------------------------------------------

namespace {

// On the host this name is only a stand-in: kernels get the device address
// taken with hipGetSymbolAddress, once per device, with that device current.
// Every GPU the library runs on holds its own copy until the process ends.
__device__ __align__(256) unsigned char scratch[ADS_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES] = {};

ads_status scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= SCRATCH_DEVICES)
        return fail(ADS_EUNSUPPORTED, "device %d: allocation-free searches support devices 0..%d", dev,
                    SCRATCH_DEVICES - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!p) return fail(ADS_EHIP, "scratch symbol address: null pointer");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ADS_OK;
}

}  // namespace

extern "C" ads_status ads_search_noalloc(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                                         const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                                         int32_t method, int32_t rerank, int64_t *ids, float *dist,
                                         int32_t *probes_out, int64_t *stats, hipStream_t stream) {
    ads_status st = check_search_args(ix, nq, k_max, nprobe_max, rerank);
    if (st != ADS_OK) return st;
    const size_t need = layout_for(ix, nq, k_max, nprobe_max, rerank).total;
    if (need > (size_t)ADS_NOALLOC_SCRATCH_BYTES)
        return fail(ADS_EINVAL,
                    "allocation-free search needs %zu bytes of workspace for these sizes; the scratch array "
                    "holds %llu (use ads_search with a workspace)",
                    need, (unsigned long long)ADS_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    st = scratch_address(&ws);
    if (st != ADS_OK) return st;
    return ads_search(ix, q, nq, K, nprobe, k_max, nprobe_max, eps0, method, rerank, ids, dist, probes_out,
                      stats, ws, stream);
}

struct ads_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" ads_status ads_plan_create(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                                      const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                                      int32_t method, int32_t rerank, int64_t *ids, float *dist,
                                      void *workspace, hipStream_t stream, ads_plan **out) {
    if (!out) return fail(ADS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!workspace) return fail(ADS_EINVAL, "a captured search needs a caller workspace");
    ads_status st = check_search_args(ix, nq, k_max, nprobe_max, rerank);
    if (st != ADS_OK) return st;
    if (nq < 1) return fail(ADS_EINVAL, "nq must be >= 1 for a plan");
    if (!q || !ids || !dist) return fail(ADS_EINVAL, "q, ids and dist must not be NULL");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    ads_plan *p = new (std::nothrow) ads_plan();
    if (!p) return fail(ADS_ENOMEM, "host allocation failed");
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "begin capture");
    }
    st = ads_search(ix, q, nq, K, nprobe, k_max, nprobe_max, eps0, method, rerank, ids, dist, nullptr,
                    nullptr, workspace, stream);
    std::string msg = g_err;
    e = hipStreamEndCapture(stream, &p->graph);
    if (st != ADS_OK) {
        if (p->graph) (void)hipGraphDestroy(p->graph);
        delete p;
        g_err = msg;
        return st;
    }
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "end capture");
    }
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(p->graph);
        delete p;
        return hip_fail(e, "instantiate graph");
    }
    *out = p;
    return ADS_OK;
}

extern "C" ads_status ads_plan_launch(ads_plan *plan, hipStream_t stream) {
    if (!plan || !plan->exec) return fail(ADS_EINVAL, "plan is NULL");
    HIP_TRY(hipGetLastError(), "pending HIP error");
    HIP_TRY(hipGraphLaunch(plan->exec, stream), "graph launch");
    return ADS_OK;
}

extern "C" ads_status ads_plan_free(ads_plan *plan) {
    if (!plan) return ADS_OK;
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return ADS_OK;
}

extern "C" ads_status ads_set_tuning(const ads_tuning *t) {
    if (!t) return fail(ADS_EINVAL, "tuning must not be NULL");
    if (!(t->dense_frac == 0.f || (t->dense_frac > 0.f && t->dense_frac <= 0.25f)))
        return fail(ADS_EINVAL, "dense_frac must be 0 (automatic) or in (0, 0.25] (got %g)", (double)t->dense_frac);
    if (t->queries_per_unit != 0 && t->queries_per_unit != 1 && t->queries_per_unit != 2 &&
        t->queries_per_unit != 4 && t->queries_per_unit != 8 && t->queries_per_unit != 16)
        return fail(ADS_EINVAL, "queries_per_unit must be 0, 1, 2, 4, 8 or 16 (got %d)", t->queries_per_unit);
    if (t->sweep_log2 < 1 || t->sweep_log2 > 6)
        return fail(ADS_EINVAL, "sweep_log2 must be in [1, 6] (got %d)", t->sweep_log2);
    if (t->grid_per_xcd < 0 || t->grid_per_xcd > 65536)
        return fail(ADS_EINVAL, "grid_per_xcd must be in [0, 65536] (got %d)", t->grid_per_xcd);
    if (t->prefetch_units < 0)
        return fail(ADS_EINVAL, "prefetch_units must be >= 0 (got %d)", t->prefetch_units);
    g_tune = *t;
    return ADS_OK;
}

extern "C" ads_status ads_get_tuning(ads_tuning *t) {
    if (!t) return fail(ADS_EINVAL, "tuning must not be NULL");
    *t = g_tune;
    return ADS_OK;
}

extern "C" ads_status ads_profile_enable(int32_t on) {
    g_prof.on = on != 0;
    return ADS_OK;
}

extern "C" ads_status ads_profile_collect(double *ms, int64_t *launches) {
    ads_status st = ADS_OK;
    for (auto &r : g_prof.recs) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && st == ADS_OK) st = hip_fail(e, "profile events");
        if (ms && r.phase >= 0 && r.phase < ADS_NPHASES) ms[r.phase] += (double)t;
        if (launches && r.phase >= 0 && r.phase < ADS_NPHASES) launches[r.phase] += 1;
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
    return st;
}

// ---------------------------------------------------------------------------
// Graph search (Section 2.2.1, Section 4, Section 5.1)
// ---------------------------------------------------------------------------

struct ads_hnsw {
    int64_t n = 0, up_rows = 0;
    int D = 0, M0 = 0, M = 0, max_level = 0, entry = 0, dd = 0, nb = 0;
    float *P = nullptr;          // NULL for unrotated vectors
    float *data = nullptr;       // [n][D] transformed vectors
    int32_t *adj0 = nullptr;     // [n][M0]
    int64_t *up_off = nullptr;   // [n]
    int32_t *up_adj = nullptr;   // [up_rows][M]
    int64_t bytes = 0;
};

namespace {

void free_hnsw(ads_hnsw *ix) {
    if (!ix) return;
    void *ptrs[] = {ix->P, ix->data, ix->adj0, ix->up_off, ix->up_adj};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete ix;
}

// One neighbour row: ids in [0, n), -1 only as padding at the end, no
// duplicates, and (above layer 0) every neighbour present on `layer`.
ads_status check_row(const int32_t *row, int width, int64_t n, const int32_t *levels, int layer,
                     int64_t v, std::vector<int32_t> &tmp) {
    tmp.clear();
    bool pad = false;
    for (int j = 0; j < width; ++j) {
        int32_t u = row[j];
        if (u < 0) {
            if (u != -1) return fail(ADS_EINVAL, "vertex %lld layer %d: neighbour id %d", (long long)v, layer, u);
            pad = true;
            continue;
        }
        if (pad) return fail(ADS_EINVAL, "vertex %lld layer %d: id after -1 padding", (long long)v, layer);
        if (u >= n) return fail(ADS_EINVAL, "vertex %lld layer %d: neighbour %d out of range", (long long)v, layer, u);
        if (layer > 0 && levels[u] < layer)
            return fail(ADS_EINVAL, "vertex %lld layer %d: neighbour %d is not on that layer", (long long)v, layer, u);
        tmp.push_back(u);
    }
    std::sort(tmp.begin(), tmp.end());
    if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end())
        return fail(ADS_EINVAL, "vertex %lld layer %d: duplicate neighbour", (long long)v, layer);
    return ADS_OK;
}

}  // namespace

extern "C" ads_status ads_hnsw_create(const float *base, int64_t n, int32_t D, const float *P,
                                      const int32_t *levels, const int32_t *adj0, int32_t M0,
                                      const int64_t *up_off, const int32_t *up_adj, int64_t up_rows,
                                      int32_t M, int32_t entry, int32_t delta_d, hipStream_t stream,
                                      ads_hnsw **out) {
    if (!out) return fail(ADS_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!base || !levels || !adj0 || !up_off) return fail(ADS_EINVAL, "base, levels, adj0 and up_off must not be NULL");
    if (n < 1 || n >= INT32_MAX) return fail(ADS_EINVAL, "n must be in [1, 2^31 - 1) (got %lld)", (long long)n);
    if (delta_d != 8 && delta_d != 16 && delta_d != 32)
        return fail(ADS_EINVAL, "delta_d must be 8, 16 or 32 (got %d)", delta_d);
    if (D < 32 || D % 32 || D / delta_d > HN_MAXBLOCKS)
        return fail(ADS_EINVAL, "D must be a multiple of 32 with D / delta_d <= %d (got D = %d)", HN_MAXBLOCKS, D);
    if (M0 < 1 || M0 > HN_MAXDEG) return fail(ADS_EINVAL, "M0 must be in [1, %d] (got %d)", HN_MAXDEG, M0);
    if (up_rows < 0) return fail(ADS_EINVAL, "up_rows must be >= 0");
    if (up_rows > 0 && (!up_adj || M < 1 || M > HN_MAXDEG))
        return fail(ADS_EINVAL, "upper rows need up_adj and M in [1, %d]", HN_MAXDEG);
    if (entry < 0 || entry >= n) return fail(ADS_EINVAL, "entry %d out of range", entry);
    const int top = levels[entry];
    std::vector<int32_t> tmp;
    for (int64_t v = 0; v < n; ++v) {
        const int lv = levels[v];
        if (lv < 0 || lv > top)
            return fail(ADS_EINVAL, "vertex %lld: level %d outside [0, level of the entry = %d]", (long long)v, lv, top);
        ads_status st = check_row(adj0 + v * M0, M0, n, levels, 0, v, tmp);
        if (st != ADS_OK) return st;
        if (lv == 0) continue;
        if (up_off[v] < 0 || up_off[v] + lv > up_rows)
            return fail(ADS_EINVAL, "vertex %lld: upper rows [%lld, %lld) outside [0, %lld)", (long long)v,
                        (long long)up_off[v], (long long)(up_off[v] + lv), (long long)up_rows);
        for (int l = 1; l <= lv; ++l) {
            st = check_row(up_adj + (up_off[v] + l - 1) * M, M, n, levels, l, v, tmp);
            if (st != ADS_OK) return st;
        }
    }
    HIP_TRY(hipGetLastError(), "pending HIP error");

    ads_hnsw *ix = new ads_hnsw();
    ix->n = n;
    ix->D = D;
    ix->M0 = M0;
    ix->M = up_rows > 0 ? M : 1;
    ix->max_level = top;
    ix->entry = entry;
    ix->dd = delta_d;
    ix->nb = D / delta_d;
    ix->up_rows = up_rows;
    hipError_t e = hipSuccess;
#define HNSW_TRY(expr, what)                                                             \
    do {                                                                                 \
        e = (expr);                                                                      \
        if (e != hipSuccess) {                                                           \
            free_hnsw(ix);                                                               \
            return e == hipErrorOutOfMemory ? fail(ADS_ENOMEM, "%s: out of device memory", what) \
                                            : hip_fail(e, what);                         \
        }                                                                                \
    } while (0)
    HNSW_TRY(dmalloc(&ix->data, (size_t)n * D, &ix->bytes), "vectors");
    HNSW_TRY(dmalloc(&ix->adj0, (size_t)n * M0, &ix->bytes), "layer-0 rows");
    HNSW_TRY(dmalloc(&ix->up_off, (size_t)n, &ix->bytes), "upper offsets");
    HNSW_TRY(dmalloc(&ix->up_adj, (size_t)(up_rows > 0 ? up_rows : 1) * ix->M, &ix->bytes), "upper rows");
    if (P) {
        HNSW_TRY(dmalloc(&ix->P, (size_t)D * D, &ix->bytes), "rotation");
        HNSW_TRY(hipMemcpyAsync(ix->P, P, (size_t)D * D * 4, hipMemcpyDeviceToDevice, stream), "copy P");
        HNSW_TRY(gemm_nt_f32(base, D, ix->P, D, ix->data, D, n, D, D, stream), "rotate vectors");
    } else {
        HNSW_TRY(hipMemcpyAsync(ix->data, base, (size_t)n * D * 4, hipMemcpyDeviceToDevice, stream), "copy vectors");
    }
    HNSW_TRY(hipMemcpyAsync(ix->adj0, adj0, (size_t)n * M0 * 4, hipMemcpyHostToDevice, stream), "copy layer 0");
    std::vector<int64_t> off(up_off, up_off + n);
    for (int64_t v = 0; v < n; ++v)
        if (levels[v] == 0) off[v] = -1;
    HNSW_TRY(hipMemcpyAsync(ix->up_off, off.data(), (size_t)n * 8, hipMemcpyHostToDevice, stream), "copy offsets");
    if (up_rows > 0)
        HNSW_TRY(hipMemcpyAsync(ix->up_adj, up_adj, (size_t)up_rows * M * 4, hipMemcpyHostToDevice, stream),
                 "copy upper rows");
    HNSW_TRY(hipStreamSynchronize(stream), "create");
#undef HNSW_TRY
    *out = ix;
    return ADS_OK;
}

namespace {

struct HnswLayout {
    size_t off_qrot, off_coef, off_vis, total;
    int64_t words;
};

HnswLayout hnsw_layout(const ads_hnsw *ix, int nq) {
    HnswLayout L;
    L.words = (ix->n + 31) / 32;
    L.off_qrot = 0;
    L.off_coef = align256((size_t)nq * ix->D * 4);
    L.off_vis = L.off_coef + align256((size_t)ix->nb * 4);
    L.total = L.off_vis + align256((size_t)nq * L.words * 4);
    return L;
}

}  // namespace

extern "C" uint64_t ads_hnsw_workspace_size(const ads_hnsw *ix, int32_t nq) {
    if (!ix || nq < 0) return 0;
    return (uint64_t)hnsw_layout(ix, nq).total;
}

extern "C" ads_status ads_hnsw_search(const ads_hnsw *ix, const float *q, int32_t nq, int32_t K, int32_t nef,
                                      float eps0, int32_t variant, int64_t *ids, float *dist, int64_t *qstats,
                                      int64_t *stats, void *workspace, hipStream_t stream) {
    if (!ix) return fail(ADS_EINVAL, "index must not be NULL");
    if (nq < 0) return fail(ADS_EINVAL, "nq must be >= 0");
    if (variant < ADS_HNSW_PLUS || variant > ADS_HNSW_PP) return fail(ADS_EINVAL, "unknown variant %d", variant);
    if (K < 1 || K > 256) return fail(ADS_EINVAL, "K must be in [1, 256] (got %d)", K);
    if (nef < 1 || nef > 4096) return fail(ADS_EINVAL, "nef must be in [1, 4096] (got %d)", nef);
    if (variant != ADS_HNSW_PP && nef < K) return fail(ADS_EINVAL, "nef (%d) must be >= K (%d)", nef, K);
    if (!(eps0 >= 0.f)) return fail(ADS_EINVAL, "eps0 must be >= 0 (got %g)", (double)eps0);
    if (!ix->P && variant != ADS_HNSW_PLAIN && !std::isinf(eps0))
        return fail(ADS_EINVAL, "ADSampling needs a rotated index (created with P); this one stores unrotated vectors");
    if (nq == 0) return ADS_OK;
    if (!q || !ids || !dist) return fail(ADS_EINVAL, "q, ids and dist must not be NULL");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(ADS_EINVAL, "workspace must be 256-byte aligned");
    const size_t smem = hnsw_smem_bytes(ix->D, ix->nb, nef, K);
    if (smem > 64 * 1024) return fail(ADS_EINVAL, "D, nef and K need %zu bytes of LDS (> 64 KiB)", smem);
    HIP_TRY(hipGetLastError(), "pending HIP error");

    const HnswLayout L = hnsw_layout(ix, nq);
    unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
    bool own = false;
    if (!ws) {
        hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&ws), L.total, stream);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(ADS_ENOMEM, "workspace: out of device memory")
                                                             : hip_fail(e, "workspace allocation");
        own = true;
    }
    float *qrot = reinterpret_cast<float *>(ws + L.off_qrot);
    float *coef = reinterpret_cast<float *>(ws + L.off_coef);
    uint32_t *vis = reinterpret_cast<uint32_t *>(ws + L.off_vis);
    auto done = [&](hipError_t err, const char *what) -> ads_status {
        if (own) (void)hipFreeAsync(ws, stream);
        return err == hipSuccess ? ADS_OK : hip_fail(err, what);
    };
    hipError_t e;
    if (ix->P)
        e = gemm_nt_f32(q, ix->D, ix->P, ix->D, qrot, ix->D, nq, ix->D, ix->D, stream);
    else
        e = hipMemcpyAsync(qrot, q, (size_t)nq * ix->D * 4, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return done(e, "rotate queries");
    const int method = variant == ADS_HNSW_PLAIN || std::isinf(eps0) ? ADS_METHOD_FDSCANNING : ADS_METHOD_ADSAMPLING;
    e = launch_hnsw_setup(coef, ix->nb, ix->dd, ix->D, (double)eps0, method, vis, (int64_t)nq * L.words, stream);
    if (e != hipSuccess) return done(e, "search setup");
    HnswArgs a;
    a.data = ix->data;
    a.adj0 = ix->adj0;
    a.up_off = ix->up_off;
    a.up_adj = ix->up_adj;
    a.qrot = qrot;
    a.coef = coef;
    a.visited = vis;
    a.vis_words = L.words;
    a.ids = ids;
    a.dist = dist;
    a.qstats = qstats;
    a.stats = reinterpret_cast<unsigned long long *>(stats);
    a.D = ix->D;
    a.nb = ix->nb;
    a.dd = ix->dd;
    a.M0 = ix->M0;
    a.M = ix->M;
    a.entry = ix->entry;
    a.max_level = ix->max_level;
    a.K = K;
    a.nef = nef;
    a.variant = variant;
    e = launch_hnsw_search(a, nq, stream);
    return done(e, "graph search");
}

extern "C" ads_status ads_hnsw_free(ads_hnsw *ix) {
    if (!ix) return ADS_OK;
    (void)hipDeviceSynchronize();
    free_hnsw(ix);
    return ADS_OK;
}

extern "C" const char *ads_last_error(void) { return g_err.c_str(); }

extern "C" const char *ads_version(void) { return "ads-mi355x 0.1.0 (gfx950)"; }
