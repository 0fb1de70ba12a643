/*
 * ads.h -- C ABI of the MI355X (gfx950) ADSampling-IVF library.
 *
 * ADSampling (Gao & Long, SIGMOD 2023) decides a distance comparison
 * operation (DCO, Definition 2.1: is dis(o, q) <= r, and if so what is dis)
 * by sampling coordinates of randomly rotated vectors incrementally and
 * stopping as soon as a hypothesis test rejects dis <= r (Algorithm 1,
 * Sections 3.1-3.3).  This library runs it inside an IVF candidate scan
 * (IVF+, Section 4) over a dimension-blocked list layout (IVF++, Section 5.2).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless the argument says "host".
 *   - Matrices are row-major and contiguous ([rows][cols]).
 *   - The rotation is y = P x with P a [D][D] row-major orthogonal matrix, so a
 *     batch of row vectors X is rotated as X * P^T (Section 3.1, Eq. 2).
 *   - Distances are Euclidean (not squared), as in Definition 2.1; the kernels
 *     compare squared values internally.
 *   - Calls are asynchronous on the given HIP stream unless stated otherwise;
 *     the caller keeps every buffer alive until the stream has passed the call.
 *   - Arguments are validated on the host before anything is launched.  On a
 *     failed validation the call returns a negative status, writes nothing and
 *     sets a thread-local message readable with ads_last_error().
 *   - A HIP error raised by a launch (or left pending by earlier asynchronous
 *     work) is returned as ADS_EHIP.
 *   - No C++ exception crosses this interface.
 */
#ifndef ADS_H
#define ADS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ADS_OK = 0,
    ADS_EINVAL = -1,        /* invalid argument (message in ads_last_error) */
    ADS_ENOMEM = -2,        /* device or host allocation failed */
    ADS_EHIP = -3,          /* HIP runtime / launch error */
    ADS_EUNSUPPORTED = -4   /* valid request the library does not support */
} ads_status;

typedef enum {
    ADS_F32 = 0,            /* rotated vectors stored as float32 */
    ADS_BF16 = 1,           /* stored as bfloat16 (round to nearest even) */
    ADS_F16 = 2             /* stored as IEEE half (round to nearest even) */
} ads_dtype;

typedef enum {
    ADS_METHOD_ADSAMPLING = 0,  /* Algorithm 1 with the test of Section 3.2 */
    ADS_METHOD_FDSCANNING = 1,  /* full-dimension distance then compare (Section 2.1) */
    ADS_METHOD_PDSCANNING = 2   /* partial-distance early stop on raw coordinates (Section 6.1) */
} ads_method;

typedef enum {
    ADS_METRIC_L2 = 0,      /* Euclidean distance (the paper's setting) */
    ADS_METRIC_COSINE = 1   /* cosine: base vectors, centres and queries are normalised to unit
                               length, then searched in L2 (Section 8, extension (1): cosine search equals
                               Euclidean search on normalised vectors) */
} ads_metric;

/* Opaque index.  Device-resident, owned by the library, read-only after
 * ads_ivf_build returns, released by ads_index_free. */
typedef struct ads_index ads_index;

/* Host-side description of an index. */
typedef struct {
    int64_t n;              /* number of stored vectors */
    int32_t D;              /* dimensionality */
    int32_t nlist;          /* number of inverted lists */
    int32_t delta_d;        /* block width of the stored layout */
    int32_t storage;        /* ads_dtype of the blocked layout */
    int32_t has_fp32_copy;  /* 1 if a float32 row copy is kept (rerank / dco source) */
    int32_t max_list;       /* largest list size */
    int32_t metric;         /* ads_metric */
    int64_t device_bytes;   /* device memory held by the index */
    int32_t rotated;        /* 1 if built with a rotation P, 0 for unrotated vectors */
    int32_t a1_dims;        /* leading coordinates stored block-major (IVF++ array A1) */
} ads_index_desc;

/* Counters accumulated by ads_search / ads_dco_batch into a caller buffer of
 * ADS_NSTATS int64 values on the device (never reset by the library). */
enum {
    ADS_STAT_DCOS = 0,          /* distance comparison operations */
    ADS_STAT_DIMS = 1,          /* coordinates sampled over all DCOs */
    ADS_STAT_POSITIVES = 2,     /* DCOs that returned positive */
    ADS_STAT_BYTES = 3,         /* bytes of stored vector data the DCOs needed */
    ADS_NSTATS = 4
};

/* --------------------------------------------------------------------------
 * Rotation (Section 3.1).
 * -------------------------------------------------------------------------- */

/*
 * ads_make_rotation -- HOST function.  Orthonormalises a Gaussian matrix into
 * the random orthogonal transformation of Section 3.1 (the paper obtains it
 * by orthonormalising a matrix of i.i.d. standard Gaussians, Section 3.1
 * footnote; Section 6.1 generates it once in the index phase).
 *   gaussian  host [D][D] float64, i.i.d. N(0,1) entries (caller's draw).
 *   D         >= 1.
 *   P_out     host [D][D] float32: P with y = P x (rows of P are the sampled
 *             directions).  Householder QR in float64, columns of Q scaled by
 *             sign(diag R) so that P is Haar distributed.
 *   P64_out   host [D][D] float64 copy of the same matrix, or NULL.
 * Errors: ADS_EINVAL for NULL inputs or D < 1; ADS_ENOMEM.  Synchronous.
 */
ads_status ads_make_rotation(const double *gaussian, int32_t D, float *P_out, double *P64_out);

/*
 * ads_rotate -- Y = X * P^T, i.e. y = P x for every row (Section 3.1, Eq. 2),
 * on the matrix cores (FP32 MFMA, FP32 accumulation).
 *   P   device [D][D] float32.   X device [n][D] float32.   Y device [n][D]
 *   float32 (must not alias X).  n >= 0 (n == 0 is a no-op), 1 <= D, D % 4 == 0.
 */
ads_status ads_rotate(const float *P, int32_t D, const float *X, int64_t n, float *Y,
                      hipStream_t stream);

/* --------------------------------------------------------------------------
 * Index phase (Section 2.2.2 IVF buckets, Section 5.2 IVF++ layout).
 * -------------------------------------------------------------------------- */

/*
 * ads_ivf_build -- builds the IVF index from a clustering supplied by the
 * caller (in the paper the k-means clustering comes from an external library,
 * Section 6.1; the index is the same for IVF, IVF+ and IVF++).
 *   base       device [n][D] float32 raw vectors; n >= 1.
 *   P          device [D][D] float32 rotation (copied into the index), or NULL
 *              for an index of the unrotated vectors: the layout of IVF** and
 *              the baseline IVF* of Section 6.1 (PDScanning on the original
 *              coordinates).  Such an index accepts FDScanning and PDScanning
 *              and rejects ADSampling with a finite eps0 (ADS_EINVAL): the test
 *              of Section 3.2 relies on the random rotation.
 *   centroids  device [nlist][D] float32 raw-space list centres.
 *   assign     device [n] int32 list id of every vector, in [0, nlist).
 *   delta_d    block width of the stored layout: D % delta_d == 0 and
 *              delta_d % 8 == 0 (a multiple of 4 suffices for ADS_F32).
 *   storage    ads_dtype of the blocked layout.
 *   keep_fp32  1 to keep a float32 copy of the rotated rows (required by the
 *              low-precision rerank and by ads_dco_batch's row source).
 *   metric     ads_metric.  ADS_METRIC_COSINE normalises every base vector and
 *              centre before rotating (a zero vector stays zero) and keeps the
 *              raw norms for ads_dco_batch_ip; searches then normalise their
 *              queries and report distances between unit vectors
 *              (cosine similarity = 1 - dist^2 / 2).
 *   out        host pointer receiving the new index.
 * Layout (IVF++, Section 5.2): for list l, the first a1_dims = min(D, max(
 * delta_d, 128 rounded down to delta_d)) coordinates of all its vectors are
 * stored block by block, [block][vector][delta_d] (the paper's array A1, its
 * first d1 coordinates of all candidates; the scan reads them a 64-vector
 * tile at a time), and the remaining D - a1_dims coordinates vector by
 * vector (array A2, so the later blocks of one candidate are contiguous).
 * Within a list, vectors keep ascending id order.
 * Synchronises the stream once (the list sizes are needed on the host).
 * Errors: ADS_EINVAL (sizes, ids out of range), ADS_ENOMEM, ADS_EHIP.
 */
ads_status ads_ivf_build(const float *base, int64_t n, int32_t D, const float *P,
                         const float *centroids, int32_t nlist, const int32_t *assign,
                         int32_t delta_d, int32_t storage, int32_t keep_fp32, int32_t metric,
                         hipStream_t stream, ads_index **out);

/*
 * ads_kmeans -- Lloyd's k-means clustering of the index phase (Section 2.2.2:
 * IVF partitions the data into the clusters of k-means; Section 6.1 runs it
 * with a library and 4,096 clusters), on the GPU, trained on all n rows.
 *   x          device [n][D] float32 rows; n >= 1, 1 <= D <= 4096.
 *   nlist      number of clusters, 1 <= nlist <= n.
 *   iters      Lloyd iterations, >= 0 (0: the seeded rows are the centres).
 *   seed       initialisation: row i draws the SplitMix64 output of the
 *              counter seed + (i + 1) * 0x9E3779B97F4A7C15 (Steele, Lea and
 *              Flood, 2014); the nlist rows with the smallest draws, in
 *              ascending draw order, are the initial centres 0..nlist-1.
 *   centroids  device [nlist][D] float32 out: final centres.
 *   assign     device [n] int32 out: list of every row under the final centres.
 * One iteration assigns every row to its nearest centre (squared distance in
 * the FP32 form |x|^2 + |c|^2 - 2 x.c, products on the matrix cores; ties to
 * the lower centre id), then hands every empty list, in ascending id order,
 * the member of the currently largest list (lower id on ties) farthest from
 * its centre (lower row on ties), then moves every centre to the mean of its
 * members (float64 sums in ascending row order, rounded once to float32).  A
 * final assignment to the final centres gives `assign`.  Deterministic.
 * Allocates device workspace (about 256 MB of centre products plus O(n)).
 * Synchronises the stream.  Errors: ADS_EINVAL, ADS_ENOMEM, ADS_EHIP.
 */
ads_status ads_kmeans(const float *x, int64_t n, int32_t D, int32_t nlist, int32_t iters, uint64_t seed,
                      float *centroids, int32_t *assign, hipStream_t stream);

/*
 * ads_build_ivf -- the whole index phase: ads_kmeans on the base vectors
 * (on the unit-normalised vectors for ADS_METRIC_COSINE), then ads_ivf_build
 * with the resulting centres and lists.  Arguments as those two calls;
 * centroids_out ([nlist][D]) and assign_out ([n]) are device buffers that
 * receive the clustering, or NULL (the library then uses its own).
 */
ads_status ads_build_ivf(const float *base, int64_t n, int32_t D, const float *P, int32_t nlist,
                         int32_t iters, uint64_t seed, int32_t delta_d, int32_t storage, int32_t keep_fp32,
                         int32_t metric, float *centroids_out, int32_t *assign_out, hipStream_t stream,
                         ads_index **out);

/* ads_index_info -- HOST: fills *info (host pointer).  ADS_EINVAL on NULL. */
ads_status ads_index_info(const ads_index *ix, ads_index_desc *info);

/*
 * ads_index_lists -- copies the list structure to caller buffers (device):
 *   offsets [nlist + 1] int64 prefix offsets, ids [n] int64 stored ids in list
 *   order; either pointer may be NULL.  rot_centroids [nlist][D] float32 (may be
 *   NULL) receives the rotated centres.
 */
ads_status ads_index_lists(const ads_index *ix, int64_t *offsets, int64_t *ids,
                           float *rot_centroids, hipStream_t stream);

/* ads_index_free -- releases the index (synchronises the device). NULL is a no-op. */
ads_status ads_index_free(ads_index *ix);

/* --------------------------------------------------------------------------
 * Query phase.
 * -------------------------------------------------------------------------- */

/*
 * ads_dco_batch -- DCOs of one rotated query against explicit candidates with
 * a fixed threshold r (Definition 2.1; Algorithm 1; the fixed-threshold
 * protocol of Section 6.2.6).
 *   q_rot     device [D] float32, already rotated (P q); the raw query for an
 *             index built without P.
 *   cand      device [m] int64 base ids; m >= 0.
 *   r         threshold distance (not squared), >= 0, +INF allowed.
 *   eps0      test parameter epsilon_0 >= 0 (Section 3.2); +INF never rejects.
 *   delta_d   coordinates sampled per step, 1 <= delta_d <= D (any value; the
 *             last step may be shorter).
 *   method    ads_method.  PDScanning runs on the coordinates the index stores
 *             (rotated, or original for an index built without P).
 *   source    0: read the blocked list layout; 1: read the float32 row copy
 *             (index built with keep_fp32).  Both give identical decisions for
 *             float32 storage (the IVF+ == IVF++ property of Section 5.2).
 *   pos_mask  device [m] uint8: 1 positive, 0 negative.
 *   dist      device [m] float32: dis for positives, +INF for negatives.
 *   dims      device [m] int32 coordinates sampled, or NULL.
 *   stats     device [ADS_NSTATS] int64 accumulators, or NULL.
 * S_d is the sum, in block order, of per-block partial sums over the index's
 * delta_d-wide blocks (each a chain of fused multiply-adds in ascending
 * coordinate order) plus the running partial of the current block; the
 * search uses the same order, so both report identical S.  The test at d < D
 * is  S_d > (d/D)(1+eps0/sqrt(d))^2 r^2  (the squared form of
 * dis' > (1+eps0/sqrt(d)) r); at d = D positive iff S_D <= r^2.
 * Errors: ADS_EINVAL (NULL, id out of range, bad parameters), ADS_EHIP.
 */
ads_status ads_dco_batch(const ads_index *ix, const float *q_rot, const int64_t *cand, int64_t m,
                         float r, float eps0, int32_t delta_d, int32_t method, int32_t source,
                         uint8_t *pos_mask, float *dist, int32_t *dims, int64_t *stats,
                         hipStream_t stream);

/*
 * ads_dco_batch_ip -- inner-product comparison <o, q> >= r for explicit
 * candidates, reduced to a DCO on unit vectors (Section 8, extension (1)):
 * <o,q> >= r  <=>  || o/|o| - q/|q| || <= sqrt(2 - 2 r / (|o| |q|)), decided by
 * Algorithm 1 (or FDScanning / PDScanning) with that per-candidate threshold.
 * Needs an index built with ADS_METRIC_COSINE (it keeps the raw norms).
 *   q        device [D] float32 RAW query (normalised and rotated inside).
 *   r        inner-product threshold (any finite value).
 *   ip       device [m] float32: <o, q> = |o||q|(1 - d^2/2) for positives,
 *            -INF for negatives (d: distance of the unit vectors).
 *   Other arguments as ads_dco_batch (source 0 only).  A candidate whose
 *   threshold is negative under the root can never reach r: negative with 0
 *   dims.  If |o||q| = 0, positive iff r <= 0.  Allocates D * 8 bytes of
 *   stream-ordered scratch.
 */
ads_status ads_dco_batch_ip(const ads_index *ix, const float *q, const int64_t *cand, int64_t m,
                            float r, float eps0, int32_t delta_d, int32_t method, uint8_t *pos_mask,
                            float *ip, int32_t *dims, int64_t *stats, hipStream_t stream);

/*
 * ads_search -- IVF+ / IVF++ KNN search (Section 2.2.2 with ADSampling as the
 * DCO, Section 4) for a batch of raw queries.
 *   q         device [nq][D] float32 raw queries (rotated inside, end to end as
 *             the paper measures, Section 6.1).
 *   nq        >= 0 (0 is a no-op).
 *   K         device [nq] int32 per-query K in [0, k_max], or NULL for k_max.
 *   nprobe    device [nq] int32 per-query N_probe in [1, nprobe_max], or NULL
 *             for nprobe_max.  Per-query values above nprobe_max are clamped.
 *   k_max     >= 1; nprobe_max in [1, nlist] and at most 4096 (above:
 *             ADS_EUNSUPPORTED).
 *   eps0      >= 0, +INF selects FDScanning (no statistical test).
 *   method    ads_method.  PDScanning compares partial distances over the
 *             coordinates the index stores: on an index built without P it is
 *             the paper's IVF* / IVF** baseline (Section 6.1); queries are then
 *             not rotated.
 *   rerank    0: plain search.  1: low-precision mode: scan with a KNN set of
 *             4K, then recompute the 4K survivors' distances from the float32
 *             row copy and return the best K (index built with keep_fp32).
 *   ids       device [nq][k_max] int64, ascending by (distance, id); entries
 *             past K[i] or past the available candidates are -1.
 *   dist      device [nq][k_max] float32 distances; padding +INF.
 *   probes_out device [nq][nprobe_max] int32 probed lists, nearest first
 *             (ties to the lower list id), or NULL.  Entries past nprobe[i] are -1.
 *   stats     device [ADS_NSTATS] int64 accumulators, or NULL.
 *   workspace device scratch of at least ads_search_workspace_size(...) bytes,
 *             256-byte aligned, or NULL to let the library allocate it on the
 *             stream (stream-ordered allocation, freed on the stream).
 * The index is read-only, so concurrent searches on different streams with
 * different workspaces are allowed.  Each query's result depends only on that
 * query, its K and nprobe, the index and (eps0, delta_d, method): not on the
 * other queries of the batch.
 */
ads_status ads_search(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                      const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                      int32_t method, int32_t rerank, int64_t *ids, float *dist,
                      int32_t *probes_out, int64_t *stats, void *workspace, hipStream_t stream);

/* ads_search_workspace_size -- HOST: bytes of workspace ads_search needs for
 * these sizes under the calling thread's queries_per_unit setting, for any
 * method and eps0 (0 on invalid arguments, with ads_last_error set). */
uint64_t ads_search_workspace_size(const ads_index *ix, int32_t nq, int32_t k_max,
                                   int32_t nprobe_max, int32_t rerank);

/*
 * ads_search_noalloc -- ads_search for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments and results as ads_search without the
 * workspace argument: the workspace is a file-scope device array of
 * ADS_NOALLOC_SCRATCH_BYTES bytes inside the library (each GPU the library
 * runs on holds its own copy until the process ends).  Calls no allocating
 * routine.  Sizes whose workspace (ads_search_workspace_size) exceeds the
 * array are rejected with ADS_EINVAL and a message.  All calls on one GPU
 * share that GPU's array: calls that overlap on one GPU (different streams
 * or threads without ordering between them) race and must be serialised by
 * the caller.  The first call on a device looks up the array's device
 * address with that device current.
 */
#define ADS_NOALLOC_SCRATCH_BYTES (256ull << 20)
ads_status ads_search_noalloc(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                              const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                              int32_t method, int32_t rerank, int64_t *ids, float *dist,
                              int32_t *probes_out, int64_t *stats, hipStream_t stream);

/* --------------------------------------------------------------------------
 * Captured searches: one graph launch per batch.
 * -------------------------------------------------------------------------- */

/* Opaque captured search: the whole ads_search launch sequence recorded once
 * into a HIP graph for fixed buffers and sizes. */
typedef struct ads_plan ads_plan;

/*
 * ads_plan_create -- records ads_search(ix, q, nq, K, nprobe, k_max,
 * nprobe_max, eps0, method, rerank, ids, dist, NULL, NULL, workspace) on
 * `stream` with stream capture and instantiates the graph.  Nothing runs at
 * creation.  Every pointer is bound into the plan: before each launch the
 * caller rewrites the contents of q (and K / nprobe, which may differ per
 * query and per launch) at the same addresses.  `workspace` is required (the
 * graph must not allocate).  The plan uses the tuning of the calling thread at
 * creation.  Errors: as ads_search, plus ADS_EINVAL for a NULL workspace and
 * ADS_EHIP if the stream cannot be captured (e.g. the legacy null stream).
 */
ads_status ads_plan_create(const ads_index *ix, const float *q, int32_t nq, const int32_t *K,
                           const int32_t *nprobe, int32_t k_max, int32_t nprobe_max, float eps0,
                           int32_t method, int32_t rerank, int64_t *ids, float *dist,
                           void *workspace, hipStream_t stream, ads_plan **out);

/* ads_plan_launch -- replays the captured search on `stream` (one graph launch). */
ads_status ads_plan_launch(ads_plan *plan, hipStream_t stream);

/* ads_plan_free -- destroys the plan (synchronises the device).  NULL is a no-op. */
ads_status ads_plan_free(ads_plan *plan);

/* --------------------------------------------------------------------------
 * Scheduling knobs of the scan (no effect on what a DCO decides).
 * -------------------------------------------------------------------------- */

typedef struct {
    float dense_frac;         /* (0, 0.25]: a 64-vector tile leaves the register-dense
                                 phase once at most this fraction of its (vector, query)
                                 pairs is alive; 0 = automatic (0.125).  Default 0. */
    int32_t queries_per_unit; /* 1, 2, 4, 8 or 16 queries per work unit; 0 = the largest
                                 power of two up to 8 whose KNN sets fit in 4 KB of LDS.
                                 Default 0. */
    int32_t sweep_log2;       /* probe ranks are scanned in sweeps [0,1), [1,g), [g,g^2), ...
                                 with g = 2^sweep_log2, sweep_log2 in [1, 6].  Default 4. */
    int32_t grid_per_xcd;     /* persistent scan workgroups per XCD, 0 = as many as the
                                 sweep has units (capped at 4096).  Default 0. */
    int32_t prefetch_units;   /* sweeps with fewer work units than this (and one wave per
                                 unit) run the scan instantiation that fetches block b+1 while
                                 block b is evaluated; 0 = 8192.  Same results either way.
                                 Default 0. */
} ads_tuning;

/* ads_set_tuning / ads_get_tuning -- HOST, per thread: knobs for later
 * ads_search calls issued by this thread.  ADS_EINVAL on values out of range. */
ads_status ads_set_tuning(const ads_tuning *t);
ads_status ads_get_tuning(ads_tuning *t);

/* --------------------------------------------------------------------------
 * Optional per-phase timing with HIP events (off by default).
 * -------------------------------------------------------------------------- */

enum {
    ADS_PHASE_ROTATE = 0,   /* query rotation GEMM */
    ADS_PHASE_PROBE = 1,    /* centre products GEMM + probe selection */
    ADS_PHASE_GROUP = 2,    /* per-query setup and grouping of (query, list) pairs */
    ADS_PHASE_SCAN = 3,     /* the DCO scan kernels (one launch per sweep) */
    ADS_PHASE_MERGE = 4,    /* per-query KNN-set merges after each sweep */
    ADS_PHASE_OUTPUT = 5,   /* output / float32 rerank */
    ADS_NPHASES = 6
};

/*
 * ads_profile_enable -- HOST.  on = 1: every later ads_search issued by this
 * thread records a pair of HIP events around each phase on its stream (small
 * overhead; not for use under stream capture).  on = 0 stops recording.
 */
ads_status ads_profile_enable(int32_t on);

/*
 * ads_profile_collect -- HOST.  Waits for the recorded events, adds the
 * elapsed milliseconds of every phase into ms[ADS_NPHASES] and the number of
 * timed launches into launches[ADS_NPHASES] (host arrays, either may be NULL),
 * then forgets the records.
 */
ads_status ads_profile_collect(double *ms, int64_t *launches);

/* --------------------------------------------------------------------------
 * Graph search: HNSW (Section 2.2.1), HNSW+ (Section 4) and HNSW++ (Section 5.1)
 * -------------------------------------------------------------------------- */

typedef struct ads_hnsw ads_hnsw;   /* opaque, device-resident, library-owned */

typedef enum {
    ADS_HNSW_PLUS = 0,   /* HNSW+: Algorithm 1 DCOs against R's largest distance */
    ADS_HNSW_PLAIN = 1,  /* HNSW: full-dimension DCOs (FDScanning) */
    ADS_HNSW_PP = 2      /* HNSW++: R1 (K exact distances) gives the threshold and the
                            answer, R2 (N_ef observed distances) drives the beam */
} ads_hnsw_variant;

/*
 * ads_hnsw_create -- builds a graph index on the device from a graph given on
 * the host (the HNSW index phase, Section 2.2.1; the method leaves the graph
 * construction unchanged, so the caller supplies it, e.g. from hnswlib or the
 * seeded builder of the test inputs).
 *
 *   base     device [n][D] float32 raw vectors, row-major.
 *   P        device [D][D] float32 rotation (y = P x, Section 3.1), copied; NULL
 *            stores the vectors unrotated (then only ADS_HNSW_PLAIN, or eps0 =
 *            +inf, may search it).
 *   levels   host [n] top layer of each vertex (>= 0).
 *   adj0     host [n][M0] layer-0 neighbour ids in the order the search examines
 *            them, -1 padded at the end of a row; no duplicates in a row.
 *   up_off   host [n]: for a vertex with levels[v] >= 1, the row of up_adj
 *            holding its layer-1 neighbours (its layer-l row is up_off[v] + l - 1);
 *            ignored for levels[v] == 0.
 *   up_adj   host [up_rows][M] upper-layer neighbour ids, -1 padded at the end;
 *            a neighbour on layer l must have levels >= l.  NULL if up_rows == 0.
 *   entry    the vertex the search starts from; levels[entry] must be the
 *            largest level.
 *   delta_d  coordinates per sampling step: 8, 16 or 32; D must be a multiple
 *            of 32 and D / delta_d <= 128.  M0, M <= 32.
 *
 * Every id and row is checked on the host before anything is copied.
 * Synchronises the stream.  Errors: ADS_EINVAL (with the offending vertex in
 * ads_last_error), ADS_ENOMEM, ADS_EHIP.
 */
ads_status ads_hnsw_create(const float *base, int64_t n, int32_t D, const float *P,
                           const int32_t *levels, const int32_t *adj0, int32_t M0,
                           const int64_t *up_off, const int32_t *up_adj, int64_t up_rows,
                           int32_t M, int32_t entry, int32_t delta_d, hipStream_t stream,
                           ads_hnsw **out);

/* ads_hnsw_workspace_size -- HOST: bytes of workspace ads_hnsw_search needs for
 * nq queries (the transformed queries, the test coefficients and one visited
 * bitmap of n bits per query); 0 for invalid arguments. */
uint64_t ads_hnsw_workspace_size(const ads_hnsw *ix, int32_t nq);

/*
 * ads_hnsw_search -- graph search of nq queries, one answer of K per query.
 *
 *   q        device [nq][D] float32 raw queries (rotated inside).
 *   K, nef   answer size and beam width N_ef (K <= nef for HNSW and HNSW+;
 *            HNSW++ keeps R1 of K and R2 of nef); 1 <= K <= 256, nef <= 4096
 *            (D, K and nef together must fit the 64 KiB of LDS a workgroup may
 *            use: 4 D + 128 D / delta_d + 9 nef + 8 K bytes, roughly).
 *   eps0     Algorithm 1's parameter (>= 0; +inf never rejects); ignored by
 *            ADS_HNSW_PLAIN.
 *   ids      device [nq][K] int64 out, ascending (distance, id); -1 padded.
 *   dist     device [nq][K] float32 out, distances (not squared); +inf padded.
 *   qstats   device [nq][3] int64 out: DCOs, sampled coordinates and layer-0
 *            expansions of each query, or NULL.
 *   stats    device [3] int64 accumulators of the same three counts, or NULL.
 *   workspace device, 256-byte aligned, >= ads_hnsw_workspace_size bytes, or
 *            NULL to allocate it on the stream.
 *
 * Asynchronous on `stream`.  Ties are ordered by id, every set is keyed by
 * (squared distance, id), and the search ends when every member of R (R2)
 * has been expanded.  Errors: ADS_EINVAL, ADS_ENOMEM, ADS_EHIP.
 */
ads_status ads_hnsw_search(const ads_hnsw *ix, const float *q, int32_t nq, int32_t K, int32_t nef,
                           float eps0, int32_t variant, int64_t *ids, float *dist, int64_t *qstats,
                           int64_t *stats, void *workspace, hipStream_t stream);

/* ads_hnsw_free -- releases the index (synchronises the device).  NULL is a no-op. */
ads_status ads_hnsw_free(ads_hnsw *ix);

/* ads_last_error -- thread-local message for the last failing call on this
 * thread ("" if none).  The pointer stays valid until the next call. */
const char *ads_last_error(void);

/* ads_version -- library version string. */
const char *ads_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ADS_H */
