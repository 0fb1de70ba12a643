/*
 * FP64 CPU oracle for ADSampling distance comparison operations inside an IVF
 * candidate scan.  TEST INFRASTRUCTURE ONLY: the GPU library never links,
 * loads or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Plain, slow, sequential C99 in double precision.  Every function follows the
 * paper's definitions in the paper's order:
 *
 *   - Definition 2.1 (Section 2.1): a DCO decides whether dis <= r and returns
 *     dis when it is;
 *   - FDScanning (Section 2.1): compute the full distance, then compare;
 *   - Section 3.1: dis' = sqrt(D/d) * || y|[1..d] ||, with y = P'(o - q),
 *     sampling the first d coordinates;
 *   - Section 3.2: reject H0 (dis <= r) iff dis' > (1 + eps0/sqrt(d)) * r;
 *   - Algorithm 1 (Section 3.3): incremental sampling with the three cases,
 *     taking delta_d more coordinates per iteration (Section 6.1, Parameter
 *     Setting), the last step possibly shorter;
 *   - Section 2.2.2 (IVF): scan the candidates of the probed lists, keep a
 *     KNN max-heap of size K whose maximum is the threshold (+inf while the
 *     heap is not full), insert a candidate whose distance is below it;
 *   - Section 4 (AKNN+): the IVF scan with Algorithm 1 as its DCO.
 *   - Section 6.1 (Algorithms): PDScanning stops scanning raw coordinates
 *     as soon as the partial distance exceeds r.
 *
 * Readings where the paper is silent: ties in the heap are broken by the
 * lower id (insert iff (dis, id) is lexicographically below the heap maximum);
 * with eps0 = +inf or r = +inf no early rejection happens; the statistical test
 * is not applied once d = D (Case 3 is the exact comparison).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Single DCOs                                                               */
/* ------------------------------------------------------------------------ */

/* FDScanning: full-dimension distance, then the comparison with r. */
int orc_fds_dco(const double *o, const double *q, int D, double r, double *dist_out)
{
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        double y = o[i] - q[i];
        s += y * y;
    }
    double dis = sqrt(s);
    if (dis <= r) {
        *dist_out = dis;
        return 1;
    }
    *dist_out = INFINITY;
    return 0;
}

/*
 * Algorithm 1 (ADSampling) on transformed vectors o' and q'.
 * Returns 1 (positive, *dist_out = dis) or 0 (negative, *dist_out = +inf);
 * *dims_out receives the number of sampled coordinates.
 */
int orc_ads_dco(const double *o, const double *q, int D, double r, double eps0,
                int delta_d, int *dims_out, double *dist_out)
{
    int d = 0;          /* number of sampled coordinates */
    double sq = 0.0;    /* || y|[1..d] ||^2 */
    while (d < D) {
        /* sample delta_d more coordinates y_i = o'_i - q'_i */
        int e = d + delta_d < D ? d + delta_d : D;
        for (int i = d; i < e; ++i) {
            double y = o[i] - q[i];
            sq += y * y;
        }
        d = e;
        double dis_approx = sqrt((double)D / (double)d * sq);
        if (d < D) {
            /* hypothesis test of H0: dis <= r */
            int reject = 0;
            if (!isinf(eps0) && !isinf(r))
                reject = dis_approx > (1.0 + eps0 / sqrt((double)d)) * r;
            if (reject) {           /* Case 1 */
                *dims_out = d;
                *dist_out = INFINITY;
                return 0;
            }
            continue;               /* Case 2 */
        }
        /* Case 3: d = D, dis' is the exact distance */
        *dims_out = D;
        if (dis_approx <= r) {
            *dist_out = dis_approx;
            return 1;
        }
        *dist_out = INFINITY;
        return 0;
    }
    *dims_out = 0;      /* D == 0: nothing to sample */
    *dist_out = 0.0 <= r ? 0.0 : INFINITY;
    return 0.0 <= r;
}

/*
 * PDScanning (Section 6.1): scan raw coordinates and stop once the partial
 * distance sqrt(sum_{i<=d} x_i^2) exceeds r.  Exact; dims counted like above.
 */
int orc_pds_dco(const double *o, const double *q, int D, double r, int delta_d,
                int *dims_out, double *dist_out)
{
    int d = 0;
    double sq = 0.0;
    while (d < D) {
        int e = d + delta_d < D ? d + delta_d : D;
        for (int i = d; i < e; ++i) {
            double y = o[i] - q[i];
            sq += y * y;
        }
        d = e;
        if (sqrt(sq) > r) {
            *dims_out = d;
            *dist_out = INFINITY;
            return 0;
        }
    }
    *dims_out = D;
    *dist_out = sqrt(sq);
    return 1;
}

/*
 * Band flag for the parity criterion: 1 if, at some coordinate count d the
 * DCO reached, its estimate lies within rel * boundary of the boundary it is
 * compared with there.  ADSampling: dis' against gamma(d) * r for d < D and
 * against r at d = D.  FDScanning: dis against r.  PDScanning: the partial
 * distance against r at every step.
 */
int orc_band(const double *o, const double *q, int D, double r, double eps0,
             int delta_d, int method, double rel)
{
    if (isinf(r)) return 0;
    if (method == 1) { eps0 = INFINITY; delta_d = D; }
    int d = 0;
    double sq = 0.0;
    while (d < D) {
        int e = d + delta_d < D ? d + delta_d : D;
        for (int i = d; i < e; ++i) {
            double y = o[i] - q[i];
            sq += y * y;
        }
        d = e;
        double est, bound;
        if (method == 2) {
            est = sqrt(sq);
            bound = r;
        } else {
            est = sqrt((double)D / (double)d * sq);
            bound = d < D ? (isinf(eps0) ? INFINITY : (1.0 + eps0 / sqrt((double)d)) * r) : r;
        }
        if (isinf(bound)) continue;
        if (fabs(est - bound) <= rel * bound) return 1;
        if (d < D && est > bound) return 0;  /* the DCO stops here */
    }
    return 0;
}

/* dco over an explicit candidate list with a fixed r (rows index base). */
void orc_dco_batch(const double *base, int D, const double *q, const int64_t *rows,
                   int64_t m, double r, double eps0, int delta_d, int method,
                   uint8_t *mask, double *dist, int32_t *dims, uint8_t *band, double band_rel)
{
    for (int64_t i = 0; i < m; ++i) {
        const double *o = base + rows[i] * (int64_t)D;
        int dd = 0;
        double dv = 0.0;
        int pos;
        if (method == 0) {
            pos = orc_ads_dco(o, q, D, r, eps0, delta_d, &dd, &dv);
        } else if (method == 1) {
            pos = orc_fds_dco(o, q, D, r, &dv);
            dd = D;
        } else {
            pos = orc_pds_dco(o, q, D, r, delta_d, &dd, &dv);
        }
        mask[i] = (uint8_t)pos;
        dist[i] = dv;
        dims[i] = dd;
        if (band) band[i] = (uint8_t)orc_band(o, q, D, r, eps0, delta_d, method, band_rel);
    }
}

/* ------------------------------------------------------------------------ */
/* KNN set: a max-heap of size K keyed by (dis, id)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double dis;
    int64_t id;
} orc_item;

static int item_less(orc_item a, orc_item b)
{
    return a.dis < b.dis || (a.dis == b.dis && a.id < b.id);
}

static void heap_sift_up(orc_item *h, int i)
{
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!item_less(h[p], h[i])) break;
        orc_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static void heap_sift_down(orc_item *h, int n, int i)
{
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < n && item_less(h[m], h[l])) m = l;
        if (r < n && item_less(h[m], h[r])) m = r;
        if (m == i) return;
        orc_item t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
}

static int cmp_item(const void *a, const void *b)
{
    orc_item x = *(const orc_item *)a, y = *(const orc_item *)b;
    if (item_less(x, y)) return -1;
    if (item_less(y, x)) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* IVF scan (Section 2.2.2) with FDScanning / ADSampling / PDScanning DCOs   */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *base;      /* [rows][D] vectors (transformed for ADSampling) */
    const double *queries;   /* [nq][D] */
    int D;
    const int64_t *list_off; /* [nlist + 1] into list_rows / list_ids */
    const int64_t *list_rows;/* row of base for each stored candidate */
    const int64_t *list_ids; /* id reported for each stored candidate */
    const int32_t *probes;   /* [nq][nprobe_max] list ids, nearest first */
    const int32_t *nprobe;   /* [nq] */
    int nprobe_max;
    const int32_t *K;        /* [nq] */
    int k_max;
    double eps0;
    int delta_d;
    int method;              /* 0 ADSampling, 1 FDScanning, 2 PDScanning */
    int64_t *out_ids;        /* [nq][k_max] */
    double *out_dist;        /* [nq][k_max] */
    int64_t *stats;          /* [nq][3]: DCOs, sampled dims, positives */
    int nq;
    int next;                /* work counter (guarded by lock) */
    pthread_mutex_t lock;
} ivf_job;

static void ivf_one_query(ivf_job *job, int qi, orc_item *heap)
{
    const int D = job->D;
    const double *q = job->queries + (int64_t)qi * D;
    int K = job->K[qi];
    int hn = 0;
    int64_t dcos = 0, dims = 0, pos_cnt = 0;
    for (int p = 0; p < job->nprobe[qi]; ++p) {
        int32_t l = job->probes[(int64_t)qi * job->nprobe_max + p];
        for (int64_t c = job->list_off[l]; c < job->list_off[l + 1]; ++c) {
            const double *o = job->base + job->list_rows[c] * (int64_t)D;
            /* threshold: the maximum of the KNN set, +inf until it holds K */
            double r = (hn < K || K == 0) ? INFINITY : heap[0].dis;
            double dis;
            int dd, pos;
            if (K == 0) {
                pos = 0; dd = 0; dis = INFINITY;
            } else if (job->method == 0) {
                pos = orc_ads_dco(o, q, D, r, job->eps0, job->delta_d, &dd, &dis);
            } else if (job->method == 1) {
                pos = orc_fds_dco(o, q, D, r, &dis);
                dd = D;
            } else {
                pos = orc_pds_dco(o, q, D, r, job->delta_d, &dd, &dis);
            }
            dcos += 1;
            dims += dd;
            if (!pos) continue;
            pos_cnt += 1;
            orc_item it = { dis, job->list_ids[c] };
            if (hn < K) {
                heap[hn] = it;
                heap_sift_up(heap, hn);
                ++hn;
            } else if (item_less(it, heap[0])) {
                heap[0] = it;
                heap_sift_down(heap, hn, 0);
            }
        }
    }
    qsort(heap, (size_t)hn, sizeof(orc_item), cmp_item);
    for (int k = 0; k < job->k_max; ++k) {
        int64_t o = (int64_t)qi * job->k_max + k;
        if (k < hn && k < K) {
            job->out_ids[o] = heap[k].id;
            job->out_dist[o] = heap[k].dis;
        } else {
            job->out_ids[o] = -1;
            job->out_dist[o] = INFINITY;
        }
    }
    job->stats[3 * (int64_t)qi + 0] = dcos;
    job->stats[3 * (int64_t)qi + 1] = dims;
    job->stats[3 * (int64_t)qi + 2] = pos_cnt;
}

static void *ivf_worker(void *arg)
{
    ivf_job *job = (ivf_job *)arg;
    orc_item *heap = (orc_item *)malloc(sizeof(orc_item) * (size_t)(job->k_max > 0 ? job->k_max : 1));
    if (!heap) return NULL;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int qi = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (qi >= job->nq) break;
        ivf_one_query(job, qi, heap);
    }
    free(heap);
    return NULL;
}

/* Returns 0 on success, -1 on allocation failure. */
int orc_ivf_search(const double *base, const double *queries, int nq, int D,
                   const int64_t *list_off, const int64_t *list_rows, const int64_t *list_ids,
                   const int32_t *probes, const int32_t *nprobe, int nprobe_max,
                   const int32_t *K, int k_max, double eps0, int delta_d, int method,
                   int64_t *out_ids, double *out_dist, int64_t *stats, int threads)
{
    ivf_job job;
    memset(&job, 0, sizeof(job));
    job.base = base; job.queries = queries; job.D = D;
    job.list_off = list_off; job.list_rows = list_rows; job.list_ids = list_ids;
    job.probes = probes; job.nprobe = nprobe; job.nprobe_max = nprobe_max;
    job.K = K; job.k_max = k_max; job.eps0 = eps0; job.delta_d = delta_d;
    job.method = method; job.out_ids = out_ids; job.out_dist = out_dist;
    job.stats = stats; job.nq = nq; job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > nq) threads = nq > 0 ? nq : 1;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    if (!tid) return -1;
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, ivf_worker, &job) == 0) ++started;
    if (started == 0) ivf_worker(&job);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    pthread_mutex_destroy(&job.lock);
    return 0;
}
