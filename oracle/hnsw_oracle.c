/*
 * FP64 CPU oracle for graph search with ADSampling DCOs: HNSW, HNSW+ and
 * HNSW++.  TEST INFRASTRUCTURE ONLY: the GPU library never links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Plain sequential C99 in double precision, one query at a time (threads over
 * queries only).  What it follows:
 *
 *   - Section 2.2.1 (HNSW): a layered graph; greedy search from the top
 *     layer's entry vertex down to layer 1 (at each step all neighbours of the
 *     current vertex are examined and the search moves to the closest one if
 *     it is closer, until no neighbour is); at layer 0 a greedy beam search
 *     with a search set S (min by distance) and a result set R bounded by
 *     N_ef: pop the nearest entry of S, run a DCO for each not yet visited
 *     neighbour against the largest distance in R, push the neighbour into S
 *     and R when it is closer (evicting R's farthest beyond N_ef), stop when
 *     the nearest entry of S is farther than R's farthest; return the K
 *     nearest of R.
 *   - Section 4 (AKNN+): the same search with Algorithm 1 as its DCO (HNSW+).
 *   - Section 5.1 (HNSW++): R is split into R1 (K entries, exact distances;
 *     its largest distance is the DCO threshold and it holds the answer) and
 *     R2 (N_ef entries keyed by the distance each DCO observed when it
 *     stopped: exact at d = D, sqrt(D/d) * ||y|[1..d]|| when it rejected at
 *     d < D); S and R2 are maintained with the observed distances exactly as
 *     HNSW+ maintains S and R.
 *   - Algorithm 1 (Section 3.3) with delta_d coordinates per step and the
 *     test of Section 3.2, as in the IVF oracle.
 *
 * Readings where the paper is silent (each also stated where the GPU path
 * implements it):
 *   - every ordering is on (distance, id), lexicographically, so no two keys
 *     tie; "closer than R's farthest" means lexicographically below it;
 *   - the threshold of R (or R1) is +inf until the set is full, so the beam
 *     does not stop and DCOs do not reject before that;
 *   - with these keys an entry evicted from R can never be expanded later
 *     (R's farthest only shrinks), so S is exactly the set of R's members
 *     not yet expanded and the search ends when every member of R has been
 *     expanded -- the same sequence of expansions as the two-heap loop;
 *   - the upper layers use the same DCO (Algorithm 1 for HNSW+ / HNSW++,
 *     full distances for HNSW) with the current vertex's distance as the
 *     threshold, and the neighbours of the vertex the pass started from are
 *     examined in stored order with the threshold updated after each move;
 *   - the entry vertex's distance is a full DCO (threshold +inf), counted;
 *     the layer-0 beam starts from the vertex the upper layers end at, with
 *     the distance already known (no second DCO);
 *   - a vertex is DCO'd at most once in layer 0 (visited set), but may be
 *     DCO'd again in every upper-layer pass that examines it.
 *
 * Graph format (also the GPU path's input): levels[n]; adj0[n][M0] layer-0
 * neighbour ids, -1 padded; for a vertex of level >= 1, its layer-l row is
 * up_adj[(up_off[v] + l - 1) * M .. + M), -1 padded; entry = the vertex the
 * search starts from at the top layer max_level.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* One DCO: Algorithm 1, reporting what HNSW++ needs                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int positive;   /* dis <= r */
    int dims;       /* coordinates sampled */
    double dis;     /* exact distance when dims == D, else +inf */
    double obs;     /* observed distance when the DCO stopped */
    int band;       /* a decision taken within rel of its boundary */
} hdco;

/*
 * method 0: Algorithm 1 (ADSampling) with eps0 and delta_d; method 1:
 * FDScanning.  r may be +inf.  The band flag is set when, at a point where the
 * DCO compares with a finite boundary, the compared value lies within
 * rel * boundary of it (rel_exact for the exact comparison at d = D).
 */
static hdco h_dco(const double *o, const double *q, int D, double r, double eps0, int delta_d,
                  int method, double rel, double rel_exact)
{
    hdco out;
    memset(&out, 0, sizeof(out));
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
        double est = sqrt((double)D / (double)d * sq);
        if (d < D) {
            if (isinf(eps0) || isinf(r)) continue;     /* no test */
            double bound = (1.0 + eps0 / sqrt((double)d)) * r;
            if (fabs(est - bound) <= rel * bound) out.band = 1;
            if (est > bound) {                          /* Case 1: reject */
                out.positive = 0;
                out.dims = d;
                out.dis = INFINITY;
                out.obs = est;
                return out;
            }
            continue;                                   /* Case 2 */
        }
        /* Case 3: exact */
        if (!isinf(r) && rel_exact > 0.0 && fabs(est - r) <= rel_exact * r) out.band = 1;
        out.positive = est <= r;
        out.dims = D;
        out.dis = est;
        out.obs = est;
        return out;
    }
    out.positive = 1;
    out.obs = out.dis = 0.0;
    return out;
}

/* ------------------------------------------------------------------------ */
/* Sorted sets keyed by (distance, id)                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double key;
    int64_t id;
    int exact;      /* key is an exact distance */
    int expanded;   /* layer-0 beam: already popped from S */
} hent;

typedef struct {
    hent *e;
    int n, cap;
} hset;

static int key_less(double ka, int64_t ia, double kb, int64_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

/* Threshold of a bounded set: its largest key once full, +inf before. */
static double hset_threshold(const hset *s)
{
    return s->n < s->cap ? INFINITY : s->e[s->n - 1].key;
}

/*
 * Near-tie flag for the parity criterion: a new key lies within rel of a key
 * already in the set with a different id, where a rounding difference could
 * change their order.  Exact keys are compared with rel_exact (0 when exact
 * distances are computed without rounding on both sides).
 */
static int hset_near(const hset *s, double k, int64_t id, int exact, double rel, double rel_exact)
{
    for (int i = 0; i < s->n; ++i) {
        if (s->e[i].id == id) continue;
        double t = (exact && s->e[i].exact) ? rel_exact : rel;
        double diff = fabs(s->e[i].key - k);
        double m = fabs(k) > fabs(s->e[i].key) ? fabs(k) : fabs(s->e[i].key);
        if (t > 0.0 && diff <= t * m) return 1;
    }
    return 0;
}

/* Inserts (k, id) when the set is not full or the key is below its largest;
 * returns the position, or -1 when not inserted. */
static int hset_insert(hset *s, double k, int64_t id, int exact)
{
    if (s->cap == 0) return -1;
    if (s->n == s->cap && !key_less(k, id, s->e[s->n - 1].key, s->e[s->n - 1].id)) return -1;
    int p = 0;
    while (p < s->n && key_less(s->e[p].key, s->e[p].id, k, id)) ++p;
    int last = s->n < s->cap ? s->n : s->cap - 1;   /* the farthest falls off when full */
    for (int i = last; i > p; --i) s->e[i] = s->e[i - 1];
    s->e[p].key = k;
    s->e[p].id = id;
    s->e[p].exact = exact;
    s->e[p].expanded = 0;
    if (s->n < s->cap) ++s->n;
    return p;
}

/* ------------------------------------------------------------------------ */
/* Search                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *base;     /* [n][D] vectors (transformed for ADSampling) */
    const double *queries;  /* [nq][D] (transformed likewise) */
    int64_t n;
    int D;
    const int32_t *levels;
    const int32_t *adj0;
    int M0;
    const int64_t *up_off;
    const int32_t *up_adj;
    int M;
    int32_t entry;
    int max_level;
    int K, nef;
    double eps0;
    int delta_d;
    int variant;            /* 0 HNSW+, 1 HNSW (FDScanning), 2 HNSW++ */
    double rel, rel_exact;
    int64_t *out_ids;       /* [nq][K] */
    double *out_dist;       /* [nq][K] */
    int64_t *stats;         /* [nq][4]: DCOs, sampled dims, layer-0 expansions, band flag */
    int nq;
    int next;
    pthread_mutex_t lock;
} hnsw_job;

static void hnsw_one_query(hnsw_job *job, int qi, uint8_t *visited, hent *rbuf, hent *r1buf)
{
    const int D = job->D;
    const double *q = job->queries + (int64_t)qi * D;
    const int method = job->variant == 1 ? 1 : 0;
    int64_t dcos = 0, dims = 0, hops = 0;
    int band = 0;

    /* entry vertex: full distance */
    int64_t cur = job->entry;
    hdco c0 = h_dco(job->base + cur * D, q, D, INFINITY, job->eps0, job->delta_d, method, job->rel,
                    job->rel_exact);
    double dcur = c0.dis;
    dcos += 1;
    dims += c0.dims;

    /* upper layers: greedy descent */
    for (int l = job->max_level; l >= 1; --l) {
        int changed = 1;
        while (changed) {
            changed = 0;
            const int32_t *row = job->up_adj + (job->up_off[cur] + (l - 1)) * (int64_t)job->M;
            for (int j = 0; j < job->M && row[j] >= 0; ++j) {
                int64_t v = row[j];
                hdco c = h_dco(job->base + v * D, q, D, dcur, job->eps0, job->delta_d, method, job->rel,
                               job->rel_exact);
                dcos += 1;
                dims += c.dims;
                band |= c.band;
                if (!c.positive) continue;
                if (job->rel_exact > 0.0 && v != cur &&
                    fabs(c.dis - dcur) <= job->rel_exact * (c.dis > dcur ? c.dis : dcur))
                    band = 1;
                if (key_less(c.dis, v, dcur, cur)) {
                    cur = v;
                    dcur = c.dis;
                    changed = 1;
                }
            }
        }
    }

    /* layer 0: beam search */
    memset(visited, 0, (size_t)job->n);
    hset R = { rbuf, 0, job->nef };
    hset R1 = { r1buf, 0, job->K };
    visited[cur] = 1;
    hset_insert(&R, dcur, cur, 1);
    if (job->variant == 2) hset_insert(&R1, dcur, cur, 1);
    for (;;) {
        int p = 0;
        while (p < R.n && R.e[p].expanded) ++p;
        if (p == R.n) break;            /* S is empty */
        R.e[p].expanded = 1;
        int64_t u = R.e[p].id;
        hops += 1;
        const int32_t *row = job->adj0 + u * (int64_t)job->M0;
        for (int j = 0; j < job->M0 && row[j] >= 0; ++j) {
            int64_t v = row[j];
            if (visited[v]) continue;
            visited[v] = 1;
            double r = job->variant == 2 ? hset_threshold(&R1) : hset_threshold(&R);
            hdco c = h_dco(job->base + v * D, q, D, r, job->eps0, job->delta_d, method, job->rel,
                           job->rel_exact);
            dcos += 1;
            dims += c.dims;
            band |= c.band;
            if (job->variant != 2) {
                if (!c.positive) continue;
                band |= hset_near(&R, c.dis, v, 1, job->rel, job->rel_exact);
                hset_insert(&R, c.dis, v, 1);
            } else {
                if (c.positive) {
                    band |= hset_near(&R1, c.dis, v, 1, job->rel, job->rel_exact);
                    hset_insert(&R1, c.dis, v, 1);
                }
                int exact = c.dims == D;
                band |= hset_near(&R, c.obs, v, exact, job->rel, job->rel_exact);
                hset_insert(&R, c.obs, v, exact);
            }
        }
    }

    const hset *res = job->variant == 2 ? &R1 : &R;
    for (int k = 0; k < job->K; ++k) {
        int64_t o = (int64_t)qi * job->K + k;
        if (k < res->n) {
            job->out_ids[o] = res->e[k].id;
            job->out_dist[o] = res->e[k].key;
        } else {
            job->out_ids[o] = -1;
            job->out_dist[o] = INFINITY;
        }
    }
    job->stats[4 * (int64_t)qi + 0] = dcos;
    job->stats[4 * (int64_t)qi + 1] = dims;
    job->stats[4 * (int64_t)qi + 2] = hops;
    job->stats[4 * (int64_t)qi + 3] = band;
}

static void *hnsw_worker(void *arg)
{
    hnsw_job *job = (hnsw_job *)arg;
    uint8_t *visited = (uint8_t *)malloc((size_t)job->n);
    hent *rbuf = (hent *)malloc(sizeof(hent) * (size_t)(job->nef > 0 ? job->nef : 1));
    hent *r1buf = (hent *)malloc(sizeof(hent) * (size_t)(job->K > 0 ? job->K : 1));
    if (visited && rbuf && r1buf) {
        for (;;) {
            pthread_mutex_lock(&job->lock);
            int qi = job->next++;
            pthread_mutex_unlock(&job->lock);
            if (qi >= job->nq) break;
            hnsw_one_query(job, qi, visited, rbuf, r1buf);
        }
    }
    free(visited);
    free(rbuf);
    free(r1buf);
    return NULL;
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int orc_hnsw_search(const double *base, int64_t n, int D, const double *queries, int nq,
                    const int32_t *levels, const int32_t *adj0, int M0,
                    const int64_t *up_off, const int32_t *up_adj, int M,
                    int32_t entry, int max_level, int K, int nef, double eps0, int delta_d,
                    int variant, double rel, double rel_exact,
                    int64_t *out_ids, double *out_dist, int64_t *stats, int threads)
{
    if (n <= 0 || D <= 0 || K < 1 || nef < 1 || entry < 0 || entry >= n) return -1;
    if (variant != 2 && nef < K) return -1;
    if (levels[entry] < max_level) return -1;
    hnsw_job job;
    memset(&job, 0, sizeof(job));
    job.base = base; job.queries = queries; job.n = n; job.D = D;
    job.levels = levels; job.adj0 = adj0; job.M0 = M0; job.up_off = up_off;
    job.up_adj = up_adj; job.M = M; job.entry = entry; job.max_level = max_level;
    job.K = K; job.nef = nef; job.eps0 = eps0; job.delta_d = delta_d;
    job.variant = variant; job.rel = rel; job.rel_exact = rel_exact;
    job.out_ids = out_ids; job.out_dist = out_dist; job.stats = stats;
    job.nq = nq; job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > nq) threads = nq > 0 ? nq : 1;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    if (!tid) return -1;
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], NULL, hnsw_worker, &job) == 0) ++started;
    if (started == 0) hnsw_worker(&job);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    pthread_mutex_destroy(&job.lock);
    return 0;
}

/* Algorithm 1 as the graph search runs it, exposed for the pins: returns the
 * positive flag; dims, exact distance (+inf when stopped early), observed
 * distance and band flag through the pointers. */
int orc_hnsw_dco(const double *o, const double *q, int D, double r, double eps0, int delta_d,
                 int method, double rel, int *dims, double *dis, double *obs, int *band)
{
    hdco c = h_dco(o, q, D, r, eps0, delta_d, method, rel, rel);
    *dims = c.dims;
    *dis = c.dis;
    *obs = c.obs;
    *band = c.band;
    return c.positive;
}
