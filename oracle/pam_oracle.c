/*
 * pam_oracle.c -- plain, slow, obviously-correct CPU reference of PAM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * What it computes (Schubert & Rousseeuw, "Fast and Eager k-Medoids
 * Clustering", arXiv 2008.05171):
 *   - the total deviation TD                         (Sec. 2, Eq. td)
 *   - PAM BUILD, the greedy initialisation           (Sec. 2, Alg. 1)
 *   - the per-object loss change of a swap           (Sec. 3, Eq. change)
 *   - PAM SWAP, best-swap steepest descent           (Sec. 2, Alg. 2)
 *   - the best-swap-per-medoid eager variant that the paper calls FastPAM2
 *     (Sec. 3.2, one sentence, no pseudocode), in the reading stated below
 *   - FasterPAM, eager swapping of each improving candidate   (Sec. 3.2, Alg. 4)
 *   - distance-weighted seeding and LAB                        (Sec. 3.3)
 *   - one FastCLARANS local search over given random draws     (Sec. 3.4)
 *   - BUILD and PAM SWAP for bichromatic medoids, separate consumers and
 *     locations                                                (Sec. 5).
 *
 * FastPAM1 (Alg. 3) performs exactly the swaps of PAM (Sec. 3.1), so the
 * plain definition -- original PAM with Eq. change -- is the reference for it.
 *
 * All arithmetic is FP64.  For integer dissimilarities every intermediate
 * value is an integer below 2^53, so FP64 is exact there.
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes of the repository):
 *   R1 BUILD self-term: by default the candidate's own gain -dn(c) is added
 *      to its change, so each BUILD step picks the candidate that lowers TD
 *      most (Sec. 2 text and the TD update of Alg. 1).  exclude_self=1 gives
 *      the literal loop bounds of Alg. 1, which skip x_c.
 *   R2, R3 Ties: every argmin keeps the first minimum in ascending order
 *      (strict "<"), BUILD over c, SWAP over (slot i, then c) as in Alg. 2.
 *   R4 A swap keeps the slot: the new medoid takes the removed one's slot.
 *   R5 nearest(o) is the smallest slot at the minimum distance; ds(o) is the
 *      minimum over all other slots (it equals dn(o) on ties).
 *   R6 FastPAM2: one search gives, per slot i, the best candidate c*_i
 *      (first minimum over ascending c).  Slots with a negative best are
 *      visited in order of (delta, i); a visit is skipped when c*_i has become
 *      a medoid meanwhile, otherwise the change of swapping (i, c*_i) is
 *      evaluated again against the current medoids and the swap is applied
 *      when that change is negative.  Converged when a search finds no
 *      negative change.
 *   R8 k == 1: SWAP is not run (the second-nearest distance does not exist);
 *      BUILD's first medoid is the medoid of the whole set (Eq. def-medoid).
 *   R13 FasterPAM (Alg. 4), with the misprints of its listing read as fixed:
 *      the candidate that was swapped in is the one remembered as the last
 *      swap, and a scan that has made no swap at all ends after one full
 *      pass.  Candidates are visited in ascending index order, cyclically,
 *      current medoids skipped.  For the visited candidate c every slot's
 *      change Delta(i, c) is evaluated against the current medoids (the sum
 *      of Eq. change, which Alg. 4 computes as the removal loss plus the
 *      shared accumulator); i* is the smallest slot with the minimum, and the
 *      swap (i*, c) is applied at once when its change is negative.  The run
 *      ends when n consecutive positions have been visited without a swap
 *      (the scan is back at the last swap's position).  Iterations count the
 *      passes begun: ceil(positions visited / n).
 *   R14 Distance-weighted seeding (Sec. 3.3, the k-means++ idea with the
 *      distance to the nearest seed as weight, the k-medoids loss term):
 *      the first seed is floor(u_0 n); seed t is the first object, in index
 *      order, whose running weight sum exceeds u_t W (W = sum of weights,
 *      summed in index order); seeds weigh 0 and are never picked again.
 *      If W = 0 the smallest-index non-seed is taken.  The uniforms u_t in
 *      [0, 1) are inputs.
 *   R15 LAB (Sec. 3.3): each BUILD step is restricted to a subsample supplied
 *      by the caller (10 + ceil(sqrt n) points, distinct): its non-medoid
 *      members are the candidates, in the order listed, and its members the
 *      objects of the change (self-term as in R1); the first strict minimum
 *      is taken.  If every member is a medoid the smallest-index non-medoid
 *      is taken.  With the whole data set listed in index order every step
 *      equals BUILD's.
 *   R16 FastCLARANS (Sec. 3.4): one local search from given medoids over a
 *      list of random draws supplied by the caller.  A draw that is a medoid
 *      is skipped; otherwise it is a candidate like in Alg. 4 (best slot,
 *      smallest on ties, swapped in when its change is negative).  Draws
 *      that do not improve count as failures; a swap resets the count.  The
 *      search ends when maxneighbor failures follow each other (a local
 *      optimum for the sampled neighbourhood) or when the list runs out
 *      (reported as not converged).  Restarts are separate searches.
 *   R17 Bichromatic medoids (Sec. 5): consumers C (the objects) and
 *      possible locations L (the candidates) are separate sets; D is the
 *      |C| x |L| matrix of consumer-location distances; the k medoids are
 *      locations and TD sums each consumer's distance to its nearest
 *      medoid.  BUILD and SWAP keep their steps (Alg. 1, Alg. 2, Eq. change)
 *      with objects = consumers and candidates = locations; no object is a
 *      candidate, so there is no self-term (with C = L and a symmetric D
 *      this is the one-set method with the self-term of R1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_MEM (-2)
#define ORC_ERR_TD (-3)      /* running TD disagrees with a fresh sum */
#define ORC_WARN_MAXITER 1

/* ------------------------------------------------------------------ */
/* Dissimilarity source: a dense n x n matrix, or points and a metric. */
/* ------------------------------------------------------------------ */
typedef struct {
    const double *D;  /* row-major n x n, D[o*n + c] = d(x_o, x_c); may be NULL */
    const double *X;  /* row-major n x dim points, used when D is NULL */
    int64_t n;
    int32_t dim;
    int32_t metric;   /* 1 = Manhattan (L1), 2 = Euclidean (L2), 3 = the Euclidean
                         distance rounded to the nearest FP32 value (the
                         entries of an FP32 dissimilarity matrix) */
} src_t;

static double dist(const src_t *s, int64_t a, int64_t b)
{
    if (s->D) return s->D[a * s->n + b];
    const double *x = s->X + a * (int64_t)s->dim;
    const double *y = s->X + b * (int64_t)s->dim;
    double acc = 0.0;
    if (s->metric == 1) {
        for (int32_t j = 0; j < s->dim; ++j) acc += fabs(x[j] - y[j]);
        return acc;
    }
    for (int32_t j = 0; j < s->dim; ++j) {
        double t = x[j] - y[j];
        acc += t * t;
    }
    if (s->metric == 3) return (double)(float)sqrt(acc);
    return sqrt(acc);
}

static int make_src(src_t *s, const double *D, const double *X, int64_t n,
                    int32_t dim, int32_t metric)
{
    if (n < 1) return ORC_ERR_ARG;
    if (!D && (!X || dim < 1 || metric < 1 || metric > 3)) return ORC_ERR_ARG;
    s->D = D; s->X = X; s->n = n; s->dim = dim; s->metric = metric;
    return ORC_OK;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops that follow (t >= 1); returns the
 * count now in effect. */
int orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t >= 1) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* Full dissimilarity matrix from points (L1 or L2), FP64. */
int orc_dist_matrix(const double *X, int64_t n, int32_t dim, int32_t metric, double *D)
{
    src_t s;
    if (!D || make_src(&s, NULL, X, n, dim, metric)) return ORC_ERR_ARG;
    #pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b < n; ++b)
            D[a * n + b] = dist(&s, a, b);
    return ORC_OK;
}

/* Selected rows of the dissimilarity matrix: out[j*n + b] = d(x_rows[j], x_b). */
int orc_dist_rows(const double *X, int64_t n, int32_t dim, int32_t metric,
                  const int64_t *rows, int64_t m, double *out)
{
    src_t s;
    if (!out || !rows || m < 0 || make_src(&s, NULL, X, n, dim, metric)) return ORC_ERR_ARG;
    for (int64_t j = 0; j < m; ++j)
        if (rows[j] < 0 || rows[j] >= n) return ORC_ERR_ARG;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t b = 0; b < n; ++b)
            out[j * n + b] = dist(&s, rows[j], b);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Nearest / second-nearest medoid of every object (reading R5).        */
/* ------------------------------------------------------------------ */
static void nearest_all(const src_t *s, const int32_t *med, int32_t k,
                        int32_t *near, double *dn, double *ds)
{
    #pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < s->n; ++o) {
        int32_t bi = 0;
        double bd = dist(s, o, med[0]);
        for (int32_t i = 1; i < k; ++i) {
            double d = dist(s, o, med[i]);
            if (d < bd) { bd = d; bi = i; }
        }
        double sd = INFINITY;
        for (int32_t i = 0; i < k; ++i) {
            if (i == bi) continue;
            double d = dist(s, o, med[i]);
            if (d < sd) sd = d;
        }
        near[o] = bi;
        dn[o] = bd;
        ds[o] = sd;
    }
}

int orc_nearest(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                const int32_t *med, int32_t k, int32_t *near, double *dn, double *ds)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 1 || !near || !dn || !ds)
        return ORC_ERR_ARG;
    nearest_all(&s, med, k, near, dn, ds);
    return ORC_OK;
}

/* Total deviation TD = sum over objects of the distance to the nearest
 * medoid (Eq. td), summed in ascending object order.  labels optional. */
double orc_td(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
              const int32_t *med, int32_t k, int32_t *labels)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 1) return NAN;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!dn || !ds || !near) { free(dn); free(ds); free(near); return NAN; }
    nearest_all(&s, med, k, near, dn, ds);
    double td = 0.0;
    for (int64_t o = 0; o < n; ++o) td += dn[o];
    if (labels) memcpy(labels, near, sizeof(int32_t) * (size_t)n);
    free(dn); free(ds); free(near);
    return td;
}

/* ------------------------------------------------------------------ */
/* Eq. change: loss change of object o when medoid m_i is replaced by x_c.
 *   d     = d(x_o, x_c)
 *   is_i  = (nearest(o) == i)
 *   dn,ds = distances of o to its nearest and second-nearest medoid     */
/* ------------------------------------------------------------------ */
double orc_change(double d, int32_t is_i, double dn, double ds)
{
    if (!is_i) {
        if (d >= dn) return 0.0;          /* case (a): stays with its medoid  */
        return d - dn;                    /* case (c): moves to x_c           */
    }
    if (d < ds) return d - dn;            /* case (b1): m_i removed, x_c wins */
    return ds - dn;                       /* case (b2): goes to second nearest */
}

/* Delta TD of replacing the medoid in slot i by x_c, given the caches:
 * the sum of Eq. change over every x_o that is not one of the other medoids
 * (Alg. 2 inner loop). */
static double delta_swap(const src_t *s, const int32_t *med, int32_t k,
                         const unsigned char *is_med, const int32_t *near,
                         const double *dn, const double *ds, int32_t i, int64_t c)
{
    double acc = 0.0;
    for (int64_t o = 0; o < s->n; ++o) {
        if (is_med[o] && o != med[i]) continue;
        acc += orc_change(dist(s, o, c), near[o] == i, dn[o], ds[o]);
    }
    (void)k;
    return acc;
}

static unsigned char *medoid_mask(int64_t n, const int32_t *med, int32_t k)
{
    unsigned char *m = (unsigned char *)calloc((size_t)n, 1);
    if (!m) return NULL;
    for (int32_t i = 0; i < k; ++i) m[med[i]] = 1;
    return m;
}

/* Delta TD of the single swap (slot i, candidate c) for the medoid set med. */
double orc_delta(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                 const int32_t *med, int32_t k, int32_t i, int64_t c)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 2 || i < 0 || i >= k || c < 0 || c >= n)
        return NAN;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char *is_med = medoid_mask(n, med, k);
    double r = NAN;
    if (dn && ds && near && is_med) {
        nearest_all(&s, med, k, near, dn, ds);
        r = is_med[c] ? NAN : delta_swap(&s, med, k, is_med, near, dn, ds, i, c);
    }
    free(dn); free(ds); free(near); free(is_med);
    return r;
}

/* ------------------------------------------------------------------ */
/* PAM BUILD (Alg. 1) with reading R1 for the self-term.                */
/* ------------------------------------------------------------------ */
int orc_build(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
              int32_t k, int32_t exclude_self, int32_t *med, double *td_out,
              double *step_delta /* optional [k]: change chosen at each step */)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || k < 1 || k > n || !med) return ORC_ERR_ARG;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *chg = (double *)malloc(sizeof(double) * (size_t)n);
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    if (!dn || !chg || !is_med) { free(dn); free(chg); free(is_med); return ORC_ERR_MEM; }

    /* First medoid: smallest sum of distances to all other objects. */
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double sum = 0.0;
        for (int64_t o = 0; o < n; ++o)
            if (o != c) sum += dist(&s, o, c);
        chg[c] = sum;
    }
    int64_t m1 = -1;
    double best = INFINITY;
    for (int64_t c = 0; c < n; ++c)
        if (chg[c] < best) { best = chg[c]; m1 = c; }
    med[0] = (int32_t)m1;
    is_med[m1] = 1;
    if (step_delta) step_delta[0] = best;
    for (int64_t o = 0; o < n; ++o) dn[o] = (o == m1) ? 0.0 : dist(&s, m1, o);

    /* Remaining medoids: the candidate with the most negative change. */
    for (int32_t t = 1; t < k; ++t) {
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c) {
            if (is_med[c]) continue;
            double acc = 0.0;
            for (int64_t o = 0; o < n; ++o) {
                if (is_med[o] || o == c) continue;
                double delta = dist(&s, o, c) - dn[o];
                if (delta < 0.0) acc += delta;
            }
            if (!exclude_self) acc -= dn[c];   /* x_c itself drops to distance 0 */
            chg[c] = acc;
        }
        int64_t bc = -1;
        double bd = INFINITY;
        for (int64_t c = 0; c < n; ++c)
            if (!is_med[c] && chg[c] < bd) { bd = chg[c]; bc = c; }
        med[t] = (int32_t)bc;
        is_med[bc] = 1;
        if (step_delta) step_delta[t] = bd;
        for (int64_t o = 0; o < n; ++o) {
            if (o == bc) { dn[o] = 0.0; continue; }
            if (is_med[o]) continue;
            double d = dist(&s, o, bc);
            if (d < dn[o]) dn[o] = d;
        }
    }
    if (td_out) {
        double td = 0.0;   /* recomputed, not the running sum */
        for (int64_t o = 0; o < n; ++o) td += dn[o];
        *td_out = td;
    }
    free(dn); free(chg); free(is_med);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* SWAP search: the change of every (slot, candidate) pair.             */
/* tab[i*n + c] = Delta TD of swap (i, c); NAN where c is a medoid.     */
/* ------------------------------------------------------------------ */
static void swap_table(const src_t *s, const int32_t *med, int32_t k,
                       const unsigned char *is_med, const int32_t *near,
                       const double *dn, const double *ds,
                       int64_t c_begin, int64_t c_end, double *tab)
{
    const int64_t n = s->n;
    #pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int32_t i = 0; i < k; ++i)
        for (int64_t c = c_begin; c < c_end; ++c)
            tab[(int64_t)i * n + c] =
                is_med[c] ? NAN : delta_swap(s, med, k, is_med, near, dn, ds, i, c);
}

/* One SWAP search over candidates in [c_begin, c_end): the best swap in the
 * order of Alg. 2 (slot outer, candidate inner, strict "<", start at 0).
 * Returns 1 if an improving swap exists, 0 if not, <0 on error. */
int orc_swap_search(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                    const int32_t *med, int32_t k, int64_t c_begin, int64_t c_end,
                    double *best_delta, int32_t *best_slot, int64_t *best_c)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 2 || k > n ||
        c_begin < 0 || c_end > n || c_begin > c_end)
        return ORC_ERR_ARG;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *tab = (double *)malloc(sizeof(double) * (size_t)n * (size_t)k);
    unsigned char *is_med = medoid_mask(n, med, k);
    int rc = ORC_ERR_MEM;
    if (dn && ds && near && tab && is_med) {
        nearest_all(&s, med, k, near, dn, ds);
        swap_table(&s, med, k, is_med, near, dn, ds, c_begin, c_end, tab);
        double bd = 0.0;
        int32_t bi = -1;
        int64_t bc = -1;
        for (int32_t i = 0; i < k; ++i)
            for (int64_t c = c_begin; c < c_end; ++c) {
                if (is_med[c]) continue;
                double v = tab[(int64_t)i * n + c];
                if (v < bd) { bd = v; bi = i; bc = c; }
            }
        if (best_delta) *best_delta = bd;
        if (best_slot) *best_slot = bi;
        if (best_c) *best_c = bc;
        rc = (bi >= 0) ? 1 : 0;
    }
    free(dn); free(ds); free(near); free(tab); free(is_med);
    return rc;
}

static int td_matches(double running, double fresh)
{
    double tol = 1e-9 * fabs(fresh) + 1e-9;
    return fabs(running - fresh) <= tol;
}

/* ------------------------------------------------------------------ */
/* Changes for a listed set of candidates, so that single steps of a    */
/* large run can be checked without a full search.                      */
/* ------------------------------------------------------------------ */

/* SWAP: out[j*k + i] = Delta TD of replacing the medoid in slot i by
 * cand[j], the sum of Eq. change over the objects of Alg. 2's inner loop
 * (ascending object order, as in a full search).  NAN where cand[j] is a
 * medoid. */
int orc_swap_list(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                  const int32_t *med, int32_t k, const int64_t *cand, int64_t m, double *out)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 2 || k > n || !cand || m < 0 || !out)
        return ORC_ERR_ARG;
    for (int64_t j = 0; j < m; ++j)
        if (cand[j] < 0 || cand[j] >= n) return ORC_ERR_ARG;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char *is_med = medoid_mask(n, med, k);
    if (!dn || !ds || !near || !is_med) {
        free(dn); free(ds); free(near); free(is_med);
        return ORC_ERR_MEM;
    }
    nearest_all(&s, med, k, near, dn, ds);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < m; ++j) {
        double *acc = out + j * (int64_t)k;
        const int64_t c = cand[j];
        for (int32_t i = 0; i < k; ++i) acc[i] = is_med[c] ? NAN : 0.0;
        if (is_med[c]) continue;
        for (int64_t o = 0; o < n; ++o) {
            const double d = dist(&s, o, c);
            for (int32_t i = 0; i < k; ++i) {
                if (is_med[o] && o != med[i]) continue;
                acc[i] += orc_change(d, near[o] == i, dn[o], ds[o]);
            }
        }
    }
    free(dn); free(ds); free(near); free(is_med);
    return ORC_OK;
}

/* BUILD (Alg. 1): the change of taking cand[j] as the next medoid after
 * med[0..t-1].  t == 0 gives the first step's sum of distances to all other
 * objects.  Self-term by reading R1 (exclude_self selects the literal loop
 * bounds).  NAN where cand[j] is already a medoid. */
int orc_build_list(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                   const int32_t *med, int32_t t, int32_t exclude_self, const int64_t *cand,
                   int64_t m, double *out)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || t < 0 || t >= n || (t > 0 && !med) || !cand ||
        m < 0 || !out)
        return ORC_ERR_ARG;
    for (int64_t j = 0; j < m; ++j)
        if (cand[j] < 0 || cand[j] >= n) return ORC_ERR_ARG;
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!is_med || !dn) { free(is_med); free(dn); return ORC_ERR_MEM; }
    for (int32_t i = 0; i < t; ++i) {
        if (med[i] < 0 || med[i] >= n || is_med[med[i]]) { free(is_med); free(dn); return ORC_ERR_ARG; }
        is_med[med[i]] = 1;
    }
    /* distance of every object to its nearest chosen medoid (0 for medoids) */
    #pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n; ++o) {
        double best = INFINITY;
        if (is_med[o]) best = 0.0;
        else
            for (int32_t i = 0; i < t; ++i) {
                double d = dist(&s, o, med[i]);
                if (d < best) best = d;
            }
        dn[o] = best;
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < m; ++j) {
        const int64_t c = cand[j];
        if (is_med[c]) { out[j] = NAN; continue; }
        double acc = 0.0;
        if (t == 0) {
            for (int64_t o = 0; o < n; ++o)
                if (o != c) acc += dist(&s, o, c);
        } else {
            for (int64_t o = 0; o < n; ++o) {
                if (is_med[o] || o == c) continue;
                double delta = dist(&s, o, c) - dn[o];
                if (delta < 0.0) acc += delta;
            }
            if (!exclude_self) acc -= dn[c];
        }
        out[j] = acc;
    }
    free(is_med); free(dn);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* PAM SWAP (Alg. 2), the FastPAM2 reading R6 and FasterPAM (R13).     */
/*   variant 1 = best swap per iteration (PAM; FastPAM1 gives the same) */
/*   variant 2 = best swap per medoid, applied eagerly (reading R6)     */
/*   variant 3 = FasterPAM, Alg. 4: first improving candidate in scan   */
/*               order, its best slot, applied at once (reading R13)     */
/* med is read (slot order) and overwritten with the result.            */
/* trace_* (optional, capacity trace_cap) receive every applied swap.   */
/* ------------------------------------------------------------------ */
int orc_swap(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
             int32_t *med, int32_t k, int32_t variant, int32_t max_iter,
             int32_t *trace_slot, int64_t *trace_c, double *trace_delta, int32_t trace_cap,
             int32_t *n_iter, int32_t *n_swaps, double *td_out)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 1 || k > n ||
        variant < 1 || variant > 3 || max_iter < 0)
        return ORC_ERR_ARG;
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    if (!is_med) return ORC_ERR_MEM;
    for (int32_t i = 0; i < k; ++i) {
        if (med[i] < 0 || med[i] >= n || is_med[med[i]]) { free(is_med); return ORC_ERR_ARG; }
        is_med[med[i]] = 1;
    }
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *tab = (k >= 2) ? (double *)malloc(sizeof(double) * (size_t)n * (size_t)k) : NULL;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    double *bdel = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t *bcand = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!dn || !ds || !near || (k >= 2 && !tab) || !order || !bdel || !bcand) {
        free(is_med); free(dn); free(ds); free(near); free(tab); free(order); free(bdel); free(bcand);
        return ORC_ERR_MEM;
    }

    int rc = ORC_OK;
    int32_t iters = 0, swaps = 0;
    nearest_all(&s, med, k, near, dn, ds);
    double td = 0.0;
    for (int64_t o = 0; o < n; ++o) td += dn[o];

    if (variant == 3 && k >= 2 && k < n) {
        /* reading R13: one candidate at a time, in scan order */
        int64_t pos = 0, visited = 0, quiet = 0;
        while (quiet < n) {
            if (visited == (int64_t)max_iter * n) { rc = ORC_WARN_MAXITER; break; }
            const int64_t c = pos;
            pos = (pos + 1 == n) ? 0 : pos + 1;
            ++visited;
            ++quiet;
            if (is_med[c]) continue;
            #pragma omp parallel for schedule(static) if (k >= 8)
            for (int32_t i = 0; i < k; ++i)
                bdel[i] = delta_swap(&s, med, k, is_med, near, dn, ds, i, c);
            int32_t bi = 0;
            for (int32_t i = 1; i < k; ++i)
                if (bdel[i] < bdel[bi]) bi = i;
            const double bd = bdel[bi];
            if (!(bd < 0.0)) continue;
            is_med[med[bi]] = 0;
            med[bi] = (int32_t)c;
            is_med[c] = 1;
            td += bd;
            if (trace_slot && swaps < trace_cap) {
                trace_slot[swaps] = bi; trace_c[swaps] = c; trace_delta[swaps] = bd;
            }
            ++swaps;
            quiet = 0;
            nearest_all(&s, med, k, near, dn, ds);
            double fresh = 0.0;
            for (int64_t o = 0; o < n; ++o) fresh += dn[o];
            if (!td_matches(td, fresh)) { rc = ORC_ERR_TD; break; }
            td = fresh;
        }
        iters = (int32_t)((visited + n - 1) / n);
    }

    while (variant != 3 && k >= 2 && k < n) {
        if (iters >= max_iter) { rc = ORC_WARN_MAXITER; break; }
        ++iters;
        swap_table(&s, med, k, is_med, near, dn, ds, 0, n, tab);
        int applied = 0;
        if (variant == 1) {
            double bd = 0.0;
            int32_t bi = -1;
            int64_t bc = -1;
            for (int32_t i = 0; i < k; ++i)
                for (int64_t c = 0; c < n; ++c) {
                    if (is_med[c]) continue;
                    double v = tab[(int64_t)i * n + c];
                    if (v < bd) { bd = v; bi = i; bc = c; }
                }
            if (bi < 0) break;   /* no swap lowers TD: converged */
            is_med[med[bi]] = 0;
            med[bi] = (int32_t)bc;
            is_med[bc] = 1;
            td += bd;
            if (trace_slot && swaps < trace_cap) {
                trace_slot[swaps] = bi; trace_c[swaps] = bc; trace_delta[swaps] = bd;
            }
            ++swaps;
            applied = 1;
            nearest_all(&s, med, k, near, dn, ds);
        } else {
            /* best candidate of every slot: first minimum over ascending c */
            int32_t m = 0;
            for (int32_t i = 0; i < k; ++i) {
                double bd = INFINITY;
                int64_t bc = -1;
                for (int64_t c = 0; c < n; ++c) {
                    if (is_med[c]) continue;
                    double v = tab[(int64_t)i * n + c];
                    if (v < bd) { bd = v; bc = c; }
                }
                bdel[i] = bd;
                bcand[i] = bc;
                if (bc >= 0 && bd < 0.0) order[m++] = i;
            }
            if (m == 0) break;
            /* visit slots by (delta, slot): insertion sort, stable on slot */
            for (int32_t a = 1; a < m; ++a) {
                int32_t v = order[a], b = a - 1;
                while (b >= 0 && bdel[order[b]] > bdel[v]) { order[b + 1] = order[b]; --b; }
                order[b + 1] = v;
            }
            for (int32_t a = 0; a < m; ++a) {
                int32_t i = order[a];
                int64_t c = bcand[i];
                if (is_med[c]) continue;
                double dcur = delta_swap(&s, med, k, is_med, near, dn, ds, i, c);
                if (!(dcur < 0.0)) continue;
                is_med[med[i]] = 0;
                med[i] = (int32_t)c;
                is_med[c] = 1;
                td += dcur;
                if (trace_slot && swaps < trace_cap) {
                    trace_slot[swaps] = i; trace_c[swaps] = c; trace_delta[swaps] = dcur;
                }
                ++swaps;
                applied = 1;
                nearest_all(&s, med, k, near, dn, ds);
            }
        }
        if (applied) {
            double fresh = 0.0;
            for (int64_t o = 0; o < n; ++o) fresh += dn[o];
            if (!td_matches(td, fresh)) { rc = ORC_ERR_TD; break; }
            td = fresh;
        }
    }
    if (n_iter) *n_iter = iters;
    if (n_swaps) *n_swaps = swaps;
    if (td_out) {
        double fresh = 0.0;
        for (int64_t o = 0; o < n; ++o) fresh += dn[o];
        *td_out = fresh;
    }
    free(is_med); free(dn); free(ds); free(near); free(tab); free(order); free(bdel); free(bcand);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Faster initialisations (Sec. 3.3): distance-weighted seeding (R14)    */
/* and LAB (R15).  med receives k object indices in slot order.          */
/* ------------------------------------------------------------------ */
int orc_init_dw(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                int32_t k, const double *u, int32_t *med)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || k < 1 || k > n || !u || !med) return ORC_ERR_ARG;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    if (!w || !is_med) { free(w); free(is_med); return ORC_ERR_MEM; }
    int64_t c = (int64_t)floor(u[0] * (double)n);
    if (c < 0) c = 0;
    if (c >= n) c = n - 1;
    med[0] = (int32_t)c;
    is_med[c] = 1;
    for (int64_t o = 0; o < n; ++o) w[o] = dist(&s, o, c);
    for (int32_t t = 1; t < k; ++t) {
        double W = 0.0;
        for (int64_t o = 0; o < n; ++o) W += w[o];
        const double target = u[t] * W;
        int64_t pick = -1;
        double run = 0.0;
        for (int64_t o = 0; o < n; ++o) {
            run += w[o];
            if (run > target) { pick = o; break; }
        }
        if (pick < 0)
            for (int64_t o = 0; o < n; ++o)
                if (!is_med[o]) { pick = o; break; }
        med[t] = (int32_t)pick;
        is_med[pick] = 1;
        for (int64_t o = 0; o < n; ++o) {
            const double d = dist(&s, o, pick);
            if (d < w[o]) w[o] = d;
        }
    }
    free(w); free(is_med);
    return ORC_OK;
}

int orc_init_lab(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                 int32_t k, const int32_t *samp, int32_t m, int32_t exclude_self, int32_t *med)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || k < 1 || k > n || !samp || m < 1 || !med)
        return ORC_ERR_ARG;
    for (int64_t j = 0; j < (int64_t)k * m; ++j)
        if (samp[j] < 0 || samp[j] >= n) return ORC_ERR_ARG;
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    if (!dn || !is_med) { free(dn); free(is_med); return ORC_ERR_MEM; }
    for (int64_t o = 0; o < n; ++o) dn[o] = INFINITY;
    for (int32_t t = 0; t < k; ++t) {
        const int32_t *S = samp + (int64_t)t * m;
        double best = INFINITY;
        int64_t bc = -1;
        for (int32_t j = 0; j < m; ++j) {
            const int64_t c = S[j];
            if (is_med[c]) continue;
            double acc = 0.0;
            for (int32_t jj = 0; jj < m; ++jj) {
                const int64_t o = S[jj];
                if (o == c) continue;
                if (t == 0) { acc += dist(&s, o, c); continue; }
                if (is_med[o]) continue;
                const double delta = dist(&s, o, c) - dn[o];
                if (delta < 0.0) acc += delta;
            }
            if (t > 0 && !exclude_self) acc -= dn[c];
            if (acc < best) { best = acc; bc = c; }
        }
        if (bc < 0)
            for (int64_t o = 0; o < n; ++o)
                if (!is_med[o]) { bc = o; break; }
        med[t] = (int32_t)bc;
        is_med[bc] = 1;
        for (int64_t o = 0; o < n; ++o) {
            const double d = dist(&s, o, bc);
            if (d < dn[o]) dn[o] = d;
        }
    }
    free(dn); free(is_med);
    return ORC_OK;
}

/* FastCLARANS local search (R16).  med (slot order) is read and
 * overwritten; trace_* (optional) receive the swaps; n_eval = draws
 * evaluated (non-medoid draws up to the end of the search). */
int orc_clarans(const double *D, const double *X, int64_t n, int32_t dim, int32_t metric,
                int32_t *med, int32_t k, const int32_t *draws, int64_t len, int64_t maxneighbor,
                int32_t *trace_slot, int64_t *trace_c, double *trace_delta, int32_t trace_cap,
                int64_t *n_eval, int32_t *n_swaps, double *td_out)
{
    src_t s;
    if (make_src(&s, D, X, n, dim, metric) || !med || k < 1 || k > n || !draws || len < 0 ||
        maxneighbor < 1)
        return ORC_ERR_ARG;
    for (int64_t j = 0; j < len; ++j)
        if (draws[j] < 0 || draws[j] >= n) return ORC_ERR_ARG;
    unsigned char *is_med = (unsigned char *)calloc((size_t)n, 1);
    double *dn = (double *)malloc(sizeof(double) * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *chg = (double *)malloc(sizeof(double) * (size_t)k);
    if (!is_med || !dn || !ds || !near || !chg) {
        free(is_med); free(dn); free(ds); free(near); free(chg);
        return ORC_ERR_MEM;
    }
    int rc = ORC_OK;
    for (int32_t i = 0; i < k; ++i) {
        if (med[i] < 0 || med[i] >= n || is_med[med[i]]) { rc = ORC_ERR_ARG; break; }
        is_med[med[i]] = 1;
    }
    int64_t evals = 0, fails = 0;
    int32_t swaps = 0;
    if (rc == ORC_OK && k >= 2 && k < n) {
        nearest_all(&s, med, k, near, dn, ds);
        double td = 0.0;
        for (int64_t o = 0; o < n; ++o) td += dn[o];
        int64_t j = 0;
        while (fails < maxneighbor) {
            if (j == len) { rc = ORC_WARN_MAXITER; break; }
            const int64_t c = draws[j++];
            if (is_med[c]) continue;
            ++evals;
            #pragma omp parallel for schedule(static) if (k >= 8)
            for (int32_t i = 0; i < k; ++i)
                chg[i] = delta_swap(&s, med, k, is_med, near, dn, ds, i, c);
            int32_t bi = 0;
            for (int32_t i = 1; i < k; ++i)
                if (chg[i] < chg[bi]) bi = i;
            if (!(chg[bi] < 0.0)) { ++fails; continue; }
            is_med[med[bi]] = 0;
            med[bi] = (int32_t)c;
            is_med[c] = 1;
            td += chg[bi];
            if (trace_slot && swaps < trace_cap) {
                trace_slot[swaps] = bi; trace_c[swaps] = c; trace_delta[swaps] = chg[bi];
            }
            ++swaps;
            fails = 0;
            nearest_all(&s, med, k, near, dn, ds);
            double fresh = 0.0;
            for (int64_t o = 0; o < n; ++o) fresh += dn[o];
            if (!td_matches(td, fresh)) { rc = ORC_ERR_TD; break; }
            td = fresh;
        }
    }
    if (n_eval) *n_eval = evals;
    if (n_swaps) *n_swaps = swaps;
    if (td_out && rc >= 0) {
        nearest_all(&s, med, k, near, dn, ds);
        double fresh = 0.0;
        for (int64_t o = 0; o < n; ++o) fresh += dn[o];
        *td_out = fresh;
    }
    free(is_med); free(dn); free(ds); free(near); free(chg);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Bichromatic medoids (R17): D is nc x nl, row-major (consumers x      */
/* locations); medoids are location indices.                           */
/* ------------------------------------------------------------------ */
static void rect_nearest(const double *D, int64_t nc, int64_t nl, const int32_t *med, int32_t k,
                         int32_t *near, double *dn, double *ds)
{
    #pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < nc; ++o) {
        double b1 = INFINITY, b2 = INFINITY;
        int32_t i1 = -1;
        for (int32_t i = 0; i < k; ++i) {
            const double d = D[o * nl + med[i]];
            if (d < b1) { b2 = b1; b1 = d; i1 = i; }
            else if (d < b2) b2 = d;
        }
        near[o] = i1; dn[o] = b1; ds[o] = b2;
    }
}

double orc_rect_td(const double *D, int64_t nc, int64_t nl, const int32_t *med, int32_t k,
                   int32_t *labels)
{
    if (!D || nc < 1 || nl < 1 || !med || k < 1) return NAN;
    double td = 0.0;
    for (int64_t o = 0; o < nc; ++o) {
        double b = INFINITY;
        int32_t bi = -1;
        for (int32_t i = 0; i < k; ++i) {
            const double d = D[o * nl + med[i]];
            if (d < b) { b = d; bi = i; }
        }
        td += b;
        if (labels) labels[o] = bi;
    }
    return td;
}

/* BUILD (Alg. 1) over locations: step 0 takes the location with the
 * smallest sum of distances to all consumers (the bichromatic medoid);
 * step t the location whose addition lowers TD most (first minimum). */
int orc_rect_build(const double *D, int64_t nc, int64_t nl, int32_t k, int32_t *med, double *td_out)
{
    if (!D || nc < 1 || nl < 1 || k < 1 || k > nl || !med) return ORC_ERR_ARG;
    double *dn = (double *)malloc(sizeof(double) * (size_t)nc);
    double *chg = (double *)malloc(sizeof(double) * (size_t)nl);
    unsigned char *is_med = (unsigned char *)calloc((size_t)nl, 1);
    if (!dn || !chg || !is_med) { free(dn); free(chg); free(is_med); return ORC_ERR_MEM; }
    for (int64_t o = 0; o < nc; ++o) dn[o] = INFINITY;
    for (int32_t t = 0; t < k; ++t) {
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nl; ++c) {
            if (is_med[c]) { chg[c] = NAN; continue; }
            double acc = 0.0;
            for (int64_t o = 0; o < nc; ++o) {
                const double d = D[o * nl + c];
                if (t == 0) acc += d;
                else if (d < dn[o]) acc += d - dn[o];
            }
            chg[c] = acc;
        }
        double best = INFINITY;
        int64_t bc = -1;
        for (int64_t c = 0; c < nl; ++c)
            if (!is_med[c] && chg[c] < best) { best = chg[c]; bc = c; }
        med[t] = (int32_t)bc;
        is_med[bc] = 1;
        for (int64_t o = 0; o < nc; ++o) {
            const double d = D[o * nl + bc];
            if (d < dn[o]) dn[o] = d;
        }
    }
    if (td_out) {
        double td = 0.0;
        for (int64_t o = 0; o < nc; ++o) td += dn[o];
        *td_out = td;
    }
    free(dn); free(chg); free(is_med);
    return ORC_OK;
}

/* PAM SWAP (Alg. 2) over locations: per search the best (change, slot,
 * location) with strict "<" in slot-outer, location-inner order; each
 * change the sum of Eq. change over all consumers. */
int orc_rect_swap(const double *D, int64_t nc, int64_t nl, int32_t *med, int32_t k,
                  int32_t max_iter, int32_t *trace_slot, int64_t *trace_c, double *trace_delta,
                  int32_t trace_cap, int32_t *n_iter, int32_t *n_swaps, double *td_out)
{
    if (!D || nc < 1 || nl < 1 || !med || k < 1 || k > nl || max_iter < 0) return ORC_ERR_ARG;
    unsigned char *is_med = (unsigned char *)calloc((size_t)nl, 1);
    if (!is_med) return ORC_ERR_MEM;
    for (int32_t i = 0; i < k; ++i) {
        if (med[i] < 0 || med[i] >= nl || is_med[med[i]]) { free(is_med); return ORC_ERR_ARG; }
        is_med[med[i]] = 1;
    }
    double *dn = (double *)malloc(sizeof(double) * (size_t)nc);
    double *ds = (double *)malloc(sizeof(double) * (size_t)nc);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
    double *tab = (double *)malloc(sizeof(double) * (size_t)nl * (size_t)k);
    if (!dn || !ds || !near || !tab) {
        free(is_med); free(dn); free(ds); free(near); free(tab);
        return ORC_ERR_MEM;
    }
    int rc = ORC_OK;
    int32_t iters = 0, swaps = 0;
    rect_nearest(D, nc, nl, med, k, near, dn, ds);
    double td = 0.0;
    for (int64_t o = 0; o < nc; ++o) td += dn[o];
    while (k >= 2 && k < nl) {
        if (iters >= max_iter) { rc = ORC_WARN_MAXITER; break; }
        ++iters;
        #pragma omp parallel for collapse(2) schedule(dynamic, 16)
        for (int32_t i = 0; i < k; ++i)
            for (int64_t c = 0; c < nl; ++c) {
                double acc = NAN;
                if (!is_med[c]) {
                    acc = 0.0;
                    for (int64_t o = 0; o < nc; ++o)
                        acc += orc_change(D[o * nl + c], near[o] == i, dn[o], ds[o]);
                }
                tab[(int64_t)i * nl + c] = acc;
            }
        double bd = 0.0;
        int32_t bi = -1;
        int64_t bc = -1;
        for (int32_t i = 0; i < k; ++i)
            for (int64_t c = 0; c < nl; ++c) {
                if (is_med[c]) continue;
                const double v = tab[(int64_t)i * nl + c];
                if (v < bd) { bd = v; bi = i; bc = c; }
            }
        if (bi < 0) break;
        is_med[med[bi]] = 0;
        med[bi] = (int32_t)bc;
        is_med[bc] = 1;
        td += bd;
        if (trace_slot && swaps < trace_cap) {
            trace_slot[swaps] = bi; trace_c[swaps] = bc; trace_delta[swaps] = bd;
        }
        ++swaps;
        rect_nearest(D, nc, nl, med, k, near, dn, ds);
        double fresh = 0.0;
        for (int64_t o = 0; o < nc; ++o) fresh += dn[o];
        if (!td_matches(td, fresh)) { rc = ORC_ERR_TD; break; }
        td = fresh;
    }
    if (n_iter) *n_iter = iters;
    if (n_swaps) *n_swaps = swaps;
    if (td_out) *td_out = orc_rect_td(D, nc, nl, med, k, NULL);
    free(is_med); free(dn); free(ds); free(near); free(tab);
    return rc;
}
