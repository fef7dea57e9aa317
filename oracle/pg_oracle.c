/*
 * pg_oracle.c -- plain FP64 CPU oracle for the proximity-graph build path of
 * "Revisiting the Index Construction of Proximity Graph-Based Approximate
 * Nearest Neighbor Search" (arXiv 2410.01231).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two are compared only
 * through their outputs on the same seeded inputs.
 *
 * Conventions (fixed for every function below):
 *   - dist is the L2 distance (Section 2, k-ANN search).  All comparisons use
 *     d2 = sum_i (x_i - y_i)^2 evaluated in double from the float inputs.
 *     d2 is monotone in dist, so every order by dist is the order by d2.
 *   - The paper never says how ties in distance are broken.  Every sort,
 *     top-k and "closest" below uses the total order on the pair (d2, id).
 *   - Random draws come from orc_hash, a counter-based generator built from
 *     the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
 *
 * Functions and the passages they follow:
 *   orc_exact_knn  k-ANN problem statement (Section 2); brute force.
 *   orc_nndescent  Initialization phase: KGraph / NN-Descent (Section 3.1,
 *                  Alg. 2 Phase 1; Section 6 Exp. 12 describes its iterations:
 *                  k random neighbours, then distances to 2-hop neighbours).
 *   orc_prune_one  Alg. 3 (Prune) plus the alpha test of Section 4.1.
 *   orc_refine     Alg. 2 Phase 3 (Refinement): prune, reverse-edge
 *                  re-prune, DFS connectivity and extra edges; the entry point
 *                  of Alg. 2 Phase 2 (closest point to the centroid).
 *   orc_search     Alg. 1 (KANNSearch, beam search).
 *   orc_search_self  the search phase of OptKCNA (Alg. 5, Phase 3).
 * Readings where the paper is silent are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-5)

#define ORC_STAGE_PRUNE 1u
#define ORC_STAGE_REVERSE 2u
#define ORC_STAGE_CONNECT 4u

/* ------------------------------------------------------------------ */
/* distances and the (d2, id) order                                    */
/* ------------------------------------------------------------------ */

static double sqdist(const float *a, const float *b, int32_t d)
{
    double s = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        double t = (double)a[i] - (double)b[i];
        s += t * t;
    }
    return s;
}

typedef struct {
    double d2;
    int32_t id;
    int32_t tag; /* carried payload: flag or position */
} orc_item;

static int item_less(const orc_item *x, const orc_item *y)
{
    if (x->d2 != y->d2)
        return x->d2 < y->d2;
    return x->id < y->id;
}

static int cmp_item(const void *a, const void *b)
{
    const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
    if (item_less(x, y))
        return -1;
    if (item_less(y, x))
        return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* counter-based random numbers                                        */
/* ------------------------------------------------------------------ */

/* SplitMix64: the state advances by the golden-ratio increment and each
 * output is the state passed through a fixed 64-bit mixing function.
 * sm(s, i) below is the i-th output (i >= 1) of a SplitMix64 generator
 * started at state s. */
static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t sm(uint64_t s, uint64_t i)
{
    return sm_mix(s + 0x9E3779B97F4A7C15ULL * i);
}

/* Exposed so the generator can be checked against published outputs. */
uint64_t orc_splitmix(uint64_t s, uint64_t i)
{
    return sm(s, i);
}

/* h(seed, stream, a, b) = sm(sm(sm(seed, stream+1), a+1), b+1). */
uint64_t orc_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    uint64_t x = sm(seed, stream + 1);
    x = sm(x, a + 1);
    return sm(x, b + 1);
}

/* ------------------------------------------------------------------ */
/* exact k nearest neighbours (brute force)                            */
/* ------------------------------------------------------------------ */

/* For every query q, the k smallest (d2(q, x_v), v) over all v in [0, n),
 * skipping v == exclude[q] when exclude is given (a data point is not its own
 * neighbour).  Missing entries are padded with id -1 and d2 = +inf.
 * A bounded insertion list keeps the k best seen so far. */
int orc_exact_knn(const float *X, int64_t n, int32_t d, int64_t ldx,
                  const float *Q, int64_t nq, int64_t ldq,
                  const int32_t *exclude, int32_t k,
                  int32_t *out_ids, double *out_d2)
{
    if (!X || !Q || n < 0 || nq < 0 || d <= 0 || k <= 0 || ldx < d || ldq < d)
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        orc_item *best = (orc_item *)malloc(sizeof(orc_item) * (size_t)k);
        if (!best) {
            bad = 1;
            continue;
        }
        int32_t m = 0;
        const float *xq = Q + q * ldq;
        for (int64_t v = 0; v < n; ++v) {
            if (exclude && exclude[q] == (int32_t)v)
                continue;
            orc_item it = {sqdist(xq, X + v * ldx, d), (int32_t)v, 0};
            if (m == k && !item_less(&it, &best[k - 1]))
                continue;
            int32_t p = (m < k) ? m++ : k - 1;
            while (p > 0 && item_less(&it, &best[p - 1])) {
                best[p] = best[p - 1];
                --p;
            }
            best[p] = it;
        }
        for (int32_t j = 0; j < k; ++j) {
            out_ids[q * k + j] = j < m ? best[j].id : -1;
            out_d2[q * k + j] = j < m ? best[j].d2 : INFINITY;
        }
        free(best);
    }
    return bad ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* NN-Descent (initialization phase)                                   */
/* ------------------------------------------------------------------ */

/*
 * Reading.  The paper builds the initial KNNG with KGraph and describes its
 * iterations only as: k random neighbours first, then each point computes
 * distances to its 2-hop neighbours to find closer ones.  We take the published
 * NN-Descent local join (Dong, Charikar & Li, WWW 2011), made synchronous and
 * deterministic:
 *
 *  iteration 0 (init): for u, attempt j = 0, 1, 2, ... draws
 *      r = h(seed, 0, u, j) mod (n - 1),  v = r + (r >= u),
 *  skipping ids already drawn, until K distinct ids are held.  The list is
 *  sorted by (d2, id) and every entry is flagged new.
 *
 *  iteration t >= 1 reads a snapshot of every list:
 *   (a) new_f(u): the min(S, #new) new-flagged entries with the smallest
 *       (h(seed, 3t, u, v) >> 32, v) (the high 32 bits of the hash, then the
 *       id); they are flagged old from now on.
 *       old_f(u): the entries flagged old in the snapshot.
 *   (b) Rnew(v) = {u : v in new_f(u)} keeping the S smallest
 *       (h(seed, 3t+1, v, u) >> 32, u);  Rold(v) likewise from old_f with
 *       stream 3t+2.
 *   (c) new(u) = new_f(u) U Rnew(u);  old(u) = (old_f(u) U Rold(u)) \ new(u).
 *   (d) local join at u: every unordered pair {v, w} of distinct members of
 *       new(u), and every pair v in new(u), w in old(u).  w is proposed to v
 *       iff (d2(v,w), w) < the K-th entry of v's snapshot list, and v to w
 *       likewise.
 *   (e) v's list becomes the K smallest distinct ids of (snapshot list U
 *       proposals); entries that were not in the snapshot are flagged new and
 *       counted as updates.
 *   (f) stop when updates <= stop_updates, or after max_iters iterations.
 *
 * The oracle evaluates (d) per target: v receives w from the join at u
 * whenever both belong to u's join set with at least one of them new.
 *
 * stats (optional, length 1 + 2 * max_iters): stats[0] = iterations run,
 * stats[1 + 2(t-1)] = updates in iteration t, stats[2 + 2(t-1)] = join pairs
 * in iteration t.
 * ids/d2/flags: n*K outputs (flags = 1 for new).
 */

typedef struct {
    int32_t *ids;
    double *d2;
    uint8_t *isnew;
} orc_lists;

static int draw_init(const float *X, int64_t n, int32_t d, int64_t ldx,
                     int32_t K, uint64_t seed, orc_lists *L)
{
    int bad = 0;
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; ++u) {
        orc_item *row = (orc_item *)malloc(sizeof(orc_item) * (size_t)K);
        if (!row) {
            bad = 1;
            continue;
        }
        int32_t m = 0;
        for (uint64_t j = 0; m < K; ++j) {
            uint64_t r = orc_hash(seed, 0, (uint64_t)u, j) % (uint64_t)(n - 1);
            int32_t v = (int32_t)(r >= (uint64_t)u ? r + 1 : r);
            int dup = 0;
            for (int32_t i = 0; i < m; ++i)
                if (row[i].id == v)
                    dup = 1;
            if (dup)
                continue;
            row[m].id = v;
            row[m].d2 = sqdist(X + u * ldx, X + (int64_t)v * ldx, d);
            row[m].tag = 1;
            ++m;
        }
        qsort(row, (size_t)K, sizeof(orc_item), cmp_item);
        for (int32_t i = 0; i < K; ++i) {
            L->ids[u * K + i] = row[i].id;
            L->d2[u * K + i] = row[i].d2;
            L->isnew[u * K + i] = 1;
        }
        free(row);
    }
    return bad ? ORC_ENOMEM : ORC_OK;
}

typedef struct {
    uint64_t h;
    int32_t id;
} orc_hkey;

static int cmp_hkey(const void *a, const void *b)
{
    const orc_hkey *x = (const orc_hkey *)a, *y = (const orc_hkey *)b;
    if (x->h != y->h)
        return x->h < y->h ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Sort ids and drop repeats; returns the new length. */
static int32_t sort_unique_ids(int32_t *a, int32_t m)
{
    /* insertion sort: the sets here hold at most a few hundred ids */
    for (int32_t i = 1; i < m; ++i) {
        int32_t x = a[i], p = i;
        while (p > 0 && a[p - 1] > x) {
            a[p] = a[p - 1];
            --p;
        }
        a[p] = x;
    }
    int32_t o = 0;
    for (int32_t i = 0; i < m; ++i)
        if (o == 0 || a[o - 1] != a[i])
            a[o++] = a[i];
    return o;
}

static int contains_sorted(const int32_t *a, int32_t m, int32_t x)
{
    int32_t lo = 0, hi = m;
    while (lo < hi) {
        int32_t mid = (lo + hi) / 2;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < m && a[lo] == x;
}

int orc_nndescent(const float *X, int64_t n, int32_t d, int64_t ldx,
                  int32_t K, int32_t S, int32_t max_iters, int64_t stop_updates,
                  uint64_t seed, int32_t *out_ids, double *out_d2,
                  uint8_t *out_flags, int64_t *stats)
{
    if (!X || d <= 0 || ldx < d || K <= 0 || K > 256 || S <= 0 || S > K ||
        max_iters < 0 || n < 2 || K > n - 1)
        return ORC_EINVAL;
    int rc = ORC_OK;
    orc_lists L = {out_ids, out_d2, out_flags};
    if ((rc = draw_init(X, n, d, ldx, K, seed, &L)) != ORC_OK)
        return rc;
    if (stats) {
        stats[0] = 0;
        for (int32_t t = 0; t < 2 * max_iters; ++t)
            stats[1 + t] = 0;
    }

    const int32_t NJ = 2 * S, OJ = K + S; /* bounds on |new(u)|, |old(u)| */
    int32_t *nf = malloc(sizeof(int32_t) * (size_t)n * S);
    int32_t *nf_c = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *of = malloc(sizeof(int32_t) * (size_t)n * K);
    int32_t *of_c = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *jn = malloc(sizeof(int32_t) * (size_t)n * (NJ + 0));
    int32_t *jn_c = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *jo = malloc(sizeof(int32_t) * (size_t)n * (OJ + 0));
    int32_t *jo_c = malloc(sizeof(int32_t) * (size_t)n);
    int64_t *roff = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *moff = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *snap_ids = malloc(sizeof(int32_t) * (size_t)n * K);
    double *snap_d2 = malloc(sizeof(double) * (size_t)n * K);
    uint8_t *snap_new = malloc((size_t)n * K);
    if (!nf || !nf_c || !of || !of_c || !jn || !jn_c || !jo || !jo_c || !roff ||
        !moff || !snap_ids || !snap_d2 || !snap_new) {
        rc = ORC_ENOMEM;
        goto done;
    }

    for (int32_t t = 1; t <= max_iters; ++t) {
        memcpy(snap_ids, L.ids, sizeof(int32_t) * (size_t)n * K);
        memcpy(snap_d2, L.d2, sizeof(double) * (size_t)n * K);
        /* (a) forward sampling */
        for (int64_t u = 0; u < n; ++u) {
            orc_hkey hk[256];
            int32_t m = 0, o = 0;
            for (int32_t j = 0; j < K; ++j) {
                int32_t v = L.ids[u * K + j];
                if (L.isnew[u * K + j]) {
                    hk[m].h = orc_hash(seed, 3 * (uint64_t)t, (uint64_t)u, (uint64_t)v) >> 32;
                    hk[m].id = v;
                    ++m;
                } else {
                    of[u * K + o++] = v;
                }
            }
            of_c[u] = o;
            qsort(hk, (size_t)m, sizeof(orc_hkey), cmp_hkey);
            int32_t take = m < S ? m : S;
            for (int32_t i = 0; i < take; ++i) {
                nf[u * S + i] = hk[i].id;
                for (int32_t j = 0; j < K; ++j)
                    if (L.ids[u * K + j] == hk[i].id)
                        L.isnew[u * K + j] = 0; /* sampled: old from now on */
            }
            nf_c[u] = take;
        }
        memcpy(snap_new, L.isnew, (size_t)n * K); /* flags after sampling */

        /* (b) reverse lists, capped at S by hash; (c) join sets */
        for (int side = 0; side < 2; ++side) {
            const int32_t *src = side == 0 ? nf : of;
            const int32_t *src_c = side == 0 ? nf_c : of_c;
            const int32_t stride = side == 0 ? S : K;
            memset(roff, 0, sizeof(int64_t) * (size_t)(n + 1));
            for (int64_t u = 0; u < n; ++u)
                for (int32_t i = 0; i < src_c[u]; ++i)
                    roff[src[u * stride + i] + 1]++;
            for (int64_t v = 0; v < n; ++v)
                roff[v + 1] += roff[v];
            int32_t *rev = malloc(sizeof(int32_t) * (size_t)(roff[n] > 0 ? roff[n] : 1));
            int64_t *cur = malloc(sizeof(int64_t) * (size_t)n);
            if (!rev || !cur) {
                free(rev);
                free(cur);
                rc = ORC_ENOMEM;
                goto done;
            }
            for (int64_t v = 0; v < n; ++v)
                cur[v] = roff[v];
            for (int64_t u = 0; u < n; ++u)
                for (int32_t i = 0; i < src_c[u]; ++i)
                    rev[cur[src[u * stride + i]]++] = (int32_t)u;
            uint64_t stream = 3 * (uint64_t)t + 1 + (uint64_t)side;
            for (int64_t v = 0; v < n; ++v) {
                int64_t cnt = roff[v + 1] - roff[v];
                orc_hkey *hk = malloc(sizeof(orc_hkey) * (size_t)(cnt > 0 ? cnt : 1));
                if (!hk) {
                    rc = ORC_ENOMEM;
                    break;
                }
                for (int64_t i = 0; i < cnt; ++i) {
                    int32_t u = rev[roff[v] + i];
                    hk[i].h = orc_hash(seed, stream, (uint64_t)v, (uint64_t)u) >> 32;
                    hk[i].id = u;
                }
                qsort(hk, (size_t)cnt, sizeof(orc_hkey), cmp_hkey);
                int32_t take = cnt < S ? (int32_t)cnt : S;
                int32_t buf[512];
                int32_t m = 0;
                if (side == 0) {
                    for (int32_t i = 0; i < nf_c[v]; ++i)
                        buf[m++] = nf[v * S + i];
                    for (int32_t i = 0; i < take; ++i)
                        buf[m++] = hk[i].id;
                    m = sort_unique_ids(buf, m);
                    memcpy(jn + v * NJ, buf, sizeof(int32_t) * (size_t)m);
                    jn_c[v] = m;
                } else {
                    for (int32_t i = 0; i < of_c[v]; ++i)
                        buf[m++] = of[v * K + i];
                    for (int32_t i = 0; i < take; ++i)
                        buf[m++] = hk[i].id;
                    m = sort_unique_ids(buf, m);
                    int32_t o = 0;
                    for (int32_t i = 0; i < m; ++i)
                        if (!contains_sorted(jn + v * NJ, jn_c[v], buf[i]))
                            jo[v * OJ + o++] = buf[i];
                    jo_c[v] = o;
                }
                free(hk);
            }
            free(rev);
            free(cur);
            if (rc != ORC_OK)
                goto done;
        }

        /* memberships: v belongs to the join set of u (role 1 = new) */
        memset(moff, 0, sizeof(int64_t) * (size_t)(n + 1));
        int64_t pairs = 0;
        for (int64_t u = 0; u < n; ++u) {
            for (int32_t i = 0; i < jn_c[u]; ++i)
                moff[jn[u * NJ + i] + 1]++;
            for (int32_t i = 0; i < jo_c[u]; ++i)
                moff[jo[u * OJ + i] + 1]++;
            int64_t a = jn_c[u], b = jo_c[u];
            pairs += a * (a - 1) / 2 + a * b;
        }
        for (int64_t v = 0; v < n; ++v)
            moff[v + 1] += moff[v];
        int32_t *mu = malloc(sizeof(int32_t) * (size_t)(moff[n] > 0 ? moff[n] : 1));
        uint8_t *mrole = malloc((size_t)(moff[n] > 0 ? moff[n] : 1));
        int64_t *cur = malloc(sizeof(int64_t) * (size_t)n);
        if (!mu || !mrole || !cur) {
            free(mu);
            free(mrole);
            free(cur);
            rc = ORC_ENOMEM;
            goto done;
        }
        for (int64_t v = 0; v < n; ++v)
            cur[v] = moff[v];
        for (int64_t u = 0; u < n; ++u) {
            for (int32_t i = 0; i < jn_c[u]; ++i) {
                int64_t p = cur[jn[u * NJ + i]]++;
                mu[p] = (int32_t)u;
                mrole[p] = 1;
            }
            for (int32_t i = 0; i < jo_c[u]; ++i) {
                int64_t p = cur[jo[u * OJ + i]]++;
                mu[p] = (int32_t)u;
                mrole[p] = 0;
            }
        }

        /* (d) + (e) per target */
        int64_t updates = 0;
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : updates)
        for (int64_t v = 0; v < n; ++v) {
            int64_t cap = K + 64, m = 0;
            orc_item *P = malloc(sizeof(orc_item) * (size_t)cap);
            if (!P) {
                bad = 1;
                continue;
            }
            for (int32_t j = 0; j < K; ++j) { /* snapshot, flags after sampling */
                P[m].d2 = snap_d2[v * K + j];
                P[m].id = snap_ids[v * K + j];
                P[m].tag = 2 + snap_new[v * K + j]; /* 2 = old, 3 = new; from snapshot */
                ++m;
            }
            orc_item kth = {snap_d2[v * K + K - 1], snap_ids[v * K + K - 1], 0};
            const float *xv = X + v * ldx;
            for (int64_t p = moff[v]; p < moff[v + 1]; ++p) {
                int32_t u = mu[p];
                for (int part = 0; part < 2; ++part) {
                    /* a new member meets all other members; an old one meets new members */
                    if (part == 1 && !mrole[p])
                        break;
                    const int32_t *set = part == 0 ? jn + (int64_t)u * NJ : jo + (int64_t)u * OJ;
                    int32_t cnt = part == 0 ? jn_c[u] : jo_c[u];
                    for (int32_t i = 0; i < cnt; ++i) {
                        int32_t w = set[i];
                        if (w == (int32_t)v)
                            continue;
                        orc_item it = {sqdist(xv, X + (int64_t)w * ldx, d), w, 1};
                        if (!item_less(&it, &kth))
                            continue;
                        if (m == cap) {
                            cap *= 2;
                            orc_item *np = realloc(P, sizeof(orc_item) * (size_t)cap);
                            if (!np) {
                                bad = 1;
                                break;
                            }
                            P = np;
                        }
                        P[m++] = it;
                    }
                }
            }
            qsort(P, (size_t)m, sizeof(orc_item), cmp_item);
            /* equal ids carry equal d2, so duplicates are adjacent; a snapshot
             * copy (tag >= 2) wins over proposal copies */
            int32_t o = 0;
            for (int64_t i = 0; i < m && o < K;) {
                int64_t j = i;
                int32_t tag = P[i].tag;
                while (j + 1 < m && P[j + 1].id == P[i].id) {
                    ++j;
                    if (P[j].tag > tag)
                        tag = P[j].tag;
                }
                L.ids[v * K + o] = P[i].id;
                L.d2[v * K + o] = P[i].d2;
                L.isnew[v * K + o] = (uint8_t)(tag == 2 ? 0 : 1);
                if (tag == 1)
                    updates++;
                ++o;
                i = j + 1;
            }
            free(P);
        }
        free(mu);
        free(mrole);
        free(cur);
        if (bad) {
            rc = ORC_ENOMEM;
            goto done;
        }
        if (stats) {
            stats[0] = t;
            stats[1 + 2 * (t - 1)] = updates;
            stats[2 + 2 * (t - 1)] = pairs;
        }
        if (updates <= stop_updates)
            break;
    }
done:
    free(nf);
    free(nf_c);
    free(of);
    free(of_c);
    free(jn);
    free(jn_c);
    free(jo);
    free(jo_c);
    free(roff);
    free(moff);
    free(snap_ids);
    free(snap_d2);
    free(snap_new);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Prune (Alg. 3) with the alpha test (Section 4.1)                    */
/* ------------------------------------------------------------------ */

/*
 * Alg. 3 visits the candidates in ascending dist(u, v) and keeps v unless an
 * already kept w has dist(v, w) < dist(u, v); it stops once M are kept.  The
 * alpha-pruning rule of Section 4.1 adds the condition angle(u w v) > alpha.
 *
 * Readings:
 *  - candidates equal to u, negative ids (padding) and repeated ids are dropped;
 *  - ties in dist(u, .) follow the (d2, id) order; by default an earlier
 *    candidate with the same dist(u, .) may occlude a later one, as Alg. 3
 *    tests only dist(v, w) < dist(u, v); strict_ties != 0 additionally
 *    requires dist(u, w) < dist(u, v), as the definition of the RNG in
 *    Section 2.1 states;
 *  - the angle at w comes from the law of cosines on a = d2(u,w), b = d2(v,w),
 *    c = d2(u,v): angle > alpha  <=>  a + b - c < 2 cos(alpha) sqrt(a b).
 *    For alpha <= 60 degrees the test is implied by the two distance
 *    conditions (Section 4.2 notes alpha = 60 gives RNG pruning), so it is
 *    skipped unless force_angle is set.  b == 0 (v coincides with w) counts as
 *    occluded for every alpha.  alpha = 90 uses 2 cos(alpha) = 0 exactly.
 *
 * dist_fn: when tab != NULL every distance comes from the float table
 * tab[(i)*(C+1)+(j)] over positions 0 = u and 1..C = cand[0..C-1]; otherwise
 * from X.
 */
typedef struct {
    const float *X;
    int64_t ldx;
    int32_t d;
    const float *tab; /* (C+1) x (C+1), or NULL */
    int32_t C;
} orc_dsrc;

static double dsrc_d2(const orc_dsrc *s, int32_t pa, int32_t ida, int32_t pb, int32_t idb)
{
    if (s->tab)
        return (double)s->tab[(int64_t)pa * (s->C + 1) + pb];
    return sqdist(s->X + (int64_t)ida * s->ldx, s->X + (int64_t)idb * s->ldx, s->d);
}

static int angle_exceeds(double a, double b, double c, double alpha_deg, int force)
{
    if (alpha_deg <= 60.0 && !force)
        return 1;
    if (b == 0.0)
        return 1;
    double kappa = (alpha_deg == 90.0) ? 0.0 : 2.0 * cos(alpha_deg * (M_PI / 180.0));
    return (a + b - c) < kappa * sqrt(a * b);
}

/* Returns the number kept (<= R) or a negative status.  out_pos (optional)
 * receives each kept candidate's position in cand. */
static int32_t prune_core(const orc_dsrc *s, int32_t u, const int32_t *cand, int32_t C,
                          int32_t R, double alpha_deg, int32_t strict, int32_t force_angle,
                          int32_t *out_ids, double *out_d2, int32_t *out_pos)
{
    orc_item *it = malloc(sizeof(orc_item) * (size_t)(C > 0 ? C : 1));
    int32_t *kept = malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    if (!it || !kept) {
        free(it);
        free(kept);
        return ORC_ENOMEM;
    }
    int32_t m = 0;
    for (int32_t i = 0; i < C; ++i) {
        int32_t v = cand[i];
        if (v < 0 || v == u)
            continue;
        it[m].id = v;
        it[m].tag = i;
        it[m].d2 = dsrc_d2(s, 0, u, i + 1, v);
        ++m;
    }
    qsort(it, (size_t)m, sizeof(orc_item), cmp_item);
    int32_t mm = 0;
    for (int32_t i = 0; i < m; ++i) /* drop repeated ids (adjacent after the sort) */
        if (mm == 0 || it[mm - 1].id != it[i].id)
            it[mm++] = it[i];
    m = mm;

    int32_t nk = 0;
    for (int32_t j = 0; j < m && nk < R; ++j) {
        double c = it[j].d2;
        int occluded = 0;
        for (int32_t q = 0; q < nk && !occluded; ++q) {
            const orc_item *w = &it[kept[q]];
            double a = w->d2;
            double b = dsrc_d2(s, w->tag + 1, w->id, it[j].tag + 1, it[j].id);
            if (b < c && (!strict || a < c) && angle_exceeds(a, b, c, alpha_deg, force_angle))
                occluded = 1;
        }
        if (!occluded)
            kept[nk++] = j;
    }
    for (int32_t q = 0; q < nk; ++q) {
        out_ids[q] = it[kept[q]].id;
        out_d2[q] = it[kept[q]].d2;
        if (out_pos)
            out_pos[q] = it[kept[q]].tag;
    }
    free(it);
    free(kept);
    return nk;
}

/* Prune one node's candidate list against the data X. */
int32_t orc_prune_one(const float *X, int64_t ldx, int32_t d, int32_t u,
                      const int32_t *cand, int32_t C, int32_t R, double alpha_deg,
                      int32_t strict_ties, int32_t force_angle,
                      int32_t *out_ids, double *out_d2)
{
    if (!X || d <= 0 || ldx < d || C < 0 || R <= 0)
        return ORC_EINVAL;
    orc_dsrc s = {X, ldx, d, NULL, C};
    return prune_core(&s, u, cand, C, R, alpha_deg, strict_ties, force_angle, out_ids,
                      out_d2, NULL);
}

/* Prune every node with all distances taken from per-node float tables:
 * tab[u] is (C+1) x (C+1) over positions 0 = u and 1..C = cand[u][0..C-1].
 * Output rows are padded with -1 / +inf; deg[u] = number kept. */
int orc_prune_table(int64_t n, const int32_t *cand, int32_t C, const float *tab,
                    int32_t R, double alpha_deg, int32_t strict_ties,
                    int32_t *out_ids, double *out_d2, int32_t *out_deg)
{
    if (!cand || !tab || n < 0 || C <= 0 || R <= 0)
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < n; ++u) {
        orc_dsrc s = {NULL, 0, 0, tab + u * (int64_t)(C + 1) * (C + 1), C};
        int32_t k = prune_core(&s, (int32_t)u, cand + u * C, C, R, alpha_deg, strict_ties, 0,
                               out_ids + u * R, out_d2 + u * R, NULL);
        if (k < 0) {
            bad = 1;
            k = 0;
        }
        for (int32_t j = k; j < R; ++j) {
            out_ids[u * R + j] = -1;
            out_d2[u * R + j] = INFINITY;
        }
        out_deg[u] = k;
    }
    return bad ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Refinement (Alg. 2 Phase 3) and the entry point                     */
/* ------------------------------------------------------------------ */

/* Entry point: Alg. 2 takes ep as the point closest to the centroid of D,
 * found there by a search from a random node.  Reading: the exact
 * argmin over v of (d2(x_v, centroid), v), with the centroid accumulated in
 * double in index order. */
int32_t orc_entry_point(const float *X, int64_t n, int32_t d, int64_t ldx)
{
    if (!X || n <= 0 || d <= 0)
        return ORC_EINVAL;
    double *c = calloc((size_t)d, sizeof(double));
    if (!c)
        return ORC_ENOMEM;
    for (int64_t v = 0; v < n; ++v)
        for (int32_t i = 0; i < d; ++i)
            c[i] += (double)X[v * ldx + i];
    for (int32_t i = 0; i < d; ++i)
        c[i] /= (double)n;
    int32_t best = -1;
    double bd = INFINITY;
    for (int64_t v = 0; v < n; ++v) {
        double s = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            double t = (double)X[v * ldx + i] - c[i];
            s += t * t;
        }
        if (s < bd) { /* strict: the smallest id wins ties */
            bd = s;
            best = (int32_t)v;
        }
    }
    free(c);
    return best;
}

/* Mark everything reachable from r over out-edges; returns nodes newly marked. */
static int64_t bfs_mark(int64_t n, const int32_t *g, int32_t R, const int32_t *deg,
                        uint8_t *seen, int32_t *queue, int32_t r)
{
    if (seen[r])
        return 0;
    int64_t head = 0, tail = 0;
    seen[r] = 1;
    queue[tail++] = r;
    while (head < tail) {
        int32_t x = queue[head++];
        for (int32_t j = 0; j < deg[x]; ++j) {
            int32_t y = g[(int64_t)x * R + j];
            if (y >= 0 && y < n && !seen[y]) {
                seen[y] = 1;
                queue[tail++] = y;
            }
        }
    }
    return tail;
}

/*
 * Refinement of Alg. 2 (Phase 3) on candidate lists cand (n x C):
 *   PRUNE:   N(u) <- Prune(u, C(u), R)                       for every u
 *   REVERSE: N(u) <- Prune(u, N(u) U {v : u in N(v)}, R)      for every u,
 *            every node reading the lists left by PRUNE (the paper's "in
 *            parallel" loop does not say; we read a snapshot);
 *   CONNECT: the paper finds connected components by DFS and adds edges
 *            between them.  Reading: mark what is reachable from ep; while a
 *            node is unreached, take the smallest unreached id r and add the
 *            edge p -> r, where p is the reached node with degree below R that
 *            is closest to r (by (d2, id)) among r's own candidates C(r); only
 *            when no candidate qualifies, p is the closest such node among all
 *            reached nodes.  Then mark what r reaches.  Extra edges are
 *            appended after the pruned ones.
 * Outputs: g_ids/g_d2 (n x R, padded with -1 / +inf), g_deg (n), *ep, and the
 * restart roots r in order (roots, capacity n) with their count *n_roots.
 * PRUNE must be among the stages.
 */
int orc_refine(const float *X, int64_t n, int32_t d, int64_t ldx,
               const int32_t *cand, int32_t C, int32_t R, double alpha_deg,
               int32_t strict_ties, uint32_t stages,
               int32_t *g_ids, double *g_d2, int32_t *g_deg, int32_t *ep,
               int32_t *roots, int32_t *n_roots)
{
    if (!X || !cand || n <= 0 || d <= 0 || ldx < d || C <= 0 || R <= 0 ||
        !(stages & ORC_STAGE_PRUNE))
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < n; ++u) {
        int32_t k = orc_prune_one(X, ldx, d, (int32_t)u, cand + u * C, C, R, alpha_deg,
                                  strict_ties, 0, g_ids + u * R, g_d2 + u * R);
        if (k < 0) {
            bad = 1;
            k = 0;
        }
        for (int32_t j = k; j < R; ++j) {
            g_ids[u * R + j] = -1;
            g_d2[u * R + j] = INFINITY;
        }
        g_deg[u] = k;
    }
    if (bad)
        return ORC_ENOMEM;

    if (stages & ORC_STAGE_REVERSE) {
        int32_t *snap = malloc(sizeof(int32_t) * (size_t)n * R);
        int32_t *sdeg = malloc(sizeof(int32_t) * (size_t)n);
        int64_t *off = calloc((size_t)n + 1, sizeof(int64_t));
        if (!snap || !sdeg || !off) {
            free(snap);
            free(sdeg);
            free(off);
            return ORC_ENOMEM;
        }
        memcpy(snap, g_ids, sizeof(int32_t) * (size_t)n * R);
        memcpy(sdeg, g_deg, sizeof(int32_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v)
            for (int32_t j = 0; j < sdeg[v]; ++j)
                off[snap[v * R + j] + 1]++;
        for (int64_t v = 0; v < n; ++v)
            off[v + 1] += off[v];
        int32_t *rev = malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
        int64_t *cur = malloc(sizeof(int64_t) * (size_t)n);
        if (!rev || !cur) {
            free(snap);
            free(sdeg);
            free(off);
            free(rev);
            free(cur);
            return ORC_ENOMEM;
        }
        for (int64_t v = 0; v < n; ++v)
            cur[v] = off[v];
        for (int64_t v = 0; v < n; ++v) /* v -> w gives w the reverse entry v */
            for (int32_t j = 0; j < sdeg[v]; ++j)
                rev[cur[snap[v * R + j]]++] = (int32_t)v;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) {
            int64_t m = sdeg[u] + (off[u + 1] - off[u]);
            int32_t *un = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
            if (!un) {
                bad = 1;
                continue;
            }
            int32_t q = 0;
            for (int32_t j = 0; j < sdeg[u]; ++j)
                un[q++] = snap[u * R + j];
            for (int64_t p = off[u]; p < off[u + 1]; ++p)
                un[q++] = rev[p];
            int32_t k = orc_prune_one(X, ldx, d, (int32_t)u, un, q, R, alpha_deg, strict_ties,
                                      0, g_ids + u * R, g_d2 + u * R);
            if (k < 0) {
                bad = 1;
                k = 0;
            }
            for (int32_t j = k; j < R; ++j) {
                g_ids[u * R + j] = -1;
                g_d2[u * R + j] = INFINITY;
            }
            g_deg[u] = k;
            free(un);
        }
        free(snap);
        free(sdeg);
        free(off);
        free(rev);
        free(cur);
        if (bad)
            return ORC_ENOMEM;
    }

    int32_t e = orc_entry_point(X, n, d, ldx);
    if (e < 0)
        return e;
    if (ep)
        *ep = e;
    if (n_roots)
        *n_roots = 0;

    if (stages & ORC_STAGE_CONNECT) {
        uint8_t *seen = calloc((size_t)n, 1);
        int32_t *queue = malloc(sizeof(int32_t) * (size_t)n);
        if (!seen || !queue) {
            free(seen);
            free(queue);
            return ORC_ENOMEM;
        }
        int64_t reached = bfs_mark(n, g_ids, R, g_deg, seen, queue, e);
        int32_t scan = 0, nr = 0;
        int rc = ORC_OK;
        while (reached < n) {
            while (seen[scan])
                ++scan;
            int32_t r = scan;
            int32_t best = -1;
            double bd = INFINITY;
            for (int32_t j = 0; j < C; ++j) { /* r's candidates first */
                int32_t p = cand[(int64_t)r * C + j];
                if (p < 0 || p >= n || p == r || !seen[p] || g_deg[p] >= R)
                    continue;
                double s = sqdist(X + (int64_t)p * ldx, X + (int64_t)r * ldx, d);
                if (s < bd || (s == bd && p < best)) {
                    bd = s;
                    best = p;
                }
            }
            const int from_cand = best >= 0;
            for (int64_t p = 0; !from_cand && p < n; ++p) { /* no candidate qualifies */
                if (!seen[p] || g_deg[p] >= R)
                    continue;
                double s = sqdist(X + p * ldx, X + (int64_t)r * ldx, d);
                if (s < bd) {
                    bd = s;
                    best = (int32_t)p;
                }
            }
            if (best < 0) {
                rc = ORC_EOVERFLOW; /* every reached node already has R edges */
                break;
            }
            g_ids[(int64_t)best * R + g_deg[best]] = r;
            g_d2[(int64_t)best * R + g_deg[best]] = bd;
            g_deg[best]++;
            if (roots)
                roots[nr] = r;
            ++nr;
            reached += bfs_mark(n, g_ids, R, g_deg, seen, queue, r);
        }
        if (n_roots)
            *n_roots = nr;
        free(seen);
        free(queue);
        if (rc != ORC_OK)
            return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Beam search (Alg. 1)                                                */
/* ------------------------------------------------------------------ */

/*
 * Alg. 1 with a set of entering points: the pool starts with every entry
 * (repeats dropped) and keeps the L closest by (d2, id).  Repeatedly the first
 * unexpanded pool entry is expanded: each out-neighbour not seen before in
 * this query is inserted with its distance and the pool is cut back to L.  The
 * search stops when the first min(L, |pool|) entries are all expanded, and
 * returns the first k (padded with -1 / +inf).  Alg. 1 itself would re-insert
 * neighbours already in the pool; the seen-set removes those repeats.
 * stats (optional, 2 per query): expansions, distance evaluations.
 */
/* One query of the beam search: pool (capacity L + n_entry + 1) holds the
 * result, *size its length; seen/touched are per-thread scratch, cleared on
 * return.  Returns expansions and distance evaluations through nexp, ndist. */
static int32_t search_one(const float *X, int64_t n, int32_t d, int64_t ldx,
                          const int32_t *g_ids, int32_t R, const int32_t *g_deg,
                          const float *xq, const int32_t *entries, int32_t n_entry, int32_t L,
                          orc_item *pool, uint8_t *seen, int32_t *touched,
                          int64_t *nexp, int64_t *ndist)
{
    int64_t nt = 0;
    int32_t size = 0;
    *nexp = 0;
    *ndist = 0;
    for (int32_t e = 0; e < n_entry; ++e) {
        int32_t v = entries[e];
        if (v < 0 || v >= n || seen[v])
            continue;
        seen[v] = 1;
        touched[nt++] = v;
        pool[size].id = v;
        pool[size].d2 = sqdist(xq, X + (int64_t)v * ldx, d);
        pool[size].tag = 0;
        ++size;
        ++*ndist;
    }
    qsort(pool, (size_t)size, sizeof(orc_item), cmp_item);
    if (size > L)
        size = L;
    for (;;) {
        int32_t i = 0;
        while (i < size && pool[i].tag)
            ++i;
        if (i >= size)
            break;
        pool[i].tag = 1;
        ++*nexp;
        int32_t x = pool[i].id;
        for (int32_t j = 0; j < g_deg[x]; ++j) {
            int32_t v = g_ids[(int64_t)x * R + j];
            if (v < 0 || v >= n || seen[v])
                continue;
            seen[v] = 1;
            touched[nt++] = v;
            orc_item it = {sqdist(xq, X + (int64_t)v * ldx, d), v, 0};
            ++*ndist;
            if (size == L && !item_less(&it, &pool[L - 1]))
                continue;
            int32_t p = size < L ? size++ : L - 1;
            while (p > 0 && item_less(&it, &pool[p - 1])) {
                pool[p] = pool[p - 1];
                --p;
            }
            pool[p] = it;
        }
    }
    for (int64_t t = 0; t < nt; ++t)
        seen[touched[t]] = 0;
    return size;
}

int orc_search(const float *X, int64_t n, int32_t d, int64_t ldx,
               const int32_t *g_ids, int32_t R, const int32_t *g_deg,
               const float *Q, int64_t nq, int64_t ldq,
               const int32_t *entries, int32_t n_entry, int32_t k, int32_t L,
               int32_t *out_ids, double *out_d2, int64_t *stats)
{
    if (!X || !g_ids || !g_deg || !Q || !entries || n <= 0 || d <= 0 || R <= 0 ||
        n_entry <= 0 || k <= 0 || L < k || ldx < d || ldq < d)
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel
    {
        uint8_t *seen = calloc((size_t)n, 1);
        int32_t *touched = malloc(sizeof(int32_t) * (size_t)n);
        orc_item *pool = malloc(sizeof(orc_item) * (size_t)(L + n_entry + 1));
        if (!seen || !touched || !pool)
            bad = 1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nq; ++q) {
            if (!seen || !touched || !pool)
                continue;
            int64_t nexp, ndist;
            const int32_t size = search_one(X, n, d, ldx, g_ids, R, g_deg, Q + q * ldq, entries,
                                            n_entry, L, pool, seen, touched, &nexp, &ndist);
            for (int32_t j = 0; j < k; ++j) {
                out_ids[q * k + j] = j < size ? pool[j].id : -1;
                out_d2[q * k + j] = j < size ? pool[j].d2 : INFINITY;
            }
            if (stats) {
                stats[2 * q] = nexp;
                stats[2 * q + 1] = ndist;
            }
        }
        free(seen);
        free(touched);
        free(pool);
    }
    return bad ? ORC_ENOMEM : ORC_OK;
}

/*
 * The search phase of OptKCNA (Alg. 5, Phase 3): for every node u,
 * KANNSearch(G, u, k, L, u), the beam search for the point x_u entering at u
 * itself.  Reading: the paper is silent on whether u may be one of its own
 * candidates; C(u) is the first k pool entries other than u (u sits in the
 * pool at distance 0 unless at least L other points coincide with it).
 * Needs k < L.
 */
int orc_search_self(const float *X, int64_t n, int32_t d, int64_t ldx,
                    const int32_t *g_ids, int32_t R, const int32_t *g_deg,
                    int32_t k, int32_t L, int32_t *out_ids, double *out_d2, int64_t *stats)
{
    if (!X || !g_ids || !g_deg || n <= 0 || d <= 0 || R <= 0 || k <= 0 || L <= k || ldx < d)
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel
    {
        uint8_t *seen = calloc((size_t)n, 1);
        int32_t *touched = malloc(sizeof(int32_t) * (size_t)n);
        orc_item *pool = malloc(sizeof(orc_item) * (size_t)(L + 2));
        if (!seen || !touched || !pool)
            bad = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < n; ++u) {
            if (!seen || !touched || !pool)
                continue;
            int64_t nexp, ndist;
            const int32_t entry = (int32_t)u;
            const int32_t size = search_one(X, n, d, ldx, g_ids, R, g_deg, X + u * ldx, &entry, 1,
                                            L, pool, seen, touched, &nexp, &ndist);
            int32_t j = 0;
            for (int32_t i = 0; i < size && j < k; ++i) {
                if (pool[i].id == (int32_t)u)
                    continue;
                out_ids[u * k + j] = pool[i].id;
                out_d2[u * k + j] = pool[i].d2;
                ++j;
            }
            for (; j < k; ++j) {
                out_ids[u * k + j] = -1;
                out_d2[u * k + j] = INFINITY;
            }
            if (stats) {
                stats[2 * u] = nexp;
                stats[2 * u + 1] = ndist;
            }
        }
        free(seen);
        free(touched);
        free(pool);
    }
    return bad ? ORC_ENOMEM : ORC_OK;
}
