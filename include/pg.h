/*
 * pg.h -- C ABI of the MI355X (gfx950) proximity-graph build library
 * (arXiv 2410.01231, "Revisiting the Index Construction of Proximity
 * Graph-Based Approximate Nearest Neighbor Search").
 *
 * The library builds an approximate k-nearest-neighbour graph by NN-Descent
 * local joins (the paper's initialization phase), refines it with the paper's
 * pruning rule (Alg. 3, with the alpha test of Section 4.1), reverse-edge
 * re-pruning and connectivity repair (Alg. 2, refinement phase), and answers
 * k-ANN queries by beam search (Alg. 1).
 *
 * Conventions shared by every entry point:
 *  - Every array argument is DEVICE memory (allocated by the caller, e.g.
 *    through torch) unless the comment says "host".  The caller owns every
 *    buffer; the library never frees or keeps a pointer after a call returns.
 *  - Vectors are float32 rows: X is n rows of d floats with leading dimension
 *    ldx (in floats).  d and ldx must be multiples of 4 and X 16-byte aligned.
 *  - Ids are int32 in [0, n); n < 2^31.  Missing entries are padded with id -1
 *    and distance +inf.
 *  - Distances are SQUARED L2 distances (monotone in the paper's dist), in
 *    float32, evaluated as s = fma(x_i - y_i, x_i - y_i, s) over i = 0..d-1 in
 *    order; the same evaluation is used by every kernel, so a pair's distance
 *    has one bit pattern wherever it is computed.
 *  - Every order and tie is the total order on (d2, id).
 *  - Calls run on the context's HIP stream.  pg_knn_build and pg_prune (with
 *    the connect stage) read small counters back and therefore return after
 *    their work has finished on the stream; the other calls only enqueue work.
 *  - Argument errors return PG_EINVAL (or PG_EUNSUPPORTED) synchronously,
 *    before any work is enqueued, with a message from pg_last_error().  Device
 *    errors surface as PG_EDEVICE.  Nothing is silently truncated: a bounded
 *    internal buffer that cannot hold a result makes the call retry
 *    deterministically, or fail with PG_EOVERFLOW.
 *  - A context is used by one host thread at a time.
 */
#ifndef PG_H
#define PG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pg_ctx pg_ctx;

typedef enum {
    PG_OK = 0,
    PG_EINVAL = -1,        /* bad argument */
    PG_ENOMEM = -2,        /* workspace too small or host allocation failed */
    PG_EDEVICE = -3,       /* HIP runtime or kernel error */
    PG_EUNSUPPORTED = -4,  /* valid but outside what the kernels implement */
    PG_EOVERFLOW = -5      /* a bounded structure could not hold the result */
} pg_status;

/* Arithmetic of the NN-Descent distance tiles.  Every list entry holds the
 * FP32 direct-form distance (the canonical chain: s = fmaf(x_i - y_i,
 * x_i - y_i, s) over i ascending), whatever the tiles compute in.
 *   PG_FP32: on data where it is provably exact (integer values with
 *     squared norms <= 2^23 and no negative value, or squared norms <= 2^22,
 *     so that every squared distance is an integer <= 2^24) the tiles run as
 *     FP32 MFMA norm expansions, otherwise as
 *     the direct form on the vector ALUs.  PG_FP32_VALU: always the direct
 *     form.
 *   PG_FP16 / PG_BF16: 16-bit MFMA tiles with FP32 accumulation.  On integer
 *     data where they are exact (|x| <= 2048 for FP16, <= 256 for BF16, and
 *     the norm condition of PG_FP32) they give the distances directly.  Otherwise
 *     (mixed precision) the tiles run on the mean-centred data and only
 *     prefilter: every pair whose estimate lies within the error bound
 *     (see margin_rel) of the cut of either end is recomputed in the direct
 *     form, and so is every value that enters a list.
 * With the rigorous bound every precision returns the same lists. */
typedef enum { PG_FP32 = 0, PG_FP16 = 1, PG_BF16 = 2, PG_FP32_VALU = 3 } pg_precision;

/* Join path a build used (pg_knn_stats.join_path). */
enum {
    PG_JOIN_VALU = 0,
    PG_JOIN_MFMA_FP32 = 1,
    PG_JOIN_MFMA_FP16 = 2,
    PG_JOIN_MFMA_BF16 = 3,
    PG_JOIN_MIXED_FP16 = 4, /* FP16 prefilter + FP32 recheck */
    PG_JOIN_MIXED_BF16 = 5  /* BF16 prefilter + FP32 recheck */
};

/* Library version (major * 10000 + minor * 100 + patch). */
int pg_version(void);

/* Message of the last failing call on this host thread (never NULL). */
const char *pg_last_error(void);

/* Create a context bound to HIP device `device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL means the null stream).  *out receives
 * the context (host pointer). */
pg_status pg_ctx_create(int device, void *hip_stream, pg_ctx **out);
pg_status pg_ctx_destroy(pg_ctx *ctx);

/* Per-kernel timing.  When enabled, every launch of the named kernels is
 * bracketed by HIP events on the context stream.  pg_ctx_kernel_time (host
 * outputs) returns, for kernel `name`, the summed event time in ms, the number
 * of launches, and the summed algorithmic work of those launches (flops for
 * the distance kernels, bytes for the others, as documented per kernel;
 * "join": 3 d flops per pair on the FP32 direct path, 2 d per pair on the
 * FP32 MFMA path, 2 d16 bytes per join-set member row on the 16-bit paths).
 * Reading the times synchronises the stream.  Names: "join", "merge", "init",
 * "sample", "prune", "search", "exact_knn", and "connect" (the whole connect
 * step of pg_prune as one region: several launches and host synchronisations). */
pg_status pg_ctx_set_timing(pg_ctx *ctx, int enable);
pg_status pg_ctx_kernel_time(pg_ctx *ctx, const char *name, double *total_ms,
                             int64_t *launches, double *work);
pg_status pg_ctx_reset_timing(pg_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Approximate kNN graph: NN-Descent (initialization phase)            */
/* ------------------------------------------------------------------ */
/*
 * Section 3.1 (Initialization) builds the initial KNNG G_k0 with KGraph;
 * Section 6, Exp. 12 describes the iterations (k random neighbours, then
 * distances to 2-hop neighbours).  The library runs NN-Descent local joins,
 * synchronous and deterministic:
 *   init:  K distinct random neighbours per node from a counter-based hash
 *          of (seed, 0, u, attempt);
 *   iteration t: sample <= S new entries per list (smallest hash keys), build
 *          reverse samples (<= S per node), join every new-new and new-old pair
 *          of each node's sample set, propose each pair to both ends when it
 *          beats the K-th entry of the end's list, and merge: each list becomes
 *          the K smallest distinct ids of (list U proposals).
 *   stop:  after max_iters iterations or when an iteration changes at most
 *          stop_updates list entries.
 * The result depends only on (X, K, S, max_iters, stop_updates, seed); the
 * tuning fields (bucket_cap, chunks) change speed and memory, never results.
 * exact != 0 computes the exact kNN lists instead (brute force).
 */
typedef struct {
    int32_t K;            /* list length, 1 <= K <= 64, K < n */
    int32_t S;            /* sample size per list, 1 <= S <= K (NN-Descent rho*K) */
    int32_t max_iters;    /* 0 <= max_iters <= 64 */
    int32_t exact;        /* nonzero: brute-force exact lists, other fields unused */
    int64_t stop_updates; /* stop when an iteration changes <= this many entries */
    uint64_t seed;
    int32_t precision;    /* pg_precision of the join tiles */
    float margin_rel;     /* mixed precision only.  >= 0: recheck margin = the
                             rigorous per-pair error bound of the 16-bit
                             estimate, plus margin_rel times the cut; < 0:
                             |margin_rel| times the cut alone (not rigorous:
                             decisions may then differ from FP32) */
    int32_t bucket_cap;   /* proposal slots per node per pass (>= 2K); 0 = 8K */
    int32_t chunks;       /* source passes in the first iteration (<= 64); 0 = 64 */
} pg_knn_params;

typedef struct {
    int32_t iters_run;
    int32_t join_path;     /* PG_JOIN_* used for the local joins */
    int64_t updates[64];   /* list entries changed in iteration t (index t-1) */
    int64_t pairs[64];     /* local-join pairs evaluated in iteration t */
    int64_t proposals[64]; /* proposals that passed the K-th filter at emission */
    int64_t retries;       /* extra join passes: a node's bucket and the spill list were full */
    int64_t spilled;       /* proposals that went past their node's bucket to the spill list */
    int64_t rechecked[64]; /* mixed precision: pairs recomputed in the direct form */
    int64_t members[64];   /* join-set members of the joining sources (rows gathered) */
} pg_knn_stats;

/* Workspace bytes needed by pg_knn_build for these sizes (host output). */
pg_status pg_knn_build_workspace(const pg_knn_params *p, int64_t n, int32_t d,
                                 size_t *bytes);

/* Build the kNN lists: knn_ids / knn_d2 are n x K (row u sorted by (d2, id),
 * never containing u).  ws is device scratch of ws_bytes >= the size above.
 * stats (host, optional) is filled when the call returns. */
pg_status pg_knn_build(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                       const pg_knn_params *p, void *ws, size_t ws_bytes,
                       int32_t *knn_ids, float *knn_d2, pg_knn_stats *stats);

/* Batched builds (several collections in one build; the batching pattern of
 * serving many uneven collections).  Collection c is rows
 * [offsets[c], offsets[c + 1]) of X (host offsets, offsets[0] = 0,
 * offsets[ncoll] = n, every collection more than K rows, same d).  Every
 * kernel of an iteration runs once over all collections; each collection
 * draws with its own local ids and stops on its own rule (an iteration that
 * changes at most stop_updates[c] of its entries, host array), so its lists
 * (knn_ids in ids local to the collection, knn_d2) equal those of
 * pg_knn_build on its rows alone with stop_updates[c].  iters (host, ncoll,
 * optional) receives each collection's iterations.  p->stop_updates and
 * p->exact are not used (exact != 0 is an error). */
pg_status pg_knn_build_batch_workspace(const pg_knn_params *p, int64_t n, int32_t d, int32_t ncoll,
                                       size_t *bytes);
pg_status pg_knn_build_batch(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                             const int64_t *offsets, int32_t ncoll, const int64_t *stop_updates,
                             const pg_knn_params *p, void *ws, size_t ws_bytes, int32_t *knn_ids,
                             float *knn_d2, int32_t *iters);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pg_knn_build
 * with its workspace taken from a static device array of PG_NOALLOC_WS_BYTES
 * that the library holds on each device it runs on, until the process ends.
 * Results are those of pg_knn_build with the same arguments.  Builds whose
 * workspace (pg_knn_build_workspace) exceeds PG_NOALLOC_WS_BYTES fail with
 * PG_ENOMEM before any work is enqueued: at K = 32, S = 16 that is up to
 * n = 30,788 rows with PG_FP32 (fewer with PG_FP16 / PG_BF16, which also keep
 * a 16-bit copy of X there: 29,074 rows at d = 128, 22,740 at d = 768).  The call allocates nothing (no hipMalloc / hipFree).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (several host threads, or several streams in flight) race and
 * corrupt each other's results, so the caller must serialise them. */
#define PG_NOALLOC_WS_BYTES ((size_t)128 << 20)
pg_status pg_knn_build_noalloc(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                               const pg_knn_params *p, int32_t *knn_ids, float *knn_d2,
                               pg_knn_stats *stats);

/* Brute-force k nearest neighbours of each query row among the rows of X
 * (k-ANN problem statement of Section 2, solved exactly).  Q is nq x d with
 * leading dimension ldq.  exclude (optional, nq ints) names a row of X to skip
 * for each query (-1 for none).  out_ids / out_d2 are nq x k, 1 <= k <= 64. */
pg_status pg_exact_knn(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                       const float *Q, int64_t nq, int64_t ldq, const int32_t *exclude,
                       int32_t k, int32_t *out_ids, float *out_d2);

/* Quality examination of Section 5.2 (the sample-size theorem; the quality
 * test that ends IterNSG's rounds, Alg. 6): for each sampled node u =
 * sample[i] the exact k nearest other points N*_k(u) (brute force over the
 * rows of X, u itself skipped) go to exact_ids / exact_d2 (ns x k, ordered by
 * (d2, id)), hits[i] (ns int32) receives |C(u)[:k] & N*_k(u)| with C(u) the
 * first k entries of row u of cand_ids (n x C, -1 pads count as misses), and
 * *estimate (device, one double) the estimated k-CNA recall
 * sum(hits) / (k ns).  The caller draws the sample (ns = (8 + 2 eps) l ln n /
 * eps^2 nodes estimate the mean within eps / 2 with probability 1 - n^-l).
 * Requires 1 <= k <= min(64, C), k < n, 1 <= ns <= n.  Only enqueues work:
 * on a stream of its own it overlaps other work (the next OptKCNA round).  A
 * sample id outside [0, n) gives hits -1 for it and a NaN estimate. */
pg_status pg_quality_examination(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                 const int32_t *cand_ids, int32_t C, int32_t k,
                                 const int32_t *sample, int64_t ns, int32_t *exact_ids,
                                 float *exact_d2, int32_t *hits, double *estimate);

/* ------------------------------------------------------------------ */
/* Refinement: Prune (Alg. 3), reverse re-prune and connect (Alg. 2)   */
/* ------------------------------------------------------------------ */
enum { PG_STAGE_PRUNE = 1, PG_STAGE_REVERSE = 2, PG_STAGE_CONNECT = 4 };

typedef struct {
    int32_t R;            /* out-degree bound M of the paper, 1 <= R <= 64 */
    float alpha_deg;      /* alpha of Section 4.1; <= 60 means RNG pruning */
    uint32_t stages;      /* PG_STAGE_* bits; PRUNE is required */
    int32_t strict_ties;  /* nonzero: w occludes v only if also d2(u,w) < d2(u,v) */
    const float *pair_d2; /* optional test hook, PRUNE stage alone: n tables of
                             (C+1) x (C+1) floats, positions 0 = u and 1..C =
                             cand_ids[u][0..C-1]; all distances are read from it */
    int32_t precision;    /* PG_FP32 (0): pairwise distances from FP16 MFMA Gram
                             tiles where they are exact (integer data, see
                             below), else from tiles on the mean-centred FP16
                             copy that only decide what their rigorous error
                             bound allows, the rest (and, with the alpha test,
                             every pair that may occlude) taking the FP32
                             chain; PG_FP32_VALU: every pairwise distance is
                             the FP32 chain.  Both give the same graph. */
    /* K2P (Section 5.4; the index is unchanged, Exp. 6).  k2p_prev_ids (n x
       k2p_prev_R, -1 pads, lengths k2p_prev_deg) holds the PRUNE-stage lists
       of the previous round over the same X with the same alpha_deg and
       strict_ties (prune_ids_out of that call).  Two candidates of u that
       both stayed in u's previous list are not tested against each other:
       the earlier did not occlude the later then, and cannot now.  Applies to
       the PRUNE stage of the MFMA kernels (given cand_d2, precision PG_FP32).
       k2p_counts (optional, device, 2 values) is added the pairs skipped and
       the pairs tested. */
    const int32_t *k2p_prev_ids;
    const int32_t *k2p_prev_deg;
    int32_t k2p_prev_R;
    unsigned long long *k2p_counts;
    int32_t *prune_ids_out;  /* optional, n x R: this call's PRUNE-stage lists */
    int32_t *prune_deg_out;  /* optional, n: their lengths (with prune_ids_out) */
} pg_prune_params;

/* Workspace bytes needed by pg_prune for n points of dimension d and C
 * candidates per point (host output). */
pg_status pg_prune_workspace(const pg_prune_params *p, int64_t n, int32_t d, int32_t C,
                             size_t *bytes);

/*
 * Refinement of Alg. 2 (Phase 3) and its entry point.
 *
 * cand_ids: n x C candidate lists (C <= 64; -1, u itself and repeats are
 * skipped).  cand_d2 (optional, n x C): d2(u, cand_ids[u][j]) as the
 * canonical FP32 chain computes it (pg_knn_build's knn_d2 qualifies); when
 * NULL the distances are computed here.  Results are the same either way.
 *
 * Stage PRUNE: N(u) <- Prune(u, C(u), R) for every u (Alg. 3 and, for
 * alpha > 60, the alpha test of Section 4.1).  The alpha test is the law of
 * cosines on the squared distances a = d2(u,w), b = d2(v,w), c = d2(u,v):
 * w occludes v when (a + b) - c < kappa * sqrt(a * b), kappa = 2 cos(alpha)
 * (0 at 90 degrees), decided as that expression evaluates in IEEE double from
 * the FP32 distances (an FP32 evaluation decides when it is provably the
 * same; otherwise the double one runs).  Stage REVERSE:
 * N(u) <- Prune(u, N(u) U {v : u in N(v)}, R), every node reading the PRUNE
 * result.  Entry point: the node closest to the centroid of X (argmin of
 * (d2, id); centroid summed in double).  Stage CONNECT: with ep as the start,
 * while some node is unreached, the smallest unreached id r gets the edge
 * p -> r, where p is the reached node below degree R closest to r among r's
 * own candidates cand_ids[r], or, when none qualifies, among all reached
 * nodes; then everything r reaches counts as reached.  Extra edges are
 * appended after the pruned ones.
 *
 * When X holds integers with |x| <= 2048 and squared norms <= 2^23 with no
 * negative value, or <= 2^22 (tested
 * on the device), the pairwise distances of PRUNE (given cand_d2) and
 * REVERSE come from FP16 MFMA Gram tiles, which are exact there.
 *
 * Outputs: g_ids / g_d2 (n x R, rows padded with -1 / +inf), g_deg (n),
 * ep (1 int), roots (optional, n ints: the roots r in order) and n_roots
 * (host, optional).  PG_EOVERFLOW if CONNECT finds every reached node at
 * degree R.
 */
pg_status pg_prune(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                   const int32_t *cand_ids, const float *cand_d2, int32_t C,
                   const pg_prune_params *p, void *ws, size_t ws_bytes, int32_t *g_ids,
                   float *g_d2, int32_t *g_deg, int32_t *ep, int32_t *roots,
                   int32_t *n_roots);

/* ------------------------------------------------------------------ */
/* Beam search (Alg. 1)                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t k;                  /* results per query, 1 <= k <= L (k < L with exclude) */
    int32_t L;                  /* pool width, L <= 2048; a query's LDS (4 d +
                                   9 L bytes, plus 16 record_L with a record,
                                   plus a 9 KB row tile) must stay within
                                   64 KB, else PG_EUNSUPPORTED */
    int32_t n_entry;            /* number of shared entering points, >= 1 */
    const int32_t *entry_ids;   /* device, n_entry ids (repeats dropped) */
    const int32_t *query_entry; /* optional, device, nq ids: query q enters at
                                   query_entry[q] alone (entry_ids unused) */
    const int32_t *exclude;     /* optional, device, nq ids: query q returns the
                                   first k pool entries other than exclude[q]
                                   (the search itself still passes through it) */
    /* P2K (Section 5.4): distances of the same query recorded by an earlier
       search, used instead of gathering the rows again. */
    const int32_t *record_ids;  /* optional, device, nq x record_L ids (-1 pads);
                                   record_d2 holds their canonical squared
                                   distances to the same query row */
    const float *record_d2;
    int32_t record_L;           /* 0 .. 1024 */
    int32_t *pool_ids;          /* optional, device, nq x L: the final pool of
                                   each query, (d2, id) order, -1 / +inf pads;
                                   the record of a later search */
    float *pool_d2;
    unsigned long long *counts; /* optional, device, 2 values added to:
                                   distances computed, distances taken from
                                   the record */
    const uint16_t *x16;        /* optional, device: an FP16 copy of X made by
                                   pg_half_rows that reported every element
                                   exact; rows are then gathered from it (half
                                   the bytes) and widened, so every distance and
                                   result is unchanged.  A copy that is not exact
                                   changes the distances: do not pass it. */
} pg_search_params;

/* KANNSearch of Alg. 1 for every query row, starting from the entering
 * points: the pool keeps the L closest by (d2, id); the closest unexpanded
 * entry is expanded until the first min(L, |pool|) are expanded.
 * g_ids is n x R with degrees g_deg.  out_ids / out_d2 are nq x k, padded
 * with -1 / +inf.  With Q = X, query_entry[u] = u and exclude[u] = u this is
 * the search phase of OptKCNA (Alg. 5, Phase 3): KANNSearch(G, u, k, L, u),
 * u not being its own candidate.
 * With a record (P2K), a candidate found there takes the recorded distance
 * instead of its row: the search, its results and its pool are the same as
 * without it, provided every recorded distance is the canonical value for
 * that query row (as pool_d2 of a search of the same row is). */
pg_status pg_search(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                    const int32_t *g_ids, int32_t R, const int32_t *g_deg,
                    const float *Q, int64_t nq, int64_t ldq,
                    const pg_search_params *p, int32_t *out_ids, float *out_d2);

/* FP16 copy of the rows of X for pg_search: X16 (device, n rows of
 * (d + 7) / 8 * 8 halves, zero padded, 16-byte aligned) receives the rounded
 * values; *exact (device int32) becomes 1 if every element converted exactly
 * (integers up to 2048 in magnitude, for instance), else 0.  Only an exact
 * copy may be passed to the search. */
pg_status pg_half_rows(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx, uint16_t *X16,
                       int32_t *exact);

/* ------------------------------------------------------------------ */
/* Global HNSW construction (Alg. 7): layer assignment                 */
/* ------------------------------------------------------------------ */
/* The highest layer of every node, as HNSW draws it (Alg. 7, first loop;
 * Section 5.3): levels[u] = floor(-ln U[u] / ln M), evaluated exactly as the
 * number of i >= 1 with U[u] * M^i <= 1 (M^i exact in double precision:
 * levels stop at 31 and at the last i with M^i below 2^53).  U (device, n doubles in (0, 1]) holds the uniform
 * draws; levels (device, n int32) receives the layers and max_level
 * (device, one int32) their maximum m_L.  The layers themselves are built
 * with pg_knn_build, pg_prune and pg_search on each layer's rows (IterNSG),
 * or as complete graphs when a layer has at most M nodes. */
pg_status pg_hnsw_levels(pg_ctx *ctx, const double *U, int64_t n, int32_t M, int32_t *levels,
                         int32_t *max_level);

#ifdef __cplusplus
}
#endif
#endif /* PG_H */
