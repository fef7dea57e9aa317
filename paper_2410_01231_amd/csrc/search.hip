// search.hip -- beam search (the paper's Alg. 1, KANNSearch) for gfx950.
//
// One wave per query.  The pool (<= L keys, ascending by (d2, id), plus an
// expanded flag) lives in LDS.  Each step expands the first unexpanded pool
// entry: its <= R out-neighbours get their squared distance to the query
// (one lane each), candidates already in the pool or not better than the
// L-th pool key are dropped, the rest are sorted with a wave64 bitonic sort
// and merged into the pool by merge-path ranks (binary searches in LDS).
//
// Alg. 1 keeps a pool only; the oracle also remembers every node it has
// evaluated.  Checking the pool alone gives the same search: a node that
// left the pool did so because L better keys arrived, and the L-th key never
// grows, so such a node would be rejected again; a node rejected on
// discovery likewise stays rejected.
#include <algorithm>

#include "pg_common.h"

namespace pgi {

// index of the first key >= x in sorted LDS array a[0..len)
__device__ __forceinline__ int lds_lower_bound(const uint64_t *a, int len, uint64_t x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64) void k_search(const float *__restrict__ X, int64_t ldx, int d,
                                               int64_t n, const int32_t *__restrict__ g, int R,
                                               const int32_t *__restrict__ deg,
                                               const float *__restrict__ Q, int64_t ldq, int64_t nq,
                                               const int32_t *__restrict__ entries, int n_entry,
                                               const int32_t *__restrict__ query_entry,
                                               const int32_t *__restrict__ exclude, int k, int L,
                                               int32_t *__restrict__ out_ids,
                                               float *__restrict__ out_d2) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *qv = reinterpret_cast<float *>(smem);
    uint64_t *pa = reinterpret_cast<uint64_t *>(qv + ((d + 3) & ~3));
    uint64_t *pb = pa + L;
    uint64_t *cand = pb + L;
    uint8_t *fa = reinterpret_cast<uint8_t *>(cand + PG_WAVE);
    uint8_t *fb = fa + L;
    const int lane = lane_id();
    const int64_t qi = blockIdx.x;
    if (qi >= nq) return;
    for (int j = lane; j < d; j += PG_WAVE) qv[j] = Q[qi * ldq + j];
    __builtin_amdgcn_wave_barrier();
    int size = 0;

    // merge the sorted, de-duplicated keys ck (one per lane, KEY_INF padded,
    // none already in the pool) into the pool; new entries are unexpanded
    auto merge_in = [&](uint64_t ck, int cm) {
        cand[lane] = ck;
        __builtin_amdgcn_wave_barrier();
        for (int p = lane; p < size; p += PG_WAVE) {
            const uint64_t x = pa[p];
            const int np = p + lds_lower_bound(cand, cm, x);
            if (np < L) {
                pb[np] = x;
                fb[np] = fa[p];
            }
        }
        if (lane < cm) {
            const int np = lane + lds_lower_bound(pa, size, ck);
            if (np < L) {
                pb[np] = ck;
                fb[np] = 0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        size = min(L, size + cm);
        for (int p = lane; p < size; p += PG_WAVE) {
            pa[p] = pb[p];
            fa[p] = fb[p];
        }
        __builtin_amdgcn_wave_barrier();
    };

    // keys of the candidate ids (one per lane) that may enter the pool
    auto prepare = [&](int32_t id) -> int {
        uint64_t key = KEY_INF;
        if (id >= 0 && id < n) key = pack_key(dist_chain(qv, X + (int64_t)id * ldx, d), id);
        if (key != KEY_INF && size == L && key >= pa[L - 1]) key = KEY_INF;
        if (key != KEY_INF && size > 0) {
            const int at = lds_lower_bound(pa, size, key);
            if (at < size && pa[at] == key) key = KEY_INF;
        }
        int dummy = 0;
        wave_sort(key, dummy);
        const uint64_t prev = shfl64(key, max(lane - 1, 0));
        const bool valid = key != KEY_INF && !(lane > 0 && prev == key);
        const int cm = wave_compact(key, dummy, valid);
        if (cm) merge_in(key, cm);
        return cm;
    };

    if (query_entry)
        prepare(lane == 0 ? query_entry[qi] : -1);
    else
        for (int b = 0; b < n_entry; b += PG_WAVE) prepare(b + lane < n_entry ? entries[b + lane] : -1);

    while (true) {
        int first = 0x7fffffff;
        const int lim = min(L, size);
        for (int p = lane; p < lim; p += PG_WAVE)
            if (!fa[p]) {
                first = p;
                break;
            }
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) first = min(first, __shfl_xor(first, o, PG_WAVE));
        if (first == 0x7fffffff) break;
        const int32_t x = key_id(pa[first]);
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) fa[first] = 1;
        __builtin_amdgcn_wave_barrier();
        const int dx = min(deg[x], R);
        for (int b = 0; b < dx; b += PG_WAVE) prepare(b + lane < dx ? g[(int64_t)x * R + b + lane] : -1);
    }
    // position of the excluded node in the pool (it appears at most once)
    int skip = 0x7fffffff;
    if (exclude) {
        const int32_t ex = exclude[qi];
        for (int p = lane; p < size; p += PG_WAVE)
            if (key_id(pa[p]) == ex) skip = p;
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) skip = min(skip, __shfl_xor(skip, o, PG_WAVE));
    }
    for (int j = lane; j < k; j += PG_WAVE) {
        const int p = j + (j >= skip ? 1 : 0);
        const bool have = p < size;
        out_ids[qi * k + j] = have ? key_id(pa[p]) : -1;
        out_d2[qi * k + j] = have ? key_d2(pa[p]) : __int_as_float(0x7f800000);
    }
}

}  // namespace pgi

using namespace pgi;

extern "C" pg_status pg_search(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                               const int32_t *g_ids, int32_t R, const int32_t *g_deg, const float *Q,
                               int64_t nq, int64_t ldq, const pg_search_params *p, int32_t *out_ids,
                               float *out_d2) {
    if (!ctx || !X || !g_ids || !g_deg || !Q || !p || !out_ids || !out_d2 ||
        (!p->entry_ids && !p->query_entry)) {
        set_error("pg_search: NULL argument");
        return PG_EINVAL;
    }
    if (n < 1 || n >= (int64_t)1 << 31 || nq < 0 || R < 1 || d <= 0 || ldx < d || ldq < d) {
        set_error("pg_search: bad sizes n=%lld nq=%lld d=%d R=%d", (long long)n, (long long)nq, d, R);
        return PG_EINVAL;
    }
    if (p->L < 1 || p->L > 1024 || p->k < 1 || p->k > p->L || (!p->query_entry && p->n_entry < 1)) {
        set_error("pg_search: need 1 <= k <= L <= 1024 and n_entry >= 1 (k=%d L=%d n_entry=%d)", p->k,
                  p->L, p->n_entry);
        return PG_EINVAL;
    }
    if (p->exclude && p->k >= p->L) {
        set_error("pg_search: with exclude, k=%d must be below L=%d", p->k, p->L);
        return PG_EINVAL;
    }
    if (d % 4 || ldx % 4 || ((uintptr_t)X & 15) || d > 8192) {
        set_error("pg_search: d (<= 8192) and ldx must be multiples of 4 and X 16-byte aligned");
        return PG_EUNSUPPORTED;
    }
    if (nq == 0) return PG_OK;
    const size_t lds = sizeof(float) * ((d + 3) & ~3) + sizeof(uint64_t) * (2 * (size_t)p->L + PG_WAVE) +
                       2 * (size_t)p->L;
    TimedLaunch tl(ctx, K_SEARCH, -1.0);
    hipLaunchKernelGGL(k_search, dim3((unsigned)nq), dim3(64), lds, ctx->stream, X, ldx, d, n, g_ids, R,
                       g_deg, Q, ldq, nq, p->entry_ids, p->n_entry, p->query_entry, p->exclude, p->k, p->L,
                       out_ids, out_d2);
    PG_HIP(hipGetLastError());
    return PG_OK;
}
