// search.hip -- beam search (the paper's Alg. 1, KANNSearch) for gfx950.
//
// A wave serves 64 / HW queries, one per segment of HW lanes, with HW the
// smallest of 32 and 64 that holds a node's R out-neighbours: at R <= 32 two
// queries share a wave and every lane computes a distance.  Each query keeps
// its pool (<= L keys, ascending by (d2, id), plus an expanded flag) in its
// own LDS slice and expands one node per step, as Alg. 1 does; the segments
// of a wave step together.
//
// A step expands the first unexpanded pool entry: the node's adjacency row
// and degree load together, its out-neighbours get their squared distance to
// the query (one lane each), candidates already in the pool or not better
// than the L-th pool key are dropped, and the rest are sorted with a bitonic
// sort over the segment.  Each candidate carries its insertion point in the
// pool (the binary search that found it absent), so the merge moves pool
// entries in place, top chunk first, by the number of candidates inserted
// below them, and drops the candidates into the gaps.  The first unexpanded
// entry is tracked from a cursor: entries below both the expanded position
// and the lowest insertion point stay expanded.
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

// bits of a wave ballot that belong to segment s of HW lanes
template <int HW>
__device__ __forceinline__ uint64_t seg_bits(uint64_t ballot, int s) {
    if constexpr (HW == PG_WAVE)
        return ballot;
    else
        return (ballot >> (s * HW)) & ((1ull << HW) - 1);
}

// ascending bitonic sort inside each segment of HW lanes; payload p travels
// with its key
template <int HW>
__device__ __forceinline__ void seg_sort(uint64_t &k, int &p) {
    const int sl = lane_id() % HW;
#pragma unroll
    for (int size = 2; size <= HW; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint64_t ok = shfl_xor64(k, j);
            const int op = (int)xor_lane((uint32_t)p, j);
            const bool asc = (sl & size) == 0;
            const bool lower = (sl & j) == 0;
            const bool take = (lower == asc) ? (ok < k) : (ok > k);
            k = take ? ok : k;
            p = take ? op : p;
        }
    }
}

// row staging: dimensions per slice, LDS floats per staged row (padded
// against bank conflicts of the per-lane row reads)
constexpr int ST_DIMS = 32;
constexpr int ST_STRIDE = 36;
constexpr size_t ST_BYTES = sizeof(float) * PG_WAVE * ST_STRIDE;
// FP16 rows: SD dimensions per slice (SD / 8 lanes of 16 bytes per row), SD +
// 8 halves per staged row.  The tile is smaller than the FP32 one, so more
// waves fit a CU: 32-dimension slices for launches that fill the chip many
// times over, 16 where the smaller tile lets a launch be resident at once.
template <int SD>
constexpr size_t st_bytes16() {
    return sizeof(uint16_t) * PG_WAVE * (SD + 8);
}
static_assert(st_bytes16<32>() <= ST_BYTES, "the FP16 tile fits the FP32 one");

// LDS bytes of one query's slice: query vector, pool keys, record table (RT
// ids and distances), pool flags
__host__ __device__ inline size_t search_slice_bytes(int d, int L, int RT) {
    return ((sizeof(float) * (size_t)((d + 3) & ~3) + sizeof(uint64_t) * (size_t)L +
             (sizeof(int32_t) + sizeof(float)) * (size_t)RT + (size_t)L) +
            15) &
           ~(size_t)15;
}

// P2K record and pool output (all optional)
struct SearchRecord {
    const int32_t *ids;        // nq x len, -1 pads
    const float *d2;
    int len;
    int bits;                  // log2 of the LDS table size (0: no record)
    int32_t *pool_ids;         // nq x L
    float *pool_d2;
    unsigned long long *counts;  // computed, taken from the record
};

__device__ __forceinline__ uint32_t record_slot(int32_t id, int bits) {
    return ((uint32_t)id * 0x9E3779B1u) >> (32 - bits);
}

template <int HW, bool H16, int SD>
__global__ __launch_bounds__(64) void k_search(const float *__restrict__ X, int64_t ldx, int d,
                                               int64_t n, const int32_t *__restrict__ g, int R,
                                               const int32_t *__restrict__ deg,
                                               const float *__restrict__ Q, int64_t ldq, int64_t nq,
                                               const int32_t *__restrict__ entries, int n_entry,
                                               const int32_t *__restrict__ query_entry,
                                               const int32_t *__restrict__ exclude, int k, int L,
                                               int32_t *__restrict__ out_ids,
                                               float *__restrict__ out_d2, SearchRecord rec,
                                               const _Float16 *__restrict__ X16, int64_t ld16) {
    constexpr int QPW = PG_WAVE / HW;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int s = lane / HW, sl = lane % HW, base = s * HW;
    const int RT = rec.bits ? 1 << rec.bits : 0;
    unsigned char *slice = smem + (size_t)s * search_slice_bytes(d, L, RT);
    float *qv = reinterpret_cast<float *>(slice);
    uint64_t *pa = reinterpret_cast<uint64_t *>(qv + ((d + 3) & ~3));
    int32_t *tid = reinterpret_cast<int32_t *>(pa + L);
    float *td = reinterpret_cast<float *>(tid + RT);
    uint8_t *fa = reinterpret_cast<uint8_t *>(td + RT);
    float *tile = reinterpret_cast<float *>(smem + QPW * search_slice_bytes(d, L, RT));
    const int64_t qi = (int64_t)blockIdx.x * QPW + s;
    const bool live = qi < nq;
    if (live)
        for (int j = sl; j < d; j += HW) qv[j] = Q[qi * ldq + j];
    // the record as an open-addressing table (at most half full)
    if (RT) {
        for (int j = sl; j < RT; j += HW) tid[j] = -1;
        __builtin_amdgcn_wave_barrier();
        if (live)
            for (int j = sl; j < rec.len; j += HW) {
                const int32_t id = rec.ids[qi * rec.len + j];
                if (id < 0 || id >= n) continue;
                const float dv = rec.d2[qi * rec.len + j];
                uint32_t h = record_slot(id, rec.bits);
                while (true) {
                    const int32_t old = atomicCAS(&tid[h], -1, id);
                    if (old == -1) {
                        td[h] = dv;
                        break;
                    }
                    if (old == id) break;
                    h = (h + 1) & (RT - 1);
                }
            }
    }
    __builtin_amdgcn_wave_barrier();
    unsigned long long n_comp = 0, n_reuse = 0;
    int size = 0;   // pool size of this lane's query (uniform over its segment)
    int lowest;     // lowest insertion point of the current step

    // keys of the candidate ids (one per lane) that enter the pool: distance,
    // filter, sort, compact, then the in-place merge
    auto prepare = [&](int32_t id) {
        if (id >= n) id = -1;
        // P2K: a candidate in the record takes the recorded distance
        bool found = false;
        float dfound = 0.f;
        if (RT && id >= 0) {
            uint32_t h = record_slot(id, rec.bits);
            while (true) {
                const int32_t t = tid[h];
                if (t == id) {
                    found = true;
                    dfound = td[h];
                    break;
                }
                if (t == -1) break;
                h = (h + 1) & (RT - 1);
            }
        }
        if (rec.counts) {
            n_comp += __popcll(__ballot(id >= 0 && !found));
            n_reuse += __popcll(__ballot(found));
        }
        const int32_t gid = found ? -1 : id;
        // canonical distance chain of each lane's row to its query; the rows
        // of the wave arrive one 32-dimension slice at a time, eight lanes per
        // row reading whole 128-byte lines, through the LDS tile, the next
        // slice loading while the current one is summed
        int32_t rid[PG_WAVE / 8];
#pragma unroll
        for (int i = 0; i < PG_WAVE / 8; ++i) rid[i] = __shfl(gid, i * 8 + (lane >> 3), PG_WAVE);
        float acc = 0.f;
        if constexpr (H16) {
            // an exact FP16 copy of the rows: 64-dimension slices, eight
            // lanes per row each reading 16 bytes of one 128-byte line; the
            // halves stay 16-bit in the tile and are widened when summed
            constexpr int ST_DIMS16 = SD, ST_STRIDE16 = SD + 8, ST_LANES16 = SD / 8;
            constexpr int RPI = PG_WAVE / ST_LANES16;  // rows per load instruction
            const int part = (lane % ST_LANES16) * 8;
            int32_t rid16[PG_WAVE / RPI];
#pragma unroll
            for (int i = 0; i < PG_WAVE / RPI; ++i) rid16[i] = __shfl(gid, i * RPI + lane / ST_LANES16, PG_WAVE);
            constexpr int NV = PG_WAVE / RPI;
            // two slices in flight: va and vb alternate, each refilled two
            // slices ahead as soon as it is in the tile
            uint4 va[NV], vb[NV];
            auto fetch = [&](uint4 (&v)[NV], int c) {
                const int w = min(ST_DIMS16, d - c);
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    v[i] = make_uint4(0u, 0u, 0u, 0u);
                    if (rid16[i] >= 0 && part < w)
                        v[i] = *reinterpret_cast<const uint4 *>(X16 + (int64_t)rid16[i] * ld16 + c + part);
                }
            };
            uint16_t *tile16 = reinterpret_cast<uint16_t *>(tile);
            auto slice = [&](uint4 (&v)[NV], int c) {
                const int w = min(ST_DIMS16, d - c);
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    *reinterpret_cast<uint4 *>(tile16 + (i * RPI + lane / ST_LANES16) * ST_STRIDE16 + part) = v[i];
                if (c + 2 * ST_DIMS16 < d) fetch(v, c + 2 * ST_DIMS16);
                __builtin_amdgcn_wave_barrier();
                for (int j = 0; j < w; j += 8) {
                    const uint4 hx = *reinterpret_cast<const uint4 *>(tile16 + lane * ST_STRIDE16 + j);
                    const float4 y0 = *reinterpret_cast<const float4 *>(qv + c + j);
                    const float4 y1 = *reinterpret_cast<const float4 *>(qv + c + j + 4);
                    const uint32_t hw[4] = {hx.x, hx.y, hx.z, hx.w};
                    const float yy[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
                    const int ne = min(8, w - j);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint16_t bits = (uint16_t)(e & 1 ? hw[e >> 1] >> 16 : hw[e >> 1] & 0xffff);
                        const float t = yy[e] - (float)__builtin_bit_cast(_Float16, bits);
                        if (e < ne) acc = fmaf(t, t, acc);
                    }
                }
                __builtin_amdgcn_wave_barrier();
            };
            fetch(va, 0);
            if (ST_DIMS16 < d) fetch(vb, ST_DIMS16);
            for (int c = 0; c < d; c += 2 * ST_DIMS16) {
                slice(va, c);
                if (c + ST_DIMS16 < d) slice(vb, c + ST_DIMS16);
            }
        } else {
            const int part = (lane & 7) * 4;
            float4 v[PG_WAVE / 8];
            auto fetch = [&](int c) {
                const int w = min(ST_DIMS, d - c);
#pragma unroll
                for (int i = 0; i < PG_WAVE / 8; ++i) {
                    v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (rid[i] >= 0 && part < w)
                        v[i] = *reinterpret_cast<const float4 *>(X + (int64_t)rid[i] * ldx + c + part);
                }
            };
            fetch(0);
            for (int c = 0; c < d; c += ST_DIMS) {
                const int w = min(ST_DIMS, d - c);
#pragma unroll
                for (int i = 0; i < PG_WAVE / 8; ++i)
                    *reinterpret_cast<float4 *>(tile + (i * 8 + (lane >> 3)) * ST_STRIDE + part) = v[i];
                // the next slice is in flight while this one is summed
                if (c + ST_DIMS < d) fetch(c + ST_DIMS);
                __builtin_amdgcn_wave_barrier();
                for (int j = 0; j < w; j += 4) {
                    const float4 x = *reinterpret_cast<const float4 *>(tile + lane * ST_STRIDE + j);
                    const float4 y = *reinterpret_cast<const float4 *>(qv + c + j);
                    float t;
                    t = y.x - x.x;
                    acc = fmaf(t, t, acc);
                    t = y.y - x.y;
                    acc = fmaf(t, t, acc);
                    t = y.z - x.z;
                    acc = fmaf(t, t, acc);
                    t = y.w - x.w;
                    acc = fmaf(t, t, acc);
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        uint64_t key = id >= 0 ? pack_key(found ? dfound : acc, id) : KEY_INF;
        int at = 0;
        if (key != KEY_INF && size == L && key >= pa[L - 1]) key = KEY_INF;
        if (key != KEY_INF && size > 0) {
            at = lds_lower_bound(pa, size, key);
            if (at < size && pa[at] == key) key = KEY_INF;
        }
        // nothing left in any query of the wave: no sort, no merge
        if (__ballot(key != KEY_INF) == 0) return;
        seg_sort<HW>(key, at);
        const uint64_t prev = shfl64(key, base + max(sl - 1, 0));
        const bool valid = key != KEY_INF && !(sl > 0 && prev == key);
        // compact the valid keys to the front of the segment
        const uint64_t m = seg_bits<HW>(__ballot(valid), s);
        const int cm = __popcll(m);
        const uint64_t below = sl ? (m & ((1ull << sl) - 1)) : 0ull;
        const uint64_t below_inv = sl ? (~m & ((1ull << sl) - 1)) : 0ull;
        const int dst = base + (valid ? __popcll(below) : cm + __popcll(below_inv));
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)key);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)(key >> 32));
        at = __builtin_amdgcn_ds_permute(dst * 4, at);
        key = (((uint64_t)hi << 32) | lo);
        // candidates j < cm, ascending, with insertion points at_j (non-
        // decreasing): candidate j goes to at_j + j, pool entry p to p plus
        // the number of j with at_j <= p
        int cmax = cm;
#pragma unroll
        for (int q = 0; q < QPW; ++q) cmax = max(cmax, __builtin_amdgcn_readlane(cm, q * HW));
        if (cmax == 0) return;
        const int at0 = __shfl(at, base, PG_WAVE);
        if (cm > 0) lowest = min(lowest, at0);
        // chunks [c_lo, c_hi) of the pool hold the entries that move
        const int c_hi = cm > 0 ? (size + HW - 1) / HW : 0;
        const int c_lo = cm > 0 ? at0 / HW : 0x7fffffff;
        int chi = c_hi, clo = c_lo;
#pragma unroll
        for (int q = 0; q < QPW; ++q) {
            chi = max(chi, __builtin_amdgcn_readlane(c_hi, q * HW));
            clo = min(clo, __builtin_amdgcn_readlane(c_lo, q * HW));
        }
        for (int c = chi - 1; c >= clo; --c) {
            const int p = c * HW + sl;
            const bool mv = cm > 0 && p < size && p >= at0;
            uint64_t v = 0;
            uint8_t f = 0;
            if (mv) {
                v = pa[p];
                f = fa[p];
            }
            // number of candidates with at_j <= p (binary lifting over the
            // ascending at_j of the segment)
            int sh = 0;
#pragma unroll
            for (int step = HW / 2; step > 0; step >>= 1) {
                const int probe = sh + step - 1;
                const int a = __shfl(at, base + probe, PG_WAVE);
                if (probe < cm && a <= p) sh += step;
            }
            {
                const int a = __shfl(at, base + min(sh, HW - 1), PG_WAVE);
                if (sh < cm && a <= p) sh += 1;
            }
            __builtin_amdgcn_wave_barrier();
            if (mv && p + sh < L) {
                pa[p + sh] = v;
                fa[p + sh] = f;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (sl < cm && at + sl < L) {
            pa[at + sl] = key;
            fa[at + sl] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        size = min(L, size + cm);
    };

    lowest = 0x7fffffff;
    if (query_entry)
        prepare((live && sl == 0) ? query_entry[qi] : -1);
    else
        for (int b = 0; b < n_entry; b += HW) prepare((live && b + sl < n_entry) ? entries[b + sl] : -1);

    int start = 0;  // every pool entry below it is expanded
    while (true) {
        // first unexpanded entry at or after start among the first min(L, size)
        int first = 0x7fffffff;
        const int lim = min(L, size);
        for (int c0 = start; c0 < lim; c0 += HW) {
            const int p = c0 + sl;
            const uint64_t m = seg_bits<HW>(__ballot(p < lim && !fa[p]), s);
            if (m) {
                first = c0 + __builtin_ctzll(m);
                break;
            }
        }
        const bool active = first != 0x7fffffff;
        if (__ballot(active) == 0) break;
        int32_t x = 0, dx = 0;
        if (active) {
            x = key_id(pa[first]);
            __builtin_amdgcn_wave_barrier();
            if (sl == 0) fa[first] = 1;
            dx = min(deg[x], R);
        }
        __builtin_amdgcn_wave_barrier();
        lowest = 0x7fffffff;
        for (int b = 0; b < R; b += HW) {
            const int j = b + sl;
            const int32_t nb = (active && j < R) ? g[(int64_t)x * R + j] : -1;
            prepare(j < dx ? nb : -1);
        }
        if (active) start = min(first + 1, lowest);
    }
    if (rec.counts && lane == 0) {
        atomicAdd(&rec.counts[0], n_comp);
        atomicAdd(&rec.counts[1], n_reuse);
    }
    if (!live) return;
    if (rec.pool_ids)
        for (int p = sl; p < L; p += HW) {
            rec.pool_ids[qi * L + p] = p < size ? key_id(pa[p]) : -1;
            rec.pool_d2[qi * L + p] = p < size ? key_d2(pa[p]) : __int_as_float(0x7f800000);
        }
    // position of the excluded node in the pool (it appears at most once)
    int skip = 0x7fffffff;
    if (exclude) {
        const int32_t ex = exclude[qi];
        for (int p = sl; p < size; p += HW)
            if (key_id(pa[p]) == ex) skip = p;
#pragma unroll
        for (int o = 1; o < HW; o <<= 1) skip = min(skip, __shfl_xor(skip, o, PG_WAVE));
    }
    for (int j = sl; j < k; j += HW) {
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
    if (p->L < 1 || p->L > 2048 || p->k < 1 || p->k > p->L || (!p->query_entry && p->n_entry < 1)) {
        set_error("pg_search: need 1 <= k <= L <= 2048 and n_entry >= 1 (k=%d L=%d n_entry=%d)", p->k,
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
    // two queries per wave when a node's out-neighbours fit 32 lanes and two
    // LDS slices stay within 64 KB
    if (p->record_L < 0 || p->record_L > 1024 || (p->record_L > 0 && (!p->record_ids || !p->record_d2)) ||
        (!p->pool_ids != !p->pool_d2)) {
        set_error("pg_search: record needs ids and d2 with 0 <= record_L <= 1024; pool_ids and pool_d2 go together");
        return PG_EINVAL;
    }
    SearchRecord rec{p->record_L ? p->record_ids : nullptr, p->record_d2, p->record_L, 0, p->pool_ids, p->pool_d2,
                     p->counts};
    if (p->record_L > 0)
        while ((1 << rec.bits) < 2 * p->record_L) ++rec.bits;
    const int RT = rec.bits ? 1 << rec.bits : 0;
    const size_t slice = search_slice_bytes(d, p->L, RT);
    const size_t stb = p->x16 ? st_bytes16<32>() : ST_BYTES;
    if (slice + stb > 65536) {
        set_error("pg_search: a query needs %zu bytes of LDS (d=%d, L=%d, record_L=%d), more than 64 KB", slice + stb,
                  d, p->L, p->record_L);
        return PG_EUNSUPPORTED;
    }
    const bool pair = R <= 32 && 2 * slice + stb <= 65536;
    if (p->x16 && ((uintptr_t)p->x16 & 15)) {
        set_error("pg_search: x16 must be 16-byte aligned");
        return PG_EINVAL;
    }
    const _Float16 *x16 = reinterpret_cast<const _Float16 *>(p->x16);
    const int64_t ld16 = ((int64_t)d + 7) & ~(int64_t)7;
    TimedLaunch tl(ctx, K_SEARCH, -1.0);
    const dim3 g2((unsigned)((nq + 1) / 2)), g1((unsigned)nq);
    const size_t l2 = 2 * slice + stb, l1 = slice + stb;
    // FP16 rows: the narrower slices where they let the whole launch be
    // resident at once and the wider ones do not
    bool narrow = false;
    const int64_t waves = pair ? (nq + 1) / 2 : nq;
    if (x16 && waves > 4 * (int64_t)ctx->num_cu) {
        const size_t nb = (pair ? 2 * slice : slice) + st_bytes16<16>();
        int o32 = 0, o16 = 0;
        if (pair) {
            PG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o32, reinterpret_cast<const void *>(&k_search<32, true, 32>), 64, l2));
            PG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o16, reinterpret_cast<const void *>(&k_search<32, true, 16>), 64, nb));
        } else {
            PG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o32, reinterpret_cast<const void *>(&k_search<64, true, 32>), 64, l1));
            PG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o16, reinterpret_cast<const void *>(&k_search<64, true, 16>), 64, nb));
        }
        narrow = waves > (int64_t)o32 * ctx->num_cu && waves <= (int64_t)o16 * ctx->num_cu;
    }
    const size_t l2n = 2 * slice + st_bytes16<16>(), l1n = slice + st_bytes16<16>();
#define PG_SEARCH_ARGS                                                                                          \
    X, ldx, d, n, g_ids, R, g_deg, Q, ldq, nq, p->entry_ids, p->n_entry, p->query_entry, p->exclude, p->k, p->L, \
        out_ids, out_d2, rec, x16, ld16
    if (pair && x16 && narrow)
        hipLaunchKernelGGL((k_search<32, true, 16>), g2, dim3(64), l2n, ctx->stream, PG_SEARCH_ARGS);
    else if (pair && x16)
        hipLaunchKernelGGL((k_search<32, true, 32>), g2, dim3(64), l2, ctx->stream, PG_SEARCH_ARGS);
    else if (pair)
        hipLaunchKernelGGL((k_search<32, false, 32>), g2, dim3(64), l2, ctx->stream, PG_SEARCH_ARGS);
    else if (x16 && narrow)
        hipLaunchKernelGGL((k_search<64, true, 16>), g1, dim3(64), l1n, ctx->stream, PG_SEARCH_ARGS);
    else if (x16)
        hipLaunchKernelGGL((k_search<64, true, 32>), g1, dim3(64), l1, ctx->stream, PG_SEARCH_ARGS);
    else
        hipLaunchKernelGGL((k_search<64, false, 32>), g1, dim3(64), l1, ctx->stream, PG_SEARCH_ARGS);
#undef PG_SEARCH_ARGS
    PG_HIP(hipGetLastError());
    return PG_OK;
}

namespace pgi {

// FP16 copy of the rows of X (row stride d rounded up to 8, zero padded);
// *exact becomes 0 if any element does not survive the round trip.  Grid
// stride; one flag update per block at most (updates of one address from
// every block serialise, so one per element group would dominate the copy).
__global__ __launch_bounds__(256) void k_half_rows(const float *__restrict__ X, int64_t n, int d, int64_t ldx,
                                                   _Float16 *__restrict__ X16, int64_t ld16,
                                                   int32_t *__restrict__ exact) {
    bool bad = false;
    const int64_t total = n * ld16;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / ld16;
        const int c = (int)(t % ld16);
        float x = 0.f;
        if (c < d) x = X[r * ldx + c];
        const _Float16 h = (_Float16)x;
        X16[t] = h;
        bad |= (float)h != x;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0 && __atomic_load_n(exact, __ATOMIC_RELAXED) != 0)
        atomicAnd(exact, 0);
}

__global__ void k_set_flag(int32_t *__restrict__ p) { *p = 1; }

}  // namespace pgi

extern "C" pg_status pg_half_rows(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                  uint16_t *X16, int32_t *exact) {
    if (!ctx || !X || !X16 || !exact) {
        set_error("pg_half_rows: NULL argument");
        return PG_EINVAL;
    }
    if (n < 1 || d < 1 || ldx < d) {
        set_error("pg_half_rows: bad sizes n=%lld d=%d ldx=%lld", (long long)n, d, (long long)ldx);
        return PG_EINVAL;
    }
    const int64_t ld16 = ((int64_t)d + 7) & ~(int64_t)7;
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, ctx->stream, exact);
    const int64_t total = n * ld16;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, (int64_t)ctx->num_cu * 16);
    hipLaunchKernelGGL(k_half_rows, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, X, n, d, ldx,
                       reinterpret_cast<_Float16 *>(X16), ld16, exact);
    PG_HIP(hipGetLastError());
    return PG_OK;
}
