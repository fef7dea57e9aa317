// knn.hip -- approximate kNN graph by NN-Descent local joins (the paper's
// initialization phase: Section 3.1 and Alg. 2 Phase 1 build G_k0 with
// KGraph; Section 6, Exp. 12: k random neighbours, then distances to 2-hop
// neighbours), plus exact brute-force kNN, for gfx950.
//
// One iteration, all kernels on the context stream:
//   k_sample      wave per node: sample <= S new entries by hash, flip them to
//                 old, list the old ones, count reverse in-degrees
//   scan x2       exclusive prefix sums of the in-degrees
//   k_rev_scatter wave per node: CSR reverse lists
//   k_build_join  wave per node: keep the S smallest-hash reverse entries,
//                 form new(u) and old(u) (the join set of u)
//   k_join        wave per source u: the join set's vectors are staged
//                 through LDS in 16-dim chunks; every new-new and new-old pair
//                 gets its squared distance in registers (micro-tiles);
//                 a pair is proposed to each end whose K-th key it beats and
//                 appended to that end's proposal bucket.  k_join_mfma runs
//                 the same join as MFMA Gram tiles on data where the norm
//                 expansion is exact; k_join_hybrid, on float data, takes
//                 16-bit MFMA estimates and the exact chains of the pairs
//                 the estimates cannot settle
//   k_merge       wave per node: each list becomes the K smallest distinct
//                 keys of (list U bucket) by wave64 bitonic sort and merge
// Sources are joined in several passes (chunks) per iteration; each pass is
// merged before the next one starts.  Merging is a set operation (K smallest
// distinct keys of a union), and a proposal rejected by the tighter K-th key
// of a later pass could not have entered the list, so the result equals the
// single synchronous iteration whatever the pass boundaries.  A bucket that
// fills up marks its node; the pass is repeated for marked nodes only, without
// the keys those nodes already list, until none overflows (each repeat
// inserts at least one new key, so the node's K-th key strictly falls).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <mutex>
#include <vector>

#include "pg_common.h"

namespace pgi {

enum {
    C_UPDATES = 0,
    C_PROPOSALS = 1,
    C_OVF = 2,
    C_PAIRS = 3,
    C_SPILL = 4,
    C_RECHECK = 5,
    C_MEMBERS = 6,  // join-set members of the sources that join (rows each join gathers)
    C_NCOUNTERS = 8
};

// Counters are striped: NSTRIPE slots of CSTRIDE words (one 128-byte line
// each), and a workgroup adds to slot blockIdx.x % NSTRIPE.  Device-scope
// atomics on one address from every XCD serialize; spread over lines they do
// not.  The spill list is cut into NSTRIPE segments of `seg` entries the same
// way, each filled through the C_SPILL word of its slot.
constexpr int NSTRIPE = 256;
constexpr int CSTRIDE = 16;
enum { C_SPILLMAX = 7 };  // reduced view only: largest (clipped) segment fill

__device__ __forceinline__ unsigned long long *stripe_of(unsigned long long *c) {
    return c + (blockIdx.x % NSTRIPE) * CSTRIDE;
}

// out[f] = sum over slots of field f; C_SPILL counts stored entries (each
// segment clipped at seg) and C_SPILLMAX the largest clipped fill.  One block
// of NSTRIPE threads.
__global__ __launch_bounds__(NSTRIPE) void k_counters_reduce(const unsigned long long *__restrict__ c, int64_t seg,
                                                             unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[C_NCOUNTERS][NSTRIPE];
    const int t = threadIdx.x;
    for (int f = 0; f < C_NCOUNTERS; ++f) {
        unsigned long long v = c[t * CSTRIDE + f];
        if (f == C_SPILL) v = min(v, (unsigned long long)seg);
        if (f == C_SPILLMAX) v = min(c[t * CSTRIDE + C_SPILL], (unsigned long long)seg);
        sh[f][t] = v;
    }
    __syncthreads();
    for (int o = NSTRIPE / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int f = 0; f < C_NCOUNTERS; ++f)
                sh[f][t] = f == C_SPILLMAX ? max(sh[f][t], sh[f][t + o]) : sh[f][t] + sh[f][t + o];
        __syncthreads();
    }
    if (t < C_NCOUNTERS) out[t] = sh[t][0];
}

__global__ __launch_bounds__(NSTRIPE) void k_counters_clear(unsigned long long *__restrict__ c, int field) {
    c[threadIdx.x * CSTRIDE + field] = 0ull;
}

// ---------------------------------------------------------------------------
// Collections.  A build may hold several collections, each a contiguous range
// of rows of X; every random draw then uses ids local to the node's
// collection, so each collection's lists are those of a build of its rows
// alone (ids, ties and hashes all shift by the same base).  of == nullptr
// means one collection of all n rows.  A frozen collection (its stop rule
// met) takes no samples, so its lists no longer change.
// ---------------------------------------------------------------------------
struct Segs {
    const int32_t *of;      // n: collection of each node
    const int64_t *off;     // ncoll + 1: first row of each collection
    const uint8_t *frozen;  // ncoll
};

__device__ __forceinline__ int64_t seg_base(const Segs &sg, int64_t u) {
    return sg.of ? sg.off[sg.of[u]] : 0;
}

// ---------------------------------------------------------------------------
// init: K distinct random neighbours, hash4(seed, 0, u, attempt) mod (n-1)
// ---------------------------------------------------------------------------
// Rows come from X, or, when X16 is given (an exact FP16 copy, rows of d16
// halves), from the copy at half the bytes: the values, and so the chains,
// are the same.
__global__ __launch_bounds__(256) void k_init(const float *__restrict__ X, int64_t ldx, int d,
                                              const _Float16 *__restrict__ X16, int d16,
                                              int64_t n, int K, uint64_t seed,
                                              uint64_t *__restrict__ keys,
                                              uint64_t *__restrict__ newm,
                                              uint64_t *__restrict__ insm, Segs sg) {
    constexpr int IDC = 32, IST = IDC + 4;  // dims per LDS chunk, row stride (floats)
    __shared__ int32_t acc_s[4][PG_WAVE];
    __shared__ __align__(16) float rows_s[4][(PG_WAVE + 1) * IST];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t u = (int64_t)blockIdx.x * 4 + w;
    if (u >= n) return;
    int32_t *acc = acc_s[w];
    int na = 0;
    uint64_t j0 = 0;
    const int64_t base = seg_base(sg, u);
    const uint64_t ul = (uint64_t)(u - base);
    const uint64_t nm1 = (uint64_t)((sg.of ? sg.off[sg.of[u] + 1] - base : n) - 1);
    while (na < K) {
        const uint64_t r = hash4(seed, 0, ul, j0 + (uint64_t)lane) % nm1;
        const int32_t c = (int32_t)(base + (int64_t)(r >= ul ? r + 1 : r));
        bool dup = false;
        for (int i = 0; i < na; ++i) dup |= (acc[i] == c);
        for (int i = 0; i < PG_WAVE - 1; ++i) {
            const int ci = __builtin_amdgcn_readlane(c, i);
            dup |= (i < lane) && (ci == c);
        }
        const uint64_t m = __ballot(!dup);
        const int rank = __popcll(m & lanemask_lt());
        if (!dup && rank < K - na) acc[na + rank] = c;
        __builtin_amdgcn_wave_barrier();
        na += min(__popcll(m), K - na);
        j0 += PG_WAVE;
    }
    const int32_t id = lane < K ? acc[lane] : -1;
    // canonical chains of u against its K draws: the 64 rows and u's row pass
    // through LDS in chunks of IDC dimensions (coalesced loads, one read each)
    float *rs = rows_s[w];
    float s = 0.0f;
    for (int c0 = 0; c0 < d; c0 += IDC) {
        const int vpr = min(IDC, d - c0) / 4;  // float4 per row in this chunk
        __builtin_amdgcn_wave_barrier();
        for (int v = lane; v < (PG_WAVE + 1) * vpr; v += PG_WAVE) {
            const int r = v / vpr, c = (v - r * vpr) * 4;
            const int64_t rid = r < PG_WAVE ? (r < K ? (int64_t)acc[r] : -1) : u;
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            if (rid >= 0) {
                if (X16) {
                    const uint2 h = *reinterpret_cast<const uint2 *>(X16 + rid * d16 + c0 + c);
                    x = make_float4((float)__builtin_bit_cast(_Float16, (uint16_t)(h.x & 0xffffu)),
                                    (float)__builtin_bit_cast(_Float16, (uint16_t)(h.x >> 16)),
                                    (float)__builtin_bit_cast(_Float16, (uint16_t)(h.y & 0xffffu)),
                                    (float)__builtin_bit_cast(_Float16, (uint16_t)(h.y >> 16)));
                } else {
                    x = *reinterpret_cast<const float4 *>(X + rid * ldx + c0 + c);
                }
            }
            *reinterpret_cast<float4 *>(rs + r * IST + c) = x;
        }
        __builtin_amdgcn_wave_barrier();
        if (id >= 0) {
            for (int q = 0; q < 4 * vpr; q += 4) {
                const float4 x = *reinterpret_cast<const float4 *>(rs + PG_WAVE * IST + q);
                const float4 y = *reinterpret_cast<const float4 *>(rs + lane * IST + q);
                float t;
                t = x.x - y.x;
                s = fmaf(t, t, s);
                t = x.y - y.y;
                s = fmaf(t, t, s);
                t = x.z - y.z;
                s = fmaf(t, t, s);
                t = x.w - y.w;
                s = fmaf(t, t, s);
            }
        }
    }
    uint64_t key = KEY_INF;
    if (id >= 0) key = pack_key(s, id);
    wave_sort(key);
    if (lane < K) keys[u * K + lane] = key;
    if (lane == 0) {
        newm[u] = (K == 64) ? ~0ull : ((1ull << K) - 1ull);
        insm[u] = 0;
    }
}

// ---------------------------------------------------------------------------
// sampling (step (a) of the iteration)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample(const uint64_t *__restrict__ keys,
                                                uint64_t *__restrict__ newm,
                                                int64_t n, int K, int S, uint64_t seed,
                                                uint64_t stream, int32_t *__restrict__ nf,
                                                int32_t *__restrict__ nf_c,
                                                int32_t *__restrict__ of,
                                                int32_t *__restrict__ of_c,
                                                int32_t *__restrict__ rn_cnt,
                                                int32_t *__restrict__ ro_cnt,
                                                int32_t *__restrict__ nf_slot,
                                                int32_t *__restrict__ of_slot, Segs sg) {
    const int lane = lane_id();
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= n) return;
    if (sg.of && sg.frozen[sg.of[u]]) {
        if (lane == 0) {
            nf_c[u] = 0;
            of_c[u] = 0;
        }
        return;
    }
    const int64_t base = seg_base(sg, u);
    const uint64_t nm = newm[u];
    const uint64_t key = lane < K ? keys[u * K + lane] : KEY_INF;
    const int32_t id = key_id(key);
    const bool isnew = lane < K && ((nm >> lane) & 1ull);
    const bool isold = lane < K && !isnew;
    uint64_t sk = isnew ? sample_key(hash4(seed, stream, (uint64_t)(u - base), (uint64_t)(id - base)), id) : KEY_INF;
    int pos = lane;
    wave_sort(sk, pos);
    const bool sel = lane < S && sk != KEY_INF;
    uint64_t selbit = sel ? (1ull << pos) : 0ull;
#pragma unroll
    for (int off = 1; off < PG_WAVE; off <<= 1) selbit |= shfl_xor64(selbit, off);
    if (sel) {
        const int32_t v = key_id(sk);
        nf[u * S + lane] = v;
        nf_slot[u * S + lane] = atomicAdd(&rn_cnt[v], 1);  // u's place in v's reverse list
    }
    const uint64_t om = __ballot(isold);
    if (isold) {
        const int at = __popcll(om & lanemask_lt());
        of[u * K + at] = id;
        of_slot[u * K + at] = atomicAdd(&ro_cnt[id], 1);
    }
    if (lane == 0) {
        nf_c[u] = min(S, __popcll(nm & ((K == 64) ? ~0ull : ((1ull << K) - 1ull))));
        of_c[u] = __popcll(om);
        newm[u] = nm & ~selbit;
    }
}

// ---------------------------------------------------------------------------
// reverse lists (CSR)
// ---------------------------------------------------------------------------
// u goes to its place (taken by the counting atomics of k_sample) in the
// reverse list of every v it sampled
__global__ __launch_bounds__(256) void k_rev_scatter(int64_t n, const int32_t *__restrict__ nf,
                                                     const int32_t *__restrict__ nf_c, int S,
                                                     const int32_t *__restrict__ of,
                                                     const int32_t *__restrict__ of_c, int K,
                                                     const int64_t *__restrict__ rn_off,
                                                     const int32_t *__restrict__ nf_slot,
                                                     int32_t *__restrict__ rn_list,
                                                     const int64_t *__restrict__ ro_off,
                                                     const int32_t *__restrict__ of_slot,
                                                     int32_t *__restrict__ ro_list) {
    const int lane = lane_id();
    const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= n) return;
    if (lane < nf_c[u]) {
        const int32_t v = nf[u * S + lane];
        rn_list[rn_off[v] + nf_slot[u * S + lane]] = (int32_t)u;
    }
    if (lane < of_c[u]) {
        const int32_t v = of[u * K + lane];
        ro_list[ro_off[v] + of_slot[u * K + lane]] = (int32_t)u;
    }
}

// S smallest sample keys among the CSR list of v (stream `stream`), ascending;
// a list of at most S entries is selected whole (ids only, in list order).
__device__ __forceinline__ uint64_t select_reverse(int64_t v, const int64_t *__restrict__ off,
                                                   const int32_t *__restrict__ list,
                                                   uint64_t seed, uint64_t stream, int S, int64_t base) {
    const int lane = lane_id();
    const int64_t beg = off[v], cnt = off[v + 1] - beg;
    if (cnt <= S)  // every entry is selected; callers use the ids only
        return lane < cnt ? (uint64_t)(uint32_t)list[beg + lane] : KEY_INF;
    uint64_t top = KEY_INF;
    int dummy = 0;
    for (int64_t b = 0; b < cnt; b += PG_WAVE) {
        uint64_t sk = KEY_INF;
        if (b + lane < cnt) {
            const int32_t x = list[beg + b + lane];
            sk = sample_key(hash4(seed, stream, (uint64_t)(v - base), (uint64_t)(x - base)), x);
        }
        int p = 0;
        wave_sort(sk, p);
        wave_merge_lowest(top, dummy, sk, p);
    }
    return top;
}

__device__ __forceinline__ bool wave_contains(uint64_t sorted, uint64_t x) {
    const int c = wave_count_less(sorted, x);
    const uint64_t at = shfl64(sorted, min(c, PG_WAVE - 1));
    return x != KEY_INF && c < PG_WAVE && at == x;
}

// ---------------------------------------------------------------------------
// join sets: new(v) = new_f(v) U Rnew(v); old(v) = (old_f(v) U Rold(v)) \ new(v)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_build_join(
    int64_t n, int K, int S, uint64_t seed, uint64_t stream_rn, uint64_t stream_ro,
    const int32_t *__restrict__ nf, const int32_t *__restrict__ nf_c,
    const int32_t *__restrict__ of, const int32_t *__restrict__ of_c,
    const int64_t *__restrict__ rn_off, const int32_t *__restrict__ rn_list,
    const int64_t *__restrict__ ro_off, const int32_t *__restrict__ ro_list,
    int32_t *__restrict__ jn, int32_t *__restrict__ jn_c, int JN, int32_t *__restrict__ jo,
    int32_t *__restrict__ jo_c, int JO, unsigned long long *__restrict__ counters, Segs sg) {
    __shared__ unsigned long long pairs_s[4], memb_s[4];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    unsigned long long pairs = 0, memb = 0;
    // grid-stride over nodes, one wave each; one counter atomic per block
    for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
        const int64_t base = seg_base(sg, v);
        const uint64_t rsel = select_reverse(v, rn_off, rn_list, seed, stream_rn, S, base);
        const uint64_t osel = select_reverse(v, ro_off, ro_list, seed, stream_ro, S, base);
        // new set (|new_f| <= S and |Rnew| <= S, S <= 32: one id per lane)
        const int nfc = nf_c[v];
        const uint64_t rsel_id = (lane < S && rsel != KEY_INF) ? (uint64_t)(uint32_t)key_id(rsel) : KEY_INF;
        uint64_t a = lane < nfc ? (uint64_t)(uint32_t)nf[v * S + lane] : KEY_INF;
        {
            const int r = lane - nfc;
            const uint64_t fromr = shfl64(rsel_id, max(0, min(r, PG_WAVE - 1)));
            if (r >= 0 && r < S) a = fromr;
        }
        int pa = 0;
        wave_sort(a, pa);
        const uint64_t prev = from_lane_below64(a);
        const int nn = wave_compact(a, pa, a != KEY_INF && (lane == 0 || prev != a));
        if (lane < nn) jn[v * JN + lane] = (int32_t)a;
        // old set
        const int ofc = of_c[v];
        uint64_t A = lane < ofc ? (uint64_t)(uint32_t)of[v * K + lane] : KEY_INF;
        int pA = 0;
        wave_sort(A, pA);
        uint64_t Bk = (lane < S && osel != KEY_INF) ? (uint64_t)(uint32_t)key_id(osel) : KEY_INF;
        int pB = 0;
        wave_sort(Bk, pB);
        // cross-lane lookups run on every lane (no short-circuit around shuffles)
        const bool b_in_A = wave_contains(A, Bk);
        const bool b_in_new = wave_contains(a, Bk);
        const bool a_in_new = wave_contains(a, A);
        const bool b_ok = Bk != KEY_INF && !b_in_A && !b_in_new;
        const bool a_ok = A != KEY_INF && !a_in_new;
        const int ca = wave_compact(A, pA, a_ok);
        const int cb = wave_compact(Bk, pB, b_ok);
        if (lane < ca) jo[v * JO + lane] = (int32_t)A;
        if (lane < cb) jo[v * JO + ca + lane] = (int32_t)Bk;
        if (lane == 0) {
            jn_c[v] = nn;
            jo_c[v] = ca + cb;
            pairs += (unsigned long long)nn * (nn - 1) / 2 + (unsigned long long)nn * (ca + cb);
            memb += (nn > 0 && nn + ca + cb >= 2) ? (unsigned long long)(nn + ca + cb) : 0ull;
        }
    }
    if (lane == 0) {
        pairs_s[w] = pairs;
        memb_s[w] = memb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = pairs_s[0] + pairs_s[1] + pairs_s[2] + pairs_s[3];
        const unsigned long long mm = memb_s[0] + memb_s[1] + memb_s[2] + memb_s[3];
        unsigned long long *cs = stripe_of(counters);
        if (t) atomicAdd(&cs[C_PAIRS], t);
        if (mm) atomicAdd(&cs[C_MEMBERS], mm);
    }
}

// ---------------------------------------------------------------------------
// local join tile
// ---------------------------------------------------------------------------
// Is `key` one of the K sorted keys of a list?  (binary search)
__device__ __forceinline__ bool list_has(const uint64_t *__restrict__ row, int K, uint64_t key) {
    int lo = 0, hi = K;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < K && row[lo] == key;
}

// Proposals beyond their node's bucket go to the workgroup's spill segment
// (a range reserved per member of the join set; cap = the segment end); when
// that is full too, the node is marked for a repeat pass.  `counters` is the
// workgroup's counter slot.
__device__ __forceinline__ void spill_put(int32_t t, uint64_t key, int64_t pos,
                                          int32_t *__restrict__ spill_t,
                                          uint64_t *__restrict__ spill_k, int64_t cap,
                                          uint8_t *__restrict__ ovf_next,
                                          unsigned long long *__restrict__ counters) {
    if (pos < cap) {
        spill_t[pos] = t;
        spill_k[pos] = key;
    } else {
        ovf_next[t] = 1;
        atomicAdd(&counters[C_OVF], 1ull);
    }
}

// Reserve this wave's bucket ranges for members i = lane + 64 j: one global
// atomic per member on its proposal counter, and one per wave and j on the
// fill counter of the workgroup's spill segment for the parts that do not fit
// in the buckets.
__device__ __forceinline__ unsigned long long reserve_ranges(
    int m, const int32_t *__restrict__ ids, int32_t *__restrict__ cnt, int32_t *__restrict__ base,
    int64_t *__restrict__ sbase, int32_t *__restrict__ pcnt, int B,
    unsigned long long *__restrict__ cslot, int64_t seg_begin) {
    const int lane = lane_id();
    unsigned long long props = 0;
    for (int j0 = 0; j0 < m; j0 += PG_WAVE) {
        const int i = j0 + lane;
        int over = 0;
        if (i < m) {
            const int c = cnt[i];
            if (c > 0) {
                const int b0 = atomicAdd(&pcnt[ids[i]], c);
                base[i] = b0;
                over = max(0, b0 + c - max(b0, B));  // entries past the bucket
                props += (unsigned long long)c;
            }
            cnt[i] = 0;
        }
        // exclusive prefix of `over` across the wave, one atomic for the total
        int incl = over;
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) {
            const int t = __shfl_up(incl, o, PG_WAVE);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, PG_WAVE - 1, PG_WAVE);
        unsigned long long sb = 0;
        if (total > 0) {
            if (lane == PG_WAVE - 1) sb = atomicAdd(&cslot[C_SPILL], (unsigned long long)total);
            sb = (unsigned long long)__shfl((long long)sb, PG_WAVE - 1, PG_WAVE);
        }
        if (over > 0) sbase[i] = seg_begin + (int64_t)(sb + (unsigned long long)(incl - over));
    }
    return props;
}

// ids per value (counting sort of small integer keys)
// The same for one member per lane (mi < 0: none), in a single pass.
__device__ __forceinline__ unsigned long long reserve_lanes(int mi, const int32_t *__restrict__ ids,
                                                           int32_t *__restrict__ cnt, int32_t *__restrict__ base,
                                                           int64_t *__restrict__ sbase, int32_t *__restrict__ pcnt,
                                                           int B, unsigned long long *__restrict__ cslot,
                                                           int64_t seg_begin) {
    const int lane = lane_id();
    unsigned long long props = 0;
    int over = 0;
    if (mi >= 0) {
        const int c = cnt[mi];
        if (c > 0) {
            const int b0 = atomicAdd(&pcnt[ids[mi]], c);
            base[mi] = b0;
            over = max(0, b0 + c - max(b0, B));
            props = (unsigned long long)c;
        }
        cnt[mi] = 0;
    }
    int incl = over;
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) {
        const int t = __shfl_up(incl, o, PG_WAVE);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, PG_WAVE - 1, PG_WAVE);
    unsigned long long sb = 0;
    if (total > 0) {
        if (lane == PG_WAVE - 1) sb = atomicAdd(&cslot[C_SPILL], (unsigned long long)total);
        sb = (unsigned long long)__shfl((long long)sb, PG_WAVE - 1, PG_WAVE);
    }
    if (over > 0) sbase[mi] = seg_begin + (int64_t)(sb + (unsigned long long)(incl - over));
    return props;
}

__global__ void k_count_ids(const int32_t *__restrict__ key, int64_t cnt, int32_t *__restrict__ kcnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) atomicAdd(&kcnt[key[i]], 1);
}

// spilled entries per target node, over every segment (grid.y = segment)
__global__ void k_spill_count(const int32_t *__restrict__ spill_t, const unsigned long long *__restrict__ c,
                              int64_t seg, int32_t *__restrict__ scnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = blockIdx.y;
    const int64_t fill = min((int64_t)c[s * CSTRIDE + C_SPILL], seg);
    if (j < fill) atomicAdd(&scnt[spill_t[s * seg + j]], 1);
}

__global__ void k_spill_scatter(const int32_t *__restrict__ spill_t, const uint64_t *__restrict__ spill_k,
                                const unsigned long long *__restrict__ c, int64_t seg,
                                const int64_t *__restrict__ soff, int32_t *__restrict__ scur,
                                uint64_t *__restrict__ sorted) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = blockIdx.y;
    const int64_t fill = min((int64_t)c[s * CSTRIDE + C_SPILL], seg);
    if (j < fill) {
        const int64_t i = s * seg + j;
        const int32_t t = spill_t[i];
        sorted[soff[t] + atomicAdd(&scur[t], 1)] = spill_k[i];
    }
}

constexpr int JW = 2;            // sources (waves) per workgroup
constexpr int JT = JW * PG_WAVE;
constexpr int JDC = 8;           // dims per LDS chunk
constexpr int TRW = 4, TCL = 8;  // largest micro-tile: 4 new members x 8 members
template <int R, int C>
struct JoinTile {
    static constexpr int rows = R, cols = C;
};
// float4 staging loads per lane and chunk for a join set of at most 160
// members (3S + K with S <= 32, K <= 64)
constexpr int JPF = (160 * (JDC / 4) + PG_WAVE - 1) / PG_WAVE;

// LDS column stride (floats) for a join set of at most maxm members: a
// multiple of 4 (16-byte reads), padded off a multiple of 8.
__host__ __device__ __forceinline__ int join_mps(int maxm) {
    const int mp = (maxm + TCL - 1) / TCL * TCL;
    return mp + 4;
}

// LDS bytes of one wave's region
__host__ __device__ __forceinline__ size_t join_wave_lds(int maxm) {
    const int mps = join_mps(maxm);
    return (size_t)JDC * mps * 4 + (size_t)mps * (8 + 8 + 4 + 4 + 4 + 4);
}

static size_t join_lds_bytes(int maxm) { return JW * join_wave_lds(maxm); }

// Local join, one wave per source u.  The join set (new members first, then
// old) is staged dim-major in the wave's LDS region, tile[k][i] = x_i[c0 + k],
// JDC dims at a time: with 4 x 8 micro-tiles a lane's 8 consecutive members
// at one dim are two conflict-free 16-byte reads and its 4 new members one
// (shared by the lanes of the same row block).  The pair set is covered by
// micro-tiles of 4 x 8, 4 x 4, 2 x 4 or 1 x 2 (new members x members, the
// smallest shape that needs no more rounds), one per lane per round; every pair's squared distance
// accumulates in registers in the canonical order (dims ascending, one fma
// per dim).  Proposals are counted per (lane, member), ranges are reserved
// per member in the node's bucket (then the spill list), and written.
// Held to three waves per SIMD (167 VGPRs with 8-dimension chunks; 16-dim
// chunks took 221 and two waves): GIST-shaped join 1.42 -> 1.32 s,
// Deep-shaped 3.13 -> 2.26 s.  Four waves would spill.
__global__ __launch_bounds__(JT, 3) void k_join(
    const float *__restrict__ X, int64_t ldx, int d, int K, const int32_t *__restrict__ jn,
    const int32_t *__restrict__ jn_c, int JN, const int32_t *__restrict__ jo,
    const int32_t *__restrict__ jo_c, int JO, const uint64_t *__restrict__ keys,
    int32_t *__restrict__ pcnt, uint64_t *__restrict__ bucket, int B,
    int32_t *__restrict__ spill_t, uint64_t *__restrict__ spill_k, int64_t seg,
    uint8_t *__restrict__ ovf_next, const uint8_t *__restrict__ mark, const int32_t *__restrict__ order,
    int64_t n, PassRange pr, int maxm, unsigned long long *__restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int MPS = join_mps(maxm);
    const int lane = lane_id();
    const int wv = threadIdx.x / PG_WAVE;
    const int64_t nlog = (pr.items + JW - 1) / JW;
    const int64_t lb = xcd_logical_block(blockIdx.x, nlog);
    const int64_t u = lb < nlog ? pass_source(order, n, pr, lb * JW + wv) : -1;
    if (u < 0) return;
    unsigned long long *cslot = stripe_of(counters);
    const int64_t seg_begin = (int64_t)(blockIdx.x % NSTRIPE) * seg, seg_end = seg_begin + seg;
    unsigned char *region = smem + (size_t)wv * join_wave_lds(maxm);
    float *tile = reinterpret_cast<float *>(region);
    uint64_t *kth = reinterpret_cast<uint64_t *>(tile + (size_t)JDC * MPS);
    int64_t *sbase = reinterpret_cast<int64_t *>(kth + MPS);
    int32_t *ids = reinterpret_cast<int32_t *>(sbase + MPS);
    int32_t *cnt = ids + MPS;
    int32_t *base = cnt + MPS;
    int32_t *mk = base + MPS;

    const int nn = jn_c[u], no = jo_c[u];
    const int m = nn + no;
    if (nn == 0 || m < 2) return;
    const int mp = (m + TCL - 1) / TCL * TCL;
    bool anymark = false;
    for (int i = lane; i < mp; i += PG_WAVE) {
        const int32_t id = i < nn ? jn[u * JN + i] : (i < m ? jo[u * JO + (i - nn)] : -1);
        ids[i] = id;
        kth[i] = id >= 0 ? keys[(int64_t)id * K + (K - 1)] : 0ull;
        cnt[i] = 0;
        const int mkv = (mark && id >= 0) ? (int)mark[id] : (mark ? 0 : 1);
        mk[i] = mkv;
        anymark |= (id >= 0 && mkv != 0);
    }
    if (__ballot(anymark) == 0) return;  // a repeat pass serves none of this source's members
    __builtin_amdgcn_wave_barrier();

    unsigned long long local_props = 0;
    // the member row behind each of this lane's staging loads
    int32_t fid[JPF];
#pragma unroll
    for (int j = 0; j < JPF; ++j) {
        const int e = lane + PG_WAVE * j;
        fid[j] = e < mp * (JDC / 4) ? ids[e / (JDC / 4)] : -1;
    }
    // micro-tiles of TR new members x TC members that hold a pair with col >
    // row: cb >= (TR rb + 1) / TC in row block rb
    auto tiles = [&](int tr, int tc) {
        const int RB = (nn + tr - 1) / tr, CB = mp / tc;
        int T = 0;
        for (int rb = 0; rb < RB; ++rb) T += CB - (tr * rb + 1) / tc;
        return T;
    };
    // one round: every lane sums the micro-tile of TR rows x TC columns at
    // (row0, col0) of the join set over all dimensions, then the pairs are
    // decided and emitted; a lane without a tile (have = false) sums rows 0
    // and emits nothing
    auto round = [&](auto shape, int row0, int col0, bool have) __attribute__((always_inline)) {
        constexpr int TR = decltype(shape)::rows, TC = decltype(shape)::cols;
        static_assert(TC % 4 == 0 || TC == 2, "micro-tile columns: one or two LDS reads");
        static_assert(TR * TC <= 32, "micro-tile shape");
        // bit c of every row of a lane's pair mask (bit a TC + c)
        constexpr uint32_t col_bits = TR == 4 ? (TC == 8 ? 0x01010101u : 0x1111u) : (TR == 2 ? 0x11u : 0x1u);
        if (!have) row0 = col0 = 0;
        float acc[TR][TC];
#pragma unroll
        for (int a = 0; a < TR; ++a)
#pragma unroll
            for (int c = 0; c < TC; ++c) acc[a][c] = 0.0f;
        // the rows of the next chunk load while the current one is summed
        float4 v[JPF];
        auto fetch = [&](int c0) {
            const int dl = min(JDC, d - c0);
#pragma unroll
            for (int j = 0; j < JPF; ++j) {
                const int q = (lane + PG_WAVE * j) % (JDC / 4);
                v[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (fid[j] >= 0 && 4 * q < dl)
                    v[j] = *reinterpret_cast<const float4 *>(X + (int64_t)fid[j] * ldx + c0 + 4 * q);
            }
        };
        fetch(0);
        for (int c0 = 0; c0 < d; c0 += JDC) {
            const int dl = min(JDC, d - c0);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < JPF; ++j) {
                const int e = lane + PG_WAVE * j;
                if (e < mp * (JDC / 4)) {
                    const int q = e % (JDC / 4), i = e / (JDC / 4);
                    tile[(4 * q + 0) * MPS + i] = v[j].x;
                    tile[(4 * q + 1) * MPS + i] = v[j].y;
                    tile[(4 * q + 2) * MPS + i] = v[j].z;
                    tile[(4 * q + 3) * MPS + i] = v[j].w;
                }
            }
            if (c0 + JDC < d) fetch(c0 + JDC);
            __builtin_amdgcn_wave_barrier();
            const float *rp = tile + row0;
            const float *cp = tile + col0;
            for (int k = 0; k < dl; ++k) {
                float rv[TR], cv[TC];
                if constexpr (TR == 4) {
                    const float4 r4 = *reinterpret_cast<const float4 *>(rp + k * MPS);
                    rv[0] = r4.x, rv[1] = r4.y, rv[2] = r4.z, rv[3] = r4.w;
                } else if constexpr (TR == 2) {
                    const float2 r2 = *reinterpret_cast<const float2 *>(rp + k * MPS);
                    rv[0] = r2.x, rv[1] = r2.y;
                } else {
                    rv[0] = rp[k * MPS];
                }
                if constexpr (TC >= 4) {
#pragma unroll
                    for (int j = 0; j < TC; j += 4) {
                        const float4 c4 = *reinterpret_cast<const float4 *>(cp + k * MPS + j);
                        cv[j] = c4.x, cv[j + 1] = c4.y, cv[j + 2] = c4.z, cv[j + 3] = c4.w;
                    }
                } else {
                    const float2 c2 = *reinterpret_cast<const float2 *>(cp + k * MPS);
                    cv[0] = c2.x, cv[1] = c2.y;
                }
#pragma unroll
                for (int a = 0; a < TR; ++a)
#pragma unroll
                    for (int c = 0; c < TC; ++c) {
                        const float t = rv[a] - cv[c];
                        acc[a][c] = fmaf(t, t, acc[a][c]);
                    }
            }
        }
        // ---- emission: decide every pair once (bit masks), one LDS offset per
        // (lane, member), reserve ranges per member, write
        uint32_t to_row = 0, to_col = 0;  // bit a*TC+c
        int off_row[TR], off_col[TC];
        if (have) {
#pragma unroll
            for (int a = 0; a < TR; ++a) {
                const int r = row0 + a;
#pragma unroll
                for (int c = 0; c < TC; ++c) {
                    const int col = col0 + c;
                    if (r >= nn || col >= m || (col < nn && col <= r)) continue;
                    const float d2 = acc[a][c];
                    const uint64_t kw = pack_key(d2, ids[col]), kv = pack_key(d2, ids[r]);
                    // a repeat pass (mark != null) skips keys already listed, so
                    // every repeat inserts at least one new key into each node it serves
                    if (mk[r] && kw < kth[r] && !(mark && list_has(keys + (int64_t)ids[r] * K, K, kw)))
                        to_row |= 1u << (a * TC + c);
                    if (mk[col] && kv < kth[col] && !(mark && list_has(keys + (int64_t)ids[col] * K, K, kv)))
                        to_col |= 1u << (a * TC + c);
                }
            }
#pragma unroll
            for (int a = 0; a < TR; ++a) {
                const int c_r = __popc((to_row >> (a * TC)) & ((1u << TC) - 1u));
                off_row[a] = c_r ? atomicAdd(&cnt[row0 + a], c_r) : 0;
            }
#pragma unroll
            for (int c = 0; c < TC; ++c) {
                const int c_c = __popc(to_col & (col_bits << c));
                off_col[c] = c_c ? atomicAdd(&cnt[col0 + c], c_c) : 0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        local_props += reserve_ranges(m, ids, cnt, base, sbase, pcnt, B, cslot, seg_begin);
        __builtin_amdgcn_wave_barrier();
        if (have) {
#pragma unroll
            for (int a = 0; a < TR; ++a) {
                const int r = row0 + a;
#pragma unroll
                for (int c = 0; c < TC; ++c) {
                    const int col = col0 + c;
                    const uint32_t bit = 1u << (a * TC + c);
                    if (!((to_row | to_col) & bit)) continue;
                    const float d2 = acc[a][c];
                    if (to_row & bit) {
                        const int32_t v = ids[r];
                        const int slot = base[r] + off_row[a]++;
                        const uint64_t kw = pack_key(d2, ids[col]);
                        if (slot < B)
                            bucket[(int64_t)v * B + slot] = kw;
                        else
                            spill_put(v, kw, sbase[r] + (slot - max(base[r], B)), spill_t, spill_k,
                                      seg_end, ovf_next, cslot);
                    }
                    if (to_col & bit) {
                        const int32_t w = ids[col];
                        const int slot = base[col] + off_col[c]++;
                        const uint64_t kv = pack_key(d2, ids[r]);
                        if (slot < B)
                            bucket[(int64_t)w * B + slot] = kv;
                        else
                            spill_put(w, kv, sbase[col] + (slot - max(base[col], B)), spill_t, spill_k,
                                      seg_end, ovf_next, cslot);
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    };
    // tile b of the row-major list of TR x TC micro-tiles (row block rb holds
    // the column blocks cb >= (TR rb + 1) / TC); rb = -1 past the end
    auto tile_at = [&](int b, int tr, int tc, int T, int &rb, int &cb) __attribute__((always_inline)) {
        rb = -1, cb = 0;
        if (b >= T) return;
        const int CB = mp / tc;
        int r = 0;
        while (b >= CB - (tr * r + 1) / tc) {
            b -= CB - (tr * r + 1) / tc;
            ++r;
        }
        rb = r;
        cb = (tr * r + 1) / tc + b;
    };
    // Every lane takes one micro-tile per round, and a round costs its wave the
    // full dimension loop (2 TR TC instructions per dimension) whatever the
    // number of busy lanes, plus a staging of the member rows.  For the same
    // number of rounds as 4 x 8 tiles, the cheapest covering is taken: a
    // smaller shape on its own grid (small join sets keep more lanes busy),
    // or 4 x 8 tiles with the last round's rem tiles split into 4 x 4, 2 x 4
    // or 1 x 2 sub-tiles when rem <= 32, 16 or 4 (that round then costs a
    // half, a quarter or a sixteenth of a full one).
    const int T48 = tiles(4, 8), T44 = tiles(4, 4), T24 = tiles(2, 4), T12 = tiles(1, 2);
    const int r48 = (T48 + PG_WAVE - 1) / PG_WAVE;
    const int rem48 = T48 - (r48 - 1) * PG_WAVE;
    const int r44 = (T44 + PG_WAVE - 1) / PG_WAVE, r24 = (T24 + PG_WAVE - 1) / PG_WAVE,
              r12 = (T12 + PG_WAVE - 1) / PG_WAVE;
    int best = 64 * (r48 - 1) + (rem48 > 32 ? 64 : rem48 > 16 ? 32 : rem48 > 4 ? 16 : 4), pick = 0;
    if (r44 <= r48 && 32 * r44 < best) best = 32 * r44, pick = 1;
    if (r24 <= r48 && 16 * r24 < best) best = 16 * r24, pick = 2;
    if (r12 <= r48 && 4 * r12 < best) best = 4 * r12, pick = 3;
    // shapes: 0 = 4 x 8, 1 = 4 x 4, 2 = 2 x 4, 3 = 1 x 2
    const int nr = pick == 0 ? r48 : pick == 1 ? r44 : pick == 2 ? r24 : r12;
    for (int r = 0; r < nr; ++r) {
        int shape, rb, cb, row0, col0;
        if (pick != 0) {
            shape = pick;
            const int tr = pick == 1 ? 4 : pick == 2 ? 2 : 1, tc = pick == 1 ? 4 : pick == 2 ? 4 : 2;
            tile_at(r * PG_WAVE + lane, tr, tc, pick == 1 ? T44 : pick == 2 ? T24 : T12, rb, cb);
            row0 = tr * rb;
            col0 = tc * cb;
        } else {
            shape = (r < nr - 1 || rem48 > 32) ? 0 : rem48 > 16 ? 1 : rem48 > 4 ? 2 : 3;
            const int sh = shape == 3 ? 4 : shape;  // log2 of the sub-tiles per 4 x 8 tile
            const int sub = lane & ((1 << sh) - 1);
            tile_at(r * PG_WAVE + (lane >> sh), 4, 8, T48, rb, cb);
            row0 = 4 * rb + (shape == 2 ? 2 * (sub >> 1) : shape == 3 ? (sub >> 2) : 0);
            col0 = 8 * cb + (shape == 1 ? 4 * sub : shape == 2 ? 4 * (sub & 1) : shape == 3 ? 2 * (sub & 3) : 0);
        }
        if (shape == 0)
            round(JoinTile<4, 8>{}, row0, col0, rb >= 0);
        else if (shape == 1)
            round(JoinTile<4, 4>{}, row0, col0, rb >= 0);
        else if (shape == 2)
            round(JoinTile<2, 4>{}, row0, col0, rb >= 0);
        else
            round(JoinTile<1, 2>{}, row0, col0, rb >= 0);
    }
    // one atomic per wave
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) {
        const unsigned long long t = __shfl_xor((long long)local_props, o, PG_WAVE);
        local_props += t;
    }
    if (lane == 0 && local_props) atomicAdd(&cslot[C_PROPOSALS], local_props);
}

// ---------------------------------------------------------------------------
// Stage and precision prep: 16-bit copies, canonical norms, exactness test.
// For integer-valued data with every squared norm <= 2^23, each product and
// every partial sum of a dot product is an integer of magnitude at most 2^23,
// and the norms add exactly.  The squared distance itself must also stay at
// or below 2^24 for the single rounding of n_x + n_y - 2 x.y and the partial
// sums of the chain to be exact: it is at most n_x + n_y <= 2^24 when no
// coordinate is negative (x.y >= 0), and at most (|x| + |y|)^2 <= 2^24 when
// every squared norm is at most 2^22.  So the MFMA norm expansion (FP32
// accumulation, any summation order) equals the canonical chain distance
// exactly when the values are integers and either no value is negative and
// the squared norms are <= 2^23, or the squared norms are <= 2^22.  FP16
// operands further need |x| <= 2048 and BF16 operands |x| <= 256.
// ---------------------------------------------------------------------------
enum { EX_NONINT = 0, EX_MAXABS = 1, EX_MAXNORM = 2, EX_NEG = 3 };

// The exactness test above, from the flags of k_prep.
static inline bool exact_integer_rows(const unsigned int he[4]) {
    float maxnorm;
    memcpy(&maxnorm, &he[EX_MAXNORM], 4);
    return he[EX_NONINT] == 0 && (maxnorm <= 4194304.0f || (he[EX_NEG] == 0 && maxnorm <= 8388608.0f));
}

// Grid-stride over rows, one wave per row.  The norm is a lane-parallel tree
// sum: it is only used where the data pass the exactness test, and there
// every order gives the same value (and a norm above 2^23 cannot come out at
// or below 2^23).  One atomic per block and flag.
__global__ __launch_bounds__(256) void k_prep(const float *__restrict__ X, int64_t ldx, int d, int d16,
                                              int64_t n, int mode, _Float16 *__restrict__ xh,
                                              __bf16 *__restrict__ xb, float *__restrict__ norms,
                                              unsigned int *__restrict__ ex) {
    __shared__ unsigned int red[4][4];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    bool nonint = false, neg = false;
    float mabs = 0.f, mnorm = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < n; i += (int64_t)gridDim.x * 4) {
        const float *x = X + i * ldx;
        float s = 0.f;
        for (int k = lane; k < d16; k += PG_WAVE) {
            const float v = k < d ? x[k] : 0.f;
            nonint |= (v != rintf(v));
            neg |= v < 0.f;
            mabs = fmaxf(mabs, fabsf(v));
            s = fmaf(v, v, s);
            if (mode == PG_FP16) xh[i * d16 + k] = (_Float16)v;
            if (mode == PG_BF16) xb[i * d16 + k] = (__bf16)v;
        }
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) s += __shfl_xor(s, o, PG_WAVE);
        if (lane == 0) norms[i] = s;
        mnorm = fmaxf(mnorm, s);
    }
    const unsigned int ni = __ballot(nonint) != 0 ? 1u : 0u;
    const unsigned int ng = __ballot(neg) != 0 ? 1u : 0u;
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) mabs = fmaxf(mabs, __shfl_xor(mabs, o, PG_WAVE));
    if (lane == 0) {
        red[wv][0] = ni;
        red[wv][1] = __float_as_uint(mabs);
        red[wv][2] = __float_as_uint(mnorm);
        red[wv][3] = ng;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int a = 0, b = 0, c = 0, e = 0;
        for (int w = 0; w < 4; ++w) {
            a |= red[w][0];
            b = max(b, red[w][1]);
            c = max(c, red[w][2]);
            e |= red[w][3];
        }
        if (a) atomicOr(&ex[EX_NONINT], 1u);
        atomicMax(&ex[EX_MAXABS], b);
        atomicMax(&ex[EX_MAXNORM], c);
        if (e) atomicOr(&ex[EX_NEG], 1u);
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision prep: the column mean mu (double partial sums over fixed
// row blocks, then a fixed-order final sum), the 16-bit copy of X - mu and
// FP32 norms of the rounded rows.  Distances do not change under the shift;
// centring shrinks the norms that the error bound of the estimates scales
// with.
// ---------------------------------------------------------------------------
constexpr int MU_ROWS = 1024;

__global__ __launch_bounds__(256) void k_colsum_partial(const float *__restrict__ X, int64_t ldx, int d, int64_t n,
                                                        double *__restrict__ part) {
    const int64_t r0 = (int64_t)blockIdx.x * MU_ROWS, r1 = min(n, r0 + MU_ROWS);
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)X[r * ldx + j];
        part[(int64_t)blockIdx.x * d + j] = s;
    }
}

__global__ __launch_bounds__(256) void k_colsum_final(const double *__restrict__ part, int64_t nb, int d, int64_t n,
                                                      float *__restrict__ mu) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d; j += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s += part[b * d + j];
        mu[j] = (float)(s / (double)n);
    }
}

// one wave per row (grid-stride): x16 = 16-bit(fl32(x - mu)), norms = FP32
// sum of the rounded squares; EX_MAXABS gets max |x - mu|
__global__ __launch_bounds__(256) void k_prep_mixed(const float *__restrict__ X, int64_t ldx, int d, int d16,
                                                    int64_t n, int mode, const float *__restrict__ mu,
                                                    _Float16 *__restrict__ xh, __bf16 *__restrict__ xb,
                                                    float *__restrict__ norms, unsigned int *__restrict__ ex) {
    __shared__ unsigned int red[4];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    float mabs = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < n; i += (int64_t)gridDim.x * 4) {
        const float *x = X + i * ldx;
        float s = 0.f;
        for (int k = lane; k < d16; k += PG_WAVE) {
            const float c = k < d ? x[k] - mu[k] : 0.f;
            mabs = fmaxf(mabs, fabsf(c));
            float r;
            if (mode == PG_FP16) {
                const _Float16 hv = (_Float16)c;
                xh[i * d16 + k] = hv;
                r = (float)hv;
            } else {
                const __bf16 bv = (__bf16)c;
                xb[i * d16 + k] = bv;
                r = (float)bv;
            }
            s = fmaf(r, r, s);
        }
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) s += __shfl_xor(s, o, PG_WAVE);
        if (lane == 0) norms[i] = s;
    }
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) mabs = fmaxf(mabs, __shfl_xor(mabs, o, PG_WAVE));
    if (lane == 0) red[wv] = __float_as_uint(mabs);
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&ex[EX_MAXABS], max(max(red[0], red[1]), max(red[2], red[3])));
}

// Error model of the mixed join (all bounds relative to the quantities the
// kernel has).  With x_c = x - mu, the 16-bit copy x^ satisfies
// |x^_i - x_c,i| <= un |x_c,i| + ea (ea: half the FP16 subnormal spacing), so
// ||e|| <= un (||x_c|| + ||y_c||) + 2 sqrt(d) ea for e = (x^ - y^) - (x_c - y_c),
// and | ||x^ - y^||^2 - ||x_c - y_c||^2 | <= 2 ||e|| ||x_c - y_c|| + ||e||^2.
// The estimate n^_x + n^_y - 2 x^.y^ (FP32 accumulation of exact products)
// is within ga (n^_x + n^_y + 2 |x^.y^|) of ||x^ - y^||^2, and the direct form
// is within gd of the exact distance.  A pair whose direct-form distance is
// at most the cut c has ||x_c - y_c|| <= sqrt(c (1 + gd)), so its estimate is
// at most c (1 + gd) + that bound: anything above cannot be accepted.
struct MixedParams {
    int on;         // 0: the tiles are exact (integer data)
    int rigorous;   // 1: rigorous bound (+ mrel * cut); 0: mrel * cut alone
    float un, ea, gd, ga, mrel, sqd;
};

__device__ __forceinline__ float mixed_bound(const MixedParams &mx, float cut, float nx, float ny, float g) {
    if (!mx.rigorous) return cut * (1.0f + mx.mrel);
    const float cg = cut * (1.0f + mx.gd);
    const float sn = (sqrtf(nx) + sqrtf(ny)) * (1.0f + 2.0f * mx.un);
    const float e = mx.un * sn + 2.0f * mx.sqd * mx.ea;
    const float b = cg + 2.0f * e * sqrtf(cg) + e * e + mx.ga * (nx + ny + 2.0f * fabsf(g)) + mx.mrel * cut;
    return b * 1.0001f + 1e-30f;  // slack for evaluating the bound itself in FP32
}

typedef float mf_f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 mf_f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));

// 32 x 32 block of x_r . x_c over all d for member rows (ra[lane%32]) and
// columns (ca[lane%32]); result in the MFMA accumulator layout: lane l,
// register g holds row 8*(g/4) + 4*(l/32) + g%4, column l%32.
template <int P>
__device__ __forceinline__ mf_f32x16 gram_tile(const float *__restrict__ X, int64_t ldx,
                                               const void *__restrict__ X16, int d, int d16,
                                               int32_t rid, int32_t cid) {
    const int h = lane_id() >> 5;
    mf_f32x16 acc;
#pragma unroll
    for (int g = 0; g < 16; ++g) acc[g] = 0.f;
    // Operands are loaded in batches of GK k-steps before their MFMAs, so a
    // tile waits for memory once per batch instead of once per step.
    if (P == PG_FP32) {
        // float4 chunk t: lane half h takes dims 4t+2h and 4t+2h+1 in two steps
        constexpr int GK = 8;
        const float *ra = X + (int64_t)rid * ldx + 2 * h;
        const float *ca = X + (int64_t)cid * ldx + 2 * h;
        for (int t0 = 0; t0 < d; t0 += 4 * GK) {
            float2 a[GK], b[GK];
#pragma unroll
            for (int j = 0; j < GK; ++j) {
                const bool in = t0 + 4 * j < d;
                a[j] = in ? *reinterpret_cast<const float2 *>(ra + t0 + 4 * j) : make_float2(0.f, 0.f);
                b[j] = in ? *reinterpret_cast<const float2 *>(ca + t0 + 4 * j) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < GK; ++j) {
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].x, b[j].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].y, b[j].y, acc, 0, 0, 0);
            }
        }
    } else {
        constexpr int GK = 4;
        typedef typename std::conditional<P == PG_FP16, mf_f16x8, mf_bf16x8>::type vec8;
        typedef typename std::conditional<P == PG_FP16, _Float16, __bf16>::type elem;
        const elem *ra = reinterpret_cast<const elem *>(X16) + (int64_t)rid * d16 + 8 * h;
        const elem *ca = reinterpret_cast<const elem *>(X16) + (int64_t)cid * d16 + 8 * h;
        for (int t0 = 0; t0 < d16; t0 += 16 * GK) {
            vec8 a[GK], b[GK];
#pragma unroll
            for (int j = 0; j < GK; ++j) {
                const bool in = t0 + 16 * j < d16;
                a[j] = in ? *reinterpret_cast<const vec8 *>(ra + t0 + 16 * j) : vec8{};
                b[j] = in ? *reinterpret_cast<const vec8 *>(ca + t0 + 16 * j) : vec8{};
            }
#pragma unroll
            for (int j = 0; j < GK; ++j) {
                if (P == PG_FP16)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[j], b[j], acc, 0, 0, 0);
                else
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[j], acc, 0, 0, 0);
            }
        }
    }
    return acc;
}

constexpr int MW = 4;  // sources (waves) per workgroup in the MFMA join

// LDS bytes of one join wave: per member kth, sbase, ids, cnt, base, mk, nrm, thr
__host__ __device__ inline size_t join_mfma_wave_bytes(int mps) {
    return (size_t)mps * (8 + 8 + 4 + 4 + 4 + 4 + 4 + 4);
}

// MFMA local join for data on which the norm expansion is exact (see k_prep):
// one wave per source, 32 x 32 Gram tiles of (new members) x (all members),
// d2 = n_r + n_c - 2 x_r.x_c, then the same decisions and reservations as the
// FP32 join.  Offsets of the proposals to a tile's row member come from
// ballots (the 32 lanes of a half share the row), so only one LDS atomic per
// (row, tile half) and one per (lane, column) are needed.
template <int P>
__global__ __launch_bounds__(MW * PG_WAVE, 4) void k_join_mfma(
    const float *__restrict__ X, int64_t ldx, const void *__restrict__ X16, int d, int d16,
    const float *__restrict__ norms, int K, const int32_t *__restrict__ jn,
    const int32_t *__restrict__ jn_c, int JN, const int32_t *__restrict__ jo,
    const int32_t *__restrict__ jo_c, int JO, const uint64_t *__restrict__ keys,
    int32_t *__restrict__ pcnt, uint64_t *__restrict__ bucket, int B,
    int32_t *__restrict__ spill_t, uint64_t *__restrict__ spill_k, int64_t seg,
    uint8_t *__restrict__ ovf_next, const uint8_t *__restrict__ mark, const int32_t *__restrict__ order,
    int64_t n, PassRange pr, int maxm, unsigned long long *__restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int MPS = (maxm + 31) / 32 * 32;
    const int lane = lane_id(), h = lane >> 5, l32 = lane & 31;
    const int wv = threadIdx.x / PG_WAVE;
    const int64_t nlog = (pr.items + MW - 1) / MW;
    const int64_t lb = xcd_logical_block(blockIdx.x, nlog);
    const int64_t u = lb < nlog ? pass_source(order, n, pr, lb * MW + wv) : -1;
    if (u < 0) return;
    unsigned long long *cslot = stripe_of(counters);
    const int64_t seg_begin = (int64_t)(blockIdx.x % NSTRIPE) * seg, seg_end = seg_begin + seg;
    unsigned char *region = smem + (size_t)wv * join_mfma_wave_bytes(MPS);
    uint64_t *kth = reinterpret_cast<uint64_t *>(region);
    int64_t *sbase = reinterpret_cast<int64_t *>(kth + MPS);
    int32_t *ids = reinterpret_cast<int32_t *>(sbase + MPS);
    int32_t *cnt = ids + MPS;
    int32_t *base = cnt + MPS;
    int32_t *mk = base + MPS;
    float *nrm = reinterpret_cast<float *>(mk + MPS);
    float *thr = nrm + MPS;  // d2 of the member's cut when it takes proposals, else -1

    const int nn = jn_c[u], no = jo_c[u];
    const int m = nn + no;
    if (nn == 0 || m < 2) return;
    const int mp = (m + 31) / 32 * 32;
    bool anymark = false;
    for (int i = lane; i < mp; i += PG_WAVE) {
        const int32_t id = i < nn ? jn[u * JN + i] : (i < m ? jo[u * JO + (i - nn)] : -1);
        ids[i] = id;
        const uint64_t kk = id >= 0 ? keys[(int64_t)id * K + (K - 1)] : 0ull;
        kth[i] = kk;
        nrm[i] = id >= 0 ? norms[id] : 0.f;
        cnt[i] = 0;
        const int mkv = (mark && id >= 0) ? (int)mark[id] : (mark ? 0 : 1);
        mk[i] = mkv;
        thr[i] = (id >= 0 && mkv) ? key_d2(kk) : -1.0f;
        anymark |= (id >= 0 && mkv != 0);
    }
    if (__ballot(anymark) == 0) return;
    __builtin_amdgcn_wave_barrier();
    const int RB = (nn + 31) / 32, CB = mp / 32;
    const int32_t id0 = ids[0];
    unsigned long long local_props = 0;
    for (int rb = 0; rb < RB; ++rb) {
        for (int cb = rb; cb < CB; ++cb) {
            // member of this lane's column and of the tile rows it loads
            const int cm = 32 * cb + l32;
            const int rm = 32 * rb + l32;
            const int32_t cid = cm < m ? ids[cm] : id0;
            const int32_t rid = rm < nn ? ids[rm] : id0;
            const mf_f32x16 g = gram_tile<P>(X, ldx, X16, d, d16, rid, cid);
            // decisions (bit g of each mask = accumulator register g)
            uint32_t to_row = 0, to_col = 0;
            const float nc = nrm[cm < mp ? cm : 0];
            const float thc = thr[cm < mp ? cm : 0];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = 32 * rb + 8 * (q / 4) + 4 * h + (q % 4);
                const float d2 = fmaxf(fmaf(-2.0f, g[q], nrm[r] + nc), 0.0f);
                // a key below an end's cut has d2 <= the cut's d2: most pairs stop here
                if (!(d2 <= thr[r]) && !(d2 <= thc)) continue;
                if (r >= nn || cm >= m || (cm < nn && cm <= r)) continue;
                const uint64_t kw = pack_key(d2, ids[cm]), kv = pack_key(d2, ids[r]);
                const bool row_ok = !(mark && list_has(keys + (int64_t)ids[r] * K, K, kw));
                const bool col_ok = !(mark && list_has(keys + (int64_t)ids[cm] * K, K, kv));
                if (mk[r] && kw < kth[r] && row_ok) to_row |= 1u << q;
                if (mk[cm] && kv < kth[cm] && col_ok) to_col |= 1u << q;
            }
            // Offsets within this tile's contribution to each target.  Each
            // (register, half) is a distinct row, so a row's count is one
            // popcount of its ballot; the two halves of a column combine by a
            // shuffle.  In a diagonal tile a member is both a row and a
            // column: its column proposals go after its row proposals.
            int off_row[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint64_t bm = __ballot((to_row >> q) & 1u);
                const uint64_t mine = h ? (bm >> 32) : (bm & 0xFFFFFFFFull);
                const int r = 32 * rb + 8 * (q / 4) + 4 * h + (q % 4);
                if (l32 == 0) cnt[r] = __popcll(mine);
                const uint64_t below = (lanemask_lt() >> (32 * h)) & 0xFFFFFFFFull;
                off_row[q] = __popcll(mine & below);
            }
            __builtin_amdgcn_wave_barrier();
            int off_col;
            {
                const int cc = __popc(to_col), cc_other = __shfl_xor(cc, 32, PG_WAVE);
                const int rows_before = (rb == cb) ? cnt[cm] : 0;
                off_col = rows_before + (h ? cc_other : 0);
                __builtin_amdgcn_wave_barrier();
                if (h == 0 && (rb == cb || cc + cc_other > 0)) cnt[cm] = rows_before + cc + cc_other;
            }
            __builtin_amdgcn_wave_barrier();
            {
                // only the tile's rows and columns can hold proposals
                const int mi = h == 0 ? 32 * rb + l32 : (cb != rb ? 32 * cb + l32 : -1);
                local_props += reserve_lanes(mi < m ? mi : -1, ids, cnt, base, sbase, pcnt, B, cslot, seg_begin);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t bit = 1u << q;
                if (!((to_row | to_col) & bit)) continue;
                const int r = 32 * rb + 8 * (q / 4) + 4 * h + (q % 4);
                const float d2 = fmaxf(fmaf(-2.0f, g[q], nrm[r] + nc), 0.0f);
                if (to_row & bit) {
                    const int32_t v = ids[r];
                    const int slot = base[r] + off_row[q];
                    const uint64_t kw = pack_key(d2, ids[cm]);
                    if (slot < B)
                        bucket[(int64_t)v * B + slot] = kw;
                    else
                        spill_put(v, kw, sbase[r] + (slot - max(base[r], B)), spill_t, spill_k, seg_end,
                                  ovf_next, cslot);
                }
                if (to_col & bit) {
                    const int32_t w = ids[cm];
                    const int slot = base[cm] + off_col++;
                    const uint64_t kv = pack_key(d2, ids[r]);
                    if (slot < B)
                        bucket[(int64_t)w * B + slot] = kv;
                    else
                        spill_put(w, kv, sbase[cm] + (slot - max(base[cm], B)), spill_t, spill_k, seg_end,
                                  ovf_next, cslot);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1)
        local_props += (unsigned long long)__shfl_xor((long long)local_props, o, PG_WAVE);
    if (lane == 0 && local_props) atomicAdd(&cslot[C_PROPOSALS], local_props);
}

static size_t join_mfma_lds_bytes(int maxm) {
    const int mps = (maxm + 31) / 32 * 32;
    return (size_t)MW * join_mfma_wave_bytes(mps);
}

// ---------------------------------------------------------------------------
// Mixed-precision local join for float data (PG_FP16 / PG_BF16 on non-exact
// rows).  One wave per source u.  The 16-bit Gram tiles of the centred copy
// give every pair's estimate; a pair whose estimate lies within the rigorous
// bound (mixed_bound) of an end's cut is a candidate for that end and goes to
// the wave's pair list; every other pair cannot beat either cut.  The list is
// then settled on the FP32 rows: the rows of the members it involves are
// staged through LDS HCH dimensions at a time, each lane accumulates the
// canonical chains of its entries (dims ascending, one fma per dim, the same
// value as everywhere else), and the exact keys are decided and emitted as in
// the FP32 join.  So every stored distance is the chain value and the lists
// equal the FP32 build's; the FP32 rows are read once per source and only
// for members that some candidate pair involves.
// ---------------------------------------------------------------------------
constexpr int HW = 3;        // sources (waves) per workgroup
constexpr int HCAP = 1024;   // pair list entries per wave (a tile adds at most 1024)
constexpr int HCH = 8;       // FP32 dims per staging chunk
constexpr int HPL = HCAP / PG_WAVE;  // list entries per lane

// LDS bytes of one hybrid-join wave: per member kth, sbase, ids, cnt, base,
// mk, nrm, thr, staging slot and slot owner; the pair list; the staging tile
__host__ __device__ inline size_t join_hybrid_wave_bytes(int mps) {
    return (size_t)mps * (8 + 8 + 4 + 4 + 4 + 4 + 4 + 4 + 4 + 4) + (size_t)HCAP * 4 +
           (size_t)mps * HCH * sizeof(float);
}

static size_t join_hybrid_lds_bytes(int maxm) {
    const int mps = (maxm + 31) / 32 * 32;
    return (size_t)HW * join_hybrid_wave_bytes(mps);
}

template <int P>
__global__ __launch_bounds__(HW * PG_WAVE, 3) void k_join_hybrid(
    const float *__restrict__ X, int64_t ldx, const void *__restrict__ X16, int d, int d16,
    const float *__restrict__ norms, int K, const int32_t *__restrict__ jn,
    const int32_t *__restrict__ jn_c, int JN, const int32_t *__restrict__ jo,
    const int32_t *__restrict__ jo_c, int JO, const uint64_t *__restrict__ keys,
    int32_t *__restrict__ pcnt, uint64_t *__restrict__ bucket, int B,
    int32_t *__restrict__ spill_t, uint64_t *__restrict__ spill_k, int64_t seg,
    uint8_t *__restrict__ ovf_next, const uint8_t *__restrict__ mark, const int32_t *__restrict__ order,
    int64_t n, PassRange pr, int maxm, MixedParams mx, unsigned long long *__restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int MPS = (maxm + 31) / 32 * 32;
    const int lane = lane_id(), h = lane >> 5, l32 = lane & 31;
    const int wv = threadIdx.x / PG_WAVE;
    const int64_t nlog = (pr.items + HW - 1) / HW;
    const int64_t lb = xcd_logical_block(blockIdx.x, nlog);
    const int64_t u = lb < nlog ? pass_source(order, n, pr, lb * HW + wv) : -1;
    if (u < 0) return;
    unsigned long long *cslot = stripe_of(counters);
    const int64_t seg_begin = (int64_t)(blockIdx.x % NSTRIPE) * seg, seg_end = seg_begin + seg;
    unsigned char *region = smem + (size_t)wv * join_hybrid_wave_bytes(MPS);
    uint64_t *kth = reinterpret_cast<uint64_t *>(region);
    int64_t *sbase = reinterpret_cast<int64_t *>(kth + MPS);
    int32_t *ids = reinterpret_cast<int32_t *>(sbase + MPS);
    int32_t *cnt = ids + MPS;
    int32_t *base = cnt + MPS;
    int32_t *mk = base + MPS;
    float *nrm = reinterpret_cast<float *>(mk + MPS);
    float *cut = nrm + MPS;     // d2 of the member's cut when it takes proposals, else -1
    int32_t *slot = reinterpret_cast<int32_t *>(cut + MPS);  // staging row of a member, or -1
    int32_t *owner = slot + MPS;                              // member of a staging row
    uint32_t *plist = reinterpret_cast<uint32_t *>(owner + MPS);
    float *stage = reinterpret_cast<float *>(plist + HCAP);  // [row][HCH]

    const int nn = jn_c[u], no = jo_c[u];
    const int m = nn + no;
    if (nn == 0 || m < 2) return;
    const int mp = (m + 31) / 32 * 32;
    bool anymark = false;
    for (int i = lane; i < mp; i += PG_WAVE) {
        const int32_t id = i < nn ? jn[u * JN + i] : (i < m ? jo[u * JO + (i - nn)] : -1);
        ids[i] = id;
        const uint64_t kk = id >= 0 ? keys[(int64_t)id * K + (K - 1)] : 0ull;
        kth[i] = kk;
        nrm[i] = id >= 0 ? norms[id] : 0.f;
        cnt[i] = 0;
        slot[i] = -1;
        const int mkv = (mark && id >= 0) ? (int)mark[id] : (mark ? 0 : 1);
        mk[i] = mkv;
        cut[i] = (id >= 0 && mkv) ? key_d2(kk) : -1.0f;
        anymark |= (id >= 0 && mkv != 0);
    }
    if (__ballot(anymark) == 0) return;
    __builtin_amdgcn_wave_barrier();
    const int RB = (nn + 31) / 32, CB = mp / 32;
    const int32_t id0 = ids[0];
    unsigned long long local_props = 0, local_rechk = 0;
    int nl = 0;  // entries in the pair list (wave-uniform)

    // settle the listed pairs on the FP32 rows and emit their proposals
    auto flush = [&]() {
        if (nl == 0) return;
        // staging rows: the members the list involves, in member order
        for (int e = lane; e < nl; e += PG_WAVE) {
            const uint32_t ent = plist[e];
            slot[ent & 0xFF] = 0;
            slot[(ent >> 8) & 0xFF] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        int ns = 0;
        for (int i0 = 0; i0 < mp; i0 += PG_WAVE) {
            const int i = i0 + lane;
            const bool inv = i < m && slot[i] == 0;
            const uint64_t bm = __ballot(inv);
            if (inv) {
                const int s = ns + __popcll(bm & lanemask_lt());
                slot[i] = s;
                owner[s] = ids[i];
            }
            ns += __popcll(bm);
        }
        __builtin_amdgcn_wave_barrier();
        // per lane: entries e = lane + 64 j, their staging rows and chains
        float acc[HPL];
        int sr[HPL], sc[HPL];
#pragma unroll
        for (int j = 0; j < HPL; ++j) {
            const int e = lane + PG_WAVE * j;
            acc[j] = 0.0f;
            sr[j] = sc[j] = 0;
            if (e < nl) {
                const uint32_t ent = plist[e];
                sr[j] = slot[ent & 0xFF] * HCH;
                sc[j] = slot[(ent >> 8) & 0xFF] * HCH;
            }
        }
        const int jmax = (nl + PG_WAVE - 1) / PG_WAVE;
        for (int c0 = 0; c0 < d; c0 += HCH) {
            __builtin_amdgcn_wave_barrier();
            for (int v = lane; v < ns * (HCH / 4); v += PG_WAVE) {
                const int s = v / (HCH / 4), q = v - s * (HCH / 4);
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (c0 + 4 * q < d) x = *reinterpret_cast<const float4 *>(X + (int64_t)owner[s] * ldx + c0 + 4 * q);
                *reinterpret_cast<float4 *>(stage + s * HCH + 4 * q) = x;
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < HPL; ++j) {
                if (j < jmax) {
#pragma unroll
                    for (int q = 0; q < HCH; q += 4) {
                        const float4 a = *reinterpret_cast<const float4 *>(stage + sr[j] + q);
                        const float4 b = *reinterpret_cast<const float4 *>(stage + sc[j] + q);
                        float s = acc[j], t;
                        t = a.x - b.x;
                        s = fmaf(t, t, s);
                        t = a.y - b.y;
                        s = fmaf(t, t, s);
                        t = a.z - b.z;
                        s = fmaf(t, t, s);
                        t = a.w - b.w;
                        s = fmaf(t, t, s);
                        acc[j] = s;
                    }
                }
            }
        }
        // exact decisions; offsets per member from LDS atomics
        uint32_t to_row = 0, to_col = 0;
        int off_r[HPL], off_c[HPL];
#pragma unroll
        for (int j = 0; j < HPL; ++j) {
            const int e = lane + PG_WAVE * j;
            off_r[j] = off_c[j] = 0;
            if (e < nl) {
                const uint32_t ent = plist[e];
                const int r = ent & 0xFF, c = (ent >> 8) & 0xFF;
                const float d2 = acc[j];
                const uint64_t kw = pack_key(d2, ids[c]), kv = pack_key(d2, ids[r]);
                if (((ent >> 16) & 1u) && kw < kth[r] && !(mark && list_has(keys + (int64_t)ids[r] * K, K, kw))) {
                    to_row |= 1u << j;
                    off_r[j] = atomicAdd(&cnt[r], 1);
                }
                if (((ent >> 17) & 1u) && kv < kth[c] && !(mark && list_has(keys + (int64_t)ids[c] * K, K, kv))) {
                    to_col |= 1u << j;
                    off_c[j] = atomicAdd(&cnt[c], 1);
                }
            }
        }
        local_rechk += (unsigned long long)(lane < nl ? (nl - lane + PG_WAVE - 1) / PG_WAVE : 0);
        __builtin_amdgcn_wave_barrier();
        local_props += reserve_ranges(m, ids, cnt, base, sbase, pcnt, B, cslot, seg_begin);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < HPL; ++j) {
            if (!(((to_row | to_col) >> j) & 1u)) continue;
            const uint32_t ent = plist[lane + PG_WAVE * j];
            const int r = ent & 0xFF, c = (ent >> 8) & 0xFF;
            const float d2 = acc[j];
            if ((to_row >> j) & 1u) {
                const int32_t v = ids[r];
                const int sl = base[r] + off_r[j];
                const uint64_t kw = pack_key(d2, ids[c]);
                if (sl < B)
                    bucket[(int64_t)v * B + sl] = kw;
                else
                    spill_put(v, kw, sbase[r] + (sl - max(base[r], B)), spill_t, spill_k, seg_end, ovf_next, cslot);
            }
            if ((to_col >> j) & 1u) {
                const int32_t w = ids[c];
                const int sl = base[c] + off_c[j];
                const uint64_t kv = pack_key(d2, ids[r]);
                if (sl < B)
                    bucket[(int64_t)w * B + sl] = kv;
                else
                    spill_put(w, kv, sbase[c] + (sl - max(base[c], B)), spill_t, spill_k, seg_end, ovf_next, cslot);
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < mp; i += PG_WAVE) slot[i] = -1;
        __builtin_amdgcn_wave_barrier();
        nl = 0;
    };

    for (int rb = 0; rb < RB; ++rb) {
        for (int cb = rb; cb < CB; ++cb) {
            const int cm = 32 * cb + l32;
            const int rm = 32 * rb + l32;
            const int32_t cid = cm < m ? ids[cm] : id0;
            const int32_t rid = rm < nn ? ids[rm] : id0;
            const mf_f32x16 g = gram_tile<P>(X, ldx, X16, d, d16, rid, cid);
            const float nc = nrm[cm < mp ? cm : 0];
            const float cc = cut[cm < mp ? cm : 0];
            // candidates: bits 2q (row end) and 2q + 1 (column end)
            uint32_t emask = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = 32 * rb + 8 * (q / 4) + 4 * h + (q % 4);
                if (r >= nn || cm >= m || (cm < nn && cm <= r)) continue;
                const float cr = cut[r];
                const float hi = fmaxf(cr, cc);
                if (hi < 0.0f) continue;
                const float d2e = fmaxf(fmaf(-2.0f, g[q], nrm[r] + nc), 0.0f);
                if (!(d2e <= mixed_bound(mx, hi, nrm[r], nc, g[q]))) continue;
                // the bound grows with the cut: the end with the larger cut is
                // a candidate, the other one when its own bound holds
                const float lo = fminf(cr, cc);
                const bool other = lo >= 0.0f && d2e <= mixed_bound(mx, lo, nrm[r], nc, g[q]);
                const bool er = cr >= 0.0f && (cr >= cc || other);
                const bool ec = cc >= 0.0f && (cc > cr || other);
                emask |= ((er ? 1u : 0u) | (ec ? 2u : 0u)) << (2 * q);
            }
            // append this lane's candidates after the lanes below it
            const uint32_t any = (emask | (emask >> 1)) & 0x55555555u;
            const int mine = __popc(any);
            int incl = mine;
#pragma unroll
            for (int o = 1; o < PG_WAVE; o <<= 1) {
                const int t = __shfl_up(incl, o, PG_WAVE);
                if (lane >= o) incl += t;
            }
            const int total = __shfl(incl, PG_WAVE - 1, PG_WAVE);
            if (nl + total > HCAP) flush();
            int at = nl + incl - mine;
            uint32_t mm = any;
            while (mm) {
                const int b = __builtin_ctz(mm);
                mm &= mm - 1;
                const int q = b >> 1;
                const int r = 32 * rb + 8 * (q / 4) + 4 * h + (q % 4);
                plist[at++] = (uint32_t)r | ((uint32_t)cm << 8) | (((emask >> b) & 3u) << 16);
            }
            nl += total;
            __builtin_amdgcn_wave_barrier();
        }
    }
    flush();
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) {
        local_props += (unsigned long long)__shfl_xor((long long)local_props, o, PG_WAVE);
        local_rechk += (unsigned long long)__shfl_xor((long long)local_rechk, o, PG_WAVE);
    }
    if (lane == 0 && local_props) atomicAdd(&cslot[C_PROPOSALS], local_props);
    if (lane == 0 && local_rechk) atomicAdd(&cslot[C_RECHECK], local_rechk);
}

// ---------------------------------------------------------------------------
// merge: list <- K smallest distinct keys of (list U bucket)
// flags per entry: bit 0 = new, bit 1 = inserted during this iteration
// ---------------------------------------------------------------------------
constexpr int MERGE_INSERT_MAX = 16;  // survivors of a batch inserted one by one

__global__ __launch_bounds__(256) void k_merge(uint64_t *__restrict__ keys,
                                               uint64_t *__restrict__ newm,
                                               uint64_t *__restrict__ insm, int64_t n, int K,
                                               int32_t *__restrict__ pcnt,
                                               const uint64_t *__restrict__ bucket, int B,
                                               const int64_t *__restrict__ soff,
                                               const uint64_t *__restrict__ spilled) {
    const int lane = lane_id();
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    const int c = pcnt[v];
    if (c == 0) return;
    uint64_t a = lane < K ? keys[v * K + lane] : KEY_INF;
    const uint64_t nm = newm[v], im = insm[v];
    int fl = lane < K ? (int)(((nm >> lane) & 1ull) | (((im >> lane) & 1ull) << 1)) : 0;
    const int cc = min(c, B);
    const int64_t s0 = soff ? soff[v] : 0;
    const int sc = soff ? (int)(soff[v + 1] - s0) : 0;
    for (int b0 = 0; b0 < cc + sc; b0 += PG_WAVE) {
        const uint64_t kth = readlane64(a, K - 1);
        const int e = b0 + lane;
        uint64_t bk = KEY_INF;
        if (e < cc)
            bk = bucket[v * B + e];
        else if (e < cc + sc)
            bk = spilled[s0 + (e - cc)];
        if (bk >= kth) bk = KEY_INF;
        const uint64_t vm = __ballot(bk != KEY_INF);
        if (vm == 0) continue;
        if (__popcll(vm) <= MERGE_INSERT_MAX) {
            // few survivors: insert them one by one (rank by ballot, shift up)
            for (uint64_t rem = vm; rem; rem &= rem - 1) {
                const uint64_t x = readlane64(bk, __ffsll((long long)rem) - 1);
                if (x >= readlane64(a, K - 1)) continue;  // not among the K smallest
                if (__ballot(a == x)) continue;       // already in the list
                const int at = __popcll(__ballot(a < x));
                const uint64_t up = from_lane_below64(a);
                const int fup = (int)from_lane_below((uint32_t)fl);
                if (lane > at) {
                    a = up;
                    fl = fup;
                } else if (lane == at) {
                    a = x;
                    fl = 3;
                }
                if (lane >= K) {
                    a = KEY_INF;
                    fl = 0;
                }
            }
            continue;
        }
        int pb = 3;
        wave_sort(bk, pb);
        const uint64_t prev = from_lane_below64(bk);
        const bool dup = lane > 0 && prev == bk;
        const bool in_list = wave_contains(a, bk);
        const bool valid = bk != KEY_INF && !dup && !in_list;
        if (wave_compact(bk, pb, valid) == 0) continue;
        wave_merge_lowest(a, fl, bk, pb);
        if (lane >= K) {
            a = KEY_INF;
            fl = 0;
        }
    }
    if (lane < K) keys[v * K + lane] = a;
    const uint64_t nmo = __ballot(lane < K && (fl & 1));
    const uint64_t imo = __ballot(lane < K && (fl & 2));
    if (lane == 0) {
        newm[v] = nmo;
        insm[v] = imo;
        pcnt[v] = 0;
    }
}

__global__ __launch_bounds__(256) void k_count_updates(uint64_t *__restrict__ insm, int64_t n,
                                                       unsigned long long *__restrict__ counters, Segs sg,
                                                       unsigned long long *__restrict__ seg_updates) {
    __shared__ unsigned long long s[256];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long c = 0;
    if (v < n) {
        c = (unsigned long long)__popcll(insm[v]);
        insm[v] = 0;
        if (sg.of && c) atomicAdd(&seg_updates[sg.of[v]], c);
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && s[0]) atomicAdd(&stripe_of(counters)[C_UPDATES], s[0]);
}

__global__ void k_unpack(const uint64_t *__restrict__ keys, int64_t total,
                         int32_t *__restrict__ ids, float *__restrict__ d2, Segs sg, int K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const uint64_t k = keys[i];
    // ids local to the node's collection
    ids[i] = k == KEY_INF ? -1 : (int32_t)(key_id(k) - seg_base(sg, i / K));
    d2[i] = k == KEY_INF ? __int_as_float(0x7f800000) : key_d2(k);
}

__global__ void k_mark_swap(uint8_t *__restrict__ mark, uint8_t *__restrict__ next, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    mark[i] = next[i];
    next[i] = 0;
}

// ---------------------------------------------------------------------------
// exact brute-force kNN: 64 queries x 64 points tiles, running top-k per query
// ---------------------------------------------------------------------------
constexpr int EQ = 64, EP = 64, EDC = 32, ESTR = EDC + 4;

__global__ __launch_bounds__(256) void k_exact_knn(const float *__restrict__ X, int64_t n, int d,
                                                   int64_t ldx, const float *__restrict__ Q,
                                                   int64_t nq, int64_t ldq,
                                                   const int32_t *__restrict__ qrow, int64_t qrow_n,
                                                   const int32_t *__restrict__ exclude,
                                                   int self_excl, int k,
                                                   int32_t *__restrict__ out_ids,
                                                   float *__restrict__ out_d2) {
    __shared__ __align__(16) float qt[EQ * ESTR];
    __shared__ __align__(16) float pt[EP * ESTR];
    __shared__ float dt[EQ * (EP + 1)];
    __shared__ uint64_t topk[EQ * PG_WAVE];
    __shared__ int32_t excl[EQ];
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int ty = tid >> 4, tx = tid & 15;
    const int64_t q0 = (int64_t)blockIdx.x * EQ;
    for (int i = tid; i < EQ * PG_WAVE; i += 256) topk[i] = KEY_INF;
    // query q reads row qrow[q] of Q when qrow is given (a row outside
    // [0, qrow_n) reads as zeros; the caller reports it), else row q
    __shared__ int64_t qoff[EQ];
    for (int i = tid; i < EQ; i += 256) {
        excl[i] = q0 + i >= nq ? -1 : (self_excl ? (int32_t)(q0 + i) : (exclude ? exclude[q0 + i] : -1));
        int64_t r = q0 + i;
        if (qrow && q0 + i < nq) {
            const int32_t qi = qrow[q0 + i];
            r = (qi >= 0 && qi < qrow_n) ? (int64_t)qi : -1;
        }
        qoff[i] = q0 + i < nq && r >= 0 ? r * ldq : -1;
    }
    __syncthreads();
    for (int64_t p0 = 0; p0 < n; p0 += EP) {
        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
        for (int c0 = 0; c0 < d; c0 += EDC) {
            __syncthreads();
            for (int e = tid; e < (EQ + EP) * (EDC / 4); e += 256) {
                const int r = e / (EDC / 4), q = e % (EDC / 4);
                float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < EQ) {
                    if (qoff[r] >= 0 && c0 + 4 * q < d)
                        val = *reinterpret_cast<const float4 *>(Q + qoff[r] + c0 + 4 * q);
                    *reinterpret_cast<float4 *>(qt + r * ESTR + 4 * q) = val;
                } else {
                    const int rr = r - EQ;
                    if (p0 + rr < n && c0 + 4 * q < d)
                        val = *reinterpret_cast<const float4 *>(X + (p0 + rr) * ldx + c0 + 4 * q);
                    *reinterpret_cast<float4 *>(pt + rr * ESTR + 4 * q) = val;
                }
            }
            __syncthreads();
            const int dlim = min(EDC, d - c0);
            for (int dd = 0; dd < dlim; dd += 4) {
                float4 r4[4], c4[4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    r4[a] = *reinterpret_cast<const float4 *>(qt + (4 * ty + a) * ESTR + dd);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    c4[b] = *reinterpret_cast<const float4 *>(pt + (4 * tx + b) * ESTR + dd);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        float s = acc[a][b], t;
                        t = r4[a].x - c4[b].x;
                        s = fmaf(t, t, s);
                        t = r4[a].y - c4[b].y;
                        s = fmaf(t, t, s);
                        t = r4[a].z - c4[b].z;
                        s = fmaf(t, t, s);
                        t = r4[a].w - c4[b].w;
                        s = fmaf(t, t, s);
                        acc[a][b] = s;
                    }
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) dt[(4 * ty + a) * (EP + 1) + 4 * tx + b] = acc[a][b];
        __syncthreads();
        for (int qq = 0; qq < EQ / 4; ++qq) {
            const int q = w * (EQ / 4) + qq;
            if (q0 + q >= nq) break;
            const int64_t pid = p0 + lane;
            uint64_t key = (pid < n && pid != excl[q]) ? pack_key(dt[q * (EP + 1) + lane], (int32_t)pid)
                                                       : KEY_INF;
            uint64_t cur = topk[q * PG_WAVE + lane];
            const uint64_t kth = shfl64(cur, k - 1);
            if (key >= kth) key = KEY_INF;
            if (__ballot(key != KEY_INF) == 0) continue;
            int pk = 0, pc = 0;
            wave_sort(key, pk);
            wave_merge_lowest(cur, pc, key, pk);
            if (lane >= k) cur = KEY_INF;
            topk[q * PG_WAVE + lane] = cur;
        }
    }
    __syncthreads();
    for (int qq = 0; qq < EQ / 4; ++qq) {
        const int q = w * (EQ / 4) + qq;
        if (q0 + q >= nq) break;
        if (lane < k) {
            const uint64_t key = topk[q * PG_WAVE + lane];
            out_ids[(q0 + q) * k + lane] = key == KEY_INF ? -1 : key_id(key);
            out_d2[(q0 + q) * k + lane] = key == KEY_INF ? __int_as_float(0x7f800000) : key_d2(key);
        }
    }
}

// ---------------------------------------------------------------------------
// locality order of the join sources: nodes grouped by their nearest pivot
// (pivots = every step-th row), so that sources sharing join-set members run
// close together in time.  Any order gives the same lists.
// ---------------------------------------------------------------------------
__global__ void k_iota(int32_t *__restrict__ order, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) order[i] = (int32_t)i;
}

__global__ void k_order_scatter(const int32_t *__restrict__ piv, int64_t n, const int64_t *__restrict__ off,
                                int32_t *__restrict__ cur, int32_t *__restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = piv[i];
    order[off[g] + atomicAdd(&cur[g], 1)] = (int32_t)i;
}

// collection of every node: the last c with off[c] <= u (binary search)
__global__ void k_seg_fill(const int64_t *__restrict__ off, int ncoll, int64_t n, int32_t *__restrict__ seg_of) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int a = 0, b = ncoll - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (off[mid] <= u)
            a = mid;
        else
            b = mid - 1;
    }
    seg_of[u] = a;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct KnnLayout {
    size_t keys, newm, insm, nf, nf_c, of, of_c, rn_cnt, ro_cnt, rn_off, ro_off, rn_list, ro_list,
        jn, jn_c, jo, jo_c, pcnt, bucket, mark, mark_next, counters, scan_tmp, spill_t, spill_k,
        spill_s, x16, norms, exflags, order, mu, mu_part, seg_of, seg_off, seg_frozen, seg_updates, total;
    int64_t mu_nb;
    int B, JN, JO, d16;
    int64_t spill_cap;
};

static int default_bucket(int K) { return 8 * K; }

static KnnLayout knn_layout(const pg_knn_params *p, int64_t n, int d, int ncoll = 0) {
    KnnLayout L{};
    L.d16 = (d + 15) / 16 * 16;
    const int64_t K = p->K, S = p->S;
    L.B = p->bucket_cap > 0 ? p->bucket_cap : default_bucket(p->K);
    L.JN = (int)(2 * S);
    L.JO = (int)(K + S);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += pg_align(bytes);
        return at;
    };
    L.keys = take(sizeof(uint64_t) * n * K);
    L.newm = take(sizeof(uint64_t) * n);
    L.insm = take(sizeof(uint64_t) * n);
    L.nf = take(sizeof(int32_t) * n * S);
    L.nf_c = take(sizeof(int32_t) * n);
    L.of = take(sizeof(int32_t) * n * K);
    L.of_c = take(sizeof(int32_t) * n);
    L.rn_cnt = take(sizeof(int32_t) * n);
    L.ro_cnt = take(sizeof(int32_t) * n);
    L.rn_off = take(sizeof(int64_t) * (n + 1));
    L.ro_off = take(sizeof(int64_t) * (n + 1));
    L.rn_list = take(sizeof(int32_t) * n * S);
    L.ro_list = take(sizeof(int32_t) * n * K);
    L.jn = take(sizeof(int32_t) * n * L.JN);
    L.jn_c = take(sizeof(int32_t) * n);
    L.jo = take(sizeof(int32_t) * n * L.JO);
    L.jo_c = take(sizeof(int32_t) * n);
    L.pcnt = take(sizeof(int32_t) * n);
    L.bucket = take(sizeof(uint64_t) * n * (size_t)L.B);
    L.mark = take(n);
    L.mark_next = take(n);
    L.counters = take(sizeof(unsigned long long) * (NSTRIPE * CSTRIDE + C_NCOUNTERS));
    L.scan_tmp = take(scan_tmp_bytes(n + 1));
    // two proposals per list entry: a full spill segment forces a repeat
    // pass, and a quarter of this (n K / 2) left the GIST-shaped build five of
    // them (join 1.31 s; 1.04 s without)
    L.spill_cap = (std::max<int64_t>(1 << 16, n * K * 2) + NSTRIPE - 1) / NSTRIPE * NSTRIPE;
    L.spill_t = take(sizeof(int32_t) * L.spill_cap);
    L.spill_k = take(sizeof(uint64_t) * L.spill_cap);
    L.spill_s = take(sizeof(uint64_t) * L.spill_cap);
    const bool half = p->precision == PG_FP16 || p->precision == PG_BF16;
    L.x16 = take(half ? (size_t)2 * n * L.d16 : 0);
    L.norms = take(sizeof(float) * n);
    L.exflags = take(sizeof(unsigned int) * 4);
    L.order = take(sizeof(int32_t) * n);
    L.mu_nb = half ? (n + MU_ROWS - 1) / MU_ROWS : 0;
    L.mu = take(half ? sizeof(float) * d : 0);
    L.mu_part = take(sizeof(double) * L.mu_nb * d);
    // collections of a batched build (none for a single build)
    L.seg_of = take(ncoll ? sizeof(int32_t) * n : 0);
    L.seg_off = take(ncoll ? sizeof(int64_t) * (ncoll + 1) : 0);
    L.seg_frozen = take(ncoll ? (size_t)ncoll : 0);
    L.seg_updates = take(ncoll ? sizeof(unsigned long long) * ncoll : 0);
    L.total = o;
    return L;
}

static pg_status check_knn(const pg_knn_params *p, int64_t n, int32_t d) {
    if (!p) {
        set_error("pg_knn_build: params is NULL");
        return PG_EINVAL;
    }
    if (n < 2 || n >= (int64_t)1 << 31) {
        set_error("pg_knn_build: n=%lld out of range [2, 2^31)", (long long)n);
        return PG_EINVAL;
    }
    if (d <= 0 || d % 4) {
        set_error("pg_knn_build: d=%d must be a positive multiple of 4", d);
        return d <= 0 ? PG_EINVAL : PG_EUNSUPPORTED;
    }
    if (p->K < 1 || p->K > 64 || p->K >= n) {
        set_error("pg_knn_build: K=%d must satisfy 1 <= K <= 64 and K < n", p->K);
        return PG_EINVAL;
    }
    if (p->exact) return PG_OK;
    if (p->S < 1 || p->S > p->K || p->S > 32) {
        set_error("pg_knn_build: S=%d must satisfy 1 <= S <= min(K, 32)", p->S);
        return PG_EINVAL;
    }
    if (p->max_iters < 0 || p->max_iters > 64) {
        set_error("pg_knn_build: max_iters=%d out of [0, 64]", p->max_iters);
        return PG_EINVAL;
    }
    if (p->precision < PG_FP32 || p->precision > PG_FP32_VALU) {
        set_error("pg_knn_build: unknown precision %d", p->precision);
        return PG_EINVAL;
    }
    if (p->bucket_cap != 0 && p->bucket_cap < 2 * p->K) {
        set_error("pg_knn_build: bucket_cap=%d must be 0 or >= 2K", p->bucket_cap);
        return PG_EINVAL;
    }
    if (p->chunks < 0) {
        set_error("pg_knn_build: chunks=%d must be >= 0", p->chunks);
        return PG_EINVAL;
    }
    if (!(p->margin_rel >= -1.0f && p->margin_rel <= 1.0f)) {
        set_error("pg_knn_build: margin_rel=%g must be in [-1, 1]", (double)p->margin_rel);
        return PG_EINVAL;
    }
    return PG_OK;
}

}  // namespace pgi

using namespace pgi;

extern "C" pg_status pg_knn_build_workspace(const pg_knn_params *p, int64_t n, int32_t d,
                                            size_t *bytes) {
    PG_TRY(check_knn(p, n, d));
    if (!bytes) {
        set_error("pg_knn_build_workspace: bytes is NULL");
        return PG_EINVAL;
    }
    *bytes = p->exact ? 0 : knn_layout(p, n, d).total;
    return PG_OK;
}

static pg_status launch_exact(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                              const float *Q, int64_t nq, int64_t ldq, const int32_t *exclude,
                              int self_excl, int32_t k, int32_t *out_ids, float *out_d2,
                              const int32_t *qrow = nullptr, int64_t qrow_n = 0) {
    if (nq == 0) return PG_OK;
    const int64_t blocks = (nq + EQ - 1) / EQ;
    TimedLaunch tl(ctx, K_EXACT, 3.0 * (double)n * (double)nq * d);
    hipLaunchKernelGGL(k_exact_knn, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, X, n, d, ldx, Q,
                       nq, ldq, qrow, qrow_n, exclude, self_excl, k, out_ids, out_d2);
    PG_HIP(hipGetLastError());
    return PG_OK;
}

extern "C" pg_status pg_exact_knn(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                  const float *Q, int64_t nq, int64_t ldq, const int32_t *exclude,
                                  int32_t k, int32_t *out_ids, float *out_d2) {
    if (!ctx || !X || !Q || !out_ids || !out_d2) {
        set_error("pg_exact_knn: NULL argument");
        return PG_EINVAL;
    }
    if (n < 1 || n >= (int64_t)1 << 31 || nq < 0 || k < 1 || k > 64 || d <= 0 || ldx < d ||
        ldq < d) {
        set_error("pg_exact_knn: bad sizes n=%lld nq=%lld d=%d k=%d", (long long)n,
                  (long long)nq, d, k);
        return PG_EINVAL;
    }
    if (d % 4 || ldx % 4 || ldq % 4 || ((uintptr_t)X & 15) || ((uintptr_t)Q & 15)) {
        set_error("pg_exact_knn: d, ldx, ldq must be multiples of 4 and X, Q 16-byte aligned");
        return PG_EUNSUPPORTED;
    }
    return launch_exact(ctx, X, n, d, ldx, Q, nq, ldq, exclude, 0, k, out_ids, out_d2);
}

static pg_status knn_exact_lists(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                 int K, int32_t *ids, float *d2) {
    // the rows of X are their own queries; each skips itself
    PG_TRY(launch_exact(ctx, X, n, d, ldx, X, n, ldx, nullptr, 1, K, ids, d2));
    PG_HIP(hipStreamSynchronize(ctx->stream));
    return PG_OK;
}

static pg_status check_build_args(const char *who, pg_ctx *ctx, const float *X, int64_t n, int32_t d,
                                  int64_t ldx, const pg_knn_params *p, int32_t *knn_ids, float *knn_d2) {
    if (!ctx || !X || !knn_ids || !knn_d2) {
        set_error("%s: NULL argument", who);
        return PG_EINVAL;
    }
    PG_TRY(check_knn(p, n, d));
    if (ldx < d || ldx % 4 || ((uintptr_t)X & 15)) {
        set_error("%s: ldx must be >= d and a multiple of 4, X 16-byte aligned", who);
        return PG_EUNSUPPORTED;
    }
    return PG_OK;
}

// The build itself, arguments already checked.  ws holds at least
// knn_layout(p, n, d).total bytes of any content: everything that must start
// at zero is cleared on the stream here.  Nothing is allocated.
// A batch (ncoll > 0) holds collections [off[c], off[c + 1]) of the rows;
// each stops on its own rule (stop[c]) and iters[c] receives its iterations.
struct BatchSpec {
    int ncoll;
    const int64_t *off;   // host, ncoll + 1
    const int64_t *stop;  // host, ncoll
    int32_t *iters;       // host, ncoll (optional)
};

static pg_status knn_build_run(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                               const pg_knn_params *p, void *ws, int32_t *knn_ids, float *knn_d2,
                               pg_knn_stats *stats, const BatchSpec &bs = BatchSpec{0, nullptr, nullptr, nullptr}) {
    if (stats) memset(stats, 0, sizeof(*stats));
    if (p->exact) return knn_exact_lists(ctx, X, n, d, ldx, p->K, knn_ids, knn_d2);
    const KnnLayout L = knn_layout(p, n, d, bs.ncoll);
    char *w = (char *)ws;
    Segs sg{nullptr, nullptr, nullptr};
    unsigned long long *seg_upd = nullptr;
    std::vector<uint8_t> frozen_h;
    if (bs.ncoll > 0) {
        int32_t *seg_of = (int32_t *)(w + L.seg_of);
        int64_t *seg_off = (int64_t *)(w + L.seg_off);
        uint8_t *seg_fr = (uint8_t *)(w + L.seg_frozen);
        seg_upd = (unsigned long long *)(w + L.seg_updates);
        PG_HIP(hipMemcpyAsync(seg_off, bs.off, sizeof(int64_t) * (bs.ncoll + 1), hipMemcpyHostToDevice,
                              ctx->stream));
        PG_HIP(hipMemsetAsync(seg_fr, 0, (size_t)bs.ncoll, ctx->stream));
        hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, seg_off,
                           bs.ncoll, n, seg_of);
        PG_HIP(hipGetLastError());
        sg = Segs{seg_of, seg_off, seg_fr};
        frozen_h.assign((size_t)bs.ncoll, 0);
        if (bs.iters)
            for (int c = 0; c < bs.ncoll; ++c) bs.iters[c] = 0;
    }
    uint64_t *keys = (uint64_t *)(w + L.keys), *newm = (uint64_t *)(w + L.newm),
             *insm = (uint64_t *)(w + L.insm);
    int32_t *nf = (int32_t *)(w + L.nf), *nf_c = (int32_t *)(w + L.nf_c), *of = (int32_t *)(w + L.of),
            *of_c = (int32_t *)(w + L.of_c), *rn_cnt = (int32_t *)(w + L.rn_cnt),
            *ro_cnt = (int32_t *)(w + L.ro_cnt), *rn_list = (int32_t *)(w + L.rn_list),
            *ro_list = (int32_t *)(w + L.ro_list), *jn = (int32_t *)(w + L.jn),
            *jn_c = (int32_t *)(w + L.jn_c), *jo = (int32_t *)(w + L.jo),
            *jo_c = (int32_t *)(w + L.jo_c), *pcnt = (int32_t *)(w + L.pcnt);
    int64_t *rn_off = (int64_t *)(w + L.rn_off), *ro_off = (int64_t *)(w + L.ro_off);
    uint64_t *bucket = (uint64_t *)(w + L.bucket);
    uint8_t *mark = (uint8_t *)(w + L.mark), *mark_next = (uint8_t *)(w + L.mark_next);
    int32_t *spill_t = (int32_t *)(w + L.spill_t);
    uint64_t *spill_k = (uint64_t *)(w + L.spill_k), *spill_s = (uint64_t *)(w + L.spill_s);
    unsigned long long *counters = (unsigned long long *)(w + L.counters);
    unsigned long long *csum = counters + NSTRIPE * CSTRIDE;  // reduced view
    const int64_t seg = L.spill_cap / NSTRIPE;                // spill entries per segment
    void *scan_tmp = w + L.scan_tmp;
    hipStream_t st = ctx->stream;
    const int K = p->K, S = p->S;
    const unsigned wave_blocks = (unsigned)((n + 3) / 4);

    PG_HIP(hipMemsetAsync(pcnt, 0, sizeof(int32_t) * n, st));
    PG_HIP(hipMemsetAsync(mark_next, 0, n, st));
    // ---- a1: precision prep and exactness test; choose the join path
    _Float16 *xh = (_Float16 *)(w + L.x16);
    __bf16 *xb = (__bf16 *)(w + L.x16);
    float *norms = (float *)(w + L.norms);
    unsigned int *exf = (unsigned int *)(w + L.exflags);
    int path = PG_JOIN_VALU;
    MixedParams mx{};
    if (p->precision != PG_FP32_VALU) {
        PG_HIP(hipMemsetAsync(exf, 0, sizeof(unsigned int) * 4, st));
        hipLaunchKernelGGL(k_prep, dim3((unsigned)std::min<int64_t>(wave_blocks, 4096)), dim3(256), 0, st, X, ldx,
                           d, L.d16, n, p->precision, xh,
                           xb, norms, exf);
        PG_HIP(hipGetLastError());
        unsigned int he[4];
        PG_HIP(hipMemcpyAsync(he, exf, sizeof(he), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        float maxabs;
        memcpy(&maxabs, &he[EX_MAXABS], 4);
        const bool ints = exact_integer_rows(he);
        if (p->precision == PG_FP32 && ints) path = PG_JOIN_MFMA_FP32;
        MixedParams none{};
        mx = none;
        if (p->precision == PG_FP16 || p->precision == PG_BF16) {
            const bool f16 = p->precision == PG_FP16;
            if (ints && maxabs <= (f16 ? 2048.0f : 256.0f)) {
                path = f16 ? PG_JOIN_MFMA_FP16 : PG_JOIN_MFMA_BF16;
            } else {
                // mixed precision: centred 16-bit prefilter, direct-form recheck
                float *mu = (float *)(w + L.mu);
                double *part = (double *)(w + L.mu_part);
                hipLaunchKernelGGL(k_colsum_partial, dim3((unsigned)L.mu_nb), dim3(256), 0, st, X, ldx, d, n, part);
                hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, part,
                                   L.mu_nb, d, n, mu);
                PG_HIP(hipMemsetAsync(exf, 0, sizeof(unsigned int) * 4, st));
                hipLaunchKernelGGL(k_prep_mixed, dim3((unsigned)std::min<int64_t>(wave_blocks, 4096)), dim3(256), 0,
                                   st, X, ldx, d, L.d16, n, p->precision, mu, xh, xb, norms, exf);
                PG_HIP(hipGetLastError());
                PG_HIP(hipMemcpyAsync(he, exf, sizeof(he), hipMemcpyDeviceToHost, st));
                PG_HIP(hipStreamSynchronize(st));
                float cmax;
                memcpy(&cmax, &he[EX_MAXABS], 4);
                if (!(cmax <= (f16 ? 32768.0f : 1e30f))) {
                    set_error("pg_knn_build: centred values up to %g do not fit the 16-bit tiles; use PG_FP32",
                              (double)cmax);
                    return PG_EUNSUPPORTED;
                }
                path = f16 ? PG_JOIN_MIXED_FP16 : PG_JOIN_MIXED_BF16;
                mx.on = 1;
                mx.rigorous = p->margin_rel >= 0.0f;
                mx.mrel = fabsf(p->margin_rel);
                const double u32 = 1.0 / 16777216.0;
                mx.un = (float)((f16 ? 1.0 / 2048.0 : 1.0 / 256.0) + 4.0 * u32);
                mx.ea = f16 ? 2.98023224e-08f : 1e-38f;  // half the 16-bit subnormal spacing
                mx.gd = (float)((d + 4) * u32 * 1.01);
                mx.ga = (float)((2.0 * d + 16) * u32 * 1.01);
                mx.sqd = sqrtf((float)d);
            }
        }
    }
    // ---- a2: init (rows from the exact FP16 copy where the join uses it)
    {
        TimedLaunch tl(ctx, K_INIT, (double)n * K * (8.0 + 4.0 * d));
        const _Float16 *x16i = path == PG_JOIN_MFMA_FP16 ? xh : nullptr;
        hipLaunchKernelGGL(k_init, dim3(wave_blocks), dim3(256), 0, st, X, ldx, d, x16i, L.d16, n, K, p->seed,
                           keys, newm, insm, sg);
        PG_HIP(hipGetLastError());
    }
    if (stats) stats->join_path = path;
    // ---- locality order of the join sources (nearest of P pivot rows).  The
    // order never changes the result.  At 10M x 96, 256 pivots against 1024
    // assign in 38 instead of 115 ms and cost the join 24 ms of locality.
    int32_t *order = (int32_t *)(w + L.order);
    {
        const int64_t P = std::min<int64_t>(256, n / 4096);
        if (P <= 1) {
            hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, order, n);
        } else {
            const int64_t step = n / P;
            int32_t *piv = jn;          // free until the first iteration
            float *pd2 = (float *)jo;
            PG_TRY(launch_exact(ctx, X, P, d, step * ldx, X, n, ldx, nullptr, 0, 1, piv, pd2));
            PG_HIP(hipMemsetAsync(rn_cnt, 0, sizeof(int32_t) * P, st));
            hipLaunchKernelGGL(k_count_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, piv, n,
                               rn_cnt);
            PG_TRY(scan_exclusive(ctx, rn_cnt, rn_off, P, scan_tmp));
            PG_HIP(hipMemsetAsync(rn_cnt, 0, sizeof(int32_t) * P, st));
            hipLaunchKernelGGL(k_order_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, piv, n,
                               rn_off, rn_cnt, order);
        }
        PG_HIP(hipGetLastError());
    }
    const int maxm = 3 * S + K;
    const bool mixed = path == PG_JOIN_MIXED_FP16 || path == PG_JOIN_MIXED_BF16;
    const size_t lds = path == PG_JOIN_VALU ? join_lds_bytes(maxm)
                                            : (mixed ? join_hybrid_lds_bytes(maxm) : join_mfma_lds_bytes(maxm));
    int iters = 0;
    int64_t prev_props = -1;
    for (int t = 1; t <= p->max_iters; ++t) {
        PG_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * (NSTRIPE * CSTRIDE + C_NCOUNTERS), st));
        PG_HIP(hipMemsetAsync(rn_cnt, 0, sizeof(int32_t) * n, st));
        PG_HIP(hipMemsetAsync(ro_cnt, 0, sizeof(int32_t) * n, st));
        {
            TimedLaunch tl(ctx, K_SAMPLE, (double)n * K * 8.0);
            // slots of the reverse entries live in jn / jo until the join sets are built
            hipLaunchKernelGGL(k_sample, dim3(wave_blocks), dim3(256), 0, st, keys, newm, n, K, S,
                               p->seed, (uint64_t)(3 * t), nf, nf_c, of, of_c, rn_cnt, ro_cnt, jn, jo, sg);
            PG_HIP(hipGetLastError());
        }
        PG_TRY(scan_exclusive(ctx, rn_cnt, rn_off, n, scan_tmp));
        PG_TRY(scan_exclusive(ctx, ro_cnt, ro_off, n, scan_tmp));
        hipLaunchKernelGGL(k_rev_scatter, dim3(wave_blocks), dim3(256), 0, st, n, nf, nf_c, S, of,
                           of_c, K, rn_off, jn, rn_list, ro_off, jo, ro_list);
        PG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_build_join, dim3(std::min<unsigned>(wave_blocks, 8192)), dim3(256), 0, st, n, K, S,
                           p->seed,
                           (uint64_t)(3 * t + 1), (uint64_t)(3 * t + 2), nf, nf_c, of, of_c, rn_off,
                           rn_list, ro_off, ro_list, jn, jn_c, L.JN, jo, jo_c, L.JO, counters, sg);
        PG_HIP(hipGetLastError());
        // Source passes: residue classes of the order positions mod 64, sized
        // r, r, 2r, 4r, ... (r = 64 / c).  Each merge tightens every K-th key,
        // so later (larger) passes emit fewer proposals; c grows with the
        // proposals of the previous iteration.  The passes never change the
        // result.
        // at most 8 boundaries: r, r, 2r, 4r, ... covering 64 residues
        int rbnd[2 + PG_PASS_PERIOD];
        int nb = 0;
        rbnd[nb++] = 0;
        {
            int64_t c0;
            if (prev_props < 0)
                c0 = p->chunks > 0 ? std::min(p->chunks, PG_PASS_PERIOD) : PG_PASS_PERIOD;
            else
                c0 = (int64_t)std::min<double>(
                    PG_PASS_PERIOD,
                    std::max<double>(1.0, std::ceil(4.0 * (double)prev_props / ((double)L.B * n))));
            int sz = std::max<int>(1, PG_PASS_PERIOD / (int)c0), at = 0;
            bool first = true;
            while (at < PG_PASS_PERIOD) {
                at = std::min(PG_PASS_PERIOD, at + sz);
                rbnd[nb++] = at;
                if (!first) sz *= 2;
                first = false;
            }
        }
        for (int ci = 0; ci + 1 < nb; ++ci) {
            PassRange pr;
            pr.lo = rbnd[ci];
            pr.w = rbnd[ci + 1] - rbnd[ci];
            pr.items = (n + PG_PASS_PERIOD - 1) / PG_PASS_PERIOD * pr.w;
            const uint8_t *mk = nullptr;
            for (int attempt = 0;; ++attempt) {
                {
                    TimedLaunch tl(ctx, K_JOIN, -1.0);
                    const unsigned mg = xcd_grid((pr.items + MW - 1) / MW);
                    const unsigned hg = xcd_grid((pr.items + HW - 1) / HW);
                    const void *x16 = (const void *)(w + L.x16);
                    if (path == PG_JOIN_VALU)
                        hipLaunchKernelGGL(k_join, dim3(xcd_grid((pr.items + JW - 1) / JW)), dim3(JT), lds, st,
                                           X, ldx, d, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys, pcnt, bucket,
                                           L.B, spill_t, spill_k, seg, mark_next, mk, order, n, pr,
                                           maxm, counters);
                    else if (path == PG_JOIN_MFMA_FP32)
                        hipLaunchKernelGGL((k_join_mfma<PG_FP32>), dim3(mg), dim3(MW * PG_WAVE), lds, st, X, ldx,
                                           x16, d, L.d16, norms, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys,
                                           pcnt, bucket, L.B, spill_t, spill_k, seg, mark_next, mk,
                                           order, n, pr, maxm, counters);
                    else if (path == PG_JOIN_MFMA_FP16)
                        hipLaunchKernelGGL((k_join_mfma<PG_FP16>), dim3(mg), dim3(MW * PG_WAVE), lds, st, X,
                                           ldx, x16, d, L.d16, norms, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys, pcnt,
                                           bucket, L.B, spill_t, spill_k, seg, mark_next, mk, order, n, pr,
                                           maxm, counters);
                    else if (path == PG_JOIN_MFMA_BF16)
                        hipLaunchKernelGGL((k_join_mfma<PG_BF16>), dim3(mg), dim3(MW * PG_WAVE), lds, st, X,
                                           ldx, x16, d, L.d16, norms, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys, pcnt,
                                           bucket, L.B, spill_t, spill_k, seg, mark_next, mk, order, n, pr,
                                           maxm, counters);
                    else if (path == PG_JOIN_MIXED_FP16)
                        hipLaunchKernelGGL((k_join_hybrid<PG_FP16>), dim3(hg), dim3(HW * PG_WAVE), lds, st, X,
                                           ldx, x16, d, L.d16, norms, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys, pcnt,
                                           bucket, L.B, spill_t, spill_k, seg, mark_next, mk, order, n, pr,
                                           maxm, mx, counters);
                    else
                        hipLaunchKernelGGL((k_join_hybrid<PG_BF16>), dim3(hg), dim3(HW * PG_WAVE), lds, st, X,
                                           ldx, x16, d, L.d16, norms, K, jn, jn_c, L.JN, jo, jo_c, L.JO, keys, pcnt,
                                           bucket, L.B, spill_t, spill_k, seg, mark_next, mk, order, n, pr,
                                           maxm, mx, counters);
                    PG_HIP(hipGetLastError());
                }
                unsigned long long hc2[C_NCOUNTERS];
                hipLaunchKernelGGL(k_counters_reduce, dim3(1), dim3(NSTRIPE), 0, st, counters, seg, csum);
                PG_HIP(hipMemcpyAsync(hc2, csum, sizeof(hc2), hipMemcpyDeviceToHost, st));
                PG_HIP(hipStreamSynchronize(st));
                const int64_t nsp = (int64_t)hc2[C_SPILL];
                const int64_t *soff = nullptr;
                if (nsp > 0) {
                    // group the spilled proposals by node (counting sort over every segment)
                    const dim3 sg((unsigned)((hc2[C_SPILLMAX] + 255) / 256), NSTRIPE);
                    PG_HIP(hipMemsetAsync(rn_cnt, 0, sizeof(int32_t) * n, st));
                    hipLaunchKernelGGL(k_spill_count, sg, dim3(256), 0, st, spill_t, counters, seg, rn_cnt);
                    PG_TRY(scan_exclusive(ctx, rn_cnt, rn_off, n, scan_tmp));
                    PG_HIP(hipMemsetAsync(rn_cnt, 0, sizeof(int32_t) * n, st));
                    hipLaunchKernelGGL(k_spill_scatter, sg, dim3(256), 0, st, spill_t, spill_k, counters, seg, rn_off,
                                       rn_cnt, spill_s);
                    hipLaunchKernelGGL(k_counters_clear, dim3(1), dim3(NSTRIPE), 0, st, counters, (int)C_SPILL);
                    PG_HIP(hipGetLastError());
                    soff = rn_off;
                    if (stats) stats->spilled += nsp;
                }
                {
                    TimedLaunch tl(ctx, K_MERGE, -1.0);
                    hipLaunchKernelGGL(k_merge, dim3(wave_blocks), dim3(256), 0, st, keys, newm, insm,
                                       n, K, pcnt, bucket, L.B, soff, spill_s);
                    PG_HIP(hipGetLastError());
                }
                if (hc2[C_OVF] == 0) break;
                if (attempt >= 1000) {
                    set_error("pg_knn_build: proposal buffers kept overflowing");
                    return PG_EOVERFLOW;
                }
                if (stats) stats->retries++;
                hipLaunchKernelGGL(k_counters_clear, dim3(1), dim3(NSTRIPE), 0, st, counters, (int)C_OVF);
                hipLaunchKernelGGL(k_mark_swap, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                                   mark, mark_next, n);
                PG_HIP(hipGetLastError());
                mk = mark;
            }
        }
        if (bs.ncoll > 0) PG_HIP(hipMemsetAsync(seg_upd, 0, sizeof(unsigned long long) * bs.ncoll, st));
        hipLaunchKernelGGL(k_count_updates, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, insm,
                           n, counters, sg, seg_upd);
        PG_HIP(hipGetLastError());
        unsigned long long hc[C_NCOUNTERS];
        hipLaunchKernelGGL(k_counters_reduce, dim3(1), dim3(NSTRIPE), 0, st, counters, seg, csum);
        PG_HIP(hipMemcpyAsync(hc, csum, sizeof(hc), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        iters = t;
        prev_props = (int64_t)hc[C_PROPOSALS];
        if (stats) {
            stats->updates[t - 1] = (int64_t)hc[C_UPDATES];
            stats->pairs[t - 1] = (int64_t)hc[C_PAIRS];
            stats->proposals[t - 1] = (int64_t)hc[C_PROPOSALS];
            stats->rechecked[t - 1] = (int64_t)hc[C_RECHECK];
            stats->members[t - 1] = (int64_t)hc[C_MEMBERS];
        }
        // algorithmic work of the joins: flops of the distance form for the
        // FP32 paths, bytes of 16-bit row gathers for the 16-bit ones
        if (path == PG_JOIN_VALU)
            ctx_add_work(ctx, K_JOIN, 3.0 * (double)hc[C_PAIRS] * d);
        else if (path == PG_JOIN_MFMA_FP32)
            ctx_add_work(ctx, K_JOIN, 2.0 * (double)hc[C_PAIRS] * d);
        else
            ctx_add_work(ctx, K_JOIN, 2.0 * (double)hc[C_MEMBERS] * L.d16);
        if (bs.ncoll == 0) {
            if ((int64_t)hc[C_UPDATES] <= p->stop_updates) break;
            continue;
        }
        // batch: freeze every collection whose iteration met its stop rule
        std::vector<unsigned long long> su((size_t)bs.ncoll);
        PG_HIP(hipMemcpyAsync(su.data(), seg_upd, sizeof(unsigned long long) * bs.ncoll, hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        bool all = true;
        for (int c = 0; c < bs.ncoll; ++c) {
            if (frozen_h[c]) continue;
            if (bs.iters) bs.iters[c] = t;
            if ((int64_t)su[c] <= bs.stop[c]) frozen_h[c] = 1;
            all = all && frozen_h[c];
        }
        if (all) break;
        PG_HIP(hipMemcpyAsync((void *)sg.frozen, frozen_h.data(), (size_t)bs.ncoll, hipMemcpyHostToDevice, st));
    }
    if (stats) stats->iters_run = iters;
    const int64_t total = n * K;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, keys, total,
                       knn_ids, knn_d2, sg, K);
    PG_HIP(hipGetLastError());
    PG_HIP(hipStreamSynchronize(st));
    return PG_OK;
}

extern "C" pg_status pg_knn_build(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                  const pg_knn_params *p, void *ws, size_t ws_bytes,
                                  int32_t *knn_ids, float *knn_d2, pg_knn_stats *stats) {
    PG_TRY(check_build_args("pg_knn_build", ctx, X, n, d, ldx, p, knn_ids, knn_d2));
    if (!p->exact) {
        const size_t need = knn_layout(p, n, d).total;
        if (!ws || ws_bytes < need) {
            set_error("pg_knn_build: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
            return PG_ENOMEM;
        }
    }
    return knn_build_run(ctx, X, n, d, ldx, p, ws, knn_ids, knn_d2, stats);
}

// ---------------------------------------------------------------------------
// Quality examination (Section 5.2): hits[i] = |C(u)[:k] & N*_k(u)| for the
// sampled u = sample[i], N*_k(u) being the exact list the brute-force kernel
// wrote for it, and the estimate sum(hits) / (k ns).  One workgroup; integer
// sums, so the estimate does not depend on the order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cna_hits(const int32_t *__restrict__ cand, int C, int k,
                                                  const int32_t *__restrict__ sample, int64_t ns, int64_t n,
                                                  const int32_t *__restrict__ exact_ids,
                                                  int32_t *__restrict__ hits, double *__restrict__ estimate) {
    __shared__ long long part[256];
    __shared__ int bad[256];
    long long acc = 0;
    int nbad = 0;
    for (int64_t i = threadIdx.x; i < ns; i += 256) {
        const int32_t u = sample[i];
        int h = -1;
        if (u >= 0 && u < n) {
            h = 0;
            const int32_t *c = cand + (int64_t)u * C;
            const int32_t *t = exact_ids + i * k;
            // the exact ids are distinct, so counting those that C(u)[:k]
            // holds counts the intersection of the two sets
            for (int a = 0; a < k; ++a) {
                const int32_t v = t[a];
                if (v < 0) continue;
                bool in = false;
                for (int b = 0; b < k; ++b) in |= c[b] == v;
                h += in ? 1 : 0;
            }
            acc += h;
        } else {
            ++nbad;
        }
        hits[i] = h;
    }
    part[threadIdx.x] = acc;
    bad[threadIdx.x] = nbad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            part[threadIdx.x] += part[threadIdx.x + o];
            bad[threadIdx.x] += bad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *estimate = bad[0] ? __longlong_as_double(0x7ff8000000000000ll)
                           : (double)part[0] / ((double)k * (double)ns);
}

extern "C" pg_status pg_quality_examination(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                            const int32_t *cand_ids, int32_t C, int32_t k,
                                            const int32_t *sample, int64_t ns, int32_t *exact_ids,
                                            float *exact_d2, int32_t *hits, double *estimate) {
    if (!ctx || !X || !cand_ids || !sample || !exact_ids || !exact_d2 || !hits || !estimate) {
        set_error("pg_quality_examination: NULL argument");
        return PG_EINVAL;
    }
    if (n < 2 || n >= (int64_t)1 << 31 || d <= 0 || ldx < d || k < 1 || k > 64 || k >= n || C < k ||
        ns < 1 || ns > n) {
        set_error("pg_quality_examination: bad sizes n=%lld d=%d k=%d C=%d ns=%lld (need 1 <= k <= min(64, C), "
                  "k < n, 1 <= ns <= n)", (long long)n, d, k, C, (long long)ns);
        return PG_EINVAL;
    }
    if (d % 4 || ldx % 4 || ((uintptr_t)X & 15)) {
        set_error("pg_quality_examination: d and ldx must be multiples of 4 and X 16-byte aligned");
        return PG_EUNSUPPORTED;
    }
    // the sampled rows are their own queries, each skipping itself
    PG_TRY(launch_exact(ctx, X, n, d, ldx, X, ns, ldx, sample, 0, k, exact_ids, exact_d2, sample, n));
    hipLaunchKernelGGL(k_cna_hits, dim3(1), dim3(256), 0, ctx->stream, cand_ids, C, k, sample, ns, n, exact_ids,
                       hits, estimate);
    PG_HIP(hipGetLastError());
    return PG_OK;
}

// ---------------------------------------------------------------------------
// Batched builds: several collections of the same dimension in one launch of
// every kernel of an iteration.
// ---------------------------------------------------------------------------
static pg_status check_batch(const char *who, const pg_knn_params *p, int64_t n, const int64_t *off, int ncoll) {
    if (ncoll < 1 || !off) {
        set_error("%s: ncoll=%d must be >= 1 with offsets", who, ncoll);
        return PG_EINVAL;
    }
    if (p && p->exact) {
        set_error("%s: exact lists are not batched (use pg_exact_knn per collection)", who);
        return PG_EINVAL;
    }
    if (off[0] != 0 || off[ncoll] != n) {
        set_error("%s: offsets must run from 0 to n=%lld", who, (long long)n);
        return PG_EINVAL;
    }
    for (int c = 0; c < ncoll; ++c)
        if (p && off[c + 1] - off[c] <= p->K) {
            set_error("%s: collection %d has %lld rows, not more than K=%d", who, c,
                      (long long)(off[c + 1] - off[c]), p->K);
            return PG_EINVAL;
        }
    return PG_OK;
}

extern "C" pg_status pg_knn_build_batch_workspace(const pg_knn_params *p, int64_t n, int32_t d, int32_t ncoll,
                                                  size_t *bytes) {
    PG_TRY(check_knn(p, n, d));
    if (!bytes || ncoll < 1) {
        set_error("pg_knn_build_batch_workspace: bytes is NULL or ncoll < 1");
        return PG_EINVAL;
    }
    *bytes = knn_layout(p, n, d, ncoll).total;
    return PG_OK;
}

extern "C" pg_status pg_knn_build_batch(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                        const int64_t *offsets, int32_t ncoll, const int64_t *stop_updates,
                                        const pg_knn_params *p, void *ws, size_t ws_bytes, int32_t *knn_ids,
                                        float *knn_d2, int32_t *iters) {
    PG_TRY(check_build_args("pg_knn_build_batch", ctx, X, n, d, ldx, p, knn_ids, knn_d2));
    PG_TRY(check_batch("pg_knn_build_batch", p, n, offsets, ncoll));
    if (!stop_updates) {
        set_error("pg_knn_build_batch: stop_updates is NULL");
        return PG_EINVAL;
    }
    const size_t need = knn_layout(p, n, d, ncoll).total;
    if (!ws || ws_bytes < need) {
        set_error("pg_knn_build_batch: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return PG_ENOMEM;
    }
    return knn_build_run(ctx, X, n, d, ldx, p, ws, knn_ids, knn_d2, nullptr,
                         BatchSpec{ncoll, offsets, stop_updates, iters});
}

// ---------------------------------------------------------------------------
// pg_knn_build_noalloc: the same build with its workspace in a file-scope
// device array, for callers that cannot allocate device memory.  Each device
// the library runs on holds its own copy of the array until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and only that address is ever handed to kernels or copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PG_NOALLOC_WS_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static pg_status scratch_of(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("pg_knn_build_noalloc: device %d beyond the %d this library tracks", device, MAX_DEVICES);
        return PG_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        PG_HIP(hipGetDevice(&cur));
        if (cur != device) PG_HIP(hipSetDevice(device));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) PG_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) {
            set_error("pg_knn_build_noalloc: hipGetSymbolAddress returned no address");
            return PG_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PG_OK;
}

extern "C" pg_status pg_knn_build_noalloc(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                                          const pg_knn_params *p, int32_t *knn_ids, float *knn_d2,
                                          pg_knn_stats *stats) {
    PG_TRY(check_build_args("pg_knn_build_noalloc", ctx, X, n, d, ldx, p, knn_ids, knn_d2));
    void *ws = nullptr;
    if (!p->exact) {
        const size_t need = knn_layout(p, n, d).total;
        if (need > (size_t)PG_NOALLOC_WS_BYTES) {
            set_error("pg_knn_build_noalloc: n=%lld, d=%d, K=%d needs %zu workspace bytes, more than the "
                      "%zu of the static scratch; use pg_knn_build with a caller workspace",
                      (long long)n, d, p->K, need, (size_t)PG_NOALLOC_WS_BYTES);
            return PG_ENOMEM;
        }
        PG_TRY(scratch_of(ctx->device, &ws));
    }
    return knn_build_run(ctx, X, n, d, ldx, p, ws, knn_ids, knn_d2, stats);
}
