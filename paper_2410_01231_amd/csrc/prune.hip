// prune.hip -- refinement of the paper's Alg. 2 (Phase 3) for gfx950:
// Prune (Alg. 3) with the alpha test of Section 4.1, reverse-edge re-pruning,
// the entry point (closest point to the centroid, Alg. 2 Phase 2) and
// connectivity repair (DFS + extra edges of Alg. 2, done here as BFS).
//
// k_prune runs one wave per node over an arbitrary-length candidate list.
// Candidates are visited in ascending (d2, id) order, 64 at a time: a round
// selects the 64 smallest distinct keys above the last one processed (wave64
// bitonic sort + merge), then computes, for candidate j (lane j), its
// squared distance to every kept node and to every earlier candidate of the
// round.  Occlusion bits live in registers (lane j owns its 64-bit mask);
// the greedy keep/drop scan of Alg. 3 is then a 64-step scalar loop.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pg_common.h"

namespace pgi {

constexpr int PRG = 16;          // rows per register group
constexpr int PDC = 64;          // dims per chunk
constexpr int PSTR = PDC + 4;    // LDS row stride

// The alpha test of Section 4.1.  With a = d2(u,w), b = d2(v,w), c = d2(u,v)
// the law of cosines gives  angle(u w v) > alpha  <=>  a + b - c < kappa sqrt(a b),
// kappa = 2 cos(alpha).  The decision is defined as that inequality evaluated
// in IEEE double from the three FP32 squared distances, in this order:
// t = (a + b) - c, r = kappa_d * sqrt(a * b), with kappa_d the double value of
// 2 cos(alpha) (0 exactly at 90 degrees).  The kernels first evaluate it in
// FP32.  Each of t and r is then within 4 ulp-units of (a + b + c) of its
// double value (t: two roundings of sums of nonnegative terms; r: the
// product, a square root within 2 ulp, kappa rounded to FP32 and the final
// product, with |r| <= a + b), and the double evaluation is within 2^-50 of
// the same scale of the real one, so outside the band
// |t - r| > 2^-20 (a + b + c) the FP32 answer is the double answer.  Inside
// the band, and whenever a b leaves the normal FP32 range, the double
// evaluation decides.  Where the distances are exact (integer data) both
// sides of a comparison with a double-precision reference therefore take the
// same decision.
struct AngleTest {
    int on;      // alpha > 60: the test applies (at or below 60 it is implied)
    float kf;    // kappa rounded to FP32
    double kd;   // kappa in double
};

__device__ __noinline__ bool angle_in_band(float a, float b, float c, double kd) {
    return ((double)a + (double)b - (double)c) < kd * sqrt((double)a * (double)b);
}

__device__ __forceinline__ bool angle_exceeds(float a, float b, float c, const AngleTest &at) {
    const float p = a * b;
    const float t = (a + b) - c;
    const float r = at.kf * sqrtf(p);
    const float band = 0x1p-20f * ((a + b) + c);
    const bool normal = p >= 0x1p-120f && p <= 0x1p120f;
    if (normal && t < r - band) return true;
    if (normal && t > r + band) return false;
    return angle_in_band(a, b, c, at.kd);
}

__device__ __forceinline__ bool occludes(float a, float b, float c, int strict, const AngleTest &at) {
    // w (a = d2(u,w)) visited before v (c = d2(u,v)); b = d2(v,w)
    if (!(b < c)) return false;
    if (strict && !(a < c)) return false;
    if (!at.on) return true;
    if (b == 0.0f) return true;
    return angle_exceeds(a, b, c, at);
}

// Distances to u come from src1_d2 / src2_d2 when given (they must be the
// canonical chain values, as pg_knn_build and this stage produce), else from X.
__global__ __launch_bounds__(64) void k_prune(
    const float *__restrict__ X, int64_t ldx, int d, int64_t n, const int32_t *__restrict__ src1,
    const float *__restrict__ src1_d2, int C1, const int32_t *__restrict__ src1_deg,
    const int64_t *__restrict__ src2_off, const int32_t *__restrict__ src2, const float *__restrict__ src2_d2,
    int R, AngleTest at, int strict,
    const float *__restrict__ tab, int32_t *__restrict__ out_ids, float *__restrict__ out_d2,
    int32_t *__restrict__ out_deg) {
    __shared__ __align__(16) float rows[PRG * PSTR];
    __shared__ uint64_t kept_key[PG_WAVE];
    __shared__ int kept_pos[PG_WAVE];
    __shared__ uint64_t chunk_key[PG_WAVE];
    __shared__ int chunk_pos[PG_WAVE];
    const int lane = lane_id();
    const int64_t u = blockIdx.x;
    const int c1 = src1_deg ? min(src1_deg[u], C1) : C1;
    const int64_t off2 = src2_off ? src2_off[u] : 0;
    const int c2 = src2_off ? (int)(src2_off[u + 1] - off2) : 0;
    const int m = c1 + c2;
    const float *xu = X + u * ldx;
    const int64_t tstride = (int64_t)(C1 + 1) * (C1 + 1);
    const float *tu = tab ? tab + u * tstride : nullptr;

    int nk = 0;
    bool first = true;
    uint64_t last = 0;
    while (true) {
        // ---- next 64 smallest distinct keys above `last`
        uint64_t top = KEY_INF;
        int tpos = -1;
        for (int b = 0; b < m; b += PG_WAVE) {
            const int idx = b + lane;
            int32_t id = -1;
            float dgiven = -1.0f;
            if (idx < c1) {
                id = src1[u * C1 + idx];
                if (src1_d2) dgiven = src1_d2[u * C1 + idx];
            } else if (idx < m) {
                id = src2[off2 + (idx - c1)];
                if (src2_d2) dgiven = src2_d2[off2 + (idx - c1)];
            }
            uint64_t key = KEY_INF;
            if (id >= 0 && id < n && id != (int32_t)u) {
                const float dd = tu ? tu[idx + 1] : (dgiven >= 0.0f ? dgiven : dist_chain(xu, X + (int64_t)id * ldx, d));
                key = pack_key(dd, id);
                if (!first && key <= last) key = KEY_INF;
            }
            int pos = idx;
            wave_sort(key, pos);
            const uint64_t prev = from_lane_below64(key);
            const bool valid = key != KEY_INF && !(lane > 0 && prev == key);
            const int cl = wave_count_less(top, key);
            const uint64_t at = shfl64(top, min(cl, PG_WAVE - 1));
            const bool in_top = key != KEY_INF && cl < PG_WAVE && at == key;
            if (wave_compact(key, pos, valid && !in_top) == 0) continue;
            wave_merge_lowest(top, tpos, key, pos);
        }
        const int cm = __popcll(__ballot(top != KEY_INF));
        if (cm == 0) break;
        chunk_key[lane] = top;
        chunk_pos[lane] = tpos;
        __builtin_amdgcn_wave_barrier();
        const int32_t myid = top != KEY_INF ? key_id(top) : -1;
        const float myc = key_d2(top);
        const float *xv = myid >= 0 ? X + (int64_t)myid * ldx : X;
        const int NR = nk + cm;
        bool occk = false;
        uint64_t occ = 0;
        for (int g0 = 0; g0 < NR; g0 += PRG) {
            float acc[PRG];
#pragma unroll
            for (int r = 0; r < PRG; ++r) acc[r] = 0.0f;
            if (!tu) {
                for (int c0 = 0; c0 < d; c0 += PDC) {
                    const int dl = min(PDC, d - c0);
                    // stage the group's rows (kept nodes first, then this round's candidates)
                    for (int e = lane; e < PRG * (PDC / 4); e += PG_WAVE) {
                        const int r = e / (PDC / 4), q = e % (PDC / 4);
                        const int row = g0 + r;
                        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (row < NR && 4 * q < dl) {
                            const int32_t rid = row < nk ? key_id(kept_key[row]) : key_id(chunk_key[row - nk]);
                            val = *reinterpret_cast<const float4 *>(X + (int64_t)rid * ldx + c0 + 4 * q);
                        }
                        *reinterpret_cast<float4 *>(rows + r * PSTR + 4 * q) = val;
                    }
                    __builtin_amdgcn_wave_barrier();
                    __syncthreads();
                    if (myid >= 0) {
                        for (int q = 0; q < dl; q += 4) {
                            const float4 cv = *reinterpret_cast<const float4 *>(xv + c0 + q);
#pragma unroll
                            for (int r = 0; r < PRG; ++r) {
                                const float4 rv = *reinterpret_cast<const float4 *>(rows + r * PSTR + q);
                                float s = acc[r], t;
                                t = rv.x - cv.x;
                                s = fmaf(t, t, s);
                                t = rv.y - cv.y;
                                s = fmaf(t, t, s);
                                t = rv.z - cv.z;
                                s = fmaf(t, t, s);
                                t = rv.w - cv.w;
                                s = fmaf(t, t, s);
                                acc[r] = s;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            if (myid >= 0) {
#pragma unroll
                for (int r = 0; r < PRG; ++r) {
                    const int row = g0 + r;
                    if (row >= NR) break;
                    const bool is_kept = row < nk;
                    const int ci = row - nk;
                    if (!is_kept && ci >= lane) continue;
                    const float a = is_kept ? key_d2(kept_key[row]) : key_d2(chunk_key[ci]);
                    float b = acc[r];
                    if (tu) {
                        const int rp = is_kept ? kept_pos[row] : chunk_pos[ci];
                        b = tu[(int64_t)(rp + 1) * (C1 + 1) + (tpos + 1)];
                    }
                    const bool cnd = occludes(a, b, myc, strict, at);
                    if (is_kept)
                        occk |= cnd;
                    else if (cnd)
                        occ |= 1ull << ci;
                }
            }
        }
        // ---- greedy scan of Alg. 3 over this round's candidates
        uint64_t keptc = 0;
        const uint64_t occk_m = __ballot(occk);
        for (int j = 0; j < cm; ++j) {
            const uint64_t oj = readlane64(occ, j);
            if (((occk_m >> j) & 1ull) || (oj & keptc)) continue;
            keptc |= 1ull << j;
            if (lane == 0) {
                kept_key[nk] = chunk_key[j];
                kept_pos[nk] = chunk_pos[j];
            }
            __builtin_amdgcn_wave_barrier();
            ++nk;
            if (nk == R) break;
        }
        if (nk == R || cm < PG_WAVE || m <= PG_WAVE) break;
        last = readlane64(top, PG_WAVE - 1);
        first = false;
    }
    __syncthreads();
    if (lane < R) {
        const bool have = lane < nk;
        const uint64_t k = have ? kept_key[lane] : KEY_INF;
        out_ids[u * R + lane] = have ? key_id(k) : -1;
        out_d2[u * R + lane] = have ? key_d2(k) : __int_as_float(0x7f800000);
    }
    if (lane == 0) out_deg[u] = nk;
}

// ---------------------------------------------------------------------------
// Exact 16-bit path.  For integer-valued X with |x| <= 2048, FP16 holds every
// coordinate exactly.  With squared norms <= 2^23 every product and partial
// sum of a dot product is an integer of magnitude at most 2^23; the squared
// distance is at most 2^24 when no coordinate is negative (then v.w >= 0 and
// d2 <= n_v + n_w), or when every squared norm is at most 2^22.  Under either
// condition, with FP32 accumulation, d2(v, w) = n_v + n_w - 2 v.w equals the
// canonical chain bit for bit (every partial sum of the chain is an integer
// <= 2^24).  The prune then takes the pairwise distances of a round from
// 32 x 32 MFMA Gram tiles over rows staged once in LDS.
// ---------------------------------------------------------------------------
enum { PX_NONINT = 0, PX_MAXABS = 1, PX_MAXNORM = 2, PX_NEG = 3 };

typedef float pm_f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 pm_f16x8 __attribute__((ext_vector_type(8)));

// grid-stride over rows, one wave per row: FP16 copy (zero padded to d16),
// norms (lane-parallel sum: only used when the data pass the test, where any
// order is exact) and the exactness flags, one atomic per block and flag
__global__ __launch_bounds__(256) void k_prune_prep(const float *__restrict__ X, int64_t ldx, int d, int d16,
                                                    int64_t n, _Float16 *__restrict__ x16,
                                                    float *__restrict__ norms, unsigned int *__restrict__ ex) {
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
            x16[i * d16 + k] = (_Float16)v;
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
        if (a) atomicOr(&ex[PX_NONINT], 1u);
        atomicMax(&ex[PX_MAXABS], b);
        atomicMax(&ex[PX_MAXNORM], c);
        if (e) atomicOr(&ex[PX_NEG], 1u);
    }
}

// ---------------------------------------------------------------------------
// Mixed 16-bit path for float data.  The Gram tiles run on the centred FP16
// copy x^ = fp16(fl32(x - mu)) with FP32 norms n^ of the rounded rows, and
// give an estimate b^ = n^_v + n^_w - 2 v^.w^ of the canonical chain b of
// the FP32 rows.  With e = un (|x^| + |y^|)(1 + 2 un) + 2 sqrt(d) ea bounding
// the rounding of the difference, and the FP32 accumulation of the estimate
// within ga (n^_v + n^_w + 2 |v^.w^|) and of the chain within gd b (the same
// error model as the mixed join):
//   b <= t  implies  b^ <= hi(t) = t' + 2 e sqrt(t') + e^2 + acc,  t' = t (1 + gd)
//   b >= t  implies  b^ >= lo(t) = t" - 2 e sqrt(t") - e^2 - acc, t" = t (1 - gd)
// (the second as long as sqrt(t") >= e; below that lo is negative and never
// decides).  So b^ > hi(c) decides b > c (no occlusion) and, without the
// angle test, b^ < lo(c) decides b < c; every other pair, and with the angle
// test every pair that may occlude, gets its canonical chain from the FP32
// rows.  The decisions are therefore those of the VALU kernel.
// ---------------------------------------------------------------------------
struct PruneMix {
    int on;
    float un, ea, gd, ga, sqd;
};

__device__ __forceinline__ float pmix_e(const PruneMix &m, float nx, float ny) {
    return m.un * (sqrtf(nx) + sqrtf(ny)) * (1.0f + 2.0f * m.un) + 2.0f * m.sqd * m.ea;
}
__device__ __forceinline__ float pmix_hi(const PruneMix &m, float t, float e, float acc) {
    const float tg = t * (1.0f + m.gd);
    const float v = tg + 2.0f * e * sqrtf(tg) + e * e + acc;
    return v + v * 1e-5f + 1e-30f;  // slack for evaluating the bound in FP32
}
__device__ __forceinline__ float pmix_lo(const PruneMix &m, float t, float e, float acc) {
    const float tl = t * (1.0f - m.gd);
    const float r = 2.0f * e * sqrtf(tl) + e * e + acc;
    return (tl - r) - (tl + r) * 1e-5f - 1e-30f;
}

// one wave per row (grid-stride): x16 = fp16(fl32(x - mu)) with mu the FP32
// rounding of the centroid, norms = FP32 sum of the rounded squares;
// PX_MAXABS gets max |x - mu|
__global__ __launch_bounds__(256) void k_prune_prep_mixed(const float *__restrict__ X, int64_t ldx, int d, int d16,
                                                          int64_t n, const double *__restrict__ cen,
                                                          _Float16 *__restrict__ x16, float *__restrict__ norms,
                                                          unsigned int *__restrict__ ex) {
    __shared__ unsigned int red[4];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    float mabs = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < n; i += (int64_t)gridDim.x * 4) {
        const float *x = X + i * ldx;
        float s = 0.f;
        for (int k = lane; k < d16; k += PG_WAVE) {
            const float c = k < d ? x[k] - (float)cen[k] : 0.f;
            mabs = fmaxf(mabs, fabsf(c));
            const _Float16 hv = (_Float16)c;
            x16[i * d16 + k] = hv;
            const float r = (float)hv;
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
    if (threadIdx.x == 0) atomicMax(&ex[PX_MAXABS], max(max(red[0], red[1]), max(red[2], red[3])));
}

constexpr int PM_DC = 32;            // dimensions per staged chunk
constexpr int PM_RS = PM_DC + 8;     // LDS row stride in halves (16-byte pad)
constexpr int PM_ROWS = 96;          // 64 round candidates, then up to 32 kept nodes
constexpr int PM_LIST = 1024;        // undecided pairs listed before their chains run
constexpr int PM_CD = 16;            // dimensions per LDS chunk of the chains' FP32 rows
constexpr int PM_CS = PM_CD + 4;     // their LDS row stride (floats; 16-byte aligned)
constexpr int PM_STAGE_D = 256;      // rows at least this long are staged for the chains
static_assert(PM_ROWS * PM_CS * 4 <= PM_ROWS * PM_RS * 2, "the chains' rows fit in the 16-bit row buffer");
constexpr int PM_PF = PM_ROWS * (PM_DC / 8) / PG_WAVE;  // 16-byte row loads per lane and chunk

// One wave per node, rounds of up to 64 candidates as in k_prune; the
// distances to u are the given (canonical) ones, the pairwise ones come from
// Gram tiles: candidates x candidates (upper tiles) and kept x candidates
// (at most 32 nodes kept in earlier rounds: the host sends the reverse
// unions, which may need several rounds, here only when R <= 32).
// Occlusion among this round's candidates is kept per occluding row (lane i
// holds the set of later candidates that i occludes); the greedy scan of
// Alg. 3 ORs in the set of every candidate it keeps.
//
// MIX (float data): the tiles give estimates on the centred copy; pairs they
// cannot decide go to a list of the tile and get their canonical chains from
// the FP32 rows, one pair per lane, and their occlusion bits through LDS.
//
// K2P (Section 5.4): prev_ids holds u's list after the PRUNE stage of the
// previous round (same alpha and tie rule).  Two candidates that both stayed
// in it were both visited then, in the same (d2, id) order, and the earlier
// did not occlude the later (else the later would have been dropped); the
// test involves only the three points, so it is skipped now.  k2p counts the
// pairs skipped and the pairs tested.
template <bool MIX, bool STG>
__global__ __launch_bounds__(64, MIX ? 3 : 4) void k_prune_mfma(
    const _Float16 *__restrict__ X16, int d16, const float *__restrict__ norms, int64_t n,
    const int32_t *__restrict__ src1, const float *__restrict__ src1_d2, int C1,
    const int32_t *__restrict__ src1_deg, const int64_t *__restrict__ src2_off,
    const int32_t *__restrict__ src2, const float *__restrict__ src2_d2, int R, AngleTest at,
    int strict, int32_t *__restrict__ out_ids, float *__restrict__ out_d2, int32_t *__restrict__ out_deg,
    const float *__restrict__ X, int64_t ldx, int d, PruneMix pmx, const int32_t *__restrict__ prev_ids,
    const int32_t *__restrict__ prev_deg, int prevR, unsigned long long *__restrict__ k2p) {
    __shared__ __align__(16) _Float16 rows[PM_ROWS * PM_RS];
    __shared__ uint64_t kept_key[PG_WAVE];
    __shared__ uint64_t chunk_key[PG_WAVE];
    __shared__ float cn[PG_WAVE], kn[PG_WAVE];
    // mixed: pairs of the current tile left to the chains (row << 6 | column),
    // and the occlusion bits they produce
    __shared__ uint16_t rl[MIX ? PM_LIST : 1];
    __shared__ unsigned long long kill_lds[MIX ? PG_WAVE : 1];
    __shared__ unsigned long long occk_lds;
    __shared__ int32_t prev_lds[PG_WAVE];
    // mixed: ids of the rows the listed pairs involve, in staging order
    __shared__ int32_t srow[STG ? PM_ROWS : 1];
    const int lane = lane_id(), h = lane >> 5, l32 = lane & 31;
    const int64_t u = blockIdx.x;
    const int c1 = src1_deg ? min(src1_deg[u], C1) : C1;
    const int64_t off2 = src2_off ? src2_off[u] : 0;
    const int c2 = src2_off ? (int)(src2_off[u + 1] - off2) : 0;
    const int m = c1 + c2;
    const int np = prev_ids ? min(prev_deg[u], prevR) : 0;
    if (prev_ids) {
        prev_lds[lane] = lane < np ? prev_ids[u * prevR + lane] : -1;
        __builtin_amdgcn_wave_barrier();
    }
    unsigned long long n_skip = 0, n_test = 0;
    uint64_t kpk = 0;  // kept nodes that were in the previous round's list

    int nk = 0;
    bool first = true;
    uint64_t last = 0;
    while (true) {
        // ---- next 64 smallest distinct keys above `last`
        uint64_t top = KEY_INF;
        int tpos = -1;
        for (int b = 0; b < m; b += PG_WAVE) {
            const int idx = b + lane;
            int32_t id = -1;
            float dd = 0.f;
            if (idx < c1) {
                id = src1[u * C1 + idx];
                dd = src1_d2[u * C1 + idx];
            } else if (idx < m) {
                id = src2[off2 + (idx - c1)];
                dd = src2_d2[off2 + (idx - c1)];
            }
            uint64_t key = KEY_INF;
            if (id >= 0 && id < n && id != (int32_t)u) {
                key = pack_key(dd, id);
                if (!first && key <= last) key = KEY_INF;
            }
            if (first && m <= PG_WAVE) {
                // a list that is already sorted, distinct and valid (a kNN
                // list, a PRUNE result) is the round as it stands
                const uint64_t prv = from_lane_below64(key);
                const bool bad = idx < m && (key == KEY_INF || (lane > 0 && !(prv < key)));
                if (__ballot(bad) == 0) {
                    top = key;
                    tpos = idx;
                    continue;
                }
            }
            int pos = idx;
            wave_sort(key, pos);
            const uint64_t prev = from_lane_below64(key);
            const bool valid = key != KEY_INF && !(lane > 0 && prev == key);
            const int cl = wave_count_less(top, key);
            const uint64_t at = shfl64(top, min(cl, PG_WAVE - 1));
            const bool in_top = key != KEY_INF && cl < PG_WAVE && at == key;
            if (wave_compact(key, pos, valid && !in_top) == 0) continue;
            wave_merge_lowest(top, tpos, key, pos);
        }
        const int cm = __popcll(__ballot(top != KEY_INF));
        if (cm == 0) break;
        chunk_key[lane] = top;
        // K2P: this round's candidates that were in the previous round's list
        uint64_t pk = 0;
        if (np > 0) {
            const int32_t cid = top != KEY_INF ? key_id(top) : -1;
            bool in = false;
            for (int t = 0; t < np; ++t) in |= cid >= 0 && prev_lds[t] == cid;
            pk = __ballot(in);
        }
        {
            const int32_t cid = top != KEY_INF ? key_id(top) : -1;
            cn[lane] = cid >= 0 ? norms[cid] : 0.f;
            const int32_t kid = lane < nk ? key_id(kept_key[lane]) : -1;
            kn[lane] = kid >= 0 ? norms[kid] : 0.f;
        }
        const bool two = cm > 32;
        if (MIX) {
            kill_lds[lane] = 0;
            if (lane == 0) occk_lds = 0;
            __builtin_amdgcn_wave_barrier();
        }
        // mixed: the undecided pairs of the round's tiles (bit g of umask:
        // register g, row rowof(g), column `col`) are listed, then decided on
        // the chains in one pass per kind; kept: the rows are kept nodes
        // (occk_lds), else candidates (kill_lds)
        int rl_n = 0;  // entries listed (the same on every lane)
        // STG (rows of PM_STAGE_D dimensions or more): the chains read the FP32 rows the listed
        // pairs involve, each row once per flush: PM_CD dimensions of every
        // involved row at a time go through LDS (four lanes load a row's 64
        // bytes), and each lane adds them to its pair's chain (dims ascending,
        // one fma per dim: the canonical chain).  GIST-shaped prune 180 -> 125
        // ms.  Short rows: each lane streams its pair's two rows (the staging
        // costs more than it saves at 96 dimensions: 265 -> 271 ms).
        auto flush = [&](bool kept) {
            if (rl_n == 0) return;
            __builtin_amdgcn_wave_barrier();
            if (!STG) {
                for (int e = lane; e < rl_n; e += PG_WAVE) {
                    const int ent = rl[e], i = ent >> 6, j = ent & 63;
                    const uint64_t ki = kept ? kept_key[i] : chunk_key[i], kj = chunk_key[j];
                    const float b = dist_chain(X + (int64_t)key_id(ki) * ldx, X + (int64_t)key_id(kj) * ldx, d);
                    if (occludes(key_d2(ki), b, key_d2(kj), strict, at)) {
                        if (kept)
                            atomicOr(&occk_lds, 1ull << j);
                        else
                            atomicOr(&kill_lds[i], 1ull << j);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                rl_n = 0;
                return;
            }
            // involved rows: candidates (bit j of m0) and kept nodes (bit i of m1)
            uint64_t m0 = 0, m1 = 0;
            for (int e = lane; e < rl_n; e += PG_WAVE) {
                const int ent = rl[e], i = ent >> 6, j = ent & 63;
                m0 |= 1ull << j;
                if (kept)
                    m1 |= 1ull << i;
                else
                    m0 |= 1ull << i;
            }
#pragma unroll
            for (int o = 1; o < PG_WAVE; o <<= 1) {
                m0 |= shfl_xor64(m0, o);
                m1 |= shfl_xor64(m1, o);
            }
            const int n0 = __popcll(m0), nr = n0 + __popcll(m1);
            if ((m0 >> lane) & 1ull) srow[__popcll(m0 & lanemask_lt())] = key_id(chunk_key[lane]);
            if ((m1 >> lane) & 1ull) srow[n0 + __popcll(m1 & lanemask_lt())] = key_id(kept_key[lane]);
            __builtin_amdgcn_wave_barrier();
            float *fr = reinterpret_cast<float *>(rows);  // nr rows of PM_CS floats
            for (int b0 = 0; b0 < rl_n; b0 += PG_WAVE) {
                const int e = b0 + lane;
                const bool have = e < rl_n;
                int i = 0, j = 0, pi = 0, pj = 0;
                if (have) {
                    const int ent = rl[e];
                    i = ent >> 6, j = ent & 63;
                    pj = __popcll(m0 & ((1ull << j) - 1ull));
                    pi = kept ? n0 + __popcll(m1 & ((1ull << i) - 1ull)) : __popcll(m0 & ((1ull << i) - 1ull));
                }
                float b = 0.0f;
                for (int c0 = 0; c0 < d; c0 += PM_CD) {
                    const int dl = min(PM_CD, d - c0);
                    __builtin_amdgcn_wave_barrier();
                    for (int v = lane; v < nr * (PM_CD / 4); v += PG_WAVE) {
                        const int r = v / (PM_CD / 4), q = v % (PM_CD / 4);
                        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (4 * q < dl) x = *reinterpret_cast<const float4 *>(X + (int64_t)srow[r] * ldx + c0 + 4 * q);
                        *reinterpret_cast<float4 *>(fr + r * PM_CS + 4 * q) = x;
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (have) {
                        const float *a = fr + pi * PM_CS, *c = fr + pj * PM_CS;
                        for (int k = 0; k < dl; ++k) {
                            const float t = a[k] - c[k];
                            b = fmaf(t, t, b);
                        }
                    }
                }
                if (have) {
                    const uint64_t ki = kept ? kept_key[i] : chunk_key[i], kj = chunk_key[j];
                    if (occludes(key_d2(ki), b, key_d2(kj), strict, at)) {
                        if (kept)
                            atomicOr(&occk_lds, 1ull << j);
                        else
                            atomicOr(&kill_lds[i], 1ull << j);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            rl_n = 0;
        };
        auto settle = [&](uint32_t umask, auto rowof, int col, bool kept) {
            const int nu = __popc(umask);
            int ro = nu;
#pragma unroll
            for (int o = 1; o < PG_WAVE; o <<= 1) {
                const int t = __shfl_up(ro, o, PG_WAVE);
                if (lane >= o) ro += t;
            }
            const int rtot = __shfl(ro, PG_WAVE - 1, PG_WAVE);
            if (rtot == 0) return;
            if (rl_n + rtot > PM_LIST) flush(kept);
            ro += rl_n - nu;
            uint32_t mm = umask;
            while (mm) {
                const int g = __builtin_ctz(mm);
                mm &= mm - 1;
                rl[ro++] = (uint16_t)((rowof(g) << 6) | col);
            }
            rl_n += rtot;
        };
        // mixed: decide a pair from its estimate when the bound allows;
        // returns 1 (occludes), 0 (does not) or 2 (undecided)
        auto decide = [&](float a, float c, float ni, float nj, float gv) -> int {
            if (strict && !(a < c)) return 0;
            const float bh = fmaxf(fmaf(-2.0f, gv, ni + nj), 0.0f);
            const float e = pmix_e(pmx, ni, nj);
            const float acc = pmx.ga * (ni + nj + 2.0f * fabsf(gv));
            if (bh > pmix_hi(pmx, c, e, acc)) return 0;
            if (!at.on && bh < pmix_lo(pmx, c, e, acc)) return 1;
            return 2;
        };
        // rows [0, nrows) of this round (candidates, then kept nodes at 64..)
        // for dimensions [c0, c0 + dc).  Mixed: the next chunk loads into
        // registers while the MFMAs read the current one from LDS (exact
        // 16-bit data: loaded chunk by chunk, four waves per SIMD)
        pm_f16x8 pf[PM_PF];
        auto fetch = [&](int c0, int dc, int nrows) {
            const int vpr = dc / 8;
#pragma unroll
            for (int t = 0; t < PM_PF; ++t) {
                const int v = lane + t * PG_WAVE;
                pf[t] = pm_f16x8{};
                if (v < nrows * vpr) {
                    const int r = v / vpr, c = (v - r * vpr) * 8;
                    int32_t id = -1;
                    if (r < 64)
                        id = r < cm ? key_id(chunk_key[r]) : -1;
                    else
                        id = r - 64 < nk ? key_id(kept_key[r - 64]) : -1;
                    if (id >= 0) pf[t] = *reinterpret_cast<const pm_f16x8 *>(X16 + (int64_t)id * d16 + c0 + c);
                }
            }
        };
        auto put = [&](int dc, int nrows) {
            const int vpr = dc / 8;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < PM_PF; ++t) {
                const int v = lane + t * PG_WAVE;
                if (v < nrows * vpr) {
                    const int r = v / vpr, c = (v - r * vpr) * 8;
                    *reinterpret_cast<pm_f16x8 *>(rows + r * PM_RS + c) = pf[t];
                }
            }
            __syncthreads();
        };
        const _Float16 *r0 = rows + l32 * PM_RS + 8 * h;
        const _Float16 *r1 = rows + (32 + l32) * PM_RS + 8 * h;
        const _Float16 *rk = rows + (64 + l32) * PM_RS + 8 * h;
        // ---- occlusion among this round's candidates: kill sets per row
        uint64_t killv = 0, occk = 0;
        {
            pm_f32x16 t00, t01, t11;
#pragma unroll
            for (int g = 0; g < 16; ++g) t00[g] = t01[g] = t11[g] = 0.f;
            const int nrows = two ? 64 : 32;
            if (MIX) fetch(0, min(PM_DC, d16), nrows);
            for (int c0 = 0; c0 < d16; c0 += PM_DC) {
                const int dc = min(PM_DC, d16 - c0);
                if (!MIX) fetch(c0, dc, nrows);
                put(dc, nrows);
                if (MIX && c0 + PM_DC < d16) fetch(c0 + PM_DC, min(PM_DC, d16 - c0 - PM_DC), nrows);
                for (int k = 0; k < dc; k += 16) {
                    const pm_f16x8 a0 = *reinterpret_cast<const pm_f16x8 *>(r0 + k);
                    t00 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, a0, t00, 0, 0, 0);
                    if (two) {
                        const pm_f16x8 a1 = *reinterpret_cast<const pm_f16x8 *>(r1 + k);
                        t01 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, a1, t01, 0, 0, 0);
                        t11 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, a1, t11, 0, 0, 0);
                    }
                }
            }
            auto cand_tile = [&](const pm_f32x16 &t, int rb, int cb) {
                const int j = 32 * cb + l32;
                const float cj = key_d2(chunk_key[j]), nj = cn[j];
                uint32_t umask = 0;
#pragma unroll
                for (int g = 0; g < 16; ++g) {
                    const int i = 32 * rb + 8 * (g / 4) + 4 * h + (g % 4);
                    bool cnd = false;
                    if (i < cm && j < cm && i < j && ((pk >> i) & (pk >> j) & 1ull)) {
                        ++n_skip;
                    } else if (i < cm && j < cm && i < j) {
                        ++n_test;
                        if (MIX) {
                            const int dv = decide(key_d2(chunk_key[i]), cj, cn[i], nj, t[g]);
                            cnd = dv == 1;
                            umask |= (dv == 2 ? 1u : 0u) << g;
                        } else {
                            const float b = fmaxf(fmaf(-2.0f, t[g], cn[i] + nj), 0.0f);
                            cnd = occludes(key_d2(chunk_key[i]), b, cj, strict, at);
                        }
                    }
                    const uint64_t bm = __ballot(cnd);
                    const int i0 = 32 * rb + 8 * (g / 4) + (g % 4);
                    if (lane == i0) killv |= (bm & 0xFFFFFFFFull) << (32 * cb);
                    if (lane == i0 + 4) killv |= (bm >> 32) << (32 * cb);
                }
                if (MIX) settle(umask, [&](int g) { return 32 * rb + 8 * (g / 4) + 4 * h + (g % 4); }, j, false);
            };
            cand_tile(t00, 0, 0);
            if (two) {
                cand_tile(t01, 0, 1);
                cand_tile(t11, 1, 1);
            }
            if (MIX) {
                flush(false);
                killv |= kill_lds[lane];
            }
        }
        // ---- occlusion by the nodes kept in earlier rounds (second pass)
        if (nk > 0) {
            pm_f32x16 k0, k1;
#pragma unroll
            for (int g = 0; g < 16; ++g) k0[g] = k1[g] = 0.f;
            if (MIX) fetch(0, min(PM_DC, d16), PM_ROWS);
            for (int c0 = 0; c0 < d16; c0 += PM_DC) {
                const int dc = min(PM_DC, d16 - c0);
                if (!MIX) fetch(c0, dc, PM_ROWS);
                put(dc, PM_ROWS);
                if (MIX && c0 + PM_DC < d16) fetch(c0 + PM_DC, min(PM_DC, d16 - c0 - PM_DC), PM_ROWS);
                for (int k = 0; k < dc; k += 16) {
                    const pm_f16x8 ak = *reinterpret_cast<const pm_f16x8 *>(rk + k);
                    const pm_f16x8 a0 = *reinterpret_cast<const pm_f16x8 *>(r0 + k);
                    k0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ak, a0, k0, 0, 0, 0);
                    if (two) {
                        const pm_f16x8 a1 = *reinterpret_cast<const pm_f16x8 *>(r1 + k);
                        k1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ak, a1, k1, 0, 0, 0);
                    }
                }
            }
            auto kept_tile = [&](const pm_f32x16 &t, int cb) {
                const int j = 32 * cb + l32;
                const float cj = key_d2(chunk_key[j]), nj = cn[j];
                uint32_t umask = 0;
#pragma unroll
                for (int g = 0; g < 16; ++g) {
                    const int k = 8 * (g / 4) + 4 * h + (g % 4);
                    bool cnd = false;
                    if (k < nk && j < cm && ((kpk >> k) & (pk >> j) & 1ull)) {
                        ++n_skip;
                    } else if (k < nk && j < cm) {
                        ++n_test;
                        if (MIX) {
                            const int dv = decide(key_d2(kept_key[k]), cj, kn[k], nj, t[g]);
                            cnd = dv == 1;
                            umask |= (dv == 2 ? 1u : 0u) << g;
                        } else {
                            const float b = fmaxf(fmaf(-2.0f, t[g], kn[k] + nj), 0.0f);
                            cnd = occludes(key_d2(kept_key[k]), b, cj, strict, at);
                        }
                    }
                    const uint64_t bm = __ballot(cnd);
                    occk |= ((bm & 0xFFFFFFFFull) | (bm >> 32)) << (32 * cb);
                }
                if (MIX) settle(umask, [&](int g) { return 8 * (g / 4) + 4 * h + (g % 4); }, j, true);
            };
            kept_tile(k0, 0);
            if (two) kept_tile(k1, 1);
            if (MIX) {
                flush(true);
                occk |= occk_lds;
            }
        }
        // ---- greedy scan of Alg. 3 over this round's candidates
        uint64_t dead = occk;
        for (int j = 0; j < cm; ++j) {
            if ((dead >> j) & 1ull) continue;
            dead |= readlane64(killv, j);
            kpk |= ((pk >> j) & 1ull) << nk;
            if (lane == 0) kept_key[nk] = chunk_key[j];
            __builtin_amdgcn_wave_barrier();
            ++nk;
            if (nk == R) break;
        }
        if (nk == R || cm < PG_WAVE || m <= PG_WAVE) break;
        last = readlane64(top, PG_WAVE - 1);
        first = false;
    }
    __syncthreads();
    if (lane < R) {
        const bool have = lane < nk;
        const uint64_t k = have ? kept_key[lane] : KEY_INF;
        out_ids[u * R + lane] = have ? key_id(k) : -1;
        out_d2[u * R + lane] = have ? key_d2(k) : __int_as_float(0x7f800000);
    }
    if (lane == 0) out_deg[u] = nk;
    if (k2p) {
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) {
            n_skip += (unsigned long long)__shfl_xor((long long)n_skip, o, PG_WAVE);
            n_test += (unsigned long long)__shfl_xor((long long)n_test, o, PG_WAVE);
        }
        if (lane == 0) {
            atomicAdd(&k2p[0], n_skip);
            atomicAdd(&k2p[1], n_test);
        }
    }
}

// ---------------------------------------------------------------------------
// reverse edges (CSR of v -> u for every u -> v)
// ---------------------------------------------------------------------------
__global__ void k_count_indeg(const int32_t *__restrict__ g, const int32_t *__restrict__ deg,
                              int64_t n, int R, int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * R) return;
    const int64_t u = i / R;
    const int j = (int)(i % R);
    if (j < deg[u]) atomicAdd(&cnt[g[i]], 1);
}

// v gets u in its reverse list for every edge u -> v, with d2(v, u) = d2(u, v)
// (the canonical chain is symmetric bit for bit)
__global__ void k_scatter_rev(const int32_t *__restrict__ g, const float *__restrict__ gd,
                              const int32_t *__restrict__ deg, int64_t n, int R,
                              const int64_t *__restrict__ off, int32_t *__restrict__ cur,
                              int32_t *__restrict__ rev, float *__restrict__ rev_d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * R) return;
    const int64_t u = i / R;
    const int j = (int)(i % R);
    if (j < deg[u]) {
        const int32_t v = g[i];
        const int64_t at = off[v] + atomicAdd(&cur[v], 1);
        rev[at] = (int32_t)u;
        rev_d2[at] = gd[i];
    }
}

// ---------------------------------------------------------------------------
// entry point: centroid (double, fixed summation tree) and argmin (d2, id)
// ---------------------------------------------------------------------------
constexpr int CB_ROWS = 1024;

__global__ __launch_bounds__(256) void k_centroid_partial(const float *__restrict__ X, int64_t n,
                                                          int d, int64_t ldx,
                                                          double *__restrict__ part) {
    const int64_t r0 = (int64_t)blockIdx.x * CB_ROWS;
    const int64_t r1 = min((int64_t)n, r0 + CB_ROWS);
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s = __dadd_rn(s, (double)X[r * ldx + j]);
        part[(int64_t)blockIdx.x * d + j] = s;
    }
}

__global__ __launch_bounds__(256) void k_centroid_final(const double *__restrict__ part, int64_t nb,
                                                        int d, int64_t n, double *__restrict__ cen) {
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s = __dadd_rn(s, part[b * d + j]);
        cen[j] = __ddiv_rn(s, (double)n);
    }
}

struct DKey {
    double d2;
    int32_t id;
};
__device__ __forceinline__ bool dkey_less(const DKey &a, const DKey &b) {
    return a.d2 < b.d2 || (a.d2 == b.d2 && a.id < b.id);
}

// One row per lane, the squared distance to the centroid summed in FP64 in
// dimension order.  The rows reach the lanes through LDS, 16 dimensions at a
// time: four lanes load one row's 64 bytes, so a load instruction touches 16
// rows instead of 64.
constexpr int AC_DC = 16;
constexpr int AC_RS = AC_DC + 1;  // LDS row stride (floats): conflict-free column reads

__global__ __launch_bounds__(256) void k_argmin_center(const float *__restrict__ X, int64_t n, int d,
                                                       int64_t ldx, const double *__restrict__ cen,
                                                       double *__restrict__ pd, int32_t *__restrict__ pid) {
    __shared__ double sd[256];
    __shared__ int32_t si[256];
    __shared__ float rows[4][PG_WAVE * AC_RS];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * 256 + wv * PG_WAVE;  // this wave's first row
    const int64_t v = row0 + lane;
    float *tile = rows[wv];
    double s = 0.0;
    for (int c0 = 0; c0 < d; c0 += AC_DC) {
        const int dl = min(AC_DC, d - c0);
#pragma unroll
        for (int k = 0; k < AC_DC / 4; ++k) {
            const int f = lane + PG_WAVE * k, r = f / (AC_DC / 4), q = f % (AC_DC / 4);
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            if (row0 + r < n && 4 * q < dl)
                x = *reinterpret_cast<const float4 *>(X + (row0 + r) * ldx + c0 + 4 * q);
            float *t = tile + r * AC_RS + 4 * q;
            t[0] = x.x, t[1] = x.y, t[2] = x.z, t[3] = x.w;
        }
        __builtin_amdgcn_wave_barrier();
        for (int j = 0; j < dl; ++j) {
            const double t = __dsub_rn((double)tile[lane * AC_RS + j], cen[c0 + j]);
            s = __dadd_rn(s, __dmul_rn(t, t));
        }
        __builtin_amdgcn_wave_barrier();
    }
    DKey best{INFINITY, 0x7fffffff};
    if (v < n) best = {s, (int32_t)v};
    sd[threadIdx.x] = best.d2;
    si[threadIdx.x] = best.id;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            DKey a{sd[threadIdx.x], si[threadIdx.x]}, b{sd[threadIdx.x + o], si[threadIdx.x + o]};
            if (dkey_less(b, a)) {
                sd[threadIdx.x] = b.d2;
                si[threadIdx.x] = b.id;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pd[blockIdx.x] = sd[0];
        pid[blockIdx.x] = si[0];
    }
}

__global__ __launch_bounds__(256) void k_argmin_final(const double *__restrict__ pd,
                                                      const int32_t *__restrict__ pid, int64_t nb,
                                                      int32_t *__restrict__ ep) {
    __shared__ double sd[256];
    __shared__ int32_t si[256];
    DKey best{INFINITY, 0x7fffffff};
    for (int64_t b = threadIdx.x; b < nb; b += 256) {
        DKey c{pd[b], pid[b]};
        if (dkey_less(c, best)) best = c;
    }
    sd[threadIdx.x] = best.d2;
    si[threadIdx.x] = best.id;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            DKey a{sd[threadIdx.x], si[threadIdx.x]}, b{sd[threadIdx.x + o], si[threadIdx.x + o]};
            if (dkey_less(b, a)) {
                sd[threadIdx.x] = b.d2;
                si[threadIdx.x] = b.id;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *ep = si[0];
}

// ---------------------------------------------------------------------------
// connectivity
//
// The connect step visits the nodes the entry point does not reach in
// increasing id order.  Each one still unreached at its turn (a root) gets one
// edge p -> r from a node p reached by then, and everything r reaches counts
// as reached from then on.  Added edges only leave reached nodes, so which
// nodes are roots and when each node becomes reached depend on the pruned
// graph alone:
//   * an unreached v is a root iff no smaller unreached node reaches v;
//   * a node p counts as reached from the turn of the smallest root reaching
//     it, and that root is the smallest unreached node reaching p.
// The roots and every node's turn ("reach time") therefore come from a
// parallel min-ancestor label propagation, every root's sorted key list from
// parallel passes, and only the degree bookkeeping (a node at degree R
// accepts no edge) runs in root order, in one wave.
//
// Degrees only grow, so every node the step can still choose lies in the
// free set F of nodes below degree R when the step starts.  A root's key list
// holds its usable candidates (reached at its turn, below degree R at list
// time), sorted; a root with fewer than GLOBAL_TAIL_BELOW of them gets the
// nearest nodes of F reached at its turn appended, sorted.  The first entry
// still below degree R at the root's turn is then exactly the rule's choice:
// the nearest usable candidate if one is left, else the nearest usable node
// of the whole graph, unless every listed node has filled up, in which case
// an exact scan over F decides.
// ---------------------------------------------------------------------------
struct ConnState {
    int32_t fcount[2];
    int32_t changed;    // label propagation: some label dropped in this round
    int32_t idx;        // next root (global index) for the matching wave
    int32_t stop_root;  // >= 0: root waiting for the exact scan over F; -1: batch done; -2: overflow
    int32_t stop_turn;  //       and its 1-based turn
    int32_t n_empty;    // roots of the current batch queued for the scan over F
    int32_t overflow;
    unsigned long long nearest;
};

// roots handled per batch of key lists
constexpr int32_t CONNECT_BATCH = 16384;
// roots with fewer usable candidates than this get the nearest free nodes
// appended to their key lists
constexpr int GLOBAL_TAIL_BELOW = 1;
// roots per block of the scan over F (four per wave)
constexpr int GQ = 16;
// free nodes per tile of that scan (one per thread)
constexpr int TG_TILE = 256;
// the scan over F aims at this many workgroups, splitting F into chunks of
// at least TG_MIN_CHUNK nodes when few roots are queued
constexpr int TG_BLOCKS = 2048;
constexpr int TG_MIN_CHUNK = 2048;

// loads that must see stores and atomics made earlier in the same kernel
__device__ __forceinline__ int32_t ld_fresh(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_flag_unreached(const int32_t *__restrict__ visited, int64_t n,
                                 int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = visited[i] == 0;
}

__global__ void k_scatter_unreached(const int32_t *__restrict__ visited, int64_t n,
                                    const int64_t *__restrict__ off, int32_t *__restrict__ U) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && visited[i] == 0) U[off[i]] = (int32_t)i;
}

__global__ void k_flag_free(const int32_t *__restrict__ deg, int64_t n, int R, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = deg[i] < R;
}

__global__ void k_scatter_free(const int32_t *__restrict__ deg, int64_t n, int R,
                               const int64_t *__restrict__ off, int32_t *__restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && deg[i] < R) F[off[i]] = (int32_t)i;
}

__global__ void k_label_init(const int32_t *__restrict__ U, int32_t nu, int32_t *__restrict__ lab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) lab[U[i]] = U[i];
}

// One round of min-ancestor labels over the unreached nodes U: every edge
// u -> v inside U lowers lab[v] to lab[u], and lab[u] drops to lab[lab[u]]
// (an ancestor of an ancestor).  Labels stay ancestors and only decrease;
// a round without a change leaves each node its smallest ancestor.
__global__ __launch_bounds__(256) void k_label_round(const int32_t *__restrict__ g,
                                                     const int32_t *__restrict__ deg, int R, int64_t n,
                                                     const int32_t *__restrict__ visited,
                                                     const int32_t *__restrict__ U, int32_t nu,
                                                     int32_t *lab, int32_t *changed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nu * R) return;
    const int32_t u = U[t / R];
    const int j = (int)(t % R);
    bool ch = false;
    if (j == 0) {
        const int32_t a = lab[u];
        const int32_t b = lab[a];
        if (b < a && atomicMin(&lab[u], b) > b) ch = true;
    }
    if (j < min(deg[u], R)) {
        const int32_t v = g[(int64_t)u * R + j];
        if (v >= 0 && v < n && !visited[v]) {
            const int32_t l = lab[u];
            if (l < lab[v] && atomicMin(&lab[v], l) > l) ch = true;
        }
    }
    if (ch) *changed = 1;
}

__global__ void k_flag_roots(const int32_t *__restrict__ U, int32_t nu, const int32_t *__restrict__ lab,
                             int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) flag[i] = lab[U[i]] == U[i];
}

// roots in increasing id order; tt[root] = its 1-based turn
__global__ void k_scatter_roots(const int32_t *__restrict__ U, int32_t nu, const int32_t *__restrict__ lab,
                                const int64_t *__restrict__ pos, int32_t *__restrict__ roots,
                                int32_t *__restrict__ tt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nu) return;
    const int32_t v = U[i];
    if (lab[v] == v) {
        roots[pos[i]] = v;
        tt[v] = (int32_t)pos[i] + 1;
    }
}

// tt[p] = turn from which p counts as reached (0: reached from the entry
// point).  Only root entries are read, and those do not change here.
__global__ void k_reach_time(const int32_t *__restrict__ U, int32_t nu, const int32_t *__restrict__ lab,
                             int32_t *tt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nu) return;
    const int32_t v = U[i], a = lab[v];
    if (a != v) tt[v] = tt[a];
}

// Sorted keys (d2, p) of the candidates of roots [b0, b1) that count as
// reached at the root's turn and are below degree R now (degrees only grow,
// so a node dropped here could not be chosen later).  Roots with fewer than
// GLOBAL_TAIL_BELOW such keys are queued, with their key count, for the scan
// over F.
__global__ __launch_bounds__(256) void k_root_lists(const float *__restrict__ X, int64_t ldx, int d,
                                                    int64_t n, int R, const int32_t *__restrict__ cand,
                                                    int C, const int32_t *__restrict__ roots, int32_t b0,
                                                    int32_t b1, const int32_t *__restrict__ tt,
                                                    const int32_t *__restrict__ deg,
                                                    uint64_t *__restrict__ keys, int32_t *__restrict__ queue,
                                                    int32_t *__restrict__ qvalid, ConnState *cs) {
    const int lane = lane_id();
    const int32_t b = b0 + (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (b >= b1) return;
    const int32_t r = roots[b];
    uint64_t key = KEY_INF;
    if (lane < C) {
        const int32_t p = cand[(int64_t)r * C + lane];
        if (p >= 0 && p < n && p != r && tt[p] <= b && deg[p] < R)
            key = pack_key(dist_chain(X + (int64_t)r * ldx, X + (int64_t)p * ldx, d), p);
    }
    int pay = 0;
    wave_sort(key, pay);
    if (lane < C) keys[(int64_t)(b - b0) * C + lane] = key;
    const int nv = __popcll(__ballot(key != KEY_INF));
    if (lane == 0 && nv < GLOBAL_TAIL_BELOW && nv < C) {
        const int32_t q = atomicAdd(&cs->n_empty, 1);
        queue[q] = b;
        qvalid[q] = nv;
    }
}

// Running C smallest keys of one root over a stream of 64-key slices (one
// key per lane, KEY_INF = none).  `top` is ascending, one key per lane.  Keys
// below the list's C-th are gathered in `pend` (lanes < np) and sorted into
// the list once 64 are waiting, so a slice costs a compare and a ballot
// unless it holds such keys.  The threshold lags the pending keys, which only
// lets more keys through: the result is the C smallest keys of the stream.
__device__ __forceinline__ void topacc_flush(uint64_t &top, uint64_t &pend, int &np) {
    if (np == 0) return;
    int pp = 0, pt = 0;
    wave_sort(pend, pp);
    wave_merge_lowest(top, pt, pend, pp);
    pend = KEY_INF;
    np = 0;
}

__device__ __forceinline__ void topacc_add(uint64_t &top, uint64_t &pend, int &np, uint64_t k, int C) {
    const int lane = lane_id();
    bool pass = k < readlane64(top, C - 1);
    uint64_t m = __ballot(pass);
    if (m == 0) return;
    if (np + __popcll(m) > PG_WAVE) {
        topacc_flush(top, pend, np);
        pass = k < readlane64(top, C - 1);
        m = __ballot(pass);
        if (m == 0) return;
    }
    const int cnt = __popcll(m);
    // a permutation of the lanes: passing keys to lanes np .. np + cnt - 1 in
    // lane order, the others to the remaining lanes
    const int below = __popcll(m & lanemask_lt());
    const int rest = lane - below;
    const int dst = pass ? np + below : (rest < np ? rest : rest + cnt);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)(k >> 32));
    if (lane >= np && lane < np + cnt) pend = ((uint64_t)hi << 32) | lo;
    np += cnt;
}

// Nearest nodes of F for the queued roots.  Block (x, y) scans chunk x of F
// for queued roots [GQ y, GQ y + GQ): every thread takes one free node per
// tile and computes the canonical distance chains to those roots; a node
// counts if it is reached at the root's turn and below degree R now.  Each
// wave keeps, for four of the roots, the C smallest keys seen so far as one
// ascending key per lane and merges a 64-key slice of the tile into it only
// when some key of the slice beats the current C-th.  With one chunk the
// result goes straight behind the root's candidate keys; otherwise into the
// per-chunk lists `part`, which k_topg_merge combines.
__global__ __launch_bounds__(256) void k_global_topg(const float *__restrict__ X, int64_t ldx, int d, int R,
                                                     const int32_t *__restrict__ roots,
                                                     const int32_t *__restrict__ tt,
                                                     const int32_t *__restrict__ deg,
                                                     const int32_t *__restrict__ F, int32_t nf, int32_t chunk,
                                                     int32_t nchunk, const int32_t *__restrict__ queue,
                                                     const int32_t *__restrict__ qvalid, int32_t nqueued,
                                                     int32_t b0, int C, uint64_t *__restrict__ keys,
                                                     uint64_t *__restrict__ part) {
    __shared__ uint64_t kb[GQ][TG_TILE];
    constexpr int PER_WAVE = GQ / 4;
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    const int q0 = (int)blockIdx.y * GQ;
    const int nq = min(GQ, nqueued - q0);
    int32_t rq[GQ], bq[GQ];
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
        bq[q] = q < nq ? queue[q0 + q] : -1;
        rq[q] = roots[q < nq ? bq[q] : queue[q0]];
    }
    uint64_t top[PER_WAVE], pend[PER_WAVE];
    int np[PER_WAVE];
#pragma unroll
    for (int s = 0; s < PER_WAVE; ++s) {
        top[s] = KEY_INF;
        pend[s] = KEY_INF;
        np[s] = 0;
    }
    const int32_t f0 = (int32_t)blockIdx.x * chunk, f1 = min(nf, f0 + chunk);
    for (int32_t t = f0; t < f1; t += TG_TILE) {
        const int32_t i = t + (int32_t)threadIdx.x;
        const int32_t p = i < f1 ? F[i] : F[f0];
        float acc[GQ];
#pragma unroll
        for (int q = 0; q < GQ; ++q) acc[q] = 0.f;
        const float *xp = X + (int64_t)p * ldx;
        for (int k = 0; k < d; k += 4) {
            const float4 x = *reinterpret_cast<const float4 *>(xp + k);
#pragma unroll
            for (int q = 0; q < GQ; ++q) {
                const float4 y = *reinterpret_cast<const float4 *>(X + (int64_t)rq[q] * ldx + k);
                float e;
                e = x.x - y.x;
                acc[q] = fmaf(e, e, acc[q]);
                e = x.y - y.y;
                acc[q] = fmaf(e, e, acc[q]);
                e = x.z - y.z;
                acc[q] = fmaf(e, e, acc[q]);
                e = x.w - y.w;
                acc[q] = fmaf(e, e, acc[q]);
            }
        }
        const int32_t tp = (i < f1 && deg[p] < R) ? tt[p] : INT32_MAX;
#pragma unroll
        for (int q = 0; q < GQ; ++q) kb[q][threadIdx.x] = tp <= bq[q] ? pack_key(acc[q], p) : KEY_INF;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PER_WAVE; ++s) {
            const int q = wv * PER_WAVE + s;
#pragma unroll
            for (int c = 0; c < TG_TILE; c += PG_WAVE) topacc_add(top[s], pend[s], np[s], kb[q][c + lane], C);
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < PER_WAVE; ++s) {
        topacc_flush(top[s], pend[s], np[s]);
        const int q = wv * PER_WAVE + s;
        if (q >= nq) continue;
        if (nchunk == 1) {
            const int nv = qvalid[q0 + q];
            if (lane < C - nv) keys[(int64_t)(bq[q] - b0) * C + nv + lane] = top[s];
        } else if (lane < C) {
            part[((int64_t)(q0 + q) * nchunk + blockIdx.x) * C + lane] = top[s];
        }
    }
}

// The same scan on data that pass the exactness test of the 16-bit path:
// block (x, y) takes queued roots [GQM y, GQM y + GQM) and chunk x of F.  Each
// wave forms 32 x 32 Gram tiles (the block's roots x 32 free nodes) with the
// roots' fragments held in registers; d2 = n_r + n_p - 2 r.p equals the
// canonical chain on such data.  A step's four tiles go through LDS to the
// waves that keep the running lists, GQM / 4 roots each.
constexpr int GQM = 32;
template <int KS>  // 16-dimension k-steps held in registers: d16 <= 16 KS
__global__ __launch_bounds__(256) void k_global_topg_mfma(
    const _Float16 *__restrict__ x16, int d16, const float *__restrict__ norms, int R,
    const int32_t *__restrict__ roots, const int32_t *__restrict__ tt, const int32_t *__restrict__ deg,
    const int32_t *__restrict__ F, int32_t nf, int32_t chunk, int32_t nchunk, const int32_t *__restrict__ queue,
    const int32_t *__restrict__ qvalid, int32_t nqueued, int32_t b0, int C, uint64_t *__restrict__ keys,
    uint64_t *__restrict__ part) {
    constexpr int OWN = GQM / 4;
    __shared__ uint64_t kb[GQM][4 * 32];
    __shared__ float rn[GQM];
    __shared__ int32_t rturn[GQM];
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6), h = lane >> 5, l32 = lane & 31;
    const int q0 = (int)blockIdx.y * GQM;
    const int nq = min(GQM, nqueued - q0);
    if (threadIdx.x < GQM) {
        const int q = (int)threadIdx.x;
        const int32_t b = queue[q0 + min(q, nq - 1)];
        rturn[q] = q < nq ? b : -1;
        rn[q] = norms[roots[b]];
    }
    // A operand: root of row l32 (rows past nq repeat the last root, masked below)
    pm_f16x8 A[KS];
    {
        const int32_t r = roots[queue[q0 + min(l32, nq - 1)]];
        const _Float16 *pa = x16 + (int64_t)r * d16 + 8 * h;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            A[s] = 16 * s < d16 ? *reinterpret_cast<const pm_f16x8 *>(pa + 16 * s) : pm_f16x8{};
    }
    uint64_t top[OWN], pend[OWN];
    int np[OWN];
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        top[o] = KEY_INF;
        pend[o] = KEY_INF;
        np[o] = 0;
    }
    __syncthreads();
    const int32_t f0 = (int32_t)blockIdx.x * chunk, f1 = min(nf, f0 + chunk);
    for (int32_t t = f0; t < f1; t += 4 * 32) {
        const int32_t i = t + wv * 32 + l32;
        const bool in = i < f1;
        const int32_t p = in ? F[i] : F[f0];
        const _Float16 *pb = x16 + (int64_t)p * d16 + 8 * h;
        pm_f16x8 B[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
            B[s] = 16 * s < d16 ? *reinterpret_cast<const pm_f16x8 *>(pb + 16 * s) : pm_f16x8{};
        pm_f32x16 acc;
#pragma unroll
        for (int g = 0; g < 16; ++g) acc[g] = 0.f;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (16 * s < d16) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[s], B[s], acc, 0, 0, 0);
        const float npn = norms[p];
        const int32_t tp = (in && deg[p] < R) ? tt[p] : INT32_MAX;
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const int row = 8 * (g / 4) + 4 * h + (g % 4);
            const float d2 = fmaxf(fmaf(-2.0f, acc[g], rn[row] + npn), 0.0f);
            kb[row][wv * 32 + l32] = tp <= rturn[row] ? pack_key(d2, p) : KEY_INF;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int q = wv * OWN + o;
            topacc_add(top[o], pend[o], np[o], kb[q][lane], C);
            topacc_add(top[o], pend[o], np[o], kb[q][PG_WAVE + lane], C);
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        topacc_flush(top[o], pend[o], np[o]);
        const int q = wv * OWN + o;
        if (q >= nq) continue;
        if (nchunk == 1) {
            const int nv = qvalid[q0 + q];
            if (lane < C - nv) keys[(int64_t)(rturn[q] - b0) * C + nv + lane] = top[o];
        } else if (lane < C) {
            part[((int64_t)(q0 + q) * nchunk + blockIdx.x) * C + lane] = top[o];
        }
    }
}

// One wave per queued root: the C smallest keys over its per-chunk lists
// (each ascending), written behind the root's candidate keys.
__global__ __launch_bounds__(256) void k_topg_merge(const uint64_t *__restrict__ part, int32_t nchunk,
                                                    const int32_t *__restrict__ queue,
                                                    const int32_t *__restrict__ qvalid, int32_t nqueued,
                                                    int32_t b0, int C, uint64_t *__restrict__ keys) {
    const int lane = lane_id();
    const int32_t qi = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (qi >= nqueued) return;
    uint64_t top = KEY_INF;
    for (int32_t c = 0; c < nchunk; ++c) {
        const uint64_t k = lane < C ? part[((int64_t)qi * nchunk + c) * C + lane] : KEY_INF;
        if (__ballot(k < readlane64(top, C - 1)) == 0) continue;
        int pt = 0;
        wave_merge_lowest(top, pt, k, 0);
    }
    const int nv = qvalid[qi];
    if (lane < C - nv) keys[(int64_t)(queue[qi] - b0) * C + nv + lane] = top;
}

// Roots in turn order: each takes the first key of its list whose node is
// still below degree R and appends the edge p -> r there.  Windows of 64
// roots, one per lane: every lane finds the first listed node below R in the
// degrees at the window's start, and counts the earlier lanes that took the
// same node.  Up to the first lane whose node that count fills (or whose list
// has no such node), every lane's choice is the rule's own: the nodes before
// it in its list were already at R, and its node still has room after the
// earlier picks.  That prefix is written at once; the root after it then
// decides with the degrees it left, over its whole list.  A root whose list
// has no node below R stops the wave (stop_root >= 0, nearest reset); the
// host then runs the exact scan over F for it and restarts the wave.  A wave
// started after a failed scan reports the overflow (stop_root = -2).
constexpr int MATCH_PROBE = 8;  // listed keys a lane examines per round
constexpr int STOP_CHAIN = 8;   // stops resolved per host synchronisation

__global__ __launch_bounds__(64) void k_match(const int32_t *__restrict__ roots, int32_t b0, int32_t b1,
                                              const uint64_t *__restrict__ keys, int C, int R, int32_t *g,
                                              float *gd, int32_t *deg, ConnState *cs) {
    const int lane = lane_id();
    if (cs->overflow) {
        if (lane == 0) cs->stop_root = -2;
        return;
    }
    int32_t b = cs->idx;
    while (b < b1) {
        const int32_t bi = b + lane;
        const bool act = bi < b1;
        int32_t p = -1, dp = 0;
        float d2 = 0.f;
        bool done = !act;
        for (int j0 = 0; j0 < C && __ballot(!done) != 0; j0 += MATCH_PROBE) {
            if (!done) {
                uint64_t kq[MATCH_PROBE];
                int32_t dq[MATCH_PROBE];
#pragma unroll
                for (int t = 0; t < MATCH_PROBE; ++t)
                    kq[t] = j0 + t < C ? keys[(int64_t)(bi - b0) * C + j0 + t] : KEY_INF;
#pragma unroll
                for (int t = 0; t < MATCH_PROBE; ++t) dq[t] = kq[t] != KEY_INF ? ld_fresh(&deg[key_id(kq[t])]) : R;
#pragma unroll
                for (int t = 0; t < MATCH_PROBE; ++t) {
                    if (!done && dq[t] < R) {
                        p = key_id(kq[t]);
                        d2 = key_d2(kq[t]);
                        dp = dq[t];
                        done = true;
                    }
                }
            }
        }
        // earlier lanes of the window that took the same node
        int cnt = 0;
#pragma unroll 8
        for (int j = 0; j < PG_WAVE; ++j) {
            const int32_t pj = __builtin_amdgcn_readlane(p, j);
            cnt += (j < lane && pj == p) ? 1 : 0;
        }
        const bool ok = !act || (p >= 0 && dp + cnt < R);
        const uint64_t bad = __ballot(!ok);
        const int ncommit = bad != 0 ? __ffsll((long long)bad) - 1 : min(PG_WAVE, b1 - b);
        if (lane < ncommit) {
            const int slot = dp + cnt;
            g[(int64_t)p * R + slot] = roots[bi];
            gd[(int64_t)p * R + slot] = d2;
            atomicAdd(&deg[p], 1);
        }
        __threadfence();
        b += ncommit;
        if (bad == 0) continue;
        // root b decides over its whole list with the degrees after the prefix
        const uint64_t kk = lane < C ? keys[(int64_t)(b - b0) * C + lane] : KEY_INF;
        const int32_t pk = kk != KEY_INF ? key_id(kk) : -1;
        const int cur = pk >= 0 ? ld_fresh(&deg[pk]) : R;
        const uint64_t okm = __ballot(pk >= 0 && cur < R);
        if (okm == 0) {
            if (lane == 0) {
                cs->idx = b;
                cs->stop_root = roots[b];
                cs->stop_turn = b + 1;
                cs->nearest = KEY_INF;
            }
            return;
        }
        const int f = __ffsll((long long)okm) - 1;  // wave-uniform
        const int32_t pp = __builtin_amdgcn_readlane(pk, f);
        const int slot = __builtin_amdgcn_readlane(cur, f);
        const uint64_t key = readlane64(kk, f);
        if (lane == 0) {
            g[(int64_t)pp * R + slot] = roots[b];
            gd[(int64_t)pp * R + slot] = key_d2(key);
            atomicAdd(&deg[pp], 1);
        }
        __threadfence();
        b += 1;
    }
    if (lane == 0) {
        cs->idx = b1;
        cs->stop_root = -1;
    }
}

__global__ void k_bfs_seed(int32_t *__restrict__ visited, int32_t *__restrict__ frontier,
                           ConnState *__restrict__ cs, const int32_t *__restrict__ src) {
    const int32_t r = *src;
    visited[r] = 1;
    frontier[0] = r;
    cs->fcount[0] = 1;
    cs->fcount[1] = 0;
}

__global__ __launch_bounds__(256) void k_bfs_step(const int32_t *__restrict__ g, int64_t n, int R,
                                                  const int32_t *__restrict__ deg,
                                                  int32_t *__restrict__ visited,
                                                  const int32_t *__restrict__ fin, int32_t nin,
                                                  int32_t *__restrict__ fout, int32_t *__restrict__ nout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool push = false;
    int32_t y = -1;
    if (i < (int64_t)nin * R) {
        const int32_t x = fin[i / R];
        const int j = (int)(i % R);
        if (j < deg[x] && j < R) {
            y = g[(int64_t)x * R + j];
            if (y >= 0 && y < n && atomicExch(&visited[y], 1) == 0) push = true;
        }
    }
    const uint64_t m = __ballot(push);
    if (m == 0) return;
    int base = 0;
    const int leader = __ffsll((long long)m) - 1;
    if (lane_id() == leader) base = atomicAdd(nout, __popcll(m));
    base = __shfl(base, leader, PG_WAVE);
    if (push) fout[base + __popcll(m & lanemask_lt())] = y;
}

// exact scan for the stopped root: nearest node of F reached at its turn and
// below degree R now (nothing when the wave has no stopped root)
__global__ __launch_bounds__(256) void k_nearest_at(const float *__restrict__ X, int64_t ldx, int d, int R,
                                                    const int32_t *__restrict__ F, int32_t nf,
                                                    const int32_t *__restrict__ tt,
                                                    const int32_t *__restrict__ deg,
                                                    ConnState *__restrict__ cs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t r = cs->stop_root, turn = cs->stop_turn;
    if (r < 0) return;  // the same for every thread of the grid
    uint64_t key = KEY_INF;
    if (i < nf) {
        const int32_t p = F[i];
        if (tt[p] < turn && deg[p] < R)
            key = pack_key(dist_chain(X + (int64_t)r * ldx, X + (int64_t)p * ldx, d), p);
    }
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) {
        const uint64_t t = shfl_xor64(key, o);
        key = t < key ? t : key;
    }
    if (lane_id() == 0 && key != KEY_INF) atomicMin(&cs->nearest, (unsigned long long)key);
}

__global__ void k_attach(int32_t *__restrict__ g, float *__restrict__ gd, int32_t *__restrict__ deg,
                         int R, ConnState *__restrict__ cs) {
    const int32_t r = cs->stop_root;
    if (r < 0) return;  // no stopped root
    const unsigned long long key = cs->nearest;
    if (key == KEY_INF) {
        cs->overflow = 1;
        return;
    }
    const int32_t p = key_id(key);
    const int j = deg[p];
    g[(int64_t)p * R + j] = r;
    gd[(int64_t)p * R + j] = key_d2(key);
    deg[p] = j + 1;
    cs->idx = cs->stop_turn;  // the next root
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct PruneLayout {
    size_t p_ids, p_d2, p_deg, cnt, off, rev, rev_d2, visited, fa, fb, cs, keys, empty, qvalid, free_ids,
        part, cpart, cen, apd, api, scan_tmp, x16, norms, exflags, total;
    int d16;
    int64_t ncb, nab;
    int64_t part_keys;  // keys the per-chunk lists of the scan over F can hold
};

static PruneLayout prune_layout(const pg_prune_params *p, int64_t n, int d) {
    PruneLayout L{};
    const int64_t R = p->R;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += pg_align(bytes);
        return at;
    };
    L.ncb = (n + CB_ROWS - 1) / CB_ROWS;
    L.nab = (n + 255) / 256;
    L.p_ids = take(sizeof(int32_t) * n * R);
    L.p_d2 = take(sizeof(float) * n * R);
    L.p_deg = take(sizeof(int32_t) * n);
    L.cnt = take(sizeof(int32_t) * n);
    L.off = take(sizeof(int64_t) * (n + 1));
    L.rev = take(sizeof(int32_t) * n * R);
    L.rev_d2 = take(sizeof(float) * n * R);
    L.visited = take(sizeof(int32_t) * n);
    L.fa = take(sizeof(int32_t) * n);
    L.fb = take(sizeof(int32_t) * n);
    L.cs = take(sizeof(ConnState));
    const int64_t nb = std::min<int64_t>(n, CONNECT_BATCH);
    L.keys = take(sizeof(uint64_t) * 64 * nb);
    L.empty = take(sizeof(int32_t) * nb);
    L.qvalid = take(sizeof(int32_t) * nb);
    L.free_ids = take(sizeof(int32_t) * n);
    // per-chunk lists of the scan over F: only written when F is split, which
    // keeps chunks x root groups below 2 TG_BLOCKS
    const int64_t groups = (nb + GQ - 1) / GQ;
    const int64_t part_blocks = std::min<int64_t>(2 * TG_BLOCKS, groups * ((n + TG_MIN_CHUNK - 1) / TG_MIN_CHUNK));
    L.part_keys = 64 * GQ * part_blocks;
    L.part = take(sizeof(uint64_t) * L.part_keys);
    L.cpart = take(sizeof(double) * L.ncb * d);
    L.cen = take(sizeof(double) * d);
    L.apd = take(sizeof(double) * L.nab);
    L.api = take(sizeof(int32_t) * L.nab);
    L.scan_tmp = take(scan_tmp_bytes(n + 1));
    L.d16 = (d + 15) / 16 * 16;
    L.x16 = take(sizeof(_Float16) * n * L.d16);
    L.norms = take(sizeof(float) * n);
    L.exflags = take(sizeof(unsigned int) * 4);
    L.total = o;
    return L;
}

// Workspace is sized for d up to this many dimensions (centroid partial sums).
constexpr int PRUNE_MAX_D = 4096;

static pg_status check_prune(const pg_prune_params *p, int64_t n, int32_t C) {
    if (!p) {
        set_error("pg_prune: params is NULL");
        return PG_EINVAL;
    }
    if (n < 1 || n >= (int64_t)1 << 31) {
        set_error("pg_prune: n=%lld out of range", (long long)n);
        return PG_EINVAL;
    }
    if (C < 1 || C > 64) {
        set_error("pg_prune: C=%d must be in [1, 64]", C);
        return PG_EINVAL;
    }
    if (p->R < 1 || p->R > 64) {
        set_error("pg_prune: R=%d must be in [1, 64]", p->R);
        return PG_EINVAL;
    }
    if (!(p->stages & PG_STAGE_PRUNE) || (p->stages & ~7u)) {
        set_error("pg_prune: stages=%u must include PG_STAGE_PRUNE and only known bits", p->stages);
        return PG_EINVAL;
    }
    if (p->pair_d2 && p->stages != PG_STAGE_PRUNE) {
        set_error("pg_prune: the pair_d2 table only serves the PRUNE stage alone");
        return PG_EINVAL;
    }
    if (p->k2p_prev_ids && (!p->k2p_prev_deg || p->k2p_prev_R < 1 || p->k2p_prev_R > 64)) {
        set_error("pg_prune: k2p_prev_ids needs k2p_prev_deg and 1 <= k2p_prev_R <= 64");
        return PG_EINVAL;
    }
    if ((p->prune_ids_out != nullptr) != (p->prune_deg_out != nullptr)) {
        set_error("pg_prune: prune_ids_out and prune_deg_out go together");
        return PG_EINVAL;
    }
    if (p->precision != PG_FP32 && p->precision != PG_FP32_VALU) {
        set_error("pg_prune: precision=%d must be PG_FP32 or PG_FP32_VALU", p->precision);
        return PG_EINVAL;
    }
    if (!(p->alpha_deg >= 0.0f && p->alpha_deg <= 180.0f)) {
        set_error("pg_prune: alpha_deg=%g must be in [0, 180]", (double)p->alpha_deg);
        return PG_EINVAL;
    }
    return PG_OK;
}

// Level-synchronous BFS over out-edges from the node *src (device).
static pg_status bfs_from(pg_ctx *ctx, const int32_t *g, int64_t n, int R, const int32_t *deg, int32_t *visited,
                          int32_t *fa, int32_t *fb, ConnState *cs, const int32_t *src) {
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_bfs_seed, dim3(1), dim3(1), 0, st, visited, fa, cs, src);
    PG_HIP(hipGetLastError());
    int32_t nin = 1;
    int32_t *fin = fa, *fout = fb;
    int parity = 0;
    while (nin > 0) {
        PG_HIP(hipMemsetAsync(&cs->fcount[parity ^ 1], 0, sizeof(int32_t), st));
        const int64_t threads = (int64_t)nin * R;
        hipLaunchKernelGGL(k_bfs_step, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, g, n, R,
                           deg, visited, fin, nin, fout, &cs->fcount[parity ^ 1]);
        PG_HIP(hipGetLastError());
        PG_HIP(hipMemcpyAsync(&nin, &cs->fcount[parity ^ 1], sizeof(int32_t), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        fin = fout;
        fout = (fout == fb) ? fa : fb;
        parity ^= 1;
    }
    return PG_OK;
}

template <typename T>
static pg_status read_back(pg_ctx *ctx, T *host, const T *dev) {
    PG_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
    PG_HIP(hipStreamSynchronize(ctx->stream));
    return PG_OK;
}

template <typename T>
static pg_status write_to(pg_ctx *ctx, T *dev, T value) {
    PG_HIP(hipMemcpyAsync(dev, &value, sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    PG_HIP(hipStreamSynchronize(ctx->stream));
    return PG_OK;
}

// The connect step (see the comment above ConnState).
// exact16: x16 and the norms hold the exact 16-bit copy (see k_prune_prep),
// so the scan over F may take its distances from MFMA Gram tiles.
static pg_status connect(pg_ctx *ctx, const PruneLayout &L, char *w, const float *X, int64_t n, int d,
                         int64_t ldx, const int32_t *cand, int C, int R, int32_t *g_ids, float *g_d2,
                         int32_t *g_deg, const int32_t *ep, int32_t *roots, int32_t *n_roots, bool exact16) {
    hipStream_t st = ctx->stream;
    int32_t *cnt = (int32_t *)(w + L.cnt), *U = (int32_t *)(w + L.rev), *visited = (int32_t *)(w + L.visited),
            *fa = (int32_t *)(w + L.fa), *fb = (int32_t *)(w + L.fb), *queue = (int32_t *)(w + L.empty),
            *qvalid = (int32_t *)(w + L.qvalid), *F = (int32_t *)(w + L.free_ids);
    int64_t *off = (int64_t *)(w + L.off);
    uint64_t *keys = (uint64_t *)(w + L.keys), *part = (uint64_t *)(w + L.part);
    ConnState *cs = (ConnState *)(w + L.cs);
    int32_t *rts = roots ? roots : (int32_t *)(w + L.p_ids);
    const unsigned nbn = (unsigned)((n + 255) / 256);

    PG_HIP(hipMemsetAsync(visited, 0, sizeof(int32_t) * n, st));
    PG_HIP(hipMemsetAsync(cs, 0, sizeof(ConnState), st));
    PG_TRY(bfs_from(ctx, g_ids, n, R, g_deg, visited, fa, fb, cs, ep));
    // unreached ids in increasing order
    hipLaunchKernelGGL(k_flag_unreached, dim3(nbn), dim3(256), 0, st, visited, n, cnt);
    PG_TRY(scan_exclusive(ctx, cnt, off, n, w + L.scan_tmp));
    hipLaunchKernelGGL(k_scatter_unreached, dim3(nbn), dim3(256), 0, st, visited, n, off, U);
    PG_HIP(hipGetLastError());
    int64_t nu64 = 0;
    PG_TRY(read_back(ctx, &nu64, off + n));
    const int32_t nu = (int32_t)nu64;
    if (nu == 0) return PG_OK;

    // min-ancestor labels (fa), roots and reach turns (fb)
    int32_t *lab = fa, *tt = fb;
    const unsigned nbu = (unsigned)((nu + 255) / 256);
    hipLaunchKernelGGL(k_label_init, dim3(nbu), dim3(256), 0, st, U, nu, lab);
    PG_HIP(hipGetLastError());
    for (;;) {
        PG_HIP(hipMemsetAsync(&cs->changed, 0, sizeof(int32_t), st));
        const int64_t threads = (int64_t)nu * R;
        hipLaunchKernelGGL(k_label_round, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, g_ids, g_deg,
                           R, n, visited, U, nu, lab, &cs->changed);
        PG_HIP(hipGetLastError());
        int32_t ch = 0;
        PG_TRY(read_back(ctx, &ch, &cs->changed));
        if (!ch) break;
    }
    hipLaunchKernelGGL(k_flag_roots, dim3(nbu), dim3(256), 0, st, U, nu, lab, cnt);
    PG_TRY(scan_exclusive(ctx, cnt, off, nu, w + L.scan_tmp));
    PG_HIP(hipMemsetAsync(tt, 0, sizeof(int32_t) * n, st));
    hipLaunchKernelGGL(k_scatter_roots, dim3(nbu), dim3(256), 0, st, U, nu, lab, off, rts, tt);
    hipLaunchKernelGGL(k_reach_time, dim3(nbu), dim3(256), 0, st, U, nu, lab, tt);
    PG_HIP(hipGetLastError());
    int64_t m64 = 0;
    PG_TRY(read_back(ctx, &m64, off + nu));
    const int32_t m = (int32_t)m64;

    // the free set F: nodes below degree R now
    hipLaunchKernelGGL(k_flag_free, dim3(nbn), dim3(256), 0, st, g_deg, n, R, cnt);
    PG_TRY(scan_exclusive(ctx, cnt, off, n, w + L.scan_tmp));
    hipLaunchKernelGGL(k_scatter_free, dim3(nbn), dim3(256), 0, st, g_deg, n, R, off, F);
    PG_HIP(hipGetLastError());
    int64_t nf64 = 0;
    PG_TRY(read_back(ctx, &nf64, off + n));
    const int32_t nf = (int32_t)nf64;
    const unsigned nbf = (unsigned)std::max<int64_t>(1, (nf + 255) / 256);

    for (int32_t b0 = 0; b0 < m; b0 += CONNECT_BATCH) {
        const int32_t b1 = std::min<int32_t>(m, b0 + CONNECT_BATCH);
        PG_HIP(hipMemsetAsync(&cs->n_empty, 0, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_root_lists, dim3((unsigned)((b1 - b0 + 3) / 4)), dim3(256), 0, st, X, ldx, d, n, R,
                           cand, C, rts, b0, b1, tt, g_deg, keys, queue, qvalid, cs);
        PG_HIP(hipGetLastError());
        int32_t ne = 0;
        PG_TRY(read_back(ctx, &ne, &cs->n_empty));
        if (ne > 0 && nf > 0) {
            const bool mf = exact16 && L.d16 <= 256;
            const int gq = mf ? GQM : GQ;
            const int64_t groups = (ne + gq - 1) / gq;
            int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((TG_BLOCKS + groups - 1) / groups,
                                                                    (nf + TG_MIN_CHUNK - 1) / TG_MIN_CHUNK));
            // the per-chunk lists (ne x nchunk lists of C keys) must fit their buffer
            nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, L.part_keys / ((int64_t)ne * C)));
            const int64_t chunk = ((nf + nchunk - 1) / nchunk + TG_TILE - 1) / TG_TILE * TG_TILE;
            nchunk = (nf + chunk - 1) / chunk;
            const _Float16 *x16 = (const _Float16 *)(w + L.x16);
            const float *nrm = (const float *)(w + L.norms);
            if (mf && L.d16 <= 128)
                hipLaunchKernelGGL(k_global_topg_mfma<8>, dim3((unsigned)nchunk, (unsigned)groups), dim3(256), 0, st,
                                   x16, L.d16, nrm, R, rts, tt, g_deg, F, nf, (int32_t)chunk, (int32_t)nchunk, queue,
                                   qvalid, ne, b0, C, keys, part);
            else if (mf)
                hipLaunchKernelGGL(k_global_topg_mfma<16>, dim3((unsigned)nchunk, (unsigned)groups), dim3(256), 0, st,
                                   x16, L.d16, nrm, R, rts, tt, g_deg, F, nf, (int32_t)chunk, (int32_t)nchunk, queue,
                                   qvalid, ne, b0, C, keys, part);
            else
                hipLaunchKernelGGL(k_global_topg, dim3((unsigned)nchunk, (unsigned)groups), dim3(256), 0, st, X, ldx,
                                   d, R, rts, tt, g_deg, F, nf, (int32_t)chunk, (int32_t)nchunk, queue, qvalid, ne, b0,
                                   C, keys, part);
            PG_HIP(hipGetLastError());
            if (nchunk > 1) {
                hipLaunchKernelGGL(k_topg_merge, dim3((unsigned)((ne + 3) / 4)), dim3(256), 0, st, part,
                                   (int32_t)nchunk, queue, qvalid, ne, b0, C, keys);
                PG_HIP(hipGetLastError());
            }
        }
        PG_TRY(write_to(ctx, &cs->idx, b0));
        hipLaunchKernelGGL(k_match, dim3(1), dim3(64), 0, st, rts, b0, b1, keys, C, R, g_ids, g_d2, g_deg, cs);
        PG_HIP(hipGetLastError());
        for (;;) {
            int32_t stop = -1;
            PG_TRY(read_back(ctx, &stop, &cs->stop_root));
            if (stop == -1) break;
            if (stop == -2) {
                set_error("pg_prune: connect found every reachable node at degree R=%d", R);
                return PG_EOVERFLOW;
            }
            // stops are resolved on the stream without waiting for each: the
            // scan and the attach do nothing once the wave has no stopped
            // root, and a wave restarted after the batch ends returns at once
            for (int c = 0; c < STOP_CHAIN; ++c) {
                hipLaunchKernelGGL(k_nearest_at, dim3(nbf), dim3(256), 0, st, X, ldx, d, R, F, nf, tt, g_deg, cs);
                hipLaunchKernelGGL(k_attach, dim3(1), dim3(1), 0, st, g_ids, g_d2, g_deg, R, cs);
                hipLaunchKernelGGL(k_match, dim3(1), dim3(64), 0, st, rts, b0, b1, keys, C, R, g_ids, g_d2, g_deg,
                                   cs);
            }
            PG_HIP(hipGetLastError());
        }
    }
    if (n_roots) *n_roots = m;
    return PG_OK;
}

}  // namespace pgi

using namespace pgi;

extern "C" pg_status pg_prune_workspace(const pg_prune_params *p, int64_t n, int32_t d, int32_t C,
                                        size_t *bytes) {
    PG_TRY(check_prune(p, n, C));
    if (!bytes) {
        set_error("pg_prune_workspace: bytes is NULL");
        return PG_EINVAL;
    }
    if (d <= 0 || d > PRUNE_MAX_D) {
        set_error("pg_prune_workspace: d=%d must be in [1, %d]", d, PRUNE_MAX_D);
        return PG_EINVAL;
    }
    *bytes = prune_layout(p, n, d).total;
    return PG_OK;
}

extern "C" pg_status pg_prune(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                              const int32_t *cand_ids, const float *cand_d2, int32_t C,
                              const pg_prune_params *p, void *ws,
                              size_t ws_bytes, int32_t *g_ids, float *g_d2, int32_t *g_deg,
                              int32_t *ep, int32_t *roots, int32_t *n_roots) {
    if (!ctx || !X || !cand_ids || !g_ids || !g_d2 || !g_deg || !ep) {
        set_error("pg_prune: NULL argument");
        return PG_EINVAL;
    }
    PG_TRY(check_prune(p, n, C));
    if (d <= 0 || d > PRUNE_MAX_D || ldx < d) {
        set_error("pg_prune: d=%d must be in [1, %d] and ldx >= d", d, PRUNE_MAX_D);
        return PG_EINVAL;
    }
    if (d % 4 || ldx % 4 || ((uintptr_t)X & 15)) {
        set_error("pg_prune: d and ldx must be multiples of 4 and X 16-byte aligned");
        return PG_EUNSUPPORTED;
    }
    const PruneLayout L = prune_layout(p, n, d);
    if (!ws || ws_bytes < L.total) {
        set_error("pg_prune: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
        return PG_ENOMEM;
    }
    char *w = (char *)ws;
    int32_t *p_ids = (int32_t *)(w + L.p_ids), *p_deg = (int32_t *)(w + L.p_deg),
            *cnt = (int32_t *)(w + L.cnt), *rev = (int32_t *)(w + L.rev),
            *visited = (int32_t *)(w + L.visited), *fa = (int32_t *)(w + L.fa),
            *fb = (int32_t *)(w + L.fb), *api = (int32_t *)(w + L.api);
    float *p_d2 = (float *)(w + L.p_d2);
    int64_t *off = (int64_t *)(w + L.off);
    ConnState *cs = (ConnState *)(w + L.cs);
    double *cpart = (double *)(w + L.cpart), *cen = (double *)(w + L.cen), *apd = (double *)(w + L.apd);
    hipStream_t st = ctx->stream;
    const int R = p->R;
    AngleTest at;
    {
        const double a = (double)p->alpha_deg;
        at.on = p->alpha_deg > 60.0f;
        at.kd = (a == 90.0) ? 0.0 : 2.0 * cos(a * (M_PI / 180.0));
        at.kf = (float)at.kd;
    }
    const bool rev_stage = (p->stages & PG_STAGE_REVERSE) != 0;

    // exactness test of the 16-bit MFMA path (needs the distances to u given)
    _Float16 *x16 = (_Float16 *)(w + L.x16);
    float *nrm = (float *)(w + L.norms);
    bool exact16 = false;
    if (!p->pair_d2) {
        unsigned int *exf = (unsigned int *)(w + L.exflags);
        PG_HIP(hipMemsetAsync(exf, 0, sizeof(unsigned int) * 4, st));
        hipLaunchKernelGGL(k_prune_prep, dim3((unsigned)std::min<int64_t>((n + 3) / 4, 4096)), dim3(256), 0, st, X,
                           ldx, d, L.d16, n, x16, nrm, exf);
        PG_HIP(hipGetLastError());
        unsigned int he[4];
        PG_HIP(hipMemcpyAsync(he, exf, sizeof(he), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        float maxabs, maxnorm;
        memcpy(&maxabs, &he[PX_MAXABS], 4);
        memcpy(&maxnorm, &he[PX_MAXNORM], 4);
        exact16 = he[PX_NONINT] == 0 && maxabs <= 2048.0f &&
                  (maxnorm <= 4194304.0f || (he[PX_NEG] == 0 && maxnorm <= 8388608.0f));
    }
    // float data: centred FP16 copy for the mixed tiles (the centroid is the
    // entry point's too)
    bool centroid_done = false, mix = false;
    PruneMix pmx{};
    if (!p->pair_d2 && !exact16 && p->precision != PG_FP32_VALU) {
        hipLaunchKernelGGL(k_centroid_partial, dim3((unsigned)L.ncb), dim3(256), 0, st, X, n, d, ldx, cpart);
        hipLaunchKernelGGL(k_centroid_final, dim3(1), dim3(256), 0, st, cpart, L.ncb, d, n, cen);
        centroid_done = true;
        unsigned int *exf = (unsigned int *)(w + L.exflags);
        PG_HIP(hipMemsetAsync(exf, 0, sizeof(unsigned int) * 4, st));
        hipLaunchKernelGGL(k_prune_prep_mixed, dim3((unsigned)std::min<int64_t>((n + 3) / 4, 4096)), dim3(256), 0,
                           st, X, ldx, d, L.d16, n, cen, x16, nrm, exf);
        PG_HIP(hipGetLastError());
        unsigned int he[4];
        PG_HIP(hipMemcpyAsync(he, exf, sizeof(he), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        float cmax;
        memcpy(&cmax, &he[PX_MAXABS], 4);
        if (cmax <= 32768.0f) {
            mix = true;
            const double u32 = 1.0 / 16777216.0;
            pmx.on = 1;
            pmx.un = (float)(1.0 / 2048.0 + 4.0 * u32);
            pmx.ea = 2.98023224e-08f;  // half the FP16 subnormal spacing
            pmx.gd = (float)((d + 4) * u32 * 1.01);
            pmx.ga = (float)((2.0 * L.d16 + 16) * u32 * 1.01);
            pmx.sqd = sqrtf((float)d);
        }
    }
    int32_t *s_ids = rev_stage ? p_ids : g_ids, *s_deg = rev_stage ? p_deg : g_deg;
    float *s_d2 = rev_stage ? p_d2 : g_d2;
    // The MFMA kernel's second pass holds at most 32 nodes kept in earlier
    // rounds.  A PRUNE list (C <= 64) takes one round; a reverse union can
    // exceed 64 candidates, so that stage runs on it only when R <= 32.
    const bool mfma_reverse = R <= 32;
    {
        TimedLaunch tl(ctx, K_PRUNE, (double)n * C * C / 2.0 * 3.0 * d);
        if ((exact16 || mix) && cand_d2)
            hipLaunchKernelGGL((exact16 ? k_prune_mfma<false, false>
                                        : (d >= PM_STAGE_D ? k_prune_mfma<true, true> : k_prune_mfma<true, false>)),
                               dim3((unsigned)n), dim3(64), 0,
                               st, x16, L.d16, nrm, n, cand_ids, cand_d2, C, (const int32_t *)nullptr,
                               (const int64_t *)nullptr, (const int32_t *)nullptr, (const float *)nullptr, R, at,
                               p->strict_ties, s_ids, s_d2, s_deg, X, ldx, d, pmx, p->k2p_prev_ids,
                               p->k2p_prev_deg, p->k2p_prev_R, p->k2p_counts);
        else
            hipLaunchKernelGGL(k_prune, dim3((unsigned)n), dim3(64), 0, st, X, ldx, d, n, cand_ids, cand_d2, C,
                               (const int32_t *)nullptr, (const int64_t *)nullptr, (const int32_t *)nullptr,
                               (const float *)nullptr, R, at, p->strict_ties, p->pair_d2,
                               s_ids, s_d2, s_deg);
        PG_HIP(hipGetLastError());
    }
    if (p->prune_ids_out) {
        PG_HIP(hipMemcpyAsync(p->prune_ids_out, s_ids, sizeof(int32_t) * n * R, hipMemcpyDeviceToDevice, st));
        PG_HIP(hipMemcpyAsync(p->prune_deg_out, s_deg, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    }
    if (rev_stage) {
        const int64_t tot = n * R;
        float *rev_d2 = (float *)(w + L.rev_d2);
        PG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, st));
        hipLaunchKernelGGL(k_count_indeg, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p_ids,
                           p_deg, n, R, cnt);
        PG_TRY(scan_exclusive(ctx, cnt, off, n, w + L.scan_tmp));
        PG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, st));
        hipLaunchKernelGGL(k_scatter_rev, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p_ids, p_d2,
                           p_deg, n, R, off, cnt, rev, rev_d2);
        PG_HIP(hipGetLastError());
        TimedLaunch tl(ctx, K_PRUNE, -1.0);
        if ((exact16 || mix) && mfma_reverse)
            hipLaunchKernelGGL((exact16 ? k_prune_mfma<false, false>
                                        : (d >= PM_STAGE_D ? k_prune_mfma<true, true> : k_prune_mfma<true, false>)),
                               dim3((unsigned)n), dim3(64), 0,
                               st, x16, L.d16, nrm, n, p_ids, p_d2, R, p_deg, off, rev, rev_d2, R, at,
                               p->strict_ties, g_ids, g_d2, g_deg, X, ldx, d, pmx, (const int32_t *)nullptr,
                               (const int32_t *)nullptr, 0, (unsigned long long *)nullptr);
        else
            hipLaunchKernelGGL(k_prune, dim3((unsigned)n), dim3(64), 0, st, X, ldx, d, n, p_ids, p_d2, R, p_deg,
                               off, rev, rev_d2, R, at, p->strict_ties, (const float *)nullptr,
                               g_ids, g_d2, g_deg);
        PG_HIP(hipGetLastError());
    }
    // entry point
    if (!centroid_done) {
        hipLaunchKernelGGL(k_centroid_partial, dim3((unsigned)L.ncb), dim3(256), 0, st, X, n, d, ldx, cpart);
        hipLaunchKernelGGL(k_centroid_final, dim3(1), dim3(256), 0, st, cpart, L.ncb, d, n, cen);
    }
    hipLaunchKernelGGL(k_argmin_center, dim3((unsigned)L.nab), dim3(256), 0, st, X, n, d, ldx, cen, apd,
                       api);
    hipLaunchKernelGGL(k_argmin_final, dim3(1), dim3(256), 0, st, apd, api, L.nab, ep);
    PG_HIP(hipGetLastError());
    if (n_roots) *n_roots = 0;
    if (p->stages & PG_STAGE_CONNECT) {
        TimedLaunch tl(ctx, K_CONNECT, -1.0);
        PG_TRY(connect(ctx, L, w, X, n, d, ldx, cand_ids, C, R, g_ids, g_d2, g_deg, ep, roots, n_roots, exact16));
    }
    return PG_OK;
}
