// pg_common.h -- internal helpers of the gfx950 proximity-graph library.
//
// Keys.  Every (distance, id) pair is packed into one 64-bit key
//   key = (bits(d2) << 32) | id
// where d2 >= +0 is a float32 squared distance.  Non-negative IEEE floats
// order like their bit patterns, so unsigned key order is the (d2, id) order
// used throughout (the paper does not say how ties break).  KEY_INF pads.
//
// Distances.  d2(x, y) = s after s = fma(x_i - y_i, x_i - y_i, s) for i = 0..d-1
// in order, starting from +0.  Every kernel evaluates it this way, so a pair
// has one bit pattern wherever it is computed, and d2(x, y) == d2(y, x).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pg.h"

#define PG_WAVE 64
#define KEY_INF 0xFFFFFFFFFFFFFFFFull

// ---------------------------------------------------------------------------
// host-side error reporting
// ---------------------------------------------------------------------------
namespace pgi {
void set_error(const char *fmt, ...);
pg_status hip_fail(hipError_t e, const char *what);
}  // namespace pgi

#define PG_HIP(call)                                           \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return pgi::hip_fail(e_, #call); \
    } while (0)

#define PG_TRY(call)                       \
    do {                                   \
        pg_status s_ = (call);             \
        if (s_ != PG_OK) return s_;        \
    } while (0)

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t pack_key(float d2, int32_t id) {
    return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
}
__device__ __forceinline__ float key_d2(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_id(uint64_t k) { return (int32_t)(uint32_t)k; }

// ---------------------------------------------------------------------------
// counter-based random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014)
// sm(s, i) is the i-th output of a SplitMix64 generator started at state s;
// hash4(seed, stream, a, b) = sm(sm(sm(seed, stream + 1), a + 1), b + 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sm_out(uint64_t s, uint64_t i) {
    uint64_t z = s + 0x9E3779B97F4A7C15ull * i;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t hash4(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
    uint64_t x = sm_out(seed, stream + 1);
    x = sm_out(x, a + 1);
    return sm_out(x, b + 1);
}
// Sampling key: the high 32 bits of the hash, then the id (a total order).
__device__ __forceinline__ uint64_t sample_key(uint64_t h, int32_t id) {
    return (h & 0xFFFFFFFF00000000ull) | (uint32_t)id;
}

// ---------------------------------------------------------------------------
// wave64 primitives.  Every helper that reads other lanes (shuffles, ballots,
// readlane) must be reached by all 64 lanes: call them from uniform control
// flow only, never behind a short-circuit && / || or a divergent branch.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (PG_WAVE - 1)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, PG_WAVE);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, PG_WAVE);
    return ((uint64_t)hi << 32) | lo;
}
// Value held by lane (lane ^ m).  Distances 1, 2 and 8 stay inside the VALU
// (DPP quad permutes and a row rotation by 8, which is the exchange of the two
// row halves); 4 and 16 are swizzles in bitmask mode (and 31, xor m, applied
// within each half-wave); other distances go through the LDS crossbar.  The
// fast forms need a constant m, which they get once the callers' loops over
// distances are unrolled.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int m) {
    switch (m) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror 8
    case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
    default: return (uint32_t)__shfl_xor((int)v, m, PG_WAVE);
    }
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = xor_lane((uint32_t)v, m);
    const uint32_t hi = xor_lane((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}
// Value held by lane - 1, lane 0 keeping its own: a DPP shift of the whole
// wave right by one lane (lane 0 has no source and keeps `old`).
__device__ __forceinline__ uint32_t from_lane_below(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x138, 0xF, 0xF, false);  // wave_shr 1
}
__device__ __forceinline__ uint64_t from_lane_below64(uint64_t v) {
    const uint32_t lo = from_lane_below((uint32_t)v);
    const uint32_t hi = from_lane_below((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of one key per lane, payload p travels with its key.
__device__ __forceinline__ void wave_sort(uint64_t &k, int &p) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= PG_WAVE; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint64_t ok = shfl_xor64(k, j);
            const int op = (int)xor_lane((uint32_t)p, j);
            const bool asc = (lane & size) == 0;
            const bool lower = (lane & j) == 0;
            const bool take = (lower == asc) ? (ok < k) : (ok > k);
            k = take ? ok : k;
            p = take ? op : p;
        }
    }
}
__device__ __forceinline__ void wave_sort(uint64_t &k) {
    int p = 0;
    wave_sort(k, p);
}

// A bitonic sequence across the wave becomes ascending.
__device__ __forceinline__ void wave_bitonic_merge(uint64_t &k, int &p) {
    const int lane = lane_id();
#pragma unroll
    for (int j = PG_WAVE / 2; j > 0; j >>= 1) {
        const uint64_t ok = shfl_xor64(k, j);
        const int op = (int)xor_lane((uint32_t)p, j);
        const bool lower = (lane & j) == 0;
        const bool take = lower ? (ok < k) : (ok > k);
        k = take ? ok : k;
        p = take ? op : p;
    }
}

// a and b ascending (one key per lane): returns the 64 smallest of a U b,
// ascending, with payloads.
__device__ __forceinline__ void wave_merge_lowest(uint64_t &a, int &pa, uint64_t b, int pb) {
    const int lane = lane_id();
    uint64_t br = shfl64(b, PG_WAVE - 1 - lane);
    int pbr = __shfl(pb, PG_WAVE - 1 - lane, PG_WAVE);
    const bool lt = br < a;
    a = lt ? br : a;
    pa = lt ? pbr : pa;
    wave_bitonic_merge(a, pa);
}

// Keep the keys of lanes where `valid` holds, in lane order, packed to the
// front; the tail becomes KEY_INF.  Returns the number kept.
__device__ __forceinline__ int wave_compact(uint64_t &k, int &p, bool valid) {
    const uint64_t m = __ballot(valid);
    const int cnt = __popcll(m);
    const int lane = lane_id();
    int dst = valid ? __popcll(m & lanemask_lt()) : cnt + __popcll(~m & lanemask_lt());
    uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)k);
    uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst * 4, (int)(uint32_t)(k >> 32));
    int np = __builtin_amdgcn_ds_permute(dst * 4, p);
    k = (lane < cnt) ? (((uint64_t)hi << 32) | lo) : KEY_INF;
    p = np;
    return cnt;
}

// Number of lanes whose key is < x, for an ascending wave-wide key list
// (binary search by shuffles; every lane may ask for its own x).
__device__ __forceinline__ int wave_count_less(uint64_t sorted, uint64_t x) {
    int lo = 0;
#pragma unroll
    for (int step = PG_WAVE / 2; step > 0; step >>= 1) {
        uint64_t probe = shfl64(sorted, lo + step - 1);
        if (probe < x) lo += step;
    }
    uint64_t last = shfl64(sorted, lo);
    return lo + ((lo < PG_WAVE && last < x) ? 1 : 0);
}

// ---------------------------------------------------------------------------
// source passes over a locality order, XCD-aware
//
// A pass covers the positions p of the order array whose residue p % 64 lies
// in [lo, lo + w); its items are i = q * w + (r - lo) for p = 64 q + r, so
// consecutive items are neighbouring positions.  Workgroups of a launch are
// spread over the 8 XCDs round-robin (workgroup b on XCD b % 8); the logical
// block of physical block b walks a contiguous range per XCD, so blocks that
// share an L2 work on neighbouring sources.
// ---------------------------------------------------------------------------
constexpr int PG_NXCD = 8;
constexpr int PG_PASS_PERIOD = 64;

struct PassRange {
    int lo, w;       // residues [lo, lo + w) of position % PG_PASS_PERIOD
    int64_t items;   // ceil(n / PG_PASS_PERIOD) * w
};

__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nlogical) {
    const int64_t per = (nlogical + PG_NXCD - 1) / PG_NXCD;
    return (b % PG_NXCD) * per + b / PG_NXCD;
}

static inline unsigned xcd_grid(int64_t nlogical) {
    return (unsigned)(((nlogical + PG_NXCD - 1) / PG_NXCD) * PG_NXCD);
}

// source node of item i of a pass, or -1 past the end
__device__ __forceinline__ int64_t pass_source(const int32_t *__restrict__ order, int64_t n, PassRange pr,
                                               int64_t i) {
    if (i >= pr.items) return -1;
    const int64_t p = (i / pr.w) * PG_PASS_PERIOD + pr.lo + (i % pr.w);
    return p < n ? (int64_t)order[p] : -1;
}

// ---------------------------------------------------------------------------
// canonical squared distance (one lane, full vectors, float4 loads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dist_chain(const float *__restrict__ a,
                                            const float *__restrict__ b, int d) {
    float s = 0.0f;
    for (int i = 0; i < d; i += 4) {
        const float4 x = *reinterpret_cast<const float4 *>(a + i);
        const float4 y = *reinterpret_cast<const float4 *>(b + i);
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
    return s;
}

// ---------------------------------------------------------------------------
// context and per-kernel timing
// ---------------------------------------------------------------------------
struct pg_ctx {
    int device;
    int num_cu;  // compute units of the device
    hipStream_t stream;
    bool timing;
    void *timing_state;  // pgi::TimingState
};

namespace pgi {
enum KernelId { K_JOIN = 0, K_MERGE, K_INIT, K_SAMPLE, K_PRUNE, K_SEARCH, K_EXACT, K_CONNECT, K_COUNT };
// Record the start/stop of a timed launch on the context stream.
struct TimedLaunch {
    pg_ctx *ctx;
    int kernel;
    double work;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(pg_ctx *c, int k, double w);
    ~TimedLaunch();
};
void ctx_add_work(pg_ctx *ctx, int kernel, double work);
pg_status scan_exclusive(pg_ctx *ctx, const int32_t *in, int64_t *out, int64_t n, void *tmp);
size_t scan_tmp_bytes(int64_t n);
}  // namespace pgi

static inline size_t pg_align(size_t x) { return (x + 255) & ~(size_t)255; }
