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

__device__ __forceinline__ bool occludes(float a, float b, float c, int strict, int use_angle,
                                         float kappa) {
    // w (a = d2(u,w)) visited before v (c = d2(u,v)); b = d2(v,w)
    if (!(b < c)) return false;
    if (strict && !(a < c)) return false;
    if (!use_angle) return true;
    if (b == 0.0f) return true;
    return (a + b - c) < kappa * sqrtf(a * b);
}

__global__ __launch_bounds__(64) void k_prune(
    const float *__restrict__ X, int64_t ldx, int d, int64_t n, const int32_t *__restrict__ src1,
    int C1, const int32_t *__restrict__ src1_deg, const int64_t *__restrict__ src2_off,
    const int32_t *__restrict__ src2, int R, float kappa, int use_angle, int strict,
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
            if (idx < c1)
                id = src1[u * C1 + idx];
            else if (idx < m)
                id = src2[off2 + (idx - c1)];
            uint64_t key = KEY_INF;
            if (id >= 0 && id < n && id != (int32_t)u) {
                const float dd = tu ? tu[idx + 1] : dist_chain(xu, X + (int64_t)id * ldx, d);
                key = pack_key(dd, id);
                if (!first && key <= last) key = KEY_INF;
            }
            int pos = idx;
            wave_sort(key, pos);
            const uint64_t prev = shfl64(key, max(lane - 1, 0));
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
                    const bool cnd = occludes(a, b, myc, strict, use_angle, kappa);
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

__global__ void k_scatter_rev(const int32_t *__restrict__ g, const int32_t *__restrict__ deg,
                              int64_t n, int R, const int64_t *__restrict__ off,
                              int32_t *__restrict__ cur, int32_t *__restrict__ rev) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * R) return;
    const int64_t u = i / R;
    const int j = (int)(i % R);
    if (j < deg[u]) {
        const int32_t v = g[i];
        rev[off[v] + atomicAdd(&cur[v], 1)] = (int32_t)u;
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

__global__ __launch_bounds__(256) void k_argmin_center(const float *__restrict__ X, int64_t n, int d,
                                                       int64_t ldx, const double *__restrict__ cen,
                                                       double *__restrict__ pd, int32_t *__restrict__ pid) {
    __shared__ double sd[256];
    __shared__ int32_t si[256];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    DKey best{INFINITY, 0x7fffffff};
    if (v < n) {
        double s = 0.0;
        for (int j = 0; j < d; ++j) {
            const double t = __dsub_rn((double)X[v * ldx + j], cen[j]);
            s = __dadd_rn(s, __dmul_rn(t, t));
        }
        best = {s, (int32_t)v};
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
// connectivity: level-synchronous BFS over out-edges + nearest reachable node
// ---------------------------------------------------------------------------
struct ConnState {
    int32_t fcount[2];
    int32_t first_unreached;  // root waiting for the global nearest-node scan
    int32_t n_roots;
    int32_t overflow;
    int32_t idx;              // next position in the list of unreached ids
    int32_t bfs_head;         // > 0: the wave handed a BFS queue[bfs_head, bfs_tail)
    int32_t bfs_tail;         //      over to the multi-block BFS
    unsigned long long nearest;
};

// a BFS that grows past this many queued nodes continues on the multi-block path
constexpr int CONNECT_WAVE_BFS = 2048;

// loads that must see stores made earlier in the same kernel (bypass L1)
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

// The connect loop of the refinement, one wave: unreached ids in increasing
// order; each still-unreached r gets the edge p -> r from its closest reached
// candidate p with degree < R, then a BFS from r marks what r reaches.  When no
// candidate of r qualifies the wave stops and leaves r in first_unreached for
// the global scan on the host side.
__global__ __launch_bounds__(64) void k_connect_loop(const float *__restrict__ X, int64_t ldx, int d,
                                                     int64_t n, int R, const int32_t *__restrict__ cand,
                                                     int C, int32_t *g, float *gd, int32_t *deg,
                                                     int32_t *visited, const int32_t *__restrict__ U,
                                                     int32_t nu, int32_t *queue, int32_t *roots,
                                                     ConnState *cs) {
    const int lane = lane_id();
    for (int32_t idx = cs->idx; idx < nu; ++idx) {
        const int32_t r = U[idx];
        if (ld_fresh(&visited[r])) continue;
        uint64_t key = KEY_INF;
        if (lane < C) {
            const int32_t p = cand[(int64_t)r * C + lane];
            if (p >= 0 && p < n && p != r && ld_fresh(&visited[p]) && ld_fresh(&deg[p]) < R)
                key = pack_key(dist_chain(X + (int64_t)r * ldx, X + (int64_t)p * ldx, d), p);
        }
#pragma unroll
        for (int o = 1; o < PG_WAVE; o <<= 1) {
            const uint64_t t = shfl_xor64(key, o);
            key = t < key ? t : key;
        }
        if (key == KEY_INF) {
            if (lane == 0) {
                cs->idx = idx;
                cs->first_unreached = r;
            }
            return;
        }
        const int32_t p = key_id(key);
        if (lane == 0) {
            const int j = ld_fresh(&deg[p]);
            g[(int64_t)p * R + j] = r;
            gd[(int64_t)p * R + j] = key_d2(key);
            deg[p] = j + 1;
            roots[cs->n_roots] = r;
            cs->n_roots += 1;
            visited[r] = 1;
            queue[0] = r;
        }
        __threadfence();
        int head = 0, tail = 1;
        while (head < tail) {
            if (tail - head > CONNECT_WAVE_BFS) {
                if (lane == 0) {
                    cs->idx = idx + 1;
                    cs->bfs_head = head;
                    cs->bfs_tail = tail;
                    cs->first_unreached = -1;
                }
                return;
            }
            const int32_t x = ld_fresh(&queue[head]);
            ++head;
            const int dx = min(ld_fresh(&deg[x]), R);
            bool push = false;
            int32_t y = -1;
            if (lane < dx) {
                y = ld_fresh(&g[(int64_t)x * R + lane]);
                if (y >= 0 && y < n && atomicExch(&visited[y], 1) == 0) push = true;
            }
            const uint64_t m = __ballot(push);
            if (push) queue[tail + __popcll(m & lanemask_lt())] = y;
            tail += __popcll(m);
            __threadfence();
        }
    }
    if (lane == 0) {
        cs->idx = nu;
        cs->first_unreached = -1;
    }
}

__global__ void k_bfs_seed(int32_t *__restrict__ visited, int32_t *__restrict__ frontier,
                           ConnState *__restrict__ cs, const int32_t *__restrict__ src_dev, int32_t src) {
    const int32_t r = src_dev ? *src_dev : src;
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

__global__ __launch_bounds__(256) void k_nearest_reached(const float *__restrict__ X, int64_t ldx,
                                                         int d, int64_t n, int R,
                                                         const int32_t *__restrict__ visited,
                                                         const int32_t *__restrict__ deg,
                                                         ConnState *__restrict__ cs) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t r = cs->first_unreached;
    uint64_t key = KEY_INF;
    if (p < n && visited[p] && deg[p] < R)
        key = pack_key(dist_chain(X + (int64_t)r * ldx, X + p * ldx, d), (int32_t)p);
#pragma unroll
    for (int o = 1; o < PG_WAVE; o <<= 1) {
        const uint64_t t = shfl_xor64(key, o);
        key = t < key ? t : key;
    }
    if (lane_id() == 0 && key != KEY_INF) atomicMin(&cs->nearest, (unsigned long long)key);
}

__global__ void k_attach(int32_t *__restrict__ g, float *__restrict__ gd, int32_t *__restrict__ deg,
                         int R, int32_t *__restrict__ roots, ConnState *__restrict__ cs) {
    const int32_t r = cs->first_unreached;
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
    if (roots) roots[cs->n_roots] = r;
    cs->n_roots += 1;
}

__global__ void k_copy_graph(const int32_t *__restrict__ si, const float *__restrict__ sd,
                             const int32_t *__restrict__ sdeg, int64_t n, int R,
                             int32_t *__restrict__ di, float *__restrict__ dd,
                             int32_t *__restrict__ ddeg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * R) return;
    di[i] = si[i];
    dd[i] = sd[i];
    if (i % R == 0) ddeg[i / R] = sdeg[i / R];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct PruneLayout {
    size_t p_ids, p_d2, p_deg, cnt, off, rev, visited, fa, fb, cs, cpart, cen, apd, api, scan_tmp,
        total;
    int64_t ncb, nab;
};

static PruneLayout prune_layout(const pg_prune_params *p, int64_t n, int d_max) {
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
    L.visited = take(sizeof(int32_t) * n);
    L.fa = take(sizeof(int32_t) * n);
    L.fb = take(sizeof(int32_t) * n);
    L.cs = take(sizeof(ConnState));
    L.cpart = take(sizeof(double) * L.ncb * d_max);
    L.cen = take(sizeof(double) * d_max);
    L.apd = take(sizeof(double) * L.nab);
    L.api = take(sizeof(int32_t) * L.nab);
    L.scan_tmp = take(scan_tmp_bytes(n + 1));
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
    if (!(p->alpha_deg >= 0.0f && p->alpha_deg <= 180.0f)) {
        set_error("pg_prune: alpha_deg=%g must be in [0, 180]", (double)p->alpha_deg);
        return PG_EINVAL;
    }
    return PG_OK;
}

// Level-synchronous BFS over out-edges.  With src_dev or src >= 0 the
// search starts there; otherwise from the nin0 nodes already queued at fin0
// (and already marked).
static pg_status bfs_from(pg_ctx *ctx, const int32_t *g, int64_t n, int R, const int32_t *deg, int32_t *visited,
                          int32_t *fa, int32_t *fb, ConnState *cs, const int32_t *src_dev, int32_t src,
                          int32_t *fin0 = nullptr, int32_t nin0 = 0) {
    hipStream_t st = ctx->stream;
    int32_t nin = 1;
    int32_t *fin = fa, *fout = fb;
    if (fin0) {
        nin = nin0;
        fin = fin0;
    } else {
        hipLaunchKernelGGL(k_bfs_seed, dim3(1), dim3(1), 0, st, visited, fa, cs, src_dev, src);
        PG_HIP(hipGetLastError());
    }
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

}  // namespace pgi

using namespace pgi;

extern "C" pg_status pg_prune_workspace(const pg_prune_params *p, int64_t n, int32_t C,
                                        size_t *bytes) {
    PG_TRY(check_prune(p, n, C));
    if (!bytes) {
        set_error("pg_prune_workspace: bytes is NULL");
        return PG_EINVAL;
    }
    *bytes = prune_layout(p, n, PRUNE_MAX_D).total;
    return PG_OK;
}

extern "C" pg_status pg_prune(pg_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                              const int32_t *cand_ids, int32_t C, const pg_prune_params *p, void *ws,
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
    const PruneLayout L = prune_layout(p, n, PRUNE_MAX_D);
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
    const bool use_angle = p->alpha_deg > 60.0f;
    const double a = (double)p->alpha_deg;
    const float kappa = (a == 90.0) ? 0.0f : (float)(2.0 * cos(a * (M_PI / 180.0)));
    const bool rev_stage = (p->stages & PG_STAGE_REVERSE) != 0;

    {
        TimedLaunch tl(ctx, K_PRUNE, (double)n * C * C / 2.0 * 3.0 * d);
        hipLaunchKernelGGL(k_prune, dim3((unsigned)n), dim3(64), 0, st, X, ldx, d, n, cand_ids, C,
                           (const int32_t *)nullptr, (const int64_t *)nullptr, (const int32_t *)nullptr, R,
                           kappa, (int)use_angle, p->strict_ties, p->pair_d2, rev_stage ? p_ids : g_ids,
                           rev_stage ? p_d2 : g_d2, rev_stage ? p_deg : g_deg);
        PG_HIP(hipGetLastError());
    }
    if (rev_stage) {
        const int64_t tot = n * R;
        PG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, st));
        hipLaunchKernelGGL(k_count_indeg, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p_ids,
                           p_deg, n, R, cnt);
        PG_TRY(scan_exclusive(ctx, cnt, off, n, w + L.scan_tmp));
        PG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * n, st));
        hipLaunchKernelGGL(k_scatter_rev, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p_ids,
                           p_deg, n, R, off, cnt, rev);
        PG_HIP(hipGetLastError());
        TimedLaunch tl(ctx, K_PRUNE, -1.0);
        hipLaunchKernelGGL(k_prune, dim3((unsigned)n), dim3(64), 0, st, X, ldx, d, n, p_ids, R, p_deg,
                           off, rev, R, kappa, (int)use_angle, p->strict_ties, (const float *)nullptr,
                           g_ids, g_d2, g_deg);
        PG_HIP(hipGetLastError());
    }
    // entry point
    hipLaunchKernelGGL(k_centroid_partial, dim3((unsigned)L.ncb), dim3(256), 0, st, X, n, d, ldx, cpart);
    hipLaunchKernelGGL(k_centroid_final, dim3(1), dim3(256), 0, st, cpart, L.ncb, d, n, cen);
    hipLaunchKernelGGL(k_argmin_center, dim3((unsigned)L.nab), dim3(256), 0, st, X, n, d, ldx, cen, apd,
                       api);
    hipLaunchKernelGGL(k_argmin_final, dim3(1), dim3(256), 0, st, apd, api, L.nab, ep);
    PG_HIP(hipGetLastError());
    if (n_roots) *n_roots = 0;
    if (p->stages & PG_STAGE_CONNECT) {
        PG_HIP(hipMemsetAsync(visited, 0, sizeof(int32_t) * n, st));
        PG_HIP(hipMemsetAsync(cs, 0, sizeof(ConnState), st));
        PG_TRY(bfs_from(ctx, g_ids, n, R, g_deg, visited, fa, fb, cs, ep, 0));
        const unsigned nb = (unsigned)((n + 255) / 256);
        // unreached ids in increasing order
        hipLaunchKernelGGL(k_flag_unreached, dim3(nb), dim3(256), 0, st, visited, n, cnt);
        PG_TRY(scan_exclusive(ctx, cnt, off, n, w + L.scan_tmp));
        hipLaunchKernelGGL(k_scatter_unreached, dim3(nb), dim3(256), 0, st, visited, n, off, rev);
        PG_HIP(hipGetLastError());
        int64_t nu64 = 0;
        PG_HIP(hipMemcpyAsync(&nu64, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PG_HIP(hipStreamSynchronize(st));
        const int32_t nu = (int32_t)nu64;
        for (int64_t restart = 0; nu > 0; ++restart) {
            hipLaunchKernelGGL(k_connect_loop, dim3(1), dim3(64), 0, st, X, ldx, d, n, R, cand_ids, C,
                               g_ids, g_d2, g_deg, visited, rev, nu, fa, roots ? roots : fb, cs);
            PG_HIP(hipGetLastError());
            ConnState h;
            PG_HIP(hipMemcpyAsync(&h, cs, sizeof(h), hipMemcpyDeviceToHost, st));
            PG_HIP(hipStreamSynchronize(st));
            if (h.bfs_head > 0) {
                // a large component: finish its BFS level-synchronously, then resume
                const int32_t hb = h.bfs_head, tb = h.bfs_tail;
                const int32_t zero2[2] = {0, 0};
                PG_HIP(hipMemcpyAsync(&cs->bfs_head, zero2, sizeof(zero2), hipMemcpyHostToDevice, st));
                PG_TRY(bfs_from(ctx, g_ids, n, R, g_deg, visited, fa + tb, fb, cs, nullptr, -1, fa + hb,
                                tb - hb));
                continue;
            }
            if (h.idx >= nu) break;
            // no candidate of r qualifies: nearest reached node over all of X
            const unsigned long long inf = KEY_INF;
            PG_HIP(hipMemcpyAsync(&cs->nearest, &inf, sizeof(inf), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_nearest_reached, dim3(nb), dim3(256), 0, st, X, ldx, d, n, R, visited,
                               g_deg, cs);
            hipLaunchKernelGGL(k_attach, dim3(1), dim3(1), 0, st, g_ids, g_d2, g_deg, R, roots, cs);
            PG_HIP(hipGetLastError());
            int32_t ovf = 0;
            PG_HIP(hipMemcpyAsync(&ovf, &cs->overflow, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            PG_HIP(hipStreamSynchronize(st));
            if (ovf) {
                set_error("pg_prune: connect found every reachable node at degree R=%d", R);
                return PG_EOVERFLOW;
            }
            PG_TRY(bfs_from(ctx, g_ids, n, R, g_deg, visited, fa, fb, cs, &cs->first_unreached, 0));
            const int32_t next = h.idx + 1;
            PG_HIP(hipMemcpyAsync(&cs->idx, &next, sizeof(int32_t), hipMemcpyHostToDevice, st));
        }
        if (n_roots) {
            int32_t nr = 0;
            PG_HIP(hipMemcpyAsync(&nr, &cs->n_roots, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            PG_HIP(hipStreamSynchronize(st));
            *n_roots = nr;
        }
    }
    return PG_OK;
}
