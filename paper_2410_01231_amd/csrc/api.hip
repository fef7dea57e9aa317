// api.hip -- context, errors, per-kernel event timing and the device prefix
// sum shared by the build kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "pg_common.h"

namespace pgi {

static thread_local char g_err[512] = "no error";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

pg_status hip_fail(hipError_t e, const char *what) {
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return PG_EDEVICE;
}

struct TimingState {
    struct Pending {
        hipEvent_t a, b;
        int kernel;
        double work;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double ms[K_COUNT] = {0};
    double work[K_COUNT] = {0};
    int64_t launches[K_COUNT] = {0};
};

static hipEvent_t get_event(TimingState *ts) {
    if (!ts->pool.empty()) {
        hipEvent_t e = ts->pool.back();
        ts->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void drain(TimingState *ts) {
    for (auto &p : ts->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
            ts->ms[p.kernel] += ms;
        ts->launches[p.kernel] += 1;
        if (p.work > 0) ts->work[p.kernel] += p.work;
        ts->pool.push_back(p.a);
        ts->pool.push_back(p.b);
    }
    ts->pending.clear();
}

TimedLaunch::TimedLaunch(pg_ctx *c, int k, double w) : ctx(c), kernel(k), work(w) {
    if (!ctx->timing) return;
    TimingState *ts = (TimingState *)ctx->timing_state;
    if (ts->pending.size() > 4096) drain(ts);
    a = get_event(ts);
    b = get_event(ts);
    if (a) (void)hipEventRecord(a, ctx->stream);
}

TimedLaunch::~TimedLaunch() {
    if (!ctx->timing || !a || !b) return;
    TimingState *ts = (TimingState *)ctx->timing_state;
    (void)hipEventRecord(b, ctx->stream);
    ts->pending.push_back({a, b, kernel, work});
}

void ctx_add_work(pg_ctx *ctx, int kernel, double work) {
    if (!ctx->timing) return;
    ((TimingState *)ctx->timing_state)->work[kernel] += work;
}

// ---------------------------------------------------------------------------
// exclusive prefix sum of int32 counts into int64 offsets (n + 1 outputs)
// three passes over 1024-element tiles; integer, so the order cannot matter
// ---------------------------------------------------------------------------
constexpr int SCAN_TILE = 1024;

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *__restrict__ in, int64_t n,
                                                    int64_t *__restrict__ tile_sum) {
    __shared__ int64_t s[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int i = threadIdx.x; i < SCAN_TILE; i += 256)
        if (base + i < n) acc += in[base + i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_scan_sums(int64_t *__restrict__ tile_sum, int64_t ntiles) {
    // single workgroup: exclusive scan of the tile sums in place
    __shared__ int64_t s[256];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += 256) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < ntiles ? tile_sum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + s[threadIdx.x] - v;
        carry += s[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                    const int64_t *__restrict__ tile_off,
                                                    int64_t *__restrict__ out) {
    __shared__ int64_t s[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // each thread owns 4 consecutive elements
    int64_t v[4], loc = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + threadIdx.x * 4 + j;
        v[j] = i < n ? in[i] : 0;
        loc += v[j];
    }
    s[threadIdx.x] = loc;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = tile_off[blockIdx.x] + s[threadIdx.x] - loc;
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + threadIdx.x * 4 + j;
        if (i < n) out[i] = run;
        run += v[j];
        if (i == n - 1) out[n] = run;
    }
}

size_t scan_tmp_bytes(int64_t n) { return sizeof(int64_t) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1); }

pg_status scan_exclusive(pg_ctx *ctx, const int32_t *in, int64_t *out, int64_t n, void *tmp) {
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *ts = (int64_t *)tmp;
    if (n == 0) {
        PG_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), ctx->stream));
        return PG_OK;
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, ctx->stream, in, n, ts);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, ctx->stream, ts, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(256), 0, ctx->stream, in, n, ts, out);
    PG_HIP(hipGetLastError());
    return PG_OK;
}

static const char *kNames[K_COUNT] = {"join", "merge", "init", "sample", "prune", "search", "exact_knn", "connect"};

}  // namespace pgi

using namespace pgi;

extern "C" int pg_version(void) { return 100; }

extern "C" const char *pg_last_error(void) { return g_err; }

extern "C" pg_status pg_ctx_create(int device, void *hip_stream, pg_ctx **out) {
    if (!out) {
        set_error("pg_ctx_create: out is NULL");
        return PG_EINVAL;
    }
    int count = 0;
    PG_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) {
        set_error("pg_ctx_create: device %d not in [0, %d)", device, count);
        return PG_EINVAL;
    }
    PG_HIP(hipSetDevice(device));
    int ncu = 0;
    PG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    pg_ctx *c = new (std::nothrow) pg_ctx;
    if (!c) {
        set_error("pg_ctx_create: out of host memory");
        return PG_ENOMEM;
    }
    c->device = device;
    c->num_cu = ncu;
    c->stream = (hipStream_t)hip_stream;
    c->timing = false;
    c->timing_state = new (std::nothrow) TimingState;
    if (!c->timing_state) {
        delete c;
        set_error("pg_ctx_create: out of host memory");
        return PG_ENOMEM;
    }
    *out = c;
    return PG_OK;
}

extern "C" pg_status pg_ctx_destroy(pg_ctx *ctx) {
    if (!ctx) return PG_OK;
    TimingState *ts = (TimingState *)ctx->timing_state;
    if (ts) {
        drain(ts);
        for (hipEvent_t e : ts->pool) (void)hipEventDestroy(e);
        delete ts;
    }
    delete ctx;
    return PG_OK;
}

extern "C" pg_status pg_ctx_set_timing(pg_ctx *ctx, int enable) {
    if (!ctx) {
        set_error("pg_ctx_set_timing: NULL context");
        return PG_EINVAL;
    }
    ctx->timing = enable != 0;
    return PG_OK;
}

extern "C" pg_status pg_ctx_reset_timing(pg_ctx *ctx) {
    if (!ctx) {
        set_error("pg_ctx_reset_timing: NULL context");
        return PG_EINVAL;
    }
    TimingState *ts = (TimingState *)ctx->timing_state;
    drain(ts);
    for (int i = 0; i < K_COUNT; ++i) {
        ts->ms[i] = 0;
        ts->work[i] = 0;
        ts->launches[i] = 0;
    }
    return PG_OK;
}

extern "C" pg_status pg_ctx_kernel_time(pg_ctx *ctx, const char *name, double *total_ms,
                                        int64_t *launches, double *work) {
    if (!ctx || !name) {
        set_error("pg_ctx_kernel_time: NULL argument");
        return PG_EINVAL;
    }
    int k = -1;
    for (int i = 0; i < K_COUNT; ++i)
        if (strcmp(name, kNames[i]) == 0) k = i;
    if (k < 0) {
        set_error("pg_ctx_kernel_time: unknown kernel name '%s'", name);
        return PG_EINVAL;
    }
    TimingState *ts = (TimingState *)ctx->timing_state;
    drain(ts);
    if (total_ms) *total_ms = ts->ms[k];
    if (launches) *launches = ts->launches[k];
    if (work) *work = ts->work[k];
    return PG_OK;
}
