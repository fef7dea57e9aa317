// hnsw.hip -- layer assignment of the global HNSW construction (the paper's
// Alg. 7, first step) for gfx950.
//
// Each node draws its highest layer the way HNSW does: l(u) =
// floor(-ln U(u) / ln M) with U(u) uniform in (0, 1] and M the out-degree
// limit.  The uniform draws are inputs.  The level is evaluated without a
// logarithm: l(u) is the number of i >= 1 with U(u) * M^i <= 1, where M^i
// is exact in double precision (an integer below 2^53) and the product is
// one correctly rounded multiplication, so every platform agrees on it.
// Levels stop at 31 and at the last i with M^i below 2^53.
#include "pg_common.h"

namespace pgi {

// levels stop here (U would have to be below M^-31)
constexpr int HNSW_MAX_LEVEL = 31;

__global__ void k_hnsw_levels(const double *__restrict__ U, int64_t n, double M, int32_t *__restrict__ lev,
                              unsigned int *__restrict__ top) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = U[i];
    int l = 0;
    double p = M;
    while (l < HNSW_MAX_LEVEL && u * p <= 1.0 && p < 9007199254740992.0) {
        ++l;
        p *= M;
    }
    lev[i] = l;
    atomicMax(top, (unsigned int)l);
}

}  // namespace pgi

using namespace pgi;

extern "C" pg_status pg_hnsw_levels(pg_ctx *ctx, const double *U, int64_t n, int32_t M, int32_t *levels,
                                    int32_t *max_level) {
    if (!ctx || !U || !levels || !max_level) {
        set_error("pg_hnsw_levels: NULL argument");
        return PG_EINVAL;
    }
    if (n < 1 || n >= (int64_t)1 << 31 || M < 2) {
        set_error("pg_hnsw_levels: need 1 <= n < 2^31 and M >= 2 (n=%lld M=%d)", (long long)n, M);
        return PG_EINVAL;
    }
    PG_HIP(hipMemsetAsync(max_level, 0, sizeof(int32_t), ctx->stream));
    hipLaunchKernelGGL(k_hnsw_levels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, U, n,
                       (double)M, levels, (unsigned int *)max_level);
    PG_HIP(hipGetLastError());
    return PG_OK;
}
