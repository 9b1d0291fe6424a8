// Input generator for the served GNN aggregation requests (not part of the
// product path): the feature matrix X of one request, n x f with nk kept
// columns, dense in those columns with values in (0, 1].  Built in one pass
// so that a request's features can be made on the device when it is
// admitted.  Bit-identical to the host generator: value e (row-major over
// the n x nk block) is k / 2^24 with k = (SplitMix64(4 e + off) >> 40) + 1,
// SplitMix64 being the finaliser of Steele, Lea and Flood (OOPSLA 2014)
// applied to its argument plus the golden-ratio increment.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_gnn_features(int64_t n, int nk,
                                                      const int32_t *__restrict__ kept,
                                                      uint64_t off, int64_t *__restrict__ rpt,
                                                      int32_t *__restrict__ col,
                                                      float *__restrict__ val) {
    const int64_t total = n * nk;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the column slot e % nk, kept up to date by adding the stride's
    // remainder instead of a 64-bit division per entry
    const int sr = (int)(stride % nk);
    int r = (int)(e0 % nk);
    for (int64_t e = e0; e < total; e += stride) {
        const uint64_t h = splitmix64((uint64_t)e * 4u + off);
        col[e] = kept[r];
        val[e] = (float)((h >> 40) + 1) * (1.0f / 16777216.0f);
        r += sr;
        if (r >= nk) r -= nk;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
        rpt[i] = i * nk;
}

}  // namespace

extern "C" int gen_gnn_features(int64_t n, int32_t nk, const int32_t *kept, uint64_t off,
                                int64_t *rpt, int32_t *col, float *val, void *stream) {
    if (n < 0 || nk <= 0 || !kept || !rpt || (n > 0 && (!col || !val))) return 1;
    const int64_t work = n * nk > n + 1 ? n * nk : n + 1;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_gnn_features, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       n, nk, kept, off, rpt, col, val);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
