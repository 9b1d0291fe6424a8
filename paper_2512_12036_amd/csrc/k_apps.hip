// Device steps of the applications that chain products (paper Section V):
//
//  * graph contraction (Algorithm 7): the transposed selector S^T, built from
//    the cluster labels by a counting sort (k rows, one entry per vertex);
//  * Markov clustering (Algorithm 6): the step after each expansion, on
//    row-stochastic storage (the transpose of the column-stochastic matrix,
//    so the paper's column operations are row operations here): raise every
//    entry to `power`, divide each row by its sum, drop entries below theta
//    (strictly), divide each row by the sum of what is kept.  Two passes: the
//    first counts what each row keeps (and records the row's two sums), the
//    second writes the kept entries in their original order.
#include "common.hpp"
#include "dev.hpp"

namespace spg {

__global__ void k_label_count(const int32_t *__restrict__ labels, int64_t n, int64_t k,
                              int64_t *__restrict__ cnt, int *__restrict__ err) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    if (l < 0 || l >= k) {
        atomicOr(err, kErrRow);
        return;
    }
    atomicAdd((unsigned long long *)&cnt[l], 1ull);
}

__global__ void k_label_scatter(const int32_t *__restrict__ labels, int64_t n, int64_t k,
                                int64_t *__restrict__ cursor, int32_t *__restrict__ col,
                                float *__restrict__ val) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    if (l < 0 || l >= k) return;
    const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&cursor[l], 1ull);
    col[pos] = (int32_t)v;
    val[pos] = 1.f;
}

__device__ __forceinline__ float mcl_pow(float x, float p) {
    return p == 2.f ? x * x : __powf(x, p);
}

// One wave per row.  rowsum[2 r] = sum of x^p, rowsum[2 r + 1] = sum of the
// kept normalised entries; keep[r] = kept count.
__global__ __launch_bounds__(256) void k_mcl_count(int64_t m, const int64_t *__restrict__ rpt,
                                                   const float *__restrict__ val, float power,
                                                   float theta, float *__restrict__ rowsum,
                                                   int64_t *__restrict__ keep) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    const int64_t s = rpt[r], e = rpt[r + 1];
    float sum = 0.f;
    for (int64_t j = s + lane; j < e; j += 64) sum += mcl_pow(val[j], power);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    float ksum = 0.f;
    int64_t kc = 0;
    if (sum > 0.f) {
        const float inv = 1.f / sum;
        for (int64_t j = s + lane; j < e; j += 64) {
            const float y = mcl_pow(val[j], power) * inv;
            if (y >= theta) {
                ksum += y;
                ++kc;
            }
        }
    } else {
        kc = 0;  // a row of zeros keeps nothing (all entries are below theta)
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ksum += __shfl_xor(ksum, off, 64);
        kc += __shfl_xor(kc, off, 64);
    }
    if (lane == 0) {
        rowsum[2 * r] = sum;
        rowsum[2 * r + 1] = ksum;
        keep[r] = kc;
    }
}

__global__ __launch_bounds__(256) void k_mcl_write(int64_t m, const int64_t *__restrict__ rpt,
                                                   const int32_t *__restrict__ col,
                                                   const float *__restrict__ val, float power,
                                                   float theta,
                                                   const float *__restrict__ rowsum,
                                                   const int64_t *__restrict__ out_rpt,
                                                   int32_t *__restrict__ out_col,
                                                   float *__restrict__ out_val) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    const float sum = rowsum[2 * r], ksum = rowsum[2 * r + 1];
    if (!(sum > 0.f)) return;
    const float inv = 1.f / sum, kinv = ksum > 0.f ? 1.f / ksum : 0.f;
    const int64_t s = rpt[r], e = rpt[r + 1];
    int64_t o = out_rpt[r];
    const int64_t oend = out_rpt[r + 1];
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t jb = s; jb < e; jb += 64) {
        const int64_t j = jb + lane;
        float y = 0.f;
        bool k = false;
        if (j < e) {
            y = mcl_pow(val[j], power) * inv;
            k = y >= theta;
        }
        const unsigned long long bal = __ballot(k);
        const int64_t at = o + __popcll(bal & lt);
        if (k && at < oend) {
            out_col[at] = col[j];
            out_val[at] = y * kinv;
        }
        o += __popcll(bal);
    }
}

void launch_selector_t(const int32_t *labels, int64_t n, int64_t k, int64_t *rpt, int32_t *col,
                       float *val, int64_t *work, void *scan_tmp, int *err, hipStream_t s) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    // work[0..k) = label counts; their exclusive scan (k + 1 entries) is rpt,
    // then work becomes the per-row write cursor
    launch_fill_i64(work, k, 0, s);
    if (n > 0)
        hipLaunchKernelGGL(k_label_count, dim3(nb), dim3(256), 0, s, labels, n, k, work, err);
    launch_scan_i64(work, rpt, k, scan_tmp, s);
    (void)hipMemcpyAsync(work, rpt, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, s);
    if (n > 0)
        hipLaunchKernelGGL(k_label_scatter, dim3(nb), dim3(256), 0, s, labels, n, k, work, col,
                           val);
}

void launch_mcl_count(int64_t m, const int64_t *rpt, const float *val, float power, float theta,
                      float *rowsum, int64_t *keep, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_mcl_count, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, m, rpt, val,
                       power, theta, rowsum, keep);
}

void launch_mcl_write(int64_t m, const int64_t *rpt, const int32_t *col, const float *val,
                      float power, float theta, const float *rowsum, const int64_t *out_rpt,
                      int32_t *out_col, float *out_val, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_mcl_write, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, m, rpt, col,
                       val, power, theta, rowsum, out_rpt, out_col, out_val);
}

}  // namespace spg
