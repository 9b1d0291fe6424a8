// Device steps of the applications that chain products (paper Section V):
//
//  * graph contraction (Algorithm 7): the transposed selector S^T, built from
//    the cluster labels by a counting sort (k rows, one entry per vertex);
//  * Markov clustering (Algorithm 6): the step after each expansion, on
//    row-stochastic storage (the transpose of the column-stochastic matrix,
//    so the paper's column operations are row operations here): raise every
//    entry to `power`, divide each row by its sum, drop entries below theta
//    (strictly), keep only the k largest (optional), divide each row by the
//    sum of what is kept.  Two passes: the first counts what each row keeps
//    (and records the row's two sums and its top-k selection), the second
//    writes the kept entries in their original order.  Then the change
//    between successive iterates (the convergence test) and the connected
//    components of the final matrix (the cluster interpretation).
#include "common.hpp"
#include "dev.hpp"

namespace spg {

__global__ void k_label_count(const int32_t *__restrict__ labels, int64_t n, int64_t k,
                              int64_t *__restrict__ cnt, int *__restrict__ err) {
    const int64_t v = lin_block() * blockDim.x + threadIdx.x;
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
    const int64_t v = lin_block() * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t l = labels[v];
    if (l < 0 || l >= k) return;
    const int64_t pos = (int64_t)atomicAdd((unsigned long long *)&cursor[l], 1ull);
    col[pos] = (int32_t)v;
    val[pos] = 1.f;
}

__device__ __forceinline__ float mcl_pow(float x, float p) {
    return p == 1.f ? x : p == 2.f ? x * x : __powf(x, p);
}

// Top-k of a row: among the entries kept by the threshold, the k largest
// input values (inputs are nonnegative, and x -> x^p / sum is increasing,
// so ordering the inputs orders the normalised values without rounding);
// equal values are taken in column (storage) order.  Radix selection on the
// FP32 bit patterns, 8 bits per pass, with a 256-bucket LDS histogram: the
// result is the k-th largest pattern `thr` and how many entries equal to it
// are kept (`ties`).  One wave (= the whole workgroup) per row.
__device__ void mcl_select(const float *__restrict__ val, int64_t s, int64_t e, float inv,
                           float power, float theta, int k, uint32_t *hist, uint32_t &thr,
                           int &ties) {
    const int lane = threadIdx.x;
    uint32_t prefix = 0, mask = 0;
    int need = k;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = lane; b < 256; b += 64) hist[b] = 0;
        __syncthreads();
        for (int64_t j = s + lane; j < e; j += 64) {
            const float x = val[j];
            const uint32_t key = __float_as_uint(x);
            if (mcl_pow(x, power) * inv >= theta && (key & mask) == prefix)
                atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        // lane l holds buckets 255 - 4l .. 252 - 4l (descending order)
        uint32_t h[4], tot = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            h[q] = hist[255 - 4 * lane - q];
            tot += h[q];
        }
        uint32_t incl = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        uint32_t above = incl - tot;
        int found = -1;
        uint32_t above_found = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (found < 0 && above < (uint32_t)need && above + h[q] >= (uint32_t)need) {
                found = 255 - 4 * lane - q;
                above_found = above;
            }
            above += h[q];
        }
        const unsigned long long bal = __ballot(found >= 0);
        const int src = __ffsll((long long)bal) - 1;
        const int b = __shfl(found, src, 64);
        need -= (int)__shfl(above_found, src, 64);
        prefix |= (uint32_t)b << shift;
        mask |= 255u << shift;
        __syncthreads();
    }
    thr = prefix;
    ties = need;
}

// One wave per row.  rowsum[2 r] = sum of x^p, rowsum[2 r + 1] = sum of the
// kept normalised entries; keep[r] = kept count; with k > 0 and more than k
// entries above the threshold, sel[2 r] / sel[2 r + 1] = the selection's
// threshold pattern and kept ties (else sel[2 r + 1] = -1: no selection).
__global__ __launch_bounds__(64) void k_mcl_count(int64_t m, const int64_t *__restrict__ rpt,
                                                  const float *__restrict__ val, float power,
                                                  float theta, int k,
                                                  float *__restrict__ rowsum,
                                                  int64_t *__restrict__ keep,
                                                  int32_t *__restrict__ sel) {
    __shared__ uint32_t hist[256];
    const int64_t r = lin_block();
    const int lane = threadIdx.x;
    if (r >= m) return;
    const int64_t s = rpt[r], e = rpt[r + 1];
    float sum = 0.f;
    for (int64_t j = s + lane; j < e; j += 64) sum += mcl_pow(val[j], power);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    float ksum = 0.f;
    int64_t kc = 0;
    const float inv = sum > 0.f ? 1.f / sum : 0.f;
    if (sum > 0.f) {
        for (int64_t j = s + lane; j < e; j += 64) {
            const float y = mcl_pow(val[j], power) * inv;
            if (y >= theta) {
                ksum += y;
                ++kc;
            }
        }
    }
    // a row of zeros keeps nothing (all entries are below theta)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ksum += __shfl_xor(ksum, off, 64);
        kc += __shfl_xor(kc, off, 64);
    }
    int32_t thr_out = 0, ties_out = -1;
    if (k > 0 && kc > k) {   // wave-uniform
        uint32_t thr;
        int ties;
        mcl_select(val, s, e, inv, power, theta, k, hist, thr, ties);
        // kept sum: entries above the threshold pattern plus `ties` equal ones
        float above = 0.f;
        for (int64_t j = s + lane; j < e; j += 64) {
            const float x = val[j];
            const float y = mcl_pow(x, power) * inv;
            if (y >= theta && __float_as_uint(x) > thr) above += y;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) above += __shfl_xor(above, off, 64);
        ksum = above + (float)ties * (mcl_pow(__uint_as_float(thr), power) * inv);
        kc = k;
        thr_out = (int32_t)thr;
        ties_out = ties;
    }
    if (lane == 0) {
        rowsum[2 * r] = sum;
        rowsum[2 * r + 1] = ksum;
        keep[r] = kc;
        sel[2 * r] = thr_out;
        sel[2 * r + 1] = ties_out;
    }
}

__global__ __launch_bounds__(256) void k_mcl_write(int64_t m, const int64_t *__restrict__ rpt,
                                                   const int32_t *__restrict__ col,
                                                   const float *__restrict__ val, float power,
                                                   float theta,
                                                   const float *__restrict__ rowsum,
                                                   const int32_t *__restrict__ sel,
                                                   const int64_t *__restrict__ out_rpt,
                                                   int32_t *__restrict__ out_col,
                                                   float *__restrict__ out_val) {
    const int64_t r = lin_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    const float sum = rowsum[2 * r], ksum = rowsum[2 * r + 1];
    if (!(sum > 0.f)) return;
    const float inv = 1.f / sum, kinv = ksum > 0.f ? 1.f / ksum : 0.f;
    const uint32_t thr = (uint32_t)sel[2 * r];
    const int ties = sel[2 * r + 1];  // -1: no top-k selection in this row
    const int64_t s = rpt[r], e = rpt[r + 1];
    int64_t o = out_rpt[r];
    const int64_t oend = out_rpt[r + 1];
    int tie_seen = 0;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t jb = s; jb < e; jb += 64) {
        const int64_t j = jb + lane;
        float y = 0.f;
        bool kp = false, tie = false;
        if (j < e) {
            const float x = val[j];
            y = mcl_pow(x, power) * inv;
            kp = y >= theta;
            if (kp && ties >= 0) {
                const uint32_t key = __float_as_uint(x);
                tie = key == thr;
                kp = key > thr;
            }
        }
        if (ties >= 0) {   // the first `ties` entries equal to the threshold
            const unsigned long long tb = __ballot(tie);
            if (tie && tie_seen + __popcll(tb & lt) < ties) kp = true;
            tie_seen += __popcll(tb);
        }
        const unsigned long long bal = __ballot(kp);
        const int64_t at = o + __popcll(bal & lt);
        if (kp && at < oend) {
            out_col[at] = col[j];
            out_val[at] = y * kinv;
        }
        o += __popcll(bal);
    }
}

// Change between successive iterates: the largest |a_ij - b_ij| over the
// union of both patterns (rows sorted by column), in FP64 from the FP32
// entries (the difference of two FP32 numbers is exact in FP64).  One thread
// per stored entry of either matrix; its row by binary search of the row
// pointers, its partner by binary search of the other row.  Nonnegative
// doubles order like their bit patterns, so the maximum is an integer
// atomicMax.
__device__ __forceinline__ int64_t row_of(const int64_t *__restrict__ rpt, int64_t m, int64_t j) {
    int64_t lo = 0, hi = m;  // last r with rpt[r] <= j
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rpt[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_mcl_change(int64_t m, const int64_t *__restrict__ rpt_a,
                             const int32_t *__restrict__ col_a, const float *__restrict__ val_a,
                             int64_t nnz_a, const int64_t *__restrict__ rpt_b,
                             const int32_t *__restrict__ col_b, const float *__restrict__ val_b,
                             int64_t nnz_b, unsigned long long *__restrict__ out) {
    const int64_t t = lin_block() * blockDim.x + threadIdx.x;
    if (t >= nnz_a + nnz_b) return;
    const bool first = t < nnz_a;
    const int64_t j = first ? t : t - nnz_a;
    const int64_t *rp = first ? rpt_a : rpt_b;
    const int32_t *cp = first ? col_a : col_b;
    const float *vp = first ? val_a : val_b;
    const int64_t *rq = first ? rpt_b : rpt_a;
    const int32_t *cq = first ? col_b : col_a;
    const float *vq = first ? val_b : val_a;
    const int64_t r = row_of(rp, m, j);
    const int32_t c = cp[j];
    int64_t lo = rq[r], hi = rq[r + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cq[mid] < c) lo = mid + 1; else hi = mid;
    }
    const bool both = lo < rq[r + 1] && cq[lo] == c;
    if (both && !first) return;  // counted once, from A's side
    const double d = fabs((double)vp[j] - (both ? (double)vq[lo] : 0.0));
    if (d > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(d));
}

// Connected components of the undirected graph of a square pattern (cluster
// interpretation): every vertex points at a parent of smaller index (at
// first itself); the hook pass, one thread per stored entry (i, j), finds
// the roots of i and j and, when they differ, lowers the larger root's
// parent to the smaller root; the compress pass points every vertex at its
// root.  Parents only decrease, so roots stay roots of their own component
// and the final root of a component is its smallest vertex.
__device__ __forceinline__ int32_t cc_root(const int32_t *lab, int32_t x) {
    int32_t p = lab[x];
    while (p != x) {
        x = p;
        p = lab[x];
    }
    return x;
}

__global__ void k_cc_init(int64_t n, int32_t *__restrict__ lab) {
    const int64_t v = lin_block() * blockDim.x + threadIdx.x;
    if (v < n) lab[v] = (int32_t)v;
}

__global__ void k_cc_hook(int64_t n, const int64_t *__restrict__ rpt,
                          const int32_t *__restrict__ col, int64_t nnz, int32_t *lab,
                          int *__restrict__ changed) {
    const int64_t j = lin_block() * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    const int32_t u = (int32_t)row_of(rpt, n, j);
    const int32_t v = col[j];
    const int32_t ru = cc_root(lab, u), rv = cc_root(lab, v);
    if (ru == rv) return;
    const int32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
    atomicMin(&lab[hi], lo);
    *changed = 1;
}

__global__ void k_cc_compress(int64_t n, int32_t *lab) {
    const int64_t v = lin_block() * blockDim.x + threadIdx.x;
    if (v < n) lab[v] = cc_root(lab, (int32_t)v);
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    const int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Inverse transform sampling (matrix-based bulk sampling, paper Section
// V-C): one thread per draw (row r, draw t).  The row's weights are summed
// in storage order in FP32 (S), x = u[r s + t] * S, and the draw is the
// column of the first entry whose running FP32 sum exceeds x (the last
// entry if rounding leaves none).  Sequential sums make the choice exactly
// reproducible.  A row of zero total weight (or no entries) draws
// `self[r]`, the row's own vertex.
__global__ void k_its_sample(int64_t m, int s, const int64_t *__restrict__ rpt,
                             const int32_t *__restrict__ col, const float *__restrict__ val,
                             const float *__restrict__ u, const int32_t *__restrict__ self,
                             int32_t *__restrict__ out) {
    const int64_t q = lin_block() * blockDim.x + threadIdx.x;
    if (q >= m * s) return;
    const int64_t r = q / s;
    const int64_t a = rpt[r], b = rpt[r + 1];
    float tot = 0.f;
    for (int64_t j = a; j < b; ++j) tot += val[j];
    if (!(tot > 0.f)) {
        out[q] = self[r];
        return;
    }
    const float x = u[q] * tot;
    float acc = 0.f;
    int32_t pick = col[b - 1];
    for (int64_t j = a; j < b; ++j) {
        acc += val[j];
        if (acc > x) {
            pick = col[j];
            break;
        }
    }
    out[q] = pick;
}

void launch_its_sample(int64_t m, int s, const int64_t *rpt, const int32_t *col, const float *val,
                       const float *u, const int32_t *self, int32_t *out, hipStream_t st) {
    const int64_t n = m * s;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_its_sample, grid1d(((n + 255) / 256), 256), dim3(256), 0, st, m, s,
                       rpt, col, val, u, self, out);
}

void launch_selector_t(const int32_t *labels, int64_t n, int64_t k, int64_t *rpt, int32_t *col,
                       float *val, int64_t *work, void *scan_tmp, int *err, hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    // work[0..k) = label counts; their exclusive scan (k + 1 entries) is rpt,
    // then work becomes the per-row write cursor
    launch_fill_i64(work, k, 0, s);
    if (n > 0)
        hipLaunchKernelGGL(k_label_count, grid1d(nb, 256), dim3(256), 0, s, labels, n, k, work, err);
    launch_scan_i64(work, rpt, k, scan_tmp, s);
    (void)hipMemcpyAsync(work, rpt, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, s);
    if (n > 0)
        hipLaunchKernelGGL(k_label_scatter, grid1d(nb, 256), dim3(256), 0, s, labels, n, k, work, col,
                           val);
}

void launch_mcl_count(int64_t m, const int64_t *rpt, const float *val, float power, float theta,
                      int k, float *rowsum, int64_t *keep, int32_t *sel, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_mcl_count, grid1d(m, 64), dim3(64), 0, s, m, rpt, val, power, theta,
                       k, rowsum, keep, sel);
}

void launch_mcl_write(int64_t m, const int64_t *rpt, const int32_t *col, const float *val,
                      float power, float theta, const float *rowsum, const int32_t *sel,
                      const int64_t *out_rpt, int32_t *out_col, float *out_val, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_mcl_write, grid1d(((m + 3) / 4), 256), dim3(256), 0, s, m, rpt, col,
                       val, power, theta, rowsum, sel, out_rpt, out_col, out_val);
}

void launch_mcl_change(int64_t m, const int64_t *rpt_a, const int32_t *col_a, const float *val_a,
                       int64_t nnz_a, const int64_t *rpt_b, const int32_t *col_b,
                       const float *val_b, int64_t nnz_b, double *out, hipStream_t s) {
    launch_fill_i64((int64_t *)out, 1, 0, s);
    const int64_t t = nnz_a + nnz_b;
    if (m <= 0 || t <= 0) return;
    hipLaunchKernelGGL(k_mcl_change, grid1d(((t + 255) / 256), 256), dim3(256), 0, s, m, rpt_a,
                       col_a, val_a, nnz_a, rpt_b, col_b, val_b, nnz_b,
                       (unsigned long long *)out);
}

void launch_cc_init(int64_t n, int32_t *lab, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cc_init, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, n, lab);
}

void launch_cc_round(int64_t n, const int64_t *rpt, const int32_t *col, int64_t nnz, int32_t *lab,
                     int *changed, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)changed, 1, 0);
    if (nnz > 0)
        hipLaunchKernelGGL(k_cc_hook, grid1d(((nnz + 255) / 256), 256), dim3(256), 0, s, n,
                           rpt, col, nnz, lab, changed);
    if (n > 0)
        hipLaunchKernelGGL(k_cc_compress, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, n,
                           lab);
}

}  // namespace spg
