// Thread-per-row kernels for the smallest rows, in the manner of the paper's
// AIA kernel (Section IV-D): one thread processes one row of A, and the
// two-level indirection rpt_B[col_A[j]], rpt_B[col_A[j] + 1] is resolved
// ahead of time into one sequential stream per row.  On the paper's system a
// near-memory engine answers a ranged indirect request with that stream; here
// a gather kernel builds it in HBM (one pass over the group's A nonzeros:
// each entry holds the B range of one A nonzero and, for the numeric phase,
// the A value), and each workgroup stages the stream of its 64 rows in LDS
// with coalesced loads before the threads walk it.
//
// Each thread keeps a private table of T slots in LDS, slot h of lane l at
// h * 64 + l so that lanes probing the same slot index hit distinct banks.
// Linear probing with Knuth's multiplicative hash; no atomics are needed
// because no other thread touches the table.  The numeric kernel compacts
// the occupied slots and writes them in column order (rank sort).
#include "common.hpp"
#include "dev.hpp"

namespace spg {

constexpr int kRtStage = 512;   // staged stream entries per 64-row workgroup

__global__ void k_rt_lens(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                          int64_t count, int64_t *__restrict__ lens) {
    const int64_t t = lin_block() * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint64_t e = items[t];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    lens[t] = P.rptA[i + 1] - P.rptA[i];
}

// The "ranged indirect" gather: for every row of the group, in map order, the
// B ranges of its A nonzeros (and their A values) as one contiguous segment.
__global__ void k_rt_gather(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                            int64_t count, const int64_t *__restrict__ off,
                            RangeEnt *__restrict__ stream, int values) {
    const int64_t t = lin_block() * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint64_t e = items[t];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t a0 = P.rptA[i], a1 = P.rptA[i + 1];
    RangeEnt *o = stream + off[t];
    for (int64_t j = a0; j < a1; ++j) {
        const int c = P.colA[j];
        const int64_t b0 = P.rptB[c];
        RangeEnt r;
        r.b0 = b0;
        r.len = (int32_t)(P.rptB[c + 1] - b0);
        r.a = values ? P.valA[j] : 0.f;
        o[j - a0] = r;
    }
}

// Stages the block's part of the stream in LDS when it fits; returns whether
// it did (block-uniform).
__device__ __forceinline__ bool rt_stage(const RangeEnt *__restrict__ stream,
                                         const int64_t *__restrict__ off, int64_t count,
                                         RangeEnt *stage, int64_t &s0) {
    const int64_t t0 = lin_block() * 64;
    const int64_t tl = t0 + 64 < count ? t0 + 64 : count;
    s0 = off[t0];
    const int64_t n = off[tl] - s0;
    if (n > kRtStage) return false;
    for (int64_t q = threadIdx.x; q < n; q += 64) stage[q] = stream[s0 + q];
    return true;
}

template <int T>
__global__ __launch_bounds__(64) void k_sym_rowthread(const ProdDev *__restrict__ prods,
                                                      const uint64_t *__restrict__ items,
                                                      int64_t count,
                                                      const int64_t *__restrict__ off,
                                                      const RangeEnt *__restrict__ stream,
                                                      int64_t *__restrict__ row_nnz,
                                                      int *__restrict__ err) {
    constexpr int LOG2T = __builtin_ctz(T);
    __shared__ int keys[T * 64];
    __shared__ RangeEnt stage[kRtStage];
    if (lin_block() * 64 >= count) return;  // block-uniform, before the barrier
    const int lane = threadIdx.x;
    for (int h = 0; h < T; ++h) keys[h * 64 + lane] = kEmptyKey;
    int64_t s0 = 0;
    const bool staged = rt_stage(stream, off, count, stage, s0);
    __syncthreads();
    const int64_t t = lin_block() * 64 + lane;
    if (t >= count) return;
    const uint64_t e = items[t];
    const ProdDev &P = prods[item_prod(e)];
    int cnt = 0;
    for (int64_t q = off[t]; q < off[t + 1]; ++q) {
        const RangeEnt r = staged ? stage[q - s0] : stream[q];
        for (int64_t p = r.b0; p < r.b0 + r.len; ++p) {
            const int c = P.colB[p];
            uint32_t h = hash_slot(c, LOG2T);
            int probe = 0;
            for (; probe < T; ++probe) {
                const int cur = keys[h * 64 + lane];
                if (cur == c) break;
                if (cur == kEmptyKey) {
                    keys[h * 64 + lane] = c;
                    ++cnt;
                    break;
                }
                h = (h + 1) & (T - 1);
            }
            if (probe == T) atomicOr(err, kErrProbe);
        }
    }
    row_nnz[P.row_base + item_row(e)] = cnt;
}

template <int T>
__global__ __launch_bounds__(64) void k_num_rowthread(const ProdDev *__restrict__ prods,
                                                      const uint64_t *__restrict__ items,
                                                      int64_t count,
                                                      const int64_t *__restrict__ off,
                                                      const RangeEnt *__restrict__ stream,
                                                      const int64_t *__restrict__ rptv,
                                                      int *__restrict__ err) {
    constexpr int LOG2T = __builtin_ctz(T);
    __shared__ int keys[T * 64];
    __shared__ float vals[T * 64];
    __shared__ RangeEnt stage[kRtStage];
    if (lin_block() * 64 >= count) return;  // block-uniform, before the barrier
    const int lane = threadIdx.x;
    for (int h = 0; h < T; ++h) {
        keys[h * 64 + lane] = kEmptyKey;
        vals[h * 64 + lane] = 0.f;
    }
    int64_t s0 = 0;
    const bool staged = rt_stage(stream, off, count, stage, s0);
    __syncthreads();
    const int64_t t = lin_block() * 64 + lane;
    if (t >= count) return;
    const uint64_t e = items[t];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    for (int64_t q = off[t]; q < off[t + 1]; ++q) {
        const RangeEnt r = staged ? stage[q - s0] : stream[q];
        for (int64_t p = r.b0; p < r.b0 + r.len; ++p) {
            const int c = P.colB[p];
            const float v = r.a * P.valB[p];
            uint32_t h = hash_slot(c, LOG2T);
            int probe = 0;
            for (; probe < T; ++probe) {
                const int cur = keys[h * 64 + lane];
                if (cur == c) {
                    vals[h * 64 + lane] += v;
                    break;
                }
                if (cur == kEmptyKey) {
                    keys[h * 64 + lane] = c;
                    vals[h * 64 + lane] = v;
                    break;
                }
                h = (h + 1) & (T - 1);
            }
            if (probe == T) atomicOr(err, kErrProbe);
        }
    }
    // compact the occupied slots to the front (in place: the write index
    // never passes the read index), then rank sort by column
    int n = 0;
    for (int h = 0; h < T; ++h) {
        const int c = keys[h * 64 + lane];
        if (c != kEmptyKey) {
            keys[n * 64 + lane] = c;
            vals[n * 64 + lane] = vals[h * 64 + lane];
            ++n;
        }
    }
    const int64_t base = c_base(P, rptv, P.row_base + i);
    if ((int64_t)n != rptv[P.row_base + i + 1] - rptv[P.row_base + i]) {
        atomicOr(err, kErrCount);
        return;
    }
    for (int a = 0; a < n; ++a) {
        const int c = keys[a * 64 + lane];
        int rank = 0;
        for (int b = 0; b < n; ++b) rank += keys[b * 64 + lane] < c;
        P.colC[base + rank] = c;
        P.valC[base + rank] = vals[a * 64 + lane];
    }
}

void launch_rt_offsets(const ProdDev *prods, const uint64_t *items, int64_t count, int64_t *lens,
                       int64_t *off, void *scan_tmp, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_rt_lens, grid1d(((count + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, count, lens);
    launch_scan_i64(lens, off, count, scan_tmp, s);
}

void launch_rt_gather(const ProdDev *prods, const uint64_t *items, int64_t count,
                      const int64_t *off, RangeEnt *stream, bool values, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_rt_gather, grid1d(((count + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, count, off, stream, values ? 1 : 0);
}

void launch_sym_rowthread(const ProdDev *prods, const uint64_t *items, int64_t count,
                          const int64_t *off, const RangeEnt *stream, int64_t *row_nnz, int *err,
                          hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_sym_rowthread<kRtSlots>, grid1d(((count + 63) / 64), 64), dim3(64), 0,
                       s, prods, items, count, off, stream, row_nnz, err);
}

void launch_num_rowthread(const ProdDev *prods, const uint64_t *items, int64_t count,
                          const int64_t *off, const RangeEnt *stream, const int64_t *rptv,
                          int *err, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_num_rowthread<kRtSlots>, grid1d(((count + 63) / 64), 64), dim3(64), 0,
                       s, prods, items, count, off, stream, rptv, err);
}

}  // namespace spg
