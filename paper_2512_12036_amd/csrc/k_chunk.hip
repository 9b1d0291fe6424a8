// Column-chunked kernels for the heaviest rows (group 7).
//
// Paper Section III-C sends rows whose table does not fit in shared memory
// to a global-memory table.  On gfx950 these rows are instead cut into column
// chunks of W columns (W * nch >= n, nch a multiple of 8) and every (row,
// chunk) pair gets one workgroup with an LDS-resident structure covering the
// chunk's columns directly (no hashing, no probing):
//   * symbolic: a W-bit bitmap; the chunk's distinct count is its popcount;
//   * numeric : a W-float dense accumulator plus the W-bit occupancy bitmap
//     (so explicit zeros from cancellation are kept); the chunk is emitted in
//     column order straight from the bitmap, so these rows need no sort.
// Chunk c of every row lands on the workgroup index c (mod 8), i.e. on
// accelerator die c mod 8, so each die's L2 only ever holds the slab of B
// columns of its chunks.
//
// With B's rows sorted, the sub-range of B row k that falls into chunk c is
// precomputed once per (A nonzero, chunk) by k_split (binary searches) and
// reused by both phases; with unsorted B rows every chunk scans whole rows and
// filters, which is correct but nch times the gather traffic.
#include "common.hpp"

namespace spg {

__device__ __forceinline__ int64_t upper_index(const int64_t *__restrict__ base, int64_t n,
                                               int64_t x) {
    // largest h in [0, n) with base[h] <= x (base non-decreasing, base[0] <= x)
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

template <int NT>
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *wsum, int64_t &total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        int64_t x = wsum[i];
        if (i < w) before += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return before + incl - v;
}

__global__ void k_heavy_prep(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                             int64_t nh, int64_t *__restrict__ alen, int64_t *__restrict__ splitlen,
                             int64_t *__restrict__ nchv) {
    int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nh) return;
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t a = P.rptA[i + 1] - P.rptA[i];
    alen[h] = a;
    splitlen[h] = a * (P.nch + 1);
    nchv[h] = P.nch;
}

__global__ void k_dense_prep(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                             int64_t nd, int64_t *__restrict__ nchv) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nd) return;
    nchv[d] = prods[item_prod(items[d])].nch;
}

// One thread per nonzero of a group-7 row: positions of the chunk bounds
// c * W (c = 0..nch) inside the nonzero's B row, relative to the row start.
__global__ __launch_bounds__(256) void k_split(const ProdDev *__restrict__ prods,
                                                const uint64_t *__restrict__ items, int64_t nh,
                                                const int64_t *__restrict__ aoff,
                                                const int64_t *__restrict__ soff,
                                                int64_t total_alen, int32_t *__restrict__ split) {
    const int64_t jj = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (jj >= total_alen) return;
    const int64_t h = upper_index(aoff, nh, jj);
    const int64_t jl = jj - aoff[h];
    const int64_t alen = aoff[h + 1] - aoff[h];
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int k = P.colA[P.rptA[i] + jl];
    const int64_t b0 = P.rptB[k], b1 = P.rptB[k + 1];
    int32_t *sp = split + soff[h] + jl;
    const int nch = P.nch;
    sp[0] = 0;
    sp[(int64_t)nch * alen] = (int32_t)(b1 - b0);
    if (!P.b_sorted) return;  // filtered scans: bounds unused
    int64_t lo = b0;
    for (int c = 1; c < nch; ++c) {
        const int bound = c * P.W;
        int64_t l = lo, r = b1;  // first index in [lo, b1) with col >= bound
        while (l < r) {
            int64_t mid = (l + r) >> 1;
            if (P.colB[mid] < bound) l = mid + 1; else r = mid;
        }
        sp[(int64_t)c * alen] = (int32_t)(l - b0);
        lo = l;
    }
}

// Stages the chunk sub-ranges of a batch of A nonzeros and enumerates their
// products flat over the workgroup.  f(col, a_value, b_index).
template <int WG, bool VALUES, typename F>
__device__ __forceinline__ void chunk_products(const ProdDev &P, int64_t a0, int64_t a1,
                                               const int32_t *sp, int64_t alen, int c, int lo,
                                               int hi, int64_t *st_s, int64_t *st_e, float *st_a,
                                               int64_t *wsum, F &&f) {
    const bool sorted = P.b_sorted != 0;
    for (int64_t jb = a0; jb < a1; jb += WG) {
        const int64_t j = jb + threadIdx.x;
        int64_t s = 0, len = 0;
        float a = 0.f;
        if (j < a1) {
            const int k = P.colA[j];
            const int64_t b0 = P.rptB[k];
            if (sorted) {
                const int32_t *q = sp + (j - a0);
                const int32_t x0 = q[(int64_t)c * alen], x1 = q[(int64_t)(c + 1) * alen];
                s = b0 + x0;
                len = x1 - x0;
            } else {
                s = b0;
                len = P.rptB[k + 1] - b0;
            }
            if (VALUES) a = P.valA[j];
        }
        int64_t total;
        const int64_t excl = block_excl_scan_i64<WG>(len, wsum, total);
        st_s[threadIdx.x] = s;
        st_e[threadIdx.x] = excl;
        if (VALUES) st_a[threadIdx.x] = a;
        __syncthreads();
        const int nv = (int)((a1 - jb) < WG ? (a1 - jb) : WG);
        for (int64_t q = threadIdx.x; q < total; q += WG) {
            int l = 0, r = nv;
            while (r - l > 1) {
                int mid = (l + r) >> 1;
                if (st_e[mid] <= q) l = mid; else r = mid;
            }
            const int64_t t = st_s[l] + (q - st_e[l]);
            const int col = P.colB[t];
            if (sorted || (col >= lo && col < hi)) f(col, VALUES ? st_a[l] : 0.f, t);
        }
        __syncthreads();
    }
}

template <int WG>
__global__ __launch_bounds__(WG) void k_sym_chunk(const ProdDev *__restrict__ prods,
                                                   const uint64_t *__restrict__ items, int64_t nh,
                                                   const int64_t *__restrict__ ibase,
                                                   const int64_t *__restrict__ aoff,
                                                   const int64_t *__restrict__ soff,
                                                   const int32_t *__restrict__ split,
                                                   int64_t *__restrict__ chunk_cnt,
                                                   int64_t *__restrict__ row_nnz) {
    __shared__ uint32_t bm[kMaxChunkCols / 32];
    __shared__ int64_t st_s[WG];
    __shared__ int64_t st_e[WG];
    __shared__ int64_t wsum[WG / 64];
    const int64_t it = blockIdx.x;
    const int64_t h = upper_index(ibase, nh, it);
    const int c = (int)(it - ibase[h]);
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int lo = c * P.W;
    const int hi = (int)((int64_t)lo + P.W < P.n ? (int64_t)lo + P.W : P.n);
    if (hi <= lo) {  // chunk past the last column
        if (threadIdx.x == 0) chunk_cnt[it] = 0;
        return;
    }
    const int nwords = (hi - lo + 31) >> 5;
    for (int w = threadIdx.x; w < nwords; w += WG) bm[w] = 0u;
    __syncthreads();
    const int64_t a0 = P.rptA[i], a1 = P.rptA[i + 1];
    chunk_products<WG, false>(P, a0, a1, split + soff[h], a1 - a0, c, lo, hi, st_s, st_e,
                              (float *)nullptr, wsum, [&](int col, float, int64_t) {
                                  const int rel = col - lo;
                                  atomicOr(&bm[rel >> 5], 1u << (rel & 31));
                              });
    int64_t cnt = 0;
    for (int w = threadIdx.x; w < nwords; w += WG) cnt += __popc(bm[w]);
    int64_t tot;
    block_excl_scan_i64<WG>(cnt, wsum, tot);
    if (threadIdx.x == 0) {
        chunk_cnt[it] = tot;
        if (tot) atomicAdd((unsigned long long *)&row_nnz[P.row_base + i], (unsigned long long)tot);
    }
}

template <int WG, int WMAX>
__global__ __launch_bounds__(WG) void k_num_chunk(
    const ProdDev *__restrict__ prods, const uint64_t *__restrict__ ditems, int64_t nd,
    const int64_t *__restrict__ dbase, const int32_t *__restrict__ hslot,
    const int64_t *__restrict__ ibase, const int64_t *__restrict__ soff,
    const int32_t *__restrict__ split, const int64_t *__restrict__ chunk_cnt,
    const int64_t *__restrict__ chunk_pos, const int64_t *__restrict__ rptv,
    int *__restrict__ err) {
    __shared__ float acc[WMAX];
    __shared__ uint32_t bm[WMAX / 32];
    __shared__ int64_t st_s[WG];
    __shared__ int64_t st_e[WG];
    __shared__ float st_a[WG];
    __shared__ int64_t wsum[WG / 64];
    constexpr int NW = WG / 64;
    const int64_t it = blockIdx.x;
    const int64_t d = upper_index(dbase, nd, it);
    const int c = (int)(it - dbase[d]);
    const uint64_t e = ditems[d];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t g = P.row_base + i;
    const int64_t h = hslot[g];
    const int64_t sit = ibase[h] + c;
    const int64_t expect = chunk_cnt[sit];
    if (expect == 0) return;
    const int lo = c * P.W;
    const int hi = (int)((int64_t)lo + P.W < P.n ? (int64_t)lo + P.W : P.n);
    const int width = hi - lo;
    const int nwords = (width + 31) >> 5;
    for (int q = threadIdx.x; q < width; q += WG) acc[q] = 0.f;
    for (int w = threadIdx.x; w < nwords; w += WG) bm[w] = 0u;
    __syncthreads();
    const int64_t a0 = P.rptA[i], a1 = P.rptA[i + 1];
    chunk_products<WG, true>(P, a0, a1, split + soff[h], a1 - a0, c, lo, hi, st_s, st_e, st_a,
                             wsum, [&](int col, float a, int64_t t) {
                                 const int rel = col - lo;
                                 atomicAdd(&acc[rel], a * P.valB[t]);
                                 atomicOr(&bm[rel >> 5], 1u << (rel & 31));
                             });
    // Emission in column order: wave w owns columns [w*span, (w+1)*span).
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int units = (width + 63) >> 6;                  // 64-column units
    const int per = (units + NW - 1) / NW;
    const int cbeg = w * per * 64;
    const int cend = min(width, (w + 1) * per * 64);
    int64_t mine = 0;
    for (int wd = (cbeg >> 5) + lane; wd < ((cend + 31) >> 5); wd += 64) mine += __popc(bm[wd]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_down(mine, off, 64);
    mine = __shfl(mine, 0, 64);
    int64_t total;
    int64_t before = block_excl_scan_i64<WG>(lane == 0 ? mine : 0, wsum, total);
    before = __shfl(before, 0, 64);
    if (threadIdx.x == 0 && total != expect) atomicOr(err, kErrChunk);
    const int64_t out0 = rptv[g] - rptv[P.row_base] + (chunk_pos[sit] - chunk_pos[ibase[h]]);
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int64_t pos = before;
    for (int col0 = cbeg; col0 < cend; col0 += 64) {
        const int col = col0 + lane;
        const bool bit = col < cend && ((bm[col >> 5] >> (col & 31)) & 1u);
        const unsigned long long m = __ballot(bit);
        if (bit) {
            const int64_t r = pos + __popcll(m & lt);
            if (r < expect) {
                P.colC[out0 + r] = lo + col;
                P.valC[out0 + r] = acc[col];
            }
        }
        pos += __popcll(m);
    }
    (void)NW;
}

void launch_heavy_prep(const ProdDev *prods, const uint64_t *items, int64_t nh, int64_t *alen,
                       int64_t *splitlen, int64_t *nchv, hipStream_t s) {
    if (nh <= 0) return;
    hipLaunchKernelGGL(k_heavy_prep, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, prods,
                       items, nh, alen, splitlen, nchv);
}

void launch_dense_prep(const ProdDev *prods, const uint64_t *items, int64_t nd, int64_t *nchv,
                       hipStream_t s) {
    if (nd <= 0) return;
    hipLaunchKernelGGL(k_dense_prep, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, s, prods,
                       items, nd, nchv);
}

void launch_split(const ProdDev *prods, const uint64_t *items, int64_t nh, const int64_t *aoff,
                  const int64_t *soff, int64_t total_alen, int32_t *split, hipStream_t s) {
    if (total_alen <= 0) return;
    hipLaunchKernelGGL(k_split, dim3((unsigned)((total_alen + 255) / 256)), dim3(256), 0, s,
                       prods, items, nh, aoff, soff, total_alen, split);
}

void launch_sym_chunk(const ProdDev *prods, const uint64_t *items, int64_t nh,
                      const int64_t *ibase, int64_t nitems, const int64_t *aoff,
                      const int64_t *soff, const int32_t *split, int64_t *chunk_cnt,
                      int64_t *row_nnz, int *err, hipStream_t s) {
    (void)err;
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_sym_chunk<256>, dim3((unsigned)nitems), dim3(256), 0, s, prods, items,
                       nh, ibase, aoff, soff, split, chunk_cnt, row_nnz);
}

void launch_num_chunk(const ProdDev *prods, const uint64_t *ditems, int64_t nd,
                      const int64_t *dbase, int64_t nitems, const int32_t *hslot,
                      const int64_t *ibase, const int64_t *aoff, const int64_t *soff,
                      const int32_t *split, const int64_t *chunk_cnt, const int64_t *chunk_pos,
                      const int64_t *rptv, int *err, hipStream_t s) {
    (void)aoff;
    if (nitems <= 0) return;
    hipLaunchKernelGGL((k_num_chunk<512, kMaxChunkCols>), dim3((unsigned)nitems), dim3(512), 0,
                       s, prods, ditems, nd, dbase, hslot, ibase, soff, split, chunk_cnt,
                       chunk_pos, rptv, err);
}

}  // namespace spg
