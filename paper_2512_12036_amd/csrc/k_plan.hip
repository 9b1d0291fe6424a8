// Row-size estimation, row grouping and scans.
//
//  * k_ipcount: intermediate products of every row (paper Algorithm 1).  The
//    nonzeros of a block of 256 rows are cut into up to kIpSlices slices, one
//    workgroup each, whose threads walk them together, so neither a row of
//    thousands of nonzeros nor a block of hub rows serialises on a few
//    lanes; per-lane counts are combined with a segmented wavefront scan, an
//    LDS atomic per row segment and a global atomic per row.  k_ip_groups
//    then builds the block's group histogram.
//  * k_scatter: the row map of paper Section III-B.  Rows are not moved; the
//    map lists rows group by group.  Positions come from an exclusive scan of
//    the per-block histograms (group-major, block-minor) plus wavefront
//    ballot ranks, so no per-row global atomics are needed (paper Section
//    IV-A names those atomics as a cost of grouping) and the map is stable.
//  * exclusive int64 scan (tile reduce / recursive scan / tile apply), used
//    for C's row pointers (paper Algorithms 2-3, last step, read as a scan of
//    per-row counts) and for all internal offsets.
#include "common.hpp"

namespace spg {

constexpr int SCAN_T = 256;
constexpr int SCAN_V = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_V;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim = NT).
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *wsum, int64_t &total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = wave_incl_scan(v);
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

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const int64_t *__restrict__ in, int64_t n,
                                                         int64_t *__restrict__ partial) {
    __shared__ int64_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
#pragma unroll
    for (int v = 0; v < SCAN_V; ++v) {
        int64_t i = base + (int64_t)v * SCAN_T + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_excl_scan<SCAN_T>(s, wsum, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Scans one tile; `offs` (may be NULL) holds the exclusive offset of each tile.
__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int64_t *__restrict__ in,
                                                        int64_t *__restrict__ out, int64_t n,
                                                        const int64_t *__restrict__ offs) {
    __shared__ int64_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_V;
    int64_t x[SCAN_V];
    int64_t s = 0;
#pragma unroll
    for (int v = 0; v < SCAN_V; ++v) {
        int64_t i = base + v;
        x[v] = i < n ? in[i] : 0;
        s += x[v];
    }
    int64_t tot;
    int64_t run = block_excl_scan<SCAN_T>(s, wsum, tot);
    const int64_t off = offs ? offs[blockIdx.x] : 0;
    run += off;
#pragma unroll
    for (int v = 0; v < SCAN_V; ++v) {
        int64_t i = base + v;
        if (i < n) out[i] = run;
        run += x[v];
    }
    const int64_t tile_end = (int64_t)(blockIdx.x + 1) * SCAN_TILE;
    if (threadIdx.x == 0 && tile_end >= n) out[n] = off + tot;
}

size_t scan_temp_bytes(int64_t n) {
    size_t t = 64;
    while (n > SCAN_TILE) {
        int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
        t += (size_t)(2 * nt + 1) * sizeof(int64_t);
        n = nt;
    }
    return t;
}

void launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s) {
    if (n <= SCAN_TILE) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_T), 0, s, in, out, n,
                           (const int64_t *)nullptr);
        return;
    }
    int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *partial = (int64_t *)temp;
    int64_t *pscan = partial + nt;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(SCAN_T), 0, s, in, n, partial);
    launch_scan_i64(partial, pscan, nt, pscan + nt + 1, s);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(SCAN_T), 0, s, in, out, n,
                       (const int64_t *)pscan);
}

// ---------------------------------------------------------------------------
// Group of a row with grouping key `key` in a product whose B has `ncols`
// columns.  A row that would go past group 4 but whose key and B both fit
// group 4's table (8 slots x 64 lanes) takes group 4: its table is then
// direct-mapped (slot = column), which needs no load-factor headroom.
__device__ __forceinline__ int group_of(int64_t key, const GroupBounds &gb, int64_t ncols) {
    if (key == 0) return 0;
#pragma unroll
    for (int t = 1; t < kGroups - 1; ++t) {
        if (key <= gb.up[t]) return t;
        if (t == 4 && ncols <= kDirectG4 && key <= kDirectG4) return 4;
    }
    return kGroups - 1;
}

// group_of, then the copy rule: a row of one A nonzero whose B rows are
// strictly ascending (`single`) that would take a later group than
// gb.copy_group takes that one (its block kernels copy the scaled B row).
__device__ __forceinline__ int group_of_row(int64_t key, const GroupBounds &gb, int64_t ncols,
                                            bool single) {
    const int g = group_of(key, gb, ncols);
    return (single && gb.copy_group > 0 && g > gb.copy_group) ? (int)gb.copy_group : g;
}

// Largest r in [0, n) with rp[r] <= j (rp non-decreasing, rp[0] <= j).
__device__ __forceinline__ int lds_upper_row(const int64_t *rp, int n, int64_t j) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (rp[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

// Grouping keys.  Symbolic: the intermediate-product count capped at B's
// column count (both bound the row's distinct outputs; the cap is the tighter
// one when B is narrow).  Numeric: the output length, raised to
// ceil(IP / kIpPerLane) (capped at B's columns) so that rows with many
// products per output get more lanes; never above the symbolic key, so a row
// chunked in the numeric phase was chunked in the symbolic one.
__device__ __forceinline__ int64_t sym_key(int64_t ip, int64_t ncols) {
    return ip < ncols ? ip : ncols;
}

__device__ __forceinline__ int64_t num_key(int64_t nnz, int64_t ip, int64_t ncols) {
    int64_t k = (ip + kIpPerLane - 1) / kIpPerLane;
    if (k > ncols) k = ncols;
    return nnz > k ? nnz : k;
}

// Histogram of groups over the block's rows (grouped by gkey; one row per
// thread, valid < nrows) plus per-product sums of `key`: total, max, and the
// group-7 (chunked) rows with their A nonzeros, split-table size and chunk
// count (nch per row).
__device__ __forceinline__ void block_histogram(int64_t key, int64_t gkey, int64_t alen, bool single,
                                                bool valid, const GroupBounds &gb, int nblk,
                                                int64_t *blkcnt, ProdStats *st, int nch,
                                                bool ip_stats, int64_t ncols) {
    __shared__ int hist[kGroups];
    __shared__ unsigned long long red[kRowBlock / 64][5];
    if (threadIdx.x < kGroups) hist[threadIdx.x] = 0;
    __syncthreads();
    const int g = valid ? group_of_row(gkey, gb, ncols, single) : -1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < kGroups; ++b) {
        unsigned long long m = __ballot(g == b);
        if (lane == 0 && m) atomicAdd(&hist[b], __popcll(m));
    }
    unsigned long long ks = valid ? (unsigned long long)key : 0ull;
    unsigned long long km = ks;
    unsigned long long hr = (g == kChunkGroup) ? 1ull : 0ull;
    unsigned long long ha = (g == kChunkGroup) ? (unsigned long long)alen : 0ull;
    unsigned long long ht = (g == kChunkGroup) ? (unsigned long long)((alen + kSabsJ - 1) / kSabsJ)
                                               : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ks += __shfl_down(ks, off, 64);
        unsigned long long o = __shfl_down(km, off, 64);
        km = o > km ? o : km;
        hr += __shfl_down(hr, off, 64);
        ha += __shfl_down(ha, off, 64);
        ht += __shfl_down(ht, off, 64);
    }
    if (lane == 0) {
        red[w][0] = ks;
        red[w][1] = km;
        red[w][2] = hr;
        red[w][3] = ha;
        red[w][4] = ht;
    }
    __syncthreads();
    if (threadIdx.x < kGroups) blkcnt[(int64_t)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
    if (threadIdx.x == 0) {
        unsigned long long s = 0, mx = 0, rows = 0, al = 0, tl = 0;
        for (int i = 0; i < kRowBlock / 64; ++i) {
            s += red[i][0];
            mx = red[i][1] > mx ? red[i][1] : mx;
            rows += red[i][2];
            al += red[i][3];
            tl += red[i][4];
        }
        if (ip_stats) {
            atomicAdd(&st->ip_sum, s);
            atomicMax(&st->ip_max, mx);
            if (rows) {
                atomicAdd(&st->h_rows, rows);
                atomicAdd(&st->h_alen, al);
                atomicAdd(&st->h_tiles, tl);
                atomicAdd(&st->h_split, al * (unsigned long long)(nch + 1));
                atomicAdd(&st->h_items, rows * (unsigned long long)nch);
            }
        } else {
            atomicAdd(&st->nnz_sum, s);
            atomicMax(&st->nnz_max, mx);
            if (rows) {
                atomicAdd(&st->d_rows, rows);
                atomicAdd(&st->d_items, rows * (unsigned long long)nch);
            }
        }
    }
}

// IP count, accumulation pass: workgroup (b, s) takes slice s of the A
// nonzeros of row block b (up to kIpSlices slices of at least kIpMinSlice
// nonzeros), so a block holding hub rows of many thousands of nonzeros is
// spread over many workgroups.  Per-lane
// B-row lengths are combined with a segmented wavefront scan and one LDS
// atomic per row segment, then added to ip[row] (zeroed beforehand) with one
// global atomic per row touched.
__global__ __launch_bounds__(kRowBlock) void k_ipcount(const ProdDev *__restrict__ prods,
                                                        const RowBlk *__restrict__ blks,
                                                        int64_t *__restrict__ ip) {
    __shared__ int64_t rp[kRowBlock + 1];
    __shared__ unsigned long long acc[kRowBlock];
    const RowBlk blk = blks[blockIdx.x];
    const ProdDev &P = prods[blk.p];
    const int nr = blk.nrows;
    // slices of at least kIpMinSlice nonzeros: most blocks need one workgroup
    const int64_t b0 = P.rptA[blk.i0], b1 = P.rptA[blk.i0 + nr];
    int64_t len_s = (b1 - b0 + kIpSlices - 1) / kIpSlices;
    if (len_s < kIpMinSlice) len_s = kIpMinSlice;
    const int64_t j0 = b0 + len_s * blockIdx.y;
    const int64_t j1 = j0 + len_s < b1 ? j0 + len_s : b1;
    if (j0 >= j1) return;  // uniform
    for (int t = threadIdx.x; t <= nr; t += kRowBlock) rp[t] = P.rptA[blk.i0 + t];
    acc[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    constexpr int U = 4;
    for (int64_t jb = j0; jb < j1; jb += (int64_t)kRowBlock * U) {
        int64_t len[U];
        int r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t j = jb + (int64_t)u * kRowBlock + threadIdx.x;
            len[u] = 0;
            r[u] = -1;
            if (j < j1) {
                int c = P.colA[j];
                len[u] = P.rptB[c + 1] - P.rptB[c];
                r[u] = lds_upper_row(rp, nr, j);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // segmented inclusive scan keyed by row (rows are contiguous)
            int64_t v = len[u];
            const int key = r[u];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                int64_t ov = __shfl_up(v, off, 64);
                int ok = __shfl_up(key, off, 64);
                if (lane >= off && ok == key) v += ov;
            }
            int nxt = __shfl_down(key, 1, 64);
            bool tail = (lane == 63) || (nxt != key);
            if (tail && key >= 0 && v) atomicAdd(&acc[key], (unsigned long long)v);
        }
    }
    __syncthreads();
    if (threadIdx.x < nr && acc[threadIdx.x])
        atomicAdd((unsigned long long *)&ip[P.row_base + blk.i0 + threadIdx.x],
                  acc[threadIdx.x]);
}

// IP count, grouping pass: the block's symbolic group histogram and the
// per-product statistics, from the finished ip[].
__global__ __launch_bounds__(kRowBlock) void k_ip_groups(const ProdDev *__restrict__ prods,
                                                          const RowBlk *__restrict__ blks,
                                                          int nblk, GroupBounds gb,
                                                          const int64_t *__restrict__ ip,
                                                          int64_t *__restrict__ blkcnt,
                                                          ProdStats *__restrict__ stats) {
    const RowBlk blk = blks[blockIdx.x];
    const ProdDev &P = prods[blk.p];
    const bool valid = threadIdx.x < blk.nrows;
    const int64_t row = blk.i0 + threadIdx.x;
    const int64_t key = valid ? ip[P.row_base + row] : 0;
    const int64_t alen = valid ? P.rptA[row + 1] - P.rptA[row] : 0;
    const bool single = alen == 1 && P.b_unique == 1;
    block_histogram(key, sym_key(key, P.n), alen, single, valid, gb, nblk, blkcnt, stats + blk.p,
                    P.nch, true, P.n);
}

__global__ __launch_bounds__(kRowBlock) void k_count_groups(const ProdDev *__restrict__ prods,
                                                             const RowBlk *__restrict__ blks,
                                                             int nblk, GroupBounds gb,
                                                             const int64_t *__restrict__ key,
                                                             const int64_t *__restrict__ ip,
                                                             int64_t *__restrict__ blkcnt,
                                                             ProdStats *__restrict__ stats) {
    const RowBlk blk = blks[blockIdx.x];
    const ProdDev &P = prods[blk.p];
    const bool valid = threadIdx.x < blk.nrows;
    const int64_t r = P.row_base + blk.i0 + threadIdx.x;
    const int64_t k = valid ? key[r] : 0;
    const int64_t gk = valid ? num_key(k, ip[r], P.n) : 0;
    const int64_t row = blk.i0 + threadIdx.x;
    const bool single = valid && P.b_unique == 1 && P.rptA[row + 1] - P.rptA[row] == 1;
    block_histogram(k, gk, 0, single, valid, gb, nblk, blkcnt, stats + blk.p, P.nch, false, P.n);
}

__global__ __launch_bounds__(kRowBlock) void k_scatter(const ProdDev *__restrict__ prods,
                                                        const RowBlk *__restrict__ blks, int nblk,
                                                        GroupBounds gb,
                                                        const int64_t *__restrict__ key,
                                                        const int64_t *__restrict__ off,
                                                        uint64_t *__restrict__ map,
                                                        int32_t *__restrict__ hslot,
                                                        const int64_t *__restrict__ ip) {
    __shared__ int wcnt[kRowBlock / 64][kGroups];
    const RowBlk blk = blks[blockIdx.x];
    const ProdDev &P = prods[blk.p];
    const bool valid = threadIdx.x < blk.nrows;
    const int64_t row = blk.i0 + threadIdx.x;
    int64_t k = 0;
    if (valid) {
        // ip NULL: key holds IP (symbolic map); else key holds output lengths
        k = key[P.row_base + row];
        k = ip ? num_key(k, ip[P.row_base + row], P.n) : sym_key(k, P.n);
    }
    const bool single = valid && P.b_unique == 1 && P.rptA[row + 1] - P.rptA[row] == 1;
    const int g = valid ? group_of_row(k, gb, P.n, single) : -1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = 0;
#pragma unroll
    for (int b = 0; b < kGroups; ++b) {
        unsigned long long m = __ballot(g == b);
        if (g == b) rank = __popcll(m & lt);
        if (lane == 0) wcnt[w][b] = __popcll(m);
    }
    __syncthreads();
    if (valid) {
        int before = 0;
        for (int i = 0; i < w; ++i) before += wcnt[i][g];
        const int64_t pos = off[(int64_t)g * nblk + blockIdx.x] + before + rank;
        map[pos] = pack_item(blk.p, row);
        if (hslot && g == kChunkGroup)
            hslot[P.row_base + row] = (int32_t)(pos - off[(int64_t)kChunkGroup * nblk]);
    }
}

__global__ void k_group_starts(const int64_t *__restrict__ off, int nblk, int64_t *__restrict__ st) {
    int g = threadIdx.x;
    if (g <= kGroups) st[g] = off[(int64_t)g * nblk];
}

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v) {
    int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_rows_local(const int64_t *__restrict__ rptv, int64_t row_base, int64_t m,
                             int64_t *__restrict__ dst) {
    int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i <= m) dst[i] = rptv[row_base + i] - rptv[row_base];
}

// Sortedness of B's rows: a row is sorted when every adjacent pair ascends.
__global__ __launch_bounds__(256) void k_detect_sorted(const int64_t *__restrict__ rpt,
                                                        const int32_t *__restrict__ col,
                                                        int64_t nrows, int *__restrict__ unsorted) {
    __shared__ int64_t rp[257];
    const int64_t i0 = lin_block() * 256;
    if (i0 >= nrows) return;  // block-uniform, before the barrier
    const int nr = (int)((nrows - i0) < 256 ? (nrows - i0) : 256);
    for (int t = threadIdx.x; t <= nr; t += 256) rp[t] = rpt[i0 + t];
    __syncthreads();
    int bad = 0;
    for (int64_t j = rp[0] + threadIdx.x; j < rp[nr]; j += 256) {
        int r = lds_upper_row(rp, nr, j);
        if (j + 1 < rp[r + 1] && col[j + 1] <= col[j]) bad = 1;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(unsorted, 1);
}

__global__ void k_set_sorted(ProdDev *prods, int nprod, const int *__restrict__ unsorted) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprod && prods[p].b_sorted == 2) {
        prods[p].b_sorted = unsorted[p] ? 0 : 1;
        prods[p].b_unique = unsorted[p] ? 0 : 1;  // ascending pairs only: no duplicates
    }
}

// hp: host copy of the descriptors; b_sorted == 2 there means "detect".
void launch_detect_sorted(ProdDev *prods, int nprod, const ProdDev *hp, int *flags,
                          hipStream_t s) {
    for (int p = 0; p < nprod; ++p) {
        if (hp[p].b_sorted != 2 || hp[p].k == 0) continue;
        const int64_t nb = (hp[p].k + 255) / 256;
        hipLaunchKernelGGL(k_detect_sorted, grid1d(nb, 256), dim3(256), 0, s, hp[p].rptB, hp[p].colB,
                           hp[p].k, flags + p);
    }
    hipLaunchKernelGGL(k_set_sorted, dim3((nprod + 255) / 256), dim3(256), 0, s, prods, nprod,
                       (const int *)flags);
}

// CSR well-formedness: row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz,
// every column in [0, ncols).
__global__ void k_validate_rows(const int64_t *__restrict__ rpt, int64_t m, int64_t nnz,
                                int *__restrict__ bad) {
    int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i > m) return;
    int b = 0;
    if (i == 0 && rpt[0] != 0) b = 1;
    if (i == m && rpt[m] != nnz) b = 1;
    if (i < m && rpt[i + 1] < rpt[i]) b = 1;
    if (b) atomicOr(bad, 1);
}

__global__ void k_validate_cols(const int32_t *__restrict__ col, int64_t nnz, int64_t ncols,
                                int *__restrict__ bad) {
    int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i < nnz) {
        int c = col[i];
        if (c < 0 || c >= ncols) atomicOr(bad, 2);
    }
}

// Row pointers are checked first; columns only when the pointers are sound
// (the host reads the flag in between), so no kernel reads out of bounds.
void launch_validate_rows(const CsrCheck &c, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_validate_rows, grid1d(((c.m + 256) / 256), 256), dim3(256), 0, s,
                       c.rpt, c.m, c.nnz, bad);
}

void launch_validate_cols(const CsrCheck &c, int *bad, hipStream_t s) {
    if (c.nnz <= 0) return;
    hipLaunchKernelGGL(k_validate_cols, grid1d(((c.nnz + 255) / 256), 256), dim3(256), 0, s,
                       c.col, c.nnz, c.ncols, bad);
}

void launch_ipcount(const ProdDev *prods, const RowBlk *blks, int nblk, GroupBounds gb,
                    int64_t *ip, int64_t *blkcnt, ProdStats *stats, int64_t nrows,
                    hipStream_t s) {
    if (nblk == 0) return;
    launch_fill_i64(ip, nrows, 0, s);
    hipLaunchKernelGGL(k_ipcount, dim3(nblk, kIpSlices), dim3(kRowBlock), 0, s, prods, blks, ip);
    hipLaunchKernelGGL(k_ip_groups, dim3(nblk), dim3(kRowBlock), 0, s, prods, blks, nblk, gb, ip,
                       blkcnt, stats);
}

void launch_count_groups(const ProdDev *prods, const RowBlk *blks, int nblk, GroupBounds gb,
                         const int64_t *key, const int64_t *ip, int64_t *blkcnt,
                         ProdStats *stats, hipStream_t s) {
    if (nblk == 0) return;
    hipLaunchKernelGGL(k_count_groups, dim3(nblk), dim3(kRowBlock), 0, s, prods, blks, nblk, gb,
                       key, ip, blkcnt, stats);
}

void launch_scatter(const ProdDev *prods, const RowBlk *blks, int nblk, GroupBounds gb,
                    const int64_t *key, const int64_t *off, uint64_t *map, int32_t *hslot,
                    const int64_t *ip, hipStream_t s) {
    if (nblk == 0) return;
    hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(kRowBlock), 0, s, prods, blks, nblk, gb, key,
                       off, map, hslot, ip);
}

void launch_group_starts(const int64_t *off, int nblk, int64_t *starts, hipStream_t s) {
    hipLaunchKernelGGL(k_group_starts, dim3(1), dim3(64), 0, s, off, nblk, starts);
}

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i64, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, p, n, v);
}

// B's rows as column bitmaps, 16 lanes per row (16 rows per 256-thread
// workgroup): the lanes OR the bits of the row's columns into the row's
// words in LDS (at most 16 of them), then write them out.  A row's lanes lie
// in one wave, so their LDS traffic is ordered without a barrier.
__global__ __launch_bounds__(256) void k_brow_bitmap(const int64_t *__restrict__ rptB,
                                                     const int32_t *__restrict__ colB,
                                                     int64_t nrows, int64_t ncols, int bmw,
                                                     uint32_t *__restrict__ out) {
    constexpr int kWords = (int)(kBitmapCols / 32);
    constexpr int kLanes = 16;
    static_assert(kLanes == kWords, "one word per lane of a row");
    __shared__ uint32_t words[256 / kLanes][kWords];
    const int sub = threadIdx.x / kLanes, lane = threadIdx.x % kLanes;
    const int64_t k = lin_block() * (256 / kLanes) + sub;
    if (k >= nrows) return;  // uniform over the row's lanes; no workgroup barrier follows
    words[sub][lane] = 0u;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const int64_t b0 = rptB[k], b1 = rptB[k + 1];
    for (int64_t t = b0 + lane; t < b1; t += kLanes) {
        const int c = colB[t];
        if (c >= 0 && c < ncols) atomicOr(&words[sub][c >> 5], 1u << (c & 31));
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (lane < bmw) out[k * bmw + lane] = words[sub][lane];
}

void launch_brow_bitmap(const int64_t *rptB, const int32_t *colB, int64_t nrows, int64_t ncols,
                        int bmw, uint32_t *out, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_brow_bitmap, grid1d((nrows + 15) / 16, 256), dim3(256), 0, s, rptB, colB,
                       nrows, ncols, bmw, out);
}

// The same for every product of a batch in one launch: workgroup row y is
// product y (products without bitmaps leave at once), and its workgroups
// walk the product's B rows with a stride of the grid's width.
__global__ __launch_bounds__(256) void k_brow_bitmap_batch(const ProdDev *__restrict__ prods) {
    constexpr int kWords = (int)(kBitmapCols / 32);
    constexpr int kLanes = 16;
    static_assert(kLanes == kWords, "one word per lane of a row");
    __shared__ uint32_t words[256 / kLanes][kWords];
    const ProdDev &P = prods[blockIdx.y];
    const int bmw = P.bmw;
    if (bmw == 0) return;  // workgroup-uniform
    const int sub = threadIdx.x / kLanes, lane = threadIdx.x % kLanes;
    uint32_t *out = const_cast<uint32_t *>(P.bmB);
    for (int64_t k = (int64_t)blockIdx.x * (256 / kLanes) + sub; k < P.k;
         k += (int64_t)gridDim.x * (256 / kLanes)) {
        words[sub][lane] = 0u;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        const int64_t b0 = P.rptB[k], b1 = P.rptB[k + 1];
        for (int64_t t = b0 + lane; t < b1; t += kLanes) {
            const int c = P.colB[t];
            if (c >= 0 && c < P.n) atomicOr(&words[sub][c >> 5], 1u << (c & 31));
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (lane < bmw) out[k * bmw + lane] = words[sub][lane];
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // words read before the next row
    }
}

void launch_brow_bitmap_batch(const ProdDev *prods, int nprod, int64_t row_blocks,
                              hipStream_t s) {
    if (nprod <= 0 || row_blocks <= 0) return;
    hipLaunchKernelGGL(k_brow_bitmap_batch, dim3((unsigned)row_blocks, (unsigned)nprod),
                       dim3(256), 0, s, prods);
}

// Every product's own row pointers (prods[q].rptC, m + 1 entries) from the
// batch's: workgroup row y is product y, its workgroups stride its rows.
__global__ __launch_bounds__(256) void k_rows_local_batch(const ProdDev *__restrict__ prods,
                                                          const int64_t *__restrict__ rptv) {
    const ProdDev &P = prods[blockIdx.y];
    const int64_t r0 = rptv[P.row_base];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= P.m;
         i += (int64_t)gridDim.x * 256)
        P.rptC[i] = rptv[P.row_base + i] - r0;
}

void launch_rows_local_batch(const ProdDev *prods, int nprod, int64_t row_blocks,
                             const int64_t *rptv, hipStream_t s) {
    if (nprod <= 0 || row_blocks <= 0) return;
    hipLaunchKernelGGL(k_rows_local_batch, dim3((unsigned)row_blocks, (unsigned)nprod),
                       dim3(256), 0, s, prods, rptv);
}

// Row-size estimation alone (Algorithm 1), aggregated: 16 lanes per row sum
// the lengths of the B rows the row's A nonzeros name; out[0] += sum of the
// rows' intermediate products, out[1] += sum of min(ip, ncols) (a bound of
// nnz(C)), out[2] = max(out[2], ip).  One global atomic per value and block.
__global__ __launch_bounds__(256) void k_ip_estimate(const int64_t *__restrict__ rptA,
                                                     const int32_t *__restrict__ colA,
                                                     const int64_t *__restrict__ rptB, int64_t m,
                                                     int64_t ncols,
                                                     unsigned long long *__restrict__ out) {
    __shared__ unsigned long long acc[3];
    if (threadIdx.x < 3) acc[threadIdx.x] = 0;
    __syncthreads();
    const int seg = threadIdx.x & 15;
    const int64_t i = lin_block() * 16 + (threadIdx.x >> 4);
    int64_t ip = 0;
    if (i < m) {
        const int64_t a0 = rptA[i], a1 = rptA[i + 1];
        for (int64_t j = a0 + seg; j < a1; j += 16) {
            const int c = colA[j];
            ip += rptB[c + 1] - rptB[c];
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) ip += __shfl_xor(ip, off, 16);
    if (seg == 0 && i < m && ip > 0) {
        atomicAdd(&acc[0], (unsigned long long)ip);
        atomicAdd(&acc[1], (unsigned long long)(ip < ncols ? ip : ncols));
        atomicMax(&acc[2], (unsigned long long)ip);
    }
    __syncthreads();
    if (threadIdx.x == 0 && acc[0] > 0) {
        atomicAdd(&out[0], acc[0]);
        atomicAdd(&out[1], acc[1]);
        atomicMax(&out[2], acc[2]);
    }
}

void launch_ip_estimate(const int64_t *rptA, const int32_t *colA, const int64_t *rptB, int64_t m,
                        int64_t ncols, int64_t *out, hipStream_t s) {
    launch_fill_i64(out, 3, 0, s);
    if (m <= 0) return;
    hipLaunchKernelGGL(k_ip_estimate, grid1d(((m + 15) / 16), 256), dim3(256), 0, s, rptA,
                       colA, rptB, m, ncols, (unsigned long long *)out);
}

__global__ void k_arena_check(const int64_t *__restrict__ rptv, int64_t mtot, int64_t capacity,
                              int *__restrict__ err, const ProdDev *__restrict__ prods, int nprod,
                              int64_t *__restrict__ offsets) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0 && rptv[mtot] > capacity) atomicOr(err, kErrCapacity);
    if (q < nprod) offsets[q] = rptv[prods[q].row_base];
    if (q == nprod) offsets[q] = rptv[mtot];
}

void launch_arena_check(const int64_t *rptv, int64_t mtot, int64_t capacity, int *err,
                        const ProdDev *prods, int nprod, int64_t *offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_arena_check, dim3((unsigned)((nprod + 1 + 255) / 256)), dim3(256), 0, s,
                       rptv, mtot, capacity, err, prods, nprod, offsets);
}

void launch_rows_local(const int64_t *rptv, int64_t row_base, int64_t m, int64_t *dst,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_rows_local, grid1d(((m + 256) / 256), 256), dim3(256), 0, s, rptv,
                       row_base, m, dst);
}

}  // namespace spg
