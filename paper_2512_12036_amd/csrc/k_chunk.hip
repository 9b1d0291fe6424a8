// Column-chunked kernels for the heaviest rows (group 7).
//
// Paper Section III-C sends rows whose table does not fit in shared memory
// to a global-memory table.  On gfx950 these rows are instead cut into column
// chunks of W columns (W * nch >= n, nch a multiple of 8) and every (row,
// chunk) pair gets one workgroup with an LDS-resident structure covering the
// chunk's columns directly (no hashing, no probing):
//   * symbolic: a W-bit bitmap; the chunk's distinct count is its popcount;
//   * numeric : a W-float dense accumulator; the chunk's structure is the
//     bitmap the symbolic phase stored (so explicit zeros from cancellation
//     are kept and no occupancy atomics are needed); the chunk is emitted in
//     column order straight from the bitmap, so these rows need no sort.
//
// Latency: a workgroup handles K chunks of one row (an item) and keeps the
// row's A nonzeros in registers across them, so per chunk only the chunk
// bounds are gathered (one chunk ahead) before the B gathers; every item has
// a 32-byte descriptor built once per phase (k_sym_desc / k_num_desc), so a
// workgroup starts with one uniform load.  With B's rows sorted, the
// position of every chunk bound inside every B row is tabulated once per
// product (k_bsplit, one binary search per (B row, bound)); a workgroup then
// finds its sub-range of each B row with one gather.  With unsorted B rows
// every chunk scans whole rows and filters, which is correct but nch times
// the gather traffic.
#include <type_traits>

#include "dev.hpp"

namespace spg {

// bsplit[k * (nch + 1) + c] = first position in B row k (relative to its
// start) whose column is >= c * W, for c = 0..nch.
__global__ __launch_bounds__(256) void k_bsplit(const int64_t *__restrict__ rptB,
                                                 const int32_t *__restrict__ colB, int64_t k_rows,
                                                 int W, int nch, int32_t *__restrict__ bsplit) {
    const int64_t x = lin_block() * 256 + threadIdx.x;
    const int64_t per = nch + 1;
    if (x >= k_rows * per) return;
    const int64_t k = x / per;
    const int c = (int)(x - k * per);
    const int64_t b0 = rptB[k], b1 = rptB[k + 1];
    int64_t pos;
    if (c == 0) {
        pos = b0;
    } else if (c == nch) {
        pos = b1;
    } else {
        const int bound = c * W;
        int64_t l = b0, r = b1;
        while (l < r) {
            const int64_t mid = (l + r) >> 1;
            if (colB[mid] < bound) l = mid + 1; else r = mid;
        }
        pos = l;
    }
    bsplit[x] = (int32_t)(pos - b0);
}

// out[base[r] .. base[r+1]) = r for r < n: the row of every chunk item.
__global__ void k_expand(const int64_t *__restrict__ base, int64_t n, int32_t *__restrict__ out) {
    int64_t r = lin_block() * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int64_t x = base[r]; x < base[r + 1]; ++x) out[x] = (int32_t)r;
}

// len[h] = A nonzeros of row h times (nch + 1): size of its sub-range table.
__global__ void k_row_splitlen(const ProdDev *__restrict__ prods,
                               const uint64_t *__restrict__ items, int64_t nh,
                               int64_t *__restrict__ len) {
    const int64_t h = lin_block() * blockDim.x + threadIdx.x;
    if (h >= nh) return;
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    len[h] = (P.rptA[i + 1] - P.rptA[i]) * (int64_t)(P.nch + 1);
}

// ntile[h] = tiles of kSabsJ A nonzeros of group-7 row h.
__global__ void k_sabs_tiles(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                             int64_t nh, int64_t *__restrict__ ntile) {
    const int64_t h = lin_block() * blockDim.x + threadIdx.x;
    if (h >= nh) return;
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    ntile[h] = (P.rptA[i + 1] - P.rptA[i] + kSabsJ - 1) / kSabsJ;
}

// Sub-range table of the group-7 rows (fast path: sorted B, < 2^30 entries):
// sabs[sbase[h] + c * alen + j] = absolute position in B of the first entry of
// B row colA[a0 + j] with column >= c * W, for c = 0..nch.  Chunk c of the row
// then reads, for every nonzero j, the range [sabs[c][j], sabs[c+1][j]) with
// two coalesced loads.  One workgroup per tile of kSabsJ nonzeros of a row, so
// a row with many nonzeros is spread over many workgroups.  The tile's bounds
// are staged in LDS kSabsC at a time: the bounds of one B row are contiguous
// in bsplit, so the gathers run with lanes over bounds and the stores with
// lanes over nonzeros, both coalesced.  With ipc, the tile's products per
// chunk are added to ipc[cbase[h] + c] (rows of at most kSabsC chunks).
__global__ __launch_bounds__(256) void k_sabs(const ProdDev *__restrict__ prods,
                                               const uint64_t *__restrict__ items,
                                               int64_t ntiles,
                                               const int32_t *__restrict__ tile_row,
                                               const int64_t *__restrict__ tbase,
                                               const int64_t *__restrict__ sbase,
                                               uint32_t *__restrict__ sabs,
                                               const int64_t *__restrict__ cbase,
                                               unsigned long long *__restrict__ ipc) {
    __shared__ uint32_t tile[kSabsC + 1][kSabsJ + 1];  // [bound][nonzero], padded
    __shared__ int32_t kk[kSabsJ];                     // B row of each nonzero of the tile
    __shared__ uint32_t bb[kSabsJ];                    // its first position in B
    const int64_t t = lin_block();
    if (t >= ntiles) return;  // block-uniform, before any barrier
    const int64_t h = tile_row[t];
    const uint64_t e = items[h];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t a0 = P.rptA[i];
    const int64_t alen = P.rptA[i + 1] - a0;
    const int64_t jt = (t - tbase[h]) * kSabsJ;
    const int nj = (int)(alen - jt < kSabsJ ? alen - jt : kSabsJ);
    const int nch = P.nch;
    const int per = nch + 1;
    const int tid = threadIdx.x;
    uint32_t *out = sabs + sbase[h];
    const bool acc = ipc != nullptr && nch <= kSabsC;
    if (tid < nj) {
        const int k = gld(P.colA + a0 + jt + tid);
        kk[tid] = k;
        bb[tid] = (uint32_t)gld(P.rptB + k);
    }
    for (int ct = 0; ct < per; ct += kSabsC) {
        const int nc = per - ct < kSabsC + 1 ? per - ct : kSabsC + 1;  // bounds staged
        const int ns = nc < kSabsC ? nc : kSabsC;                      // bounds stored
        __syncthreads();
        for (int f = tid; f < nj * nc; f += 256) {
            const int jl = f / nc, cl = f - jl * nc;
            tile[cl][jl] = bb[jl] + (uint32_t)gld(P.bsplit + (int64_t)kk[jl] * per + ct + cl);
        }
        __syncthreads();
        for (int f = tid; f < ns * kSabsJ; f += 256) {
            const int cl = f / kSabsJ, jl = f - cl * kSabsJ;
            if (jl < nj) out[(int64_t)(ct + cl) * alen + jt + jl] = tile[cl][jl];
        }
        if (acc && tid < nch) {  // one staged tile holds every bound of the row
            unsigned long long sum = 0ull;
            for (int jl = 0; jl < nj; ++jl) sum += tile[tid + 1][jl] - tile[tid][jl];
            if (sum) atomicAdd(ipc + cbase[h] + tid, sum);
        }
    }
}

// Work items of the group-7 rows when adjacent chunks are merged, one wave
// per row: chunks are merged in column order while their intermediate
// products (ipc) together stay within `cap` and at most `merge` of them are
// taken; mstart[cbase[h] + k] = first chunk of item k and nitem[h] = the
// row's item count.  A merged item therefore has at most cap outputs.  Rows
// of more than kSabsC chunks keep one item per chunk.
__global__ __launch_bounds__(256) void k_chunk_items(const ProdDev *__restrict__ prods,
                                                      const uint64_t *__restrict__ items,
                                                      int64_t nh, int merge, int64_t cap,
                                                      const int64_t *__restrict__ cbase,
                                                      const unsigned long long *__restrict__ ipc,
                                                      int32_t *__restrict__ mstart,
                                                      int64_t *__restrict__ nitem) {
    static_assert(kSabsC <= 64, "one chunk per lane");
    const int64_t h = lin_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (h >= nh) return;  // wave-uniform
    const int nch = prods[item_prod(items[h])].nch;
    int32_t *ms = mstart + cbase[h];
    if (nch > kSabsC) {
        for (int c = lane; c < nch; c += 64) ms[c] = c;
        if (lane == 0) nitem[h] = nch;
        return;
    }
    // lane c holds chunk c's products, saturated at cap + 1 (32 bits)
    const unsigned long long v = lane < nch ? ipc[cbase[h] + lane] : 0ull;
    const uint32_t sat = (uint32_t)(cap < 0x7ffffffe ? cap + 1 : 0x7fffffff);
    const uint32_t mine = v < sat ? (uint32_t)v : sat;
    int k = 0;
    for (int c = 0; c < nch;) {
        uint64_t sum = __builtin_amdgcn_readlane(mine, c);
        int e2 = c + 1;
        while (e2 < nch && e2 - c < merge) {
            const uint64_t x = __builtin_amdgcn_readlane(mine, e2);
            if (sum + x > (uint64_t)cap) break;
            sum += x;
            ++e2;
        }
        if (lane == 0) ms[k] = c;
        ++k;
        c = e2;
    }
    if (lane == 0) nitem[h] = k;
}

// dnch[r] = items of numeric group-7 row r: those its symbolic row was given.
__global__ void k_num_nitems(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ ditems,
                             int64_t n, const int32_t *__restrict__ hslot,
                             const int64_t *__restrict__ nitem, int64_t *__restrict__ dnch) {
    const int64_t r = lin_block() * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t e = ditems[r];
    dnch[r] = nitem[hslot[prods[item_prod(e)].row_base + item_row(e)]];
}

// nchv[r] = chunks of row r divided by div (div = 1: chunks, div = K: items).
__global__ void k_nch_of(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                         int64_t n, int div, int64_t *__restrict__ nchv) {
    int64_t r = lin_block() * blockDim.x + threadIdx.x;
    if (r < n) nchv[r] = prods[item_prod(items[r])].nch / div;
}

// Item `it` of row r covers the chunks q, q + Q, q + 2Q, ... (Q = nch / K
// items per row, K chunks per item): strided, so that every item mixes dense
// and sparse column ranges (column densities are skewed) and items carry
// similar work.  One workgroup per item amortises the row's A staging over
// K chunks.
// The item order inside a row is rotated by the row index, so that with
// skewed column densities the dense column ranges of successive rows do not
// land on the same positions of the launch (workgroups are dealt out to the
// eight dies in turn).
__device__ __forceinline__ int item_q(int64_t it, int64_t base, int64_t row, int nitems_row) {
    return (int)((it - base + row) % nitems_row);
}

// Symbolic items: desc.out0 = batch row, desc.slot0 = first chunk-count slot
// of the row.  With merged items the launch covers an upper bound of the item
// count and *nlim is the exact one.
__global__ void k_sym_desc(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ items,
                           const int32_t *__restrict__ item_of, const int64_t *__restrict__ ibase,
                           const int64_t *__restrict__ cbase,
                           const int64_t *__restrict__ sbase, int64_t nitems, int kper,
                           const int32_t *__restrict__ mstart, const int64_t *__restrict__ nlim,
                           ChunkDesc *__restrict__ desc) {
    const int64_t it = lin_block() * blockDim.x + threadIdx.x;
    if (it >= nitems || (nlim && it >= *nlim)) return;
    const int64_t h = item_of[it];
    const uint64_t e = items[h];
    const int p = item_prod(e);
    const ProdDev &P = prods[p];
    const int64_t i = item_row(e);
    ChunkDesc d;
    d.a0 = P.rptA[i];
    d.alen = (int32_t)(P.rptA[i + 1] - d.a0);
    d.out0 = P.row_base + i;
    d.prod = p;
    d.slot0 = cbase[h];
    d.sb = sbase ? sbase[h] : -1;
    d.pad = 0;
    d.pad2 = 0;
    if (mstart) {  // merged items: item k covers chunks mstart[k] .. mstart[k + 1] - 1
        const int nr = (int)(ibase[h + 1] - ibase[h]);
        const int k = item_q(it, ibase[h], h, nr);
        const int32_t *ms = mstart + cbase[h];
        d.q = ms[k];
        d.span = (k + 1 < nr ? ms[k + 1] : P.nch) - d.q;
    } else {
        d.q = item_q(it, ibase[h], h, P.nch / kper);
        d.span = 1;
    }
    desc[it] = d;
}

// Numeric items: desc.out0 = output offset of the row inside C_p.  With
// merged items the launch covers an upper bound of the item count and *nlim
// is the exact one.
__global__ void k_num_desc(const ProdDev *__restrict__ prods, const uint64_t *__restrict__ ditems,
                           const int32_t *__restrict__ item_of, const int64_t *__restrict__ dbase,
                           int64_t nitems, int kper, const int32_t *__restrict__ hslot,
                           const int64_t *__restrict__ cbase, const int64_t *__restrict__ sbase,
                           const int64_t *__restrict__ rptv, const int32_t *__restrict__ mstart,
                           const int64_t *__restrict__ nlim, ChunkDesc *__restrict__ desc) {
    const int64_t it = lin_block() * blockDim.x + threadIdx.x;
    if (it >= nitems || (nlim && it >= *nlim)) return;
    const int64_t dr = item_of[it];
    const uint64_t e = ditems[dr];
    const int p = item_prod(e);
    const ProdDev &P = prods[p];
    const int64_t i = item_row(e);
    const int64_t g = P.row_base + i;
    ChunkDesc d;
    d.a0 = P.rptA[i];
    d.alen = (int32_t)(P.rptA[i + 1] - d.a0);
    d.out0 = c_base(P, rptv, g);
    d.prod = p;
    const int64_t h = hslot[g];
    d.slot0 = cbase[h];
    d.sb = sbase ? sbase[h] : -1;
    d.pad = 0;
    d.pad2 = 0;
    if (mstart) {
        const int nr = (int)(dbase[dr + 1] - dbase[dr]);
        const int k = item_q(it, dbase[dr], dr, nr);
        const int32_t *ms = mstart + cbase[h];
        d.q = ms[k];
        d.span = (k + 1 < nr ? ms[k + 1] : P.nch) - d.q;
    } else {
        d.q = item_q(it, dbase[dr], dr, P.nch / kper);
        d.span = 1;
    }
    desc[it] = d;
}

// One chunk of one row: stages the chunk's sub-range of every B row named
// by the row's A nonzeros and enumerates the products flat over the
// workgroup.  When the row has at most WG nonzeros (`resident`), the caller
// has already loaded them: thread t holds nonzero t as (b0, a) and the
// chunk bounds x0/x1 of its B row; otherwise the nonzeros are loaded here in
// batches of WG.
// FAST: B rows sorted and fewer than 2^30 entries in B -- a batch then has at
// most WG * W products (32-bit indices) and B positions fit 32 bits.
// Otherwise 64-bit indices, and unsorted B rows are scanned whole and
// filtered to the chunk.  f(col, a_value, b_value).
template <int WG, int VT, bool VALUES, bool FAST, typename F>
__device__ __forceinline__ void chunk_pass(const ProdDev &P, const ChunkDesc &d, int c, int lo,
                                           int hi, const uint32_t *sabs, bool resident,
                                           int64_t rb0, float ra, int32_t rx0, int32_t rx1,
                                           void *st_s_raw, void *st_e_raw, float *st_a,
                                           void *wsum_raw, F &&f) {
    using E = typename std::conditional<FAST, int, int64_t>::type;
    using S = typename std::conditional<FAST, uint32_t, int64_t>::type;
    S *st_s = (S *)st_s_raw;
    E *st_e = (E *)st_e_raw;
    E *wsum = (E *)wsum_raw;
    // st_e holds WG + 1 entries; st_e[WG] = batch total
    const bool sorted = FAST || P.b_sorted == 1;
    const int64_t per = P.nch + 1;
    const int64_t a0 = d.a0, alen = d.alen, a1 = a0 + alen;
    const uint32_t *sc = FAST ? sabs + d.sb + (int64_t)c * alen : nullptr;
    for (int64_t jb = a0; jb < a1; jb += WG) {
        const int64_t j = jb + threadIdx.x;
        int64_t s = 0;
        E len = 0;
        float a = 0.f;
        if (j < a1) {
            if (FAST) {
                const uint32_t x0 = gld(sc + (j - a0)), x1 = gld(sc + alen + (j - a0));
                if (VALUES) a = gld(P.valA + j);
                s = x0;
                len = (E)(x1 - x0);
            } else if (resident) {
                s = rb0 + rx0;
                len = (E)(rx1 - rx0);
                a = ra;
            } else {
                const int k = gld(P.colA + j);
                if (VALUES) a = gld(P.valA + j);
                const int64_t b0 = gld(P.rptB + k);
                if (sorted) {
                    const int32_t *q = P.bsplit + (int64_t)k * per + c;
                    const int32_t x0 = gld(q), x1 = gld(q + 1);
                    s = b0 + x0;
                    len = (E)(x1 - x0);
                } else {
                    s = b0;
                    len = (E)(gld(P.rptB + k + 1) - b0);
                }
            }
        }
        E total;
        const E excl = block_excl_scan<WG, E>(len, wsum, total);
        st_s[threadIdx.x] = (S)s;
        st_e[threadIdx.x] = excl;
        if (threadIdx.x == 0) st_e[WG] = total;
        if (VALUES) st_a[threadIdx.x] = a;
        __syncthreads();
        const int nv = (int)((a1 - jb) < WG ? (a1 - jb) : WG);
        if (sorted) {
            staged_products<WG, VT, VALUES, E, S>(st_s, st_e, st_a, nv, total, P.colB, P.valB,
                                                  f);
        } else {
            staged_products<WG, VT, VALUES, E, S>(
                st_s, st_e, st_a, nv, total, P.colB, P.valB, [&](int col, float av, float bv) {
                    if (col >= lo && col < hi) f(col, av, bv);
                });
        }
        __syncthreads();
    }
}

// Loads the row's nonzero owned by this thread (resident rows) and the chunk
// bounds of its B row for chunk c.
__device__ __forceinline__ void resident_load(const ProdDev &P, int64_t a0, int64_t alen,
                                              bool values, int &k, int64_t &b0, float &a) {
    k = 0;
    b0 = 0;
    a = 0.f;
    if ((int64_t)threadIdx.x < alen) {
        k = gld(P.colA + a0 + threadIdx.x);
        if (values) a = gld(P.valA + a0 + threadIdx.x);
        b0 = gld(P.rptB + k);
    }
}

__device__ __forceinline__ void resident_bounds(const ProdDev &P, int64_t alen, int k, int c,
                                                int32_t &x0, int32_t &x1) {
    x0 = 0;
    x1 = 0;
    if ((int64_t)threadIdx.x < alen) {
        if (P.b_sorted == 1) {
            const int32_t *q = P.bsplit + (int64_t)k * (P.nch + 1) + c;
            x0 = gld(q);
            x1 = gld(q + 1);
        } else {
            const int64_t b0 = gld(P.rptB + k);
            x1 = (int32_t)(gld(P.rptB + k + 1) - b0);
        }
    }
}

template <int WG, int WMAX, bool FAST>
__global__ __launch_bounds__(WG) void k_sym_chunk(const ProdDev *__restrict__ prods,
                                                   const ChunkDesc *__restrict__ desc,
                                                   int64_t nitems,
                                                   const uint32_t *__restrict__ sabs, int kper,
                                                   int64_t *__restrict__ chunk_cnt,
                                                   int64_t *__restrict__ row_nnz,
                                                   uint32_t *__restrict__ sbits, int wpc) {
    __shared__ uint32_t bm[WMAX / 32];
    __shared__ int64_t st_s[WG];
    __shared__ int64_t st_e[WG + 1];
    __shared__ int64_t wsum[WG / 64];
    const int64_t item = lin_block();
    if (item >= nitems) return;  // block-uniform, before any barrier
    const ChunkDesc d = desc[item];
    const ProdDev &P = prods[d.prod];
    const int Q = P.nch / kper;
    const bool resident = !FAST && d.alen <= WG;
    int k = 0;
    int64_t b0 = 0;
    float a = 0.f;
    if (resident) resident_load(P, d.a0, d.alen, false, k, b0, a);
    int32_t nx0 = 0, nx1 = 0;
    if (resident) resident_bounds(P, d.alen, k, d.q, nx0, nx1);
    for (int x = threadIdx.x; x < WMAX / 32; x += WG) bm[x] = 0u;
    int64_t row_total = 0;
    for (int t = 0; t < kper; ++t) {
        const int c = d.q + Q * t;
        const int32_t x0 = nx0, x1 = nx1;
        if (resident && t + 1 < kper) resident_bounds(P, d.alen, k, c + Q, nx0, nx1);  // prefetch
        const int lo = c * P.W;
        const int hi = (int)((int64_t)lo + P.W < P.n ? (int64_t)lo + P.W : P.n);
        if (hi <= lo) {  // chunk past the last column
            if (threadIdx.x == 0) chunk_cnt[d.slot0 + c] = 0;
            continue;
        }
        const int nwords = (hi - lo + 31) >> 5;
        __syncthreads();  // bitmap clear (first chunk) / previous count done
        chunk_pass<WG, 8, false, FAST>(P, d, c, lo, hi, sabs, resident, b0, 0.f, x0, x1,
                                       st_s, st_e, (float *)nullptr, wsum,
                                       [&](int col, float, float) {
                                           const int rel = col - lo;
                                           atomicOr(&bm[rel >> 5], 1u << (rel & 31));
                                       });
        int64_t cnt = 0;
        uint32_t *keep = sbits ? sbits + (d.slot0 + c) * (int64_t)wpc : nullptr;
        for (int x = threadIdx.x; x < nwords; x += WG) {
            const uint32_t wv = bm[x];
            cnt += __popc(wv);
            if (keep) gst(keep + x, wv);  // the chunk's structure, reused by the numeric phase
            bm[x] = 0u;                   // clear for the next chunk
        }
        const int64_t tot = block_sum<WG, int64_t>(cnt, wsum);
        if (threadIdx.x == 0) chunk_cnt[d.slot0 + c] = tot;
        row_total += tot;
    }
    if (threadIdx.x == 0 && row_total)
        atomicAdd((unsigned long long *)&row_nnz[d.out0], (unsigned long long)row_total);
}

constexpr int NVT = 8;        // products per lane per round in the numeric chunk kernels
constexpr int kDenseVT = 16;  // same for dense chunks (more gathers in flight per wave)
constexpr int kEmitU = 8;     // columns per thread per round of the dense emission
#ifndef SPG_RANK_ITEMS
#define SPG_RANK_ITEMS 1
#endif
constexpr int kRankItems = SPG_RANK_ITEMS;  // consecutive items per wave of the rank kernel
#ifndef SPG_RANK_WAVES
#define SPG_RANK_WAVES 1
#endif
constexpr int kRankWaves = SPG_RANK_WAVES;  // independent waves (items) per workgroup

template <int WG, int WMAX, bool FAST>
__global__ __launch_bounds__(WG) void k_num_chunk(const ProdDev *__restrict__ prods,
                                                   const ChunkDesc *__restrict__ desc,
                                                   int64_t nitems,
                                                   const uint32_t *__restrict__ sabs, int kper,
                                                   const int64_t *__restrict__ chunk_cnt,
                                                   const int64_t *__restrict__ chunk_pos,
                                                   const uint32_t *__restrict__ sbits, int wpc,
                                                   int *__restrict__ err) {
    __shared__ float acc[WMAX];
    __shared__ int64_t st_s[WG];
    __shared__ int64_t st_e[WG + 1];
    __shared__ float st_a[WG];
    __shared__ int64_t wsum[WG / 64];
    const int64_t item = lin_block();
    if (item >= nitems) return;  // block-uniform, before any barrier
    const ChunkDesc d = desc[item];
    const ProdDev &P = prods[d.prod];
    const int Q = P.nch / kper;
    const bool resident = !FAST && d.alen <= WG;
    int k = 0;
    int64_t b0 = 0;
    float a = 0.f;
    if (resident) resident_load(P, d.a0, d.alen, true, k, b0, a);
    int32_t nx0 = 0, nx1 = 0;
    if (resident) resident_bounds(P, d.alen, k, d.q, nx0, nx1);
    // clear once; the emission clears every slot it reads
    for (int q = threadIdx.x; q < WMAX; q += WG) acc[q] = 0.f;
    const int64_t pos0 = chunk_pos[d.slot0];
    for (int t = 0; t < kper; ++t) {
        const int c = d.q + Q * t;
        const int32_t x0 = nx0, x1 = nx1;
        if (resident && t + 1 < kper) resident_bounds(P, d.alen, k, c + Q, nx0, nx1);  // prefetch
        const int64_t expect = chunk_cnt[d.slot0 + c];
        if (expect == 0) continue;
        const int64_t out0 = d.out0 + (chunk_pos[d.slot0 + c] - pos0);
        const int lo = c * P.W;
        const int hi = (int)((int64_t)lo + P.W < P.n ? (int64_t)lo + P.W : P.n);
        const int width = hi - lo;
        if (width > WMAX) {  // the plan picks WMAX >= W; never taken
            if (threadIdx.x == 0) atomicOr(err, kErrRow);
            return;
        }
        // The chunk's structure words are fetched before the products, so their
        // latency hides behind the gathers (one word per lane when W <= 32*WG).
        const int nwords = (width + 31) >> 5;
        const uint32_t *bits = sbits + (d.slot0 + c) * (int64_t)wpc;
        const uint32_t first_word = threadIdx.x < nwords ? gld(bits + threadIdx.x) : 0u;
        __syncthreads();  // clear (first chunk) / previous emission done
        chunk_pass<WG, NVT, true, FAST>(P, d, c, lo, hi, sabs, resident, b0, a, x0, x1, st_s,
                                        st_e, st_a, wsum, [&](int col, float av, float bv) {
                                            lds_fadd(&acc[col - lo], av * bv);
                                        });
        // Emission in column order from the chunk's structure (the symbolic
        // phase's bitmap, so no occupancy atomics here): one word (32
        // columns) per lane, the word's output position from a block scan of
        // the popcounts; a lane walks only its set bits and clears the
        // accumulator slots it reads.
        int64_t base = 0;
        for (int w0 = 0; w0 < nwords; w0 += WG) {
            const int x = w0 + threadIdx.x;
            uint32_t word = w0 == 0 ? first_word : (x < nwords ? gld(bits + x) : 0u);
            int64_t total;
            const int64_t pre = block_excl_scan<WG, int64_t>(__popc(word), wsum, total);
            int64_t r = base + pre;
            int32_t *colC = P.colC + out0;
            float *valC = P.valC + out0;
            while (word) {
                const int b = __builtin_ctz(word);
                word &= word - 1u;
                const int rel = (x << 5) + b;
                const float v = acc[rel];
                acc[rel] = 0.f;
                if (r < expect) {
                    gst(colC + r, lo + rel);
                    gst(valC + r, v);
                }
                ++r;
            }
            base += total;
        }
        if (threadIdx.x == 0 && base != expect) atomicOr(err, kErrChunk);
    }
}

// ---------------------------------------------------------------------------
// Pipelined chunk kernels (sorted B with 32-bit positions, one chunk per
// item).  A fixed grid of workgroups walks the items with a stride of the
// grid size; while one item is processed, the inputs of the next one (its
// descriptor, the slices of its B rows, its A values, its counts and first
// structure word) are already in flight, and the workgroup's barriers order
// LDS only, so those loads are not drained by them.  Per item, only the
// gathers of B are then exposed to memory latency.  The accumulator / bitmap
// is cleared once per workgroup; every item leaves it clear again.

constexpr int kDescWords = (int)(sizeof(ChunkDesc) / 8);
static_assert(sizeof(ChunkDesc) % 8 == 0 && kDescWords <= 64, "descriptor layout");

// Lane l < kDescWords loads 8-byte word l of descriptor `it`.
__device__ __forceinline__ uint64_t desc_word(const ChunkDesc *desc, int64_t it) {
    const int lane = threadIdx.x & 63;
    return lane < kDescWords ? gld((const uint64_t *)(desc + it) + lane) : 0ull;
}

__device__ __forceinline__ ChunkDesc desc_unpack(uint64_t w) {
    ChunkDesc d;
    d.a0 = (int64_t)readlane64(w, 0);
    d.out0 = (int64_t)readlane64(w, 1);
    d.slot0 = (int64_t)readlane64(w, 2);
    d.sb = (int64_t)readlane64(w, 3);
    const uint64_t w4 = readlane64(w, 4), w5 = readlane64(w, 5);
    d.alen = (int32_t)(uint32_t)w4;
    d.q = (int32_t)(uint32_t)(w4 >> 32);
    d.prod = (int32_t)(uint32_t)w5;
    d.pad = (int32_t)(uint32_t)(w5 >> 32);
    const uint64_t w6 = readlane64(w, 6);
    d.span = (int32_t)(uint32_t)w6;
    d.pad2 = (int32_t)(uint32_t)(w6 >> 32);
    return d;
}

// What a thread prefetches of one item: the slice of the B row named by the
// row's A nonzero `threadIdx.x` (first staging round) and, for the numeric
// phase, its A value, the chunk's output count and offsets and the thread's
// first structure word.
struct ItemIn {
    uint32_t x0, x1;
    float a;
    uint32_t word;
    int64_t cnt, pos, pos0;
};

template <bool NUMERIC>
__device__ __forceinline__ ItemIn item_load(const ProdDev *prods, const ChunkDesc &d,
                                            const uint32_t *sabs, const int64_t *chunk_cnt,
                                            const int64_t *chunk_pos, const uint32_t *sbits,
                                            int wpc, bool resolved = false) {
    ItemIn in;
    in.x0 = in.x1 = 0u;
    in.a = 0.f;
    in.word = 0u;
    in.cnt = in.pos = in.pos0 = 0;
    const int c = d.q;
    const int j = threadIdx.x;
    if (j < d.alen) {
        const uint32_t *sc = sabs + d.sb + (int64_t)c * d.alen;
        in.x0 = gld(sc + j);
        in.x1 = gld(sc + (int64_t)d.span * d.alen + j);
        if (NUMERIC) in.a = gld(prods[d.prod].valA + d.a0 + j);
    }
    if (NUMERIC) {
        const int64_t slot = d.slot0 + c;
        if (resolved) {  // count and offset already in the descriptor
            in.cnt = d.pad;
            in.pos = in.pos0 = 0;
        } else {
            in.cnt = gld(chunk_cnt + slot);
            in.pos = gld(chunk_pos + slot);
            in.pos0 = gld(chunk_pos + d.slot0);
        }
        if (j < wpc) in.word = gld(sbits + slot * (int64_t)wpc + j);
    }
    return in;
}

// Stages the row's B slices for chunk [lo, hi) in rounds of WG A nonzeros
// (the first round from the prefetched `in`) and hands every product to f.
// WAVE: a single wave working on its own (tid = lane), ordering its LDS
// traffic by itself instead of with workgroup barriers.
template <int WG, int VT, bool VALUES, bool WAVE = false, bool CLAMP = true, typename F>
__device__ __forceinline__ void pipe_products(const ProdDev &P, const ChunkDesc &d,
                                              const ItemIn &in, const uint32_t *sabs,
                                              uint32_t *st_s, int *st_e, float *st_a, int *wsum,
                                              F &&f, int tid = threadIdx.x) {
    static_assert(!WAVE || WG == 64, "a wave-local pass is 64 lanes wide");
    const int alen = d.alen;
    const uint32_t *sc = sabs + d.sb + (int64_t)d.q * alen;
    const int64_t send = (int64_t)d.span * alen;  // the item's end bound
    uint32_t x0 = in.x0, x1 = in.x1;
    float a = in.a;
    for (int jb = 0; jb < alen; jb += WG) {
        int total;
        const int excl = wg_excl_scan<WG, int>((int)(x1 - x0), wsum, total);
        st_s[tid] = x0;
        st_e[tid] = excl;
        if (VALUES) st_a[tid] = a;
        if (tid == 0) st_e[WG] = total;
        if (WAVE) wave_lds_sync(); else lds_sync();
        const int nv = alen - jb < WG ? alen - jb : WG;
        // the next batch's bounds, loaded while this batch's products run
        const int jn = jb + WG + tid;
        uint32_t nx0 = 0u, nx1 = 0u;
        float na = 0.f;
        if (jn < alen) {
            nx0 = gld(sc + jn);
            nx1 = gld(sc + send + jn);
            if (VALUES) na = gld(P.valA + d.a0 + jn);
        }
        if (total > 0)
            striped_products<WG, VT, VALUES, int, uint32_t, CLAMP>(st_s, st_e, st_a, nv, total,
                                                                   P.colB, P.valB, f, tid, excl);
        if (WAVE) wave_lds_sync(); else lds_sync();
        x0 = nx0;
        x1 = nx1;
        a = na;
    }
}

template <int WG, int WMAX>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8))) void k_sym_chunk_pipe(const ProdDev *__restrict__ prods,
                                                       const ChunkDesc *__restrict__ desc,
                                                       int64_t nitems,
                                                       const uint32_t *__restrict__ sabs,
                                                       int64_t *__restrict__ chunk_cnt,
                                                       int64_t *__restrict__ row_nnz,
                                                       uint32_t *__restrict__ sbits, int wpc,
                                                       int *__restrict__ err) {
    __shared__ uint32_t bm[WMAX / 32];
    __shared__ uint32_t st_s[WG];
    __shared__ int st_e[WG + 1];
    __shared__ int64_t wsum[WG / 64];
    int64_t w = blockIdx.x;  // walk index; the item is xcd_unit(w, nitems)
    const int64_t stride = gridDim.x;
    if (w >= nitems) return;
    int clean = 0;  // bitmap words [0, clean) are zero (each item re-zeroes what it used)
    ChunkDesc d = desc_unpack(desc_word(desc, xcd_unit(w, nitems)));
    ItemIn in = item_load<false>(prods, d, sabs, nullptr, nullptr, nullptr, 0);
    uint64_t wnext = w + stride < nitems ? desc_word(desc, xcd_unit(w + stride, nitems)) : 0ull;
    for (;;) {
        const int64_t wn = w + stride;
        const bool more = wn < nitems;
        ChunkDesc dn;
        ItemIn inn;
        if (more) {
            dn = desc_unpack(wnext);
            inn = item_load<false>(prods, dn, sabs, nullptr, nullptr, nullptr, 0);
            wnext = wn + stride < nitems ? desc_word(desc, xcd_unit(wn + stride, nitems)) : 0ull;
        }
        const ProdDev &P = prods[d.prod];
        const int c = d.q;
        const int lo = c * P.W;
        const int64_t end = (int64_t)lo + (int64_t)d.span * P.W;
        const int hi = (int)(end < P.n ? end : P.n);
        if (hi - lo > WMAX) {  // the plan picks WMAX >= the widest item; never taken
            if (threadIdx.x == 0) atomicOr(err, kErrRow);
            return;
        }
        int64_t cnt = 0;
        if (hi > lo) {
            const int nw = (hi - lo + 31) >> 5;
            if (nw > clean) {
                for (int x = clean + (int)threadIdx.x; x < nw; x += WG) bm[x] = 0u;
                clean = nw;
            }
            lds_sync();  // bitmap clear done
            pipe_products<WG, 8, false>(
                P, d, in, sabs, st_s, st_e, nullptr, (int *)wsum,
                [&](const int *cc, const float *, const float *, const bool *ok) {
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        const int rel = cc[v] - lo;
                        if (ok[v]) atomicOr(&bm[rel >> 5], 1u << (rel & 31));
                    }
                });
            const int nwords = (hi - lo + 31) >> 5;
            uint32_t *keep = sbits + (d.slot0 + c) * (int64_t)wpc;
#pragma unroll 4
            for (int x = threadIdx.x; x < nwords; x += WG) {
                const uint32_t wv = bm[x];
                cnt += __popc(wv);
                gst(keep + x, wv);  // the chunk's structure, reused by the numeric phase
                bm[x] = 0u;
            }
        }
        // an item's count is at most its width (< 2^31)
        const int64_t tot = wg_sum<WG, int>((int)cnt, (int *)wsum);
        if (threadIdx.x == 0) {
            chunk_cnt[d.slot0 + c] = tot;
            if (tot) atomicAdd((unsigned long long *)&row_nnz[d.out0], (unsigned long long)tot);
        } else if ((int)threadIdx.x < d.span) {
            chunk_cnt[d.slot0 + c + threadIdx.x] = 0;  // chunks merged into this item
        }
        if (!more) break;
        w = wn;
        d = dn;
        in = inn;
    }
}

// The dense accumulator's LDS allows four 256-thread workgroups per compute
// unit at 8,192 columns, so the kernel asks for registers for four waves per
// SIMD: one register more would cost a quarter of the occupancy.
template <int WG, int WMAX>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void k_num_chunk_pipe(const ProdDev *__restrict__ prods,
                                                       const ChunkDesc *__restrict__ desc,
                                                       int64_t nitems,
                                                       const uint32_t *__restrict__ sabs,
                                                       const int64_t *__restrict__ chunk_cnt,
                                                       const int64_t *__restrict__ chunk_pos,
                                                       const uint32_t *__restrict__ sbits,
                                                       int wpc, int64_t min_expect, int resolved,
                                                       int *__restrict__ err) {
    // + one dummy slot per lane for unused batch entries
    __shared__ __attribute__((aligned(16))) float acc[WMAX + 64];
    __shared__ uint2 sw[WMAX / 32];   // structure words and their first output slot
    __shared__ uint32_t st_s[WG];
    __shared__ int st_e[WG + 1];
    __shared__ float st_a[WG];
    __shared__ int wsum[WG / 64];
    int64_t w = blockIdx.x;  // walk index; the item is xcd_unit(w, nitems)
    const int64_t stride = gridDim.x;
    if (w >= nitems) return;
    bool cleared = false;  // the accumulator is cleared before the first item taken
    ChunkDesc d = desc_unpack(desc_word(desc, xcd_unit(w, nitems)));
    ItemIn in = item_load<true>(prods, d, sabs, chunk_cnt, chunk_pos, sbits, wpc, resolved);
    uint64_t wnext = w + stride < nitems ? desc_word(desc, xcd_unit(w + stride, nitems)) : 0ull;
    for (;;) {
        const int64_t wn = w + stride;
        const bool more = wn < nitems;
        ChunkDesc dn;
        ItemIn inn;
        if (more) {
            dn = desc_unpack(wnext);
            inn = item_load<true>(prods, dn, sabs, chunk_cnt, chunk_pos, sbits, wpc, resolved);
            wnext = wn + stride < nitems ? desc_word(desc, xcd_unit(wn + stride, nitems)) : 0ull;
        }
        const ProdDev &P = prods[d.prod];
        const int c = d.q;
        const int lo = c * P.W;
        const int64_t end = (int64_t)lo + (int64_t)d.span * P.W;
        const int hi = (int)(end < P.n ? end : P.n);
        const int width = hi - lo;
        // the count is the same in every lane; make it a scalar
        const int64_t expect = (int64_t)readlane64((uint64_t)in.cnt, 0);
        if (width > WMAX) {  // the plan picks WMAX >= W; never taken
            if (threadIdx.x == 0) atomicOr(err, kErrRow);
            return;
        }
        if (expect > min_expect) {  // smaller chunks belong to k_num_chunk_rank
            if (!cleared) {  // 16-byte stores
                static_assert((WMAX + 64) % 4 == 0, "accumulator size");
                float4 *acc4 = reinterpret_cast<float4 *>(acc);
                for (int q = threadIdx.x; q < (WMAX + 64) / 4; q += WG)
                    acc4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                cleared = true;
            }
            const int64_t out0 = d.out0 + (in.pos - in.pos0);
            lds_sync();  // clear (first item) done
            const int dummy = WMAX + (threadIdx.x & 63);
            pipe_products<WG, kDenseVT, true>(
                P, d, in, sabs, st_s, st_e, st_a, wsum,
                [&](const int *cc, const float *aa, const float *vv, const bool *ok) {
                    int idx[kDenseVT];
                    float add[kDenseVT];
#pragma unroll
                    for (int v = 0; v < kDenseVT; ++v) {
                        idx[v] = ok[v] ? cc[v] - lo : dummy;
                        add[v] = ok[v] ? aa[v] * vv[v] : 0.f;
                    }
                    lds_fadd_many<kDenseVT>(acc, idx, add);
                });
            // Emission from the chunk's structure (the symbolic bitmap): a scan
            // of the words' popcounts gives each word its first output slot;
            // then thread t takes columns t, t + WG, ...: the output slot of a
            // set column is its word's slot plus the set bits below it, so
            // consecutive set columns go to consecutive slots (coalesced
            // writes, already in column order), and every set slot of the
            // accumulator is cleared for the next chunk.  kEmitU columns per
            // thread are read from LDS together, so that one LDS round trip
            // serves all of them.
            const int nwords = (width + 31) >> 5;
            const uint32_t *bits = sbits + (d.slot0 + c) * (int64_t)wpc;
            int32_t *colC = P.colC + out0;
            float *valC = P.valC + out0;
            int base = 0;
            for (int w0 = 0; w0 < nwords; w0 += WG) {
                const int x = w0 + threadIdx.x;
                const uint32_t word = x < nwords ? (w0 == 0 ? in.word : gld(bits + x)) : 0u;
                int total;
                const int pre = wg_excl_scan<WG, int>(__popc(word), wsum, total);
                if (x < nwords) sw[x] = make_uint2(word, (uint32_t)(base + pre));
                base += total;
            }
            lds_sync();
            const int ncol = nwords * 32;
            const int ex = (int)expect;
            for (int c0 = threadIdx.x; c0 < ncol; c0 += kEmitU * WG) {
                uint2 e[kEmitU];
                float v[kEmitU];
#pragma unroll
                for (int u = 0; u < kEmitU; ++u) {
                    const int col = c0 + u * WG;
                    const int cc = col < ncol ? col : 0;
                    e[u] = sw[cc >> 5];
                    v[u] = acc[cc];
                    if (col >= ncol) e[u].x = 0u;
                }
#pragma unroll
                for (int u = 0; u < kEmitU; ++u) {
                    const int col = c0 + u * WG;
                    const uint32_t bit = 1u << (col & 31);
                    if (e[u].x & bit) {
                        // for the workgroup's next item; the products only
                        // ever touch the chunk's structure, so the other
                        // slots are still zero
                        if (more) acc[col] = 0.f;
                        const int r = (int)e[u].y + __popc(e[u].x & (bit - 1u));
                        if (r < ex) {
                            gst(colC + r, lo + col);
                            gst(valC + r, v[u]);
                        }
                    }
                }
            }
            if (threadIdx.x == 0 && base != expect) atomicOr(err, kErrChunk);
        }
        if (!more) break;
        w = wn;
        d = dn;
        in = inn;
    }
}

// Numeric kernel for chunks with at most CAP outputs (most chunks of a
// skewed product): one wave per chunk.  The chunk's structure (the bitmap the
// symbolic phase stored) gives every output column its rank among the
// chunk's outputs -- a perfect, collision-free hash -- so the accumulator is
// a compact array of CAP floats rather than one slot per column, a chunk
// needs a few KB of LDS and many chunks are resident per compute unit.  The
// values leave as one contiguous (coalesced) copy, already in column order;
// the columns are written from the bitmap.  A lane loads its structure
// words into registers first, so the rank table is written in one LDS pass.
// A wave may take IPW consecutive items (mostly chunks of one row), loading
// the next item's inputs while it works on the current one; the registers
// that costs lower the occupancy, and one item per wave measured fastest.

// What a lane holds of one item before it is processed.
template <int KMAX>
struct RankIn {
    ChunkDesc d;
    int64_t expect;  // the item's output count (0: nothing to do here)
    uint32_t x0, x1;
    float a;
    uint32_t wv[KMAX];  // structure words lane*K .. lane*K + K - 1
};

template <int WMAX, int CAP>
__device__ __forceinline__ RankIn<WMAX / 2048> rank_load(const ProdDev *prods, uint64_t w,
                                                         const uint32_t *sabs,
                                                         const int64_t *chunk_cnt,
                                                         const uint32_t *sbits, int wpc,
                                                         int resolved) {
    constexpr int KMAX = WMAX / 2048;
    const int lane = threadIdx.x & 63;
    RankIn<KMAX> in;
    in.d = desc_unpack(w);
    const ChunkDesc &d = in.d;
    const int64_t slot = d.slot0 + d.q;
    in.expect =
        resolved ? (int64_t)d.pad : (int64_t)readlane64((uint64_t)gld(chunk_cnt + slot), 0);
    in.x0 = in.x1 = 0u;
    in.a = 0.f;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) in.wv[k] = 0u;
    if (in.expect == 0 || in.expect > CAP) {
        in.expect = 0;  // empty, or a dense chunk (k_num_chunk_pipe)
        return in;
    }
    const ProdDev &P = prods[d.prod];
    if (lane < d.alen) {
        const uint32_t *sc = sabs + d.sb + (int64_t)d.q * d.alen;
        in.x0 = gld(sc + lane);
        in.x1 = gld(sc + (int64_t)d.span * d.alen + lane);
        in.a = gld(P.valA + d.a0 + lane);
    }
    const int lo = d.q * P.W;
    const int64_t end = (int64_t)lo + (int64_t)d.span * P.W;
    const int hi = (int)(end < P.n ? end : P.n);
    const int nwords = hi > lo ? (hi - lo + 31) >> 5 : 0;
    const int K = (nwords + 63) >> 6;
    const uint32_t *bits = sbits + slot * (int64_t)wpc;
    if (K <= KMAX) {
        if ((K & 3) == 0 && nwords == K * 64 && (wpc & 3) == 0) {  // 16-byte loads
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int k = 0; k < KMAX; k += 4)
                if (k < K) {
                    const u32x4 w4 = gld((const u32x4 *)(bits + lane * K + k));
                    in.wv[k] = w4.x;
                    in.wv[k + 1] = w4.y;
                    in.wv[k + 2] = w4.z;
                    in.wv[k + 3] = w4.w;
                }
        } else {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int x = lane * K + k;
                if (k < K && x < nwords) in.wv[k] = gld(bits + x);
            }
        }
    }
    return in;
}

// Acc: the accumulator type.  double (the FP64-accumulation option): every
// product a * b is formed exactly in FP64 (two FP32 significands fit in
// FP64's), the sums are FP64 LDS atomics, and each output is rounded to FP32
// once, on its way out.
template <int WMAX, int CAP, int IPW, int WAVES, typename Acc = float>
__global__ __launch_bounds__(64 * WAVES) void k_num_chunk_rank(const ProdDev *__restrict__ prods,
                                                       const ChunkDesc *__restrict__ desc,
                                                       int64_t nitems,
                                                       const uint32_t *__restrict__ sabs,
                                                       const int64_t *__restrict__ chunk_cnt,
                                                       const int64_t *__restrict__ chunk_pos,
                                                       const uint32_t *__restrict__ sbits,
                                                       int wpc, int resolved,
                                                       int *__restrict__ err) {
    constexpr int NWD = WMAX / 32;  // structure words of the widest item
    constexpr int KMAX = NWD / 64;  // of them per lane
    static_assert(NWD >= 64 && NWD % 64 == 0, "chunk width");
    // each wave of the workgroup takes its own items, with its own LDS
    // slices; the waves never meet at a barrier
    __shared__ uint2 sw_all[WAVES][NWD];         // {word, outputs before the word}
    __shared__ Acc cacc_all[WAVES][CAP + 64];  // + one dummy slot per lane
    __shared__ uint32_t st_s_all[WAVES][64];
    __shared__ int st_e_all[WAVES][65];
    __shared__ float st_a_all[WAVES][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint2 *sw = sw_all[wave];
    Acc *cacc = cacc_all[wave];
    uint32_t *st_s = st_s_all[wave];
    int *st_e = st_e_all[wave];
    float *st_a = st_a_all[wave];
    const int64_t first = (xcd_unit(lin_block(), (nitems + WAVES * IPW - 1) / (WAVES * IPW)) *
                               WAVES + wave) * IPW;
    if (first >= nitems) return;  // wave-uniform
    const int64_t last = first + IPW < nitems ? first + IPW : nitems;
    RankIn<KMAX> cur = rank_load<WMAX, CAP>(prods, desc_word(desc, first), sabs, chunk_cnt,
                                            sbits, wpc, resolved);
    uint64_t wnext = first + 1 < last ? desc_word(desc, first + 1) : 0ull;
    bool stray = false;
    for (int64_t item = first; item < last; ++item) {
        const bool more = IPW > 1 && item + 1 < last;
        RankIn<KMAX> nxt;
        if (IPW > 1 && more) {  // the next item's inputs, loaded while this one is processed
            nxt = rank_load<WMAX, CAP>(prods, wnext, sabs, chunk_cnt, sbits, wpc, resolved);
            wnext = item + 2 < last ? desc_word(desc, item + 2) : 0ull;
        }
        const ChunkDesc &d = cur.d;
        const int64_t expect = cur.expect;
        if (expect > 0) {
            const ProdDev &P = prods[d.prod];
            const int c = d.q;
            const int64_t slot = d.slot0 + c;
            const int64_t out0 =
                resolved ? d.out0 : d.out0 + (gld(chunk_pos + slot) - gld(chunk_pos + d.slot0));
            const int lo = c * P.W;
            const int64_t end = (int64_t)lo + (int64_t)d.span * P.W;
            const int hi = (int)(end < P.n ? end : P.n);
            const int nwords = (hi - lo + 31) >> 5;
            if (hi - lo > WMAX) {  // the plan picks WMAX >= the widest item; never taken
                if (lane == 0) atomicOr(err, kErrRow);
                return;
            }
            // sw[x] = {word x, outputs before word x}; lane l holds words
            // l*K .. l*K + K - 1
            const int K = (nwords + 63) >> 6;
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) cnt += __popc(cur.wv[k]);
            int total;
            int pre = wg_excl_scan<64, int>(cnt, nullptr, total);
            const int pre0 = pre;  // the rank of the lane's first output
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < K) {
                    sw[lane * K + k] = make_uint2(cur.wv[k], (uint32_t)pre);
                    pre += __popc(cur.wv[k]);
                }
            for (int r = lane; r < expect; r += 64) cacc[r] = Acc(0);
            cacc[CAP + lane] = Acc(0);
            if (lane == 0 && total != expect) atomicOr(err, kErrChunk);
            wave_lds_sync();
            const int dummy = CAP + lane;
            ItemIn in;
            in.x0 = cur.x0;
            in.x1 = cur.x1;
            in.a = cur.a;
            // items of more than 1,024 outputs are long enough for branch-free
            // (clamped) loads to pay; shorter ones keep masked loads
            pipe_products<64, NVT, true, true, (CAP >= 2048)>(
                P, d, in, sabs, st_s, st_e, st_a, nullptr,
                [&](const int *cc, const float *aa, const float *vv, const bool *ok) {
                    int idx[NVT];
                    Acc add[NVT];
#pragma unroll
                    for (int v = 0; v < NVT; ++v) {
                        const int rel = cc[v] - lo;
                        const uint2 e = sw[(ok[v] ? rel : 0) >> 5];
                        const uint32_t bit = 1u << (rel & 31);
                        const bool in_structure = (e.x & bit) != 0u;
                        stray |= ok[v] && !in_structure;
                        const bool take = ok[v] && in_structure;
                        idx[v] = take ? (int)e.y + __popc(e.x & (bit - 1u)) : dummy;
                        add[v] = take ? Acc(aa[v]) * Acc(vv[v]) : Acc(0);
                    }
                    if constexpr (std::is_same<Acc, float>::value) {
                        lds_fadd_many<NVT>(cacc, idx, add);
                    } else {
#pragma unroll
                        for (int v = 0; v < NVT; ++v)
                            __hip_atomic_fetch_add(cacc + idx[v], add[v], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                },
                lane);
            wave_lds_sync();
            const int ex = (int)expect;
            float *valC = P.valC + out0;
            int32_t *colC = P.colC + out0;
            // The values leave first, coalesced and already in column order.
            for (int r = lane; r < ex; r += 64) gst(valC + r, (float)cacc[r]);
            // The columns, balanced over the lanes.  The structure's non-empty
            // words are listed in column order in the rank table's space (no
            // longer read), each as {word, (word index << 16) | rank of its
            // first output}; lane l then emits the ranks [l S, l S + S),
            // S = ceil(ex / 64): a binary search for the word that holds its
            // first rank, then a walk through the set bits of that word and
            // the next ones.  (A lane expanding its own words would take as
            // many steps as the densest lane's words hold bits: about six
            // times as many on R-MAT chunks.)  The columns are staged in the
            // accumulator, whose values have left, and copied out coalesced.
            int nzc = 0;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) nzc += (k < K && cur.wv[k] != 0u) ? 1 : 0;
            int m;
            int pos = wg_excl_scan<64, int>(nzc, nullptr, m);
            {
                int pre = pre0;
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    if (k < K) {
                        const uint32_t w = cur.wv[k];
                        if (w) {
                            sw[pos] = make_uint2(w, ((uint32_t)(lane * K + k) << 16) | (uint32_t)pre);
                            ++pos;
                        }
                        pre += __popc(w);
                    }
            }
            wave_lds_sync();  // the list is written; the values have been read
            int *ccol = reinterpret_cast<int *>(cacc);
            const int S = (ex + 63) >> 6;
            const int t0 = lane * S;
            const int t1 = t0 + S < ex ? t0 + S : ex;
            if (t0 < t1 && m > 0) {
                int jl = 0, jh = m - 1;  // the last listed word whose first rank is <= t0
                while (jl < jh) {
                    const int mid = (jl + jh + 1) >> 1;
                    if ((int)(sw[mid].y & 0xffffu) <= t0) jl = mid;
                    else jh = mid - 1;
                }
                uint2 e = sw[jl];
                uint32_t w = e.x;
                for (int q = t0 - (int)(e.y & 0xffffu); q > 0 && w; --q) w &= w - 1u;
                int xb = lo + (int)((e.y >> 16) << 5);
                int j = jl;
                for (int t = t0; t < t1; ++t) {
                    while (w == 0u && j + 1 < m) {
                        ++j;
                        e = sw[j];
                        w = e.x;
                        xb = lo + (int)((e.y >> 16) << 5);
                    }
                    if (w == 0u) break;  // fewer set bits than outputs (flagged above)
                    ccol[t] = xb + __builtin_ctz(w);
                    w &= w - 1u;
                }
            }
            wave_lds_sync();
            for (int r = lane; r < ex; r += 64) gst(colC + r, ccol[r]);
            wave_lds_sync();  // the accumulator and structure are reused by the next item
        }
        if (IPW == 1 || !more) break;
        cur = nxt;
    }
    if (stray) atomicOr(err, kErrChunk);  // a product outside the symbolic structure
}

// Workgroups of a pipelined launch: wgs_per_cu per compute unit (a multiple
// of 8 in total, so that the grid covers the eight dies evenly), or one per
// item when wgs_per_cu is 0; never more than there are items, nor more than a
// 1-D grid holds (the workgroups walk the items with a stride of the grid).
static unsigned pipe_grid(int wgs_per_cu, int64_t nitems, int threads) {
    const int64_t limit = int64_t(0xFFFFFFFF) / threads;
    if (wgs_per_cu <= 0) return (unsigned)(nitems < limit ? nitems : limit);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 8;
    int64_t g = (int64_t)wgs_per_cu * cus;
    g -= g % 8;
    if (g < 8) g = 8;
    if (g > nitems) g = nitems;
    return (unsigned)g;
}

// Splits the numeric chunk items (one chunk per item) into five parts,
// keeping the order within each: items with more than `cap` outputs (dense),
// single chunks with more than cap / 2 outputs, single chunks with at most
// cap / 2, merged items with more than cap / 2, merged items with at most
// cap / 2 (a merged item never has more than cap).  The halves get their own
// launches with a half-size accumulator, so more of them fit in a compute
// unit's LDS.  Two flag words per item each pack two counters (low and high
// 32 bits): fa = dense | small single, fb = large merged | small merged; an
// exclusive scan of each gives every item its position.  The launches cover
// an upper bound of the item count; nlim (if set) points at the exact count.
__global__ void k_desc_flag(const ChunkDesc *__restrict__ desc, int64_t nitems,
                            const int64_t *__restrict__ chunk_cnt, int64_t cap,
                            const int64_t *__restrict__ nlim, int64_t *__restrict__ fa,
                            int64_t *__restrict__ fb) {
    const int64_t it = lin_block() * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    int64_t a = 0, b = 0;
    if (!(nlim && it >= *nlim)) {
        const ChunkDesc d = desc[it];
        const int64_t cnt = chunk_cnt[d.slot0 + d.q];
        const bool small = cnt <= cap / 2;
        if (cnt > cap) a = 1;
        else if (d.span > 1) b = small ? (int64_t(1) << 32) : 1;
        else if (small) a = int64_t(1) << 32;
    }
    fa[it] = a;
    fb[it] = b;
}

// The split descriptors are resolved: out0 is the item's own first output
// slot in C_p and pad its output count, so the numeric kernels need no
// further look-ups of the chunk counts and offsets.
__global__ void k_desc_split(const ChunkDesc *__restrict__ desc, int64_t nitems,
                             const int64_t *__restrict__ fa, const int64_t *__restrict__ fapos,
                             const int64_t *__restrict__ fb, const int64_t *__restrict__ fbpos,
                             const int64_t *__restrict__ chunk_cnt,
                             const int64_t *__restrict__ chunk_pos,
                             const int64_t *__restrict__ nlim, ChunkDesc *__restrict__ out) {
    const int64_t it = lin_block() * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    const int64_t n = nlim ? *nlim : nitems;
    if (it >= n) return;
    constexpr int64_t LO = 0xffffffffll;
    const int64_t ta = fapos[nitems], tb = fbpos[nitems];
    const int64_t n_dense = ta & LO, n_s0 = ta >> 32, n_m1 = tb & LO, n_m0 = tb >> 32;
    const int64_t n_s1 = n - n_dense - n_s0 - n_m1 - n_m0;
    const int64_t pa = fapos[it], pb = fbpos[it];
    const int64_t a = fa[it], b = fb[it];
    int64_t pos;
    if (a & LO) pos = pa & LO;                                          // dense
    else if (a >> 32) pos = n_dense + n_s1 + (pa >> 32);                // small single
    else if (b & LO) pos = n_dense + n_s1 + n_s0 + (pb & LO);           // large merged
    else if (b >> 32) pos = n_dense + n_s1 + n_s0 + n_m1 + (pb >> 32);  // small merged
    else pos = n_dense + (it - (pa & LO) - (pa >> 32) - (pb & LO) - (pb >> 32));  // large single
    ChunkDesc d = desc[it];
    const int64_t slot = d.slot0 + d.q;
    d.out0 += chunk_pos[slot] - chunk_pos[d.slot0];
    d.pad = (int32_t)chunk_cnt[slot];
    out[pos] = d;
}

void launch_desc_flag(const ChunkDesc *desc, int64_t nitems, const int64_t *chunk_cnt,
                      int64_t cap, const int64_t *nlim, int64_t *fa, int64_t *fb, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_desc_flag, grid1d(((nitems + 255) / 256), 256), dim3(256), 0, s, desc,
                       nitems, chunk_cnt, cap, nlim, fa, fb);
}

void launch_desc_split(const ChunkDesc *desc, int64_t nitems, const int64_t *fa,
                       const int64_t *fapos, const int64_t *fb, const int64_t *fbpos,
                       const int64_t *chunk_cnt, const int64_t *chunk_pos, const int64_t *nlim,
                       ChunkDesc *out, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_desc_split, grid1d(((nitems + 255) / 256), 256), dim3(256), 0, s,
                       desc, nitems, fa, fapos, fb, fbpos, chunk_cnt, chunk_pos, nlim, out);
}

void launch_bsplit(const int64_t *rptB, const int32_t *colB, int64_t k_rows, int W, int nch,
                   int32_t *bsplit, hipStream_t s) {
    const int64_t n = k_rows * (nch + 1);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bsplit, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, rptB, colB,
                       k_rows, W, nch, bsplit);
}

void launch_nch_of(const ProdDev *prods, const uint64_t *items, int64_t n, int div,
                   int64_t *nchv, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_nch_of, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, n, div, nchv);
}

void launch_expand(const int64_t *base, int64_t n, int32_t *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_expand, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, base, n, out);
}

void launch_sym_desc(const ProdDev *prods, const uint64_t *items, const int32_t *item_of,
                     const int64_t *ibase, const int64_t *cbase, const int64_t *sbase,
                     int64_t nitems, int kper, const int32_t *mstart, const int64_t *nlim,
                     ChunkDesc *desc, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_sym_desc, grid1d(((nitems + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, item_of, ibase, cbase, sbase, nitems, kper, mstart, nlim, desc);
}

void launch_row_splitlen(const ProdDev *prods, const uint64_t *items, int64_t nh, int64_t *len,
                         hipStream_t s) {
    if (nh <= 0) return;
    hipLaunchKernelGGL(k_row_splitlen, grid1d(((nh + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, nh, len);
}

void launch_sabs_tiles(const ProdDev *prods, const uint64_t *items, int64_t nh, int64_t *ntile,
                       hipStream_t s) {
    if (nh <= 0) return;
    hipLaunchKernelGGL(k_sabs_tiles, grid1d(((nh + 255) / 256), 256), dim3(256), 0, s, prods,
                       items, nh, ntile);
}

void launch_sabs(const ProdDev *prods, const uint64_t *items, int64_t ntiles,
                 const int32_t *tile_row, const int64_t *tbase, const int64_t *sbase,
                 uint32_t *sabs, const int64_t *cbase, unsigned long long *ipc, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_sabs, grid1d(ntiles, 256), dim3(256), 0, s, prods, items, ntiles, tile_row,
                       tbase, sbase, sabs, cbase, ipc);
}

void launch_chunk_items(const ProdDev *prods, const uint64_t *items, int64_t nh, int merge,
                        int64_t cap, const int64_t *cbase, const unsigned long long *ipc,
                        int32_t *mstart, int64_t *nitem, hipStream_t s) {
    if (nh <= 0) return;
    hipLaunchKernelGGL(k_chunk_items, grid1d(((nh + 3) / 4), 256), dim3(256), 0, s, prods,
                       items, nh, merge, cap, cbase, ipc, mstart, nitem);
}

void launch_num_nitems(const ProdDev *prods, const uint64_t *ditems, int64_t n,
                       const int32_t *hslot, const int64_t *nitem, int64_t *dnch, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_num_nitems, grid1d(((n + 255) / 256), 256), dim3(256), 0, s, prods,
                       ditems, n, hslot, nitem, dnch);
}

void launch_num_desc(const ProdDev *prods, const uint64_t *ditems, const int32_t *item_of,
                     const int64_t *dbase, int64_t nitems, int kper, const int32_t *hslot,
                     const int64_t *cbase, const int64_t *sbase, const int64_t *rptv,
                     const int32_t *mstart, const int64_t *nlim, ChunkDesc *desc, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_num_desc, grid1d(((nitems + 255) / 256), 256), dim3(256), 0, s, prods,
                       ditems, item_of, dbase, nitems, kper, hslot, cbase, sbase, rptv, mstart,
                       nlim, desc);
}

template <bool FAST>
static void sym_chunk_launch(int wmax, const ProdDev *prods, const ChunkDesc *desc,
                             const uint32_t *sabs, int64_t nitems, int kper, int64_t *chunk_cnt,
                             int64_t *row_nnz, uint32_t *sbits, int wpc, hipStream_t s) {
    if (wmax <= 2048)
        hipLaunchKernelGGL((k_sym_chunk<64, 2048, FAST>), grid1d(nitems, 64), dim3(64), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, row_nnz, sbits, wpc);
    else if (wmax <= 4096)
        hipLaunchKernelGGL((k_sym_chunk<128, 4096, FAST>), grid1d(nitems, 128), dim3(128), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, row_nnz, sbits, wpc);
    else if (wmax <= 8192)
        hipLaunchKernelGGL((k_sym_chunk<256, 8192, FAST>), grid1d(nitems, 256), dim3(256), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, row_nnz, sbits, wpc);
    else
        hipLaunchKernelGGL((k_sym_chunk<256, kMaxChunkCols, FAST>), grid1d(nitems, 256), dim3(256), 0, s,
                           prods, desc, nitems, sabs, kper, chunk_cnt, row_nnz, sbits, wpc);
}

template <int WG, int WMAX>
static void sym_pipe_launch(const ProdDev *prods, const ChunkDesc *desc, const uint32_t *sabs,
                            int64_t nitems, int64_t *chunk_cnt, int64_t *row_nnz,
                            uint32_t *sbits, int wpc, int wgs_per_cu, int *err, hipStream_t s) {
    const unsigned g = pipe_grid(wgs_per_cu, nitems, WG);
    hipLaunchKernelGGL((k_sym_chunk_pipe<WG, WMAX>), dim3(g), dim3(WG), 0, s, prods, desc, nitems,
                       sabs, chunk_cnt, row_nnz, sbits, wpc, err);
}

template <int WMAX>
static void sym_pipe_wg(int wg, const ProdDev *prods, const ChunkDesc *desc, const uint32_t *sabs,
                        int64_t nitems, int64_t *chunk_cnt, int64_t *row_nnz, uint32_t *sbits,
                        int wpc, int wgs_per_cu, int *err, hipStream_t s) {
    switch (wg) {
    case 64:
        sym_pipe_launch<64, WMAX>(prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                                  wgs_per_cu, err, s);
        break;
    case 128:
        sym_pipe_launch<128, WMAX>(prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                                   wgs_per_cu, err, s);
        break;
    case 512:
        sym_pipe_launch<512, WMAX>(prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                                   wgs_per_cu, err, s);
        break;
    default:
        sym_pipe_launch<256, WMAX>(prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                                   wgs_per_cu, err, s);
    }
}

// wmax: widest item (merged items included).
void launch_sym_chunk(int wmax, bool fast, const ProdDev *prods, const ChunkDesc *desc,
                      const uint32_t *sabs, int64_t nitems, int kper, int64_t *chunk_cnt,
                      int64_t *row_nnz, uint32_t *sbits, int wpc, int wgs_per_cu, int threads,
                      int *err, hipStream_t s) {
    if (nitems <= 0) return;
    if (fast && kper == 1) {
        const int t = threads ? threads : 64;
        if (wmax <= 2048)
            sym_pipe_wg<2048>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                              wgs_per_cu, err, s);
        else if (wmax <= 4096)
            sym_pipe_wg<4096>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                              wgs_per_cu, err, s);
        else if (wmax <= 8192)
            sym_pipe_wg<8192>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                              wgs_per_cu, err, s);
        else if (wmax <= 16384)
            sym_pipe_wg<16384>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                               wgs_per_cu, err, s);
        else if (wmax <= 32768)
            sym_pipe_wg<32768>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits, wpc,
                               wgs_per_cu, err, s);
        else
            sym_pipe_wg<kMaxItemCols>(t, prods, desc, sabs, nitems, chunk_cnt, row_nnz, sbits,
                                      wpc, wgs_per_cu, err, s);
        return;
    }
    if (fast)
        sym_chunk_launch<true>(wmax, prods, desc, sabs, nitems, kper, chunk_cnt, row_nnz, sbits,
                               wpc, s);
    else
        sym_chunk_launch<false>(wmax, prods, desc, sabs, nitems, kper, chunk_cnt, row_nnz, sbits,
                                wpc, s);
}

template <bool FAST>
static void num_chunk_launch(int wmax, const ProdDev *prods, const ChunkDesc *desc,
                             const uint32_t *sabs, int64_t nitems, int kper,
                             const int64_t *chunk_cnt, const int64_t *chunk_pos,
                             const uint32_t *sbits, int wpc, int *err, hipStream_t s) {
    if (wmax <= 2048)
        hipLaunchKernelGGL((k_num_chunk<64, 2048, FAST>), grid1d(nitems, 64), dim3(64), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, chunk_pos, sbits, wpc, err);
    else if (wmax <= 4096)
        hipLaunchKernelGGL((k_num_chunk<128, 4096, FAST>), grid1d(nitems, 128), dim3(128), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, chunk_pos, sbits, wpc, err);
    else if (wmax <= 8192)
        hipLaunchKernelGGL((k_num_chunk<256, 8192, FAST>), grid1d(nitems, 256), dim3(256), 0, s, prods,
                           desc, nitems, sabs, kper, chunk_cnt, chunk_pos, sbits, wpc, err);
    else
        hipLaunchKernelGGL((k_num_chunk<512, kMaxChunkCols, FAST>), grid1d(nitems, 512), dim3(512), 0, s,
                           prods, desc, nitems, sabs, kper, chunk_cnt, chunk_pos, sbits, wpc, err);
}

template <int WG, int WMAX>
static void num_pipe_launch(const ProdDev *prods, const ChunkDesc *desc, const uint32_t *sabs,
                            int64_t nitems, const int64_t *chunk_cnt, const int64_t *chunk_pos,
                            const uint32_t *sbits, int wpc, int wgs_per_cu, int rank_cap,
                            bool resolved, int *err, hipStream_t s) {
    const unsigned g = pipe_grid(wgs_per_cu, nitems, WG);
    hipLaunchKernelGGL((k_num_chunk_pipe<WG, WMAX>), dim3(g), dim3(WG), 0, s, prods, desc, nitems,
                       sabs, chunk_cnt, chunk_pos, sbits, wpc, (int64_t)rank_cap,
                       resolved ? 1 : 0, err);
}

template <int RW>
static void num_rank_launch(const ProdDev *prods, const ChunkDesc *desc, const uint32_t *sabs,
                            int64_t nitems, const int64_t *chunk_cnt, const int64_t *chunk_pos,
                            const uint32_t *sbits, int wpc, int rank_cap, bool resolved, int *err,
                            hipStream_t s) {
    const int res = resolved ? 1 : 0;
    constexpr int IPW = kRankItems, WV = kRankWaves;
    const int64_t per_wg = (int64_t)IPW * WV;
    const dim3 grid = grid1d((nitems + per_wg - 1) / per_wg, 64 * WV), block(64 * WV);
    if (rank_cap <= 256)
        hipLaunchKernelGGL((k_num_chunk_rank<RW, 256, IPW, WV>), grid, block, 0, s, prods, desc,
                           nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
    else if (rank_cap <= 512)
        hipLaunchKernelGGL((k_num_chunk_rank<RW, 512, IPW, WV>), grid, block, 0, s, prods, desc,
                           nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
    else if (rank_cap <= 1024)
        hipLaunchKernelGGL((k_num_chunk_rank<RW, 1024, IPW, WV>), grid, block, 0, s, prods,
                           desc, nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
    else
        hipLaunchKernelGGL((k_num_chunk_rank<RW, 2048, IPW, WV>), grid, block, 0, s, prods,
                           desc, nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
}

bool num_chunk_rank_used(bool fast, int kper, int rank_cap) {
    return fast && kper == 1 && rank_cap > 0;
}

// FP64 accumulation: the plan keeps every item within 2048 columns (chunks
// of at most 2048 columns, not merged), so only that width is instantiated.
static bool num_rank_launch_f64(int wmax, const ProdDev *prods, const ChunkDesc *desc,
                                const uint32_t *sabs, int64_t nitems, const int64_t *chunk_cnt,
                                const int64_t *chunk_pos, const uint32_t *sbits, int wpc,
                                int rank_cap, bool resolved, int *err, hipStream_t s) {
    if (wmax > 2048 || rank_cap < 1024) return false;
    const int res = resolved ? 1 : 0;
    const dim3 grid = grid1d(nitems, 64), block(64);
    if (rank_cap <= 1024)
        hipLaunchKernelGGL((k_num_chunk_rank<2048, 1024, 1, 1, double>), grid, block, 0, s,
                           prods, desc, nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
    else
        hipLaunchKernelGGL((k_num_chunk_rank<2048, 2048, 1, 1, double>), grid, block, 0, s,
                           prods, desc, nitems, sabs, chunk_cnt, chunk_pos, sbits, wpc, res, err);
    return true;
}

// wmax: widest item of the launch.  f64: accumulate in FP64 (returns false,
// launching nothing, for a shape the FP64 kernel does not cover).
bool launch_num_chunk_rank(int wmax, const ProdDev *prods, const ChunkDesc *desc,
                           const uint32_t *sabs, int64_t nitems, const int64_t *chunk_cnt,
                           const int64_t *chunk_pos, const uint32_t *sbits, int wpc, int rank_cap,
                           bool resolved, int *err, hipStream_t s, bool f64) {
    if (nitems <= 0 || rank_cap <= 0) return true;
    if (f64)
        return num_rank_launch_f64(wmax, prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits,
                                   wpc, rank_cap, resolved, err, s);
    if (wmax <= 2048)
        num_rank_launch<2048>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                              rank_cap, resolved, err, s);
    else if (wmax <= 4096)
        num_rank_launch<4096>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                              rank_cap, resolved, err, s);
    else if (wmax <= 8192)
        num_rank_launch<8192>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                              rank_cap, resolved, err, s);
    else if (wmax <= 16384)
        num_rank_launch<16384>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                               rank_cap, resolved, err, s);
    else if (wmax <= 32768)
        num_rank_launch<32768>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                               rank_cap, resolved, err, s);
    else
        num_rank_launch<kMaxItemCols>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits,
                                      wpc, rank_cap, resolved, err, s);
    return true;
}

template <int WMAX>
static void num_pipe_wg(int wg, const ProdDev *prods, const ChunkDesc *desc, const uint32_t *sabs,
                        int64_t nitems, const int64_t *chunk_cnt, const int64_t *chunk_pos,
                        const uint32_t *sbits, int wpc, int wgs_per_cu, int rank_cap,
                        bool resolved, int *err, hipStream_t s) {
    switch (wg) {
    case 64:
        num_pipe_launch<64, WMAX>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                                  wgs_per_cu, rank_cap, resolved, err, s);
        break;
    case 128:
        num_pipe_launch<128, WMAX>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                                   wgs_per_cu, rank_cap, resolved, err, s);
        break;
    case 512:
        num_pipe_launch<512, WMAX>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                                   wgs_per_cu, rank_cap, resolved, err, s);
        break;
    default:
        num_pipe_launch<256, WMAX>(prods, desc, sabs, nitems, chunk_cnt, chunk_pos, sbits, wpc,
                                   wgs_per_cu, rank_cap, resolved, err, s);
    }
}

void launch_num_chunk(int wmax, bool fast, const ProdDev *prods, const ChunkDesc *desc,
                      const uint32_t *sabs, int64_t nitems, int kper, const int64_t *chunk_cnt,
                      const int64_t *chunk_pos, const uint32_t *sbits, int wpc, int wgs_per_cu,
                      int threads, int rank_cap, bool resolved, int *err, hipStream_t s) {
    if (nitems <= 0) return;
    if (fast && kper == 1) {
        if (wmax <= 2048)
            num_pipe_wg<2048>(threads ? threads : 64, prods, desc, sabs, nitems, chunk_cnt,
                              chunk_pos, sbits, wpc, wgs_per_cu, rank_cap, resolved, err, s);
        else if (wmax <= 4096)
            num_pipe_wg<4096>(threads ? threads : 128, prods, desc, sabs, nitems, chunk_cnt,
                              chunk_pos, sbits, wpc, wgs_per_cu, rank_cap, resolved, err, s);
        else if (wmax <= 8192)
            num_pipe_wg<8192>(threads ? threads : 256, prods, desc, sabs, nitems, chunk_cnt,
                              chunk_pos, sbits, wpc, wgs_per_cu, rank_cap, resolved, err, s);
        else
            num_pipe_wg<kMaxChunkCols>(threads ? threads : 512, prods, desc, sabs, nitems,
                                       chunk_cnt, chunk_pos, sbits, wpc, wgs_per_cu, rank_cap, resolved, err, s);
        return;
    }
    if (fast)
        num_chunk_launch<true>(wmax, prods, desc, sabs, nitems, kper, chunk_cnt, chunk_pos, sbits,
                               wpc, err, s);
    else
        num_chunk_launch<false>(wmax, prods, desc, sabs, nitems, kper, chunk_cnt, chunk_pos,
                                sbits, wpc, err, s);
}

}  // namespace spg
