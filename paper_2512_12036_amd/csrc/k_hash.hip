// Hash-table kernels of the allocation (symbolic) and accumulation (numeric)
// phases, paper Sections III-C / III-D, Algorithms 2-5.
//
// Open addressing with linear probing in LDS (paper Algorithm 4): a slot holds
// -1 when empty, a key is claimed with a compare-and-swap, the claiming lane
// counts one distinct column, and the numeric variant adds the FP32 product
// into the value slot with an LDS float atomic.  Tables are sized so that
// they are never more than half full; a probe-count guard turns an
// impossible overflow into an error flag instead of a hang.
//
// Work mapping for 64-lane wavefronts (the paper's mappings, Algorithms 2-3,
// are written for 32-lane warps and are not kept):
//  * group kernels: G = 8/16/32/64 lanes per row, 256/G rows per workgroup,
//    a table of 8G slots per row.  The G lanes load G nonzeros of the A row,
//    scan their B-row lengths with lane shuffles and then walk the
//    concatenated products G at a time, each lane finding its product's
//    owner by a binary search over the shuffled prefix.  All lanes stay busy
//    whatever the B-row lengths are.
//  * block kernels: one row per 256- or 512-thread workgroup, tables up to
//    32 K keys (symbolic) or 16 K key/value pairs (numeric).  Batches of A
//    nonzeros are staged in LDS with the start of their B row and a block
//    prefix of the lengths; the products are then enumerated flat, so the
//    whole workgroup is busy even for rows of few, long B rows.
//  * numeric epilogue (paper Section III-D): occupied slots are gathered,
//    sorted by column (rank sort in the group kernels, as the paper's
//    comparison-based ranking; bitonic sort in LDS in the block kernels, as
//    paper Algorithm 5) and written to the row's segment of C.
#include "dev.hpp"

namespace spg {

__device__ __forceinline__ int lds_insert(int *tab, uint32_t mask, int log2T, int c, int *err) {
    uint32_t h = hash_slot(c, log2T);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        int cur = tab[h];
        if (cur == c) return 0;
        if (cur == kEmptyKey) {
            int old = atomicCAS(&tab[h], kEmptyKey, c);
            if (old == kEmptyKey) return 1;
            if (old == c) return 0;
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrProbe);
    return 0;
}

__device__ __forceinline__ void lds_add(int *tab, float *vals, uint32_t mask, int log2T, int c,
                                        float v, int *err) {
    uint32_t h = hash_slot(c, log2T);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        int cur = tab[h];
        if (cur == c) { lds_fadd(&vals[h], v); return; }
        if (cur == kEmptyKey) {
            int old = atomicCAS(&tab[h], kEmptyKey, c);
            if (old == kEmptyKey || old == c) { lds_fadd(&vals[h], v); return; }
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrProbe);
}

// Slot of key c in the table, inserting it when absent (linear probing from
// slot h); -1 after the probe guard tripped.
__device__ __forceinline__ int lds_slot(int *tab, uint32_t mask, uint32_t h, int c, int *err) {
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const int cur = tab[h];
        if (cur == c) return (int)h;
        if (cur == kEmptyKey) {
            const int old = atomicCAS(&tab[h], kEmptyKey, c);
            if (old == kEmptyKey || old == c) return (int)h;
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrProbe);
    return -1;
}

// Batched forms of lds_insert / lds_add for U products of a lane: the home
// slots of all U keys are read before any is compared, so the common case
// (key already at its home slot) costs one LDS round trip for all U; the
// rest take the probing path one by one.  For the accumulation the values
// then go through lds_fadd_many; unused entries (ok false) add 0 to the
// lane's private dummy slot `dummy` of vals.
template <int U>
__device__ __forceinline__ int lds_insert_many(int *tab, uint32_t mask, int log2T, const int *cc,
                                               const bool *ok, int *err) {
    int k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = ok[u] ? tab[hash_slot(cc[u], log2T)] : 0;
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (ok[u] && k[u] != cc[u]) cnt += lds_insert(tab, mask, log2T, cc[u], err);
    return cnt;
}

template <int U>
__device__ __forceinline__ void lds_add_many(int *tab, float *vals, uint32_t mask, int log2T,
                                             const int *cc, const float *add, const bool *ok,
                                             int dummy, int *err) {
    uint32_t h[U];
    int k[U], slot[U];
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        h[u] = hash_slot(cc[u], log2T);
        k[u] = ok[u] ? tab[h[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int sl = dummy;
        if (ok[u]) {
            sl = k[u] == cc[u] ? (int)h[u] : lds_slot(tab, mask, h[u], cc[u], err);
            if (sl < 0) sl = dummy;
        }
        slot[u] = sl;
        v[u] = sl != dummy ? add[u] : 0.f;
    }
    lds_fadd_many<U>(vals, slot, v);
}

// Direct-mapped forms, for rows whose B has no more columns than the table
// has slots: the slot of column c is c itself -- no hashing, no probing, and
// the occupied slots are already in column order, so no sort follows.
template <int U>
__device__ __forceinline__ int lds_mark_many(int *tab, const int *cc, const bool *ok) {
    int k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = ok[u] ? tab[cc[u]] : 0;
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (ok[u] && k[u] != cc[u]) cnt += atomicCAS(&tab[cc[u]], kEmptyKey, cc[u]) == kEmptyKey;
    return cnt;
}

template <int U>
__device__ __forceinline__ void lds_add_direct_many(int *tab, float *vals, const int *cc,
                                                    const float *add, const bool *ok, int dummy) {
    int slot[U];
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        slot[u] = ok[u] ? cc[u] : dummy;
        v[u] = ok[u] ? add[u] : 0.f;
        if (ok[u]) tab[cc[u]] = cc[u];  // every writer stores the same key
    }
    lds_fadd_many<U>(vals, slot, v);
}

// Direct-mapped accumulation without keys, for the group kernels: a value
// slot that no product reached holds the bit pattern kEmptyVal.  The first
// product of a slot adds to 0 (as a zero-initialised slot would), and a sum
// whose bits happen to equal kEmptyVal (a NaN) is stored as the canonical
// quiet NaN, so a slot is occupied exactly when its bits differ from
// kEmptyVal.  This saves the key store of every product.  Unused entries
// (ok false) add 0 to the lane's dummy slot, which starts at 0.
constexpr uint32_t kEmptyVal = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t fold_slot(uint32_t cur, float add) {
    const float base = cur == kEmptyVal ? 0.f : __uint_as_float(cur);
    const uint32_t r = __float_as_uint(base + add);
    return r == kEmptyVal ? 0x7FC00000u : r;
}

template <int U>
__device__ __forceinline__ void lds_add_direct_nokey(float *vals, const int *cc, const float *add,
                                                     const bool *ok, int dummy) {
    uint32_t *q = reinterpret_cast<uint32_t *>(vals);
    int slot[U];
    float v[U];
    uint32_t cur[U], prev[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        slot[u] = ok[u] ? cc[u] : dummy;
        v[u] = ok[u] ? add[u] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        cur[u] = __hip_atomic_load(q + slot[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int u = 0; u < U; ++u) prev[u] = atomicCAS(q + slot[u], cur[u], fold_slot(cur[u], v[u]));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        uint32_t c = prev[u];
        bool pending = prev[u] != cur[u];
        while (pending) {
            const uint32_t p = atomicCAS(q + slot[u], c, fold_slot(c, v[u]));
            pending = p != c;
            c = p;
        }
    }
}

template <int N>
struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <>
struct Log2<1> { static constexpr int v = 0; };

__device__ __forceinline__ int ceil_log2(int64_t x) {
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

// ---------------------------------------------------------------------------
// Group kernels: G lanes per row.
// ---------------------------------------------------------------------------
// The output columns of row i of a direct-mapped product (P.n <= 8 G) from
// B's row bitmaps: the OR of the bitmaps of the B rows that the row's A
// nonzeros name, without visiting a product.  ws lanes per stride (a power
// of two >= P.bmw, at most G / 4), one word each, G / ws A nonzeros at a
// time; returns in every lane word (lane & (ws - 1)) of the row's bitmap
// (zero past P.bmw).
template <int G>
__device__ __forceinline__ uint32_t row_bitmap_word(const ProdDev &P, int64_t i, int lane,
                                                    int &ws) {
    const int bmw = P.bmw;
    ws = 1;
    while (ws < bmw) ws <<= 1;
    const int w = lane & (ws - 1), r = lane / ws, R = G / ws;
    const int64_t a0 = gld(P.rptA + i), a1 = gld(P.rptA + i + 1);
    uint32_t acc = 0u;
    if (w < bmw)
        for (int64_t j = a0 + r; j < a1; j += R)
            acc |= gld(P.bmB + (int64_t)gld(P.colA + j) * bmw + w);
    for (int off = ws; off < G; off <<= 1) acc |= __shfl_xor(acc, off, G);
    return acc;
}

// Walks every intermediate product of row i of P with the G lanes of a group
// and calls f(col_b, a_value, b_value) for each.  The row's A nonzeros are
// staged G at a time in the group's LDS slice (B-row start, exclusive prefix
// of the B-row lengths, A value); lane l then takes products l, l + G, ...
// (consecutive lanes read consecutive B entries) and finds each product's B
// row by walking forward through the staged prefix, one LDS read per B-row
// boundary crossed.  A group lives inside one wave, so its LDS traffic is
// ordered without a barrier.  Group-uniform control flow; U products per lane
// per round (U gathers in flight), handed to f(cc, aa, vv, ok) as arrays.
template <int G, int U, bool VALUES, typename F>
__device__ __forceinline__ void group_products(const ProdDev &P, int64_t i, int lane,
                                               int64_t *gs_s, int *gs_e, float *gs_a, F &&f) {
    static_assert(64 % G == 0, "a group must live inside one wave");
    const int64_t a0 = gld(P.rptA + i), a1 = gld(P.rptA + i + 1);
    const int32_t *colB = P.colB;
    const float *valB = P.valB;
    for (int64_t jb = a0; jb < a1; jb += G) {
        const int64_t j = jb + lane;
        int64_t s = 0;
        int len = 0;
        float a = 0.f;
        if (j < a1) {
            const int k = gld(P.colA + j);
            s = gld(P.rptB + k);
            len = (int)(gld(P.rptB + k + 1) - s);
            if (VALUES) a = gld(P.valA + j);
        }
        const int incl = seg_incl_scan<G>(len);
        const int total = seg_last<G>(incl);
        gs_s[lane] = s;
        gs_e[lane] = incl - len;
        if (VALUES) gs_a[lane] = a;
        if (lane == G - 1) gs_e[G] = total;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        int o = 0;
        int e0 = 0, e1 = gs_e[1];
        int64_t base = gs_s[0];
        float av = VALUES ? gs_a[0] : 0.f;
        for (int qb = 0; qb < total; qb += G * U) {
            int cc[U];
            float aa[U], vv[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = qb + u * G + lane;
                ok[u] = q < total;
                cc[u] = 0;
                aa[u] = 0.f;
                vv[u] = 0.f;
                if (ok[u]) {
                    while (q >= e1) {
                        ++o;
                        e0 = e1;
                        e1 = gs_e[o + 1];
                        base = gs_s[o];
                        if (VALUES) av = gs_a[o];
                    }
                    cc[u] = gld(colB + base + (q - e0));
                    if (VALUES) vv[u] = gld(valB + base + (q - e0));
                    aa[u] = av;
                }
            }
            f(cc, aa, vv, ok);
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // staging reads done
    }
}

// The rows blk * R .. blk * R + R - 1 of the group (one block's share).
template <int G>
__device__ __forceinline__ void sym_group_rows(const ProdDev *__restrict__ prods,
                                               const uint64_t *__restrict__ items, int64_t count,
                                               int64_t *__restrict__ row_nnz,
                                               int *__restrict__ err, int64_t blk) {
    constexpr int T = 8 * G, R = 256 / G, LOG2T = Log2<T>::v;
    __shared__ int keys[R * T];
    __shared__ int64_t st_s[256];
    __shared__ int st_e[R * (G + 1)];
    for (int s = threadIdx.x; s < R * T; s += 256) keys[s] = kEmptyKey;
    __syncthreads();
    const int gi = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t it = blk * R + gi;
    if (it >= count) return;  // group-uniform; no block barrier follows
    const uint64_t e = items[it];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    int *tab = keys + gi * T;
    int cnt = 0;
    const bool direct = P.n <= T;
    if (direct && P.bmw > 0) {
        // the count from B's row bitmaps: each word once (lanes < ws)
        int ws;
        const uint32_t word = row_bitmap_word<G>(P, i, lane, ws);
        cnt = lane < ws ? __popc(word) : 0;
    } else {
        group_products<G, 4, false>(
            P, i, lane, st_s + gi * G, st_e + gi * (G + 1), nullptr,
            [&](const int *cc, const float *, const float *, const bool *ok) {
                cnt += direct ? lds_mark_many<4>(tab, cc, ok)
                              : lds_insert_many<4>(tab, T - 1, LOG2T, cc, ok, err);
            });
    }
    cnt = seg_last<G>(seg_incl_scan<G>(cnt));
    if (lane == 0) row_nnz[P.row_base + i] = cnt;
}

// A workgroup takes the R rows of block blockIdx.x.  Host-sized launches
// cover the group exactly; device-sized ones (DEV) cover an upper bound of
// its rows, read the group's range from the device and exit past its end.
// Empty workgroups cost a few hundred cycles, far less than a work counter
// shared by a whole grid of short blocks.
template <int G, bool DEV>
__global__ __launch_bounds__(256) void k_sym_group(const ProdDev *__restrict__ prods,
                                                    const uint64_t *__restrict__ items,
                                                    int64_t count, int64_t *__restrict__ row_nnz,
                                                    int *__restrict__ err,
                                                    const int64_t *__restrict__ gstart, int gsel) {
    constexpr int R = 256 / G;
    const int64_t blk = lin_block();
    if constexpr (DEV) {
        group_range(gstart, gsel, items, count);
        if (blk * R >= count) return;  // block-uniform
    }
    sym_group_rows<G>(prods, items, count, row_nnz, err, blk);
}

// TB threads per workgroup: TB / G rows, each a group of G lanes.  DONLY:
// every product's B fits the direct-mapped table (the launcher checked), so
// no key table is held and the workgroup needs less LDS.
template <int G, int TB, bool DONLY>
__device__ __forceinline__ void num_group_rows(const ProdDev *__restrict__ prods,
                                               const uint64_t *__restrict__ items, int64_t count,
                                               const int64_t *__restrict__ rptv,
                                               int *__restrict__ err, int64_t blk) {
    constexpr int T = 8 * G, R = TB / G, LOG2T = Log2<T>::v, PER = T / G;
    __shared__ int keys[DONLY ? 1 : R * T];
    __shared__ float vals[R * (T + G)];  // per group: T slots + G dummy slots
    __shared__ int64_t st_s[TB];
    __shared__ int st_e[R * (G + 1)];
    __shared__ float st_a[TB];
    const int gi = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t it = blk * R + gi;
    const bool active = it < count;
    int *tab = keys + (DONLY ? 0 : gi * T);  // not used when DONLY
    float *tv = vals + gi * (T + G);
    uint32_t *tvb = reinterpret_cast<uint32_t *>(tv);
    uint64_t e = 0;
    bool direct = DONLY;
    if (active) {
        e = items[it];
        direct = DONLY || prods[item_prod(e)].n <= T;
    }
    // each group clears its own table: direct-mapped ones hold no keys and
    // mark untouched value slots with kEmptyVal
    if (!direct)
        for (int s = lane; s < T; s += G) tab[s] = kEmptyKey;
    const uint32_t fill = direct ? kEmptyVal : 0u;
    for (int s = lane; s < T; s += G) tvb[s] = fill;
    tvb[T + lane] = 0u;
    __syncthreads();
    if (active) {
        const ProdDev &P = prods[item_prod(e)];
        group_products<G, 4, true>(
            P, item_row(e), lane, st_s + gi * G, st_e + gi * (G + 1), st_a + gi * G,
            [&](const int *cc, const float *aa, const float *vb, const bool *ok) {
                float add[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) add[u] = aa[u] * vb[u];
                if (direct)
                    lds_add_direct_nokey<4>(tv, cc, add, ok, T + lane);
                else
                    lds_add_many<4>(tab, tv, T - 1, LOG2T, cc, add, ok, T + lane, err);
            });
    }
    __syncthreads();
    // gather: each lane owns slots lane + G*r (round r of the group covers
    // slots r*G .. r*G + G - 1, in lane order)
    int kk[PER];
    float vv[PER];
    int mine = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        if (direct) {
            const int q = lane + G * r;
            const uint32_t b = tvb[q];
            kk[r] = b != kEmptyVal ? q : kEmptyKey;
            vv[r] = __uint_as_float(b);
        } else {
            const int q = lane + G * r;
            kk[r] = tab[q];
            vv[r] = tv[q];
        }
        mine += kk[r] != kEmptyKey;
    }
    const int incl = seg_incl_scan<G>(mine);
    const int n = seg_last<G>(incl);
    int pos = incl - mine;
    __syncthreads();
    if (active && !direct) {
#pragma unroll
        for (int r = 0; r < PER; ++r)
            if (kk[r] != kEmptyKey) { tab[pos] = kk[r]; ++pos; }
    }
    __syncthreads();
    if (!active) return;  // no block barrier follows
    const ProdDev &P = prods[item_prod(e)];
    const int64_t g = P.row_base + item_row(e);
    const int64_t expect = rptv[g + 1] - rptv[g];
    if (lane == 0 && n != expect) atomicOr(err, kErrCount);
    if (direct) {
        // slot = column, so the rounds are in column order: an entry's
        // place is the entries of the earlier rounds plus the group's lanes
        // below it in its round (a ballot over the group's lanes), and each
        // round's stores are consecutive
        const int64_t base = c_base(P, rptv, g);
        const int gbase = (int)(threadIdx.x & 63) & ~(G - 1);  // group's first lane in the wave
        const uint64_t below = (1ull << lane) - 1ull;
        int run = 0;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const bool occ = kk[r] != kEmptyKey;
            uint64_t b = __ballot(occ);
            if (G < 64) b = (b >> gbase) & ((1ull << (G & 63)) - 1ull);
            if (occ) {
                const int q = run + __popcll(b & below);
                if (q < expect) {
                    gst(P.colC + base + q, kk[r]);
                    gst(P.valC + base + q, vv[r]);
                }
            }
            run += __popcll(b);
        }
        return;
    }
    // rank of each held key among the n gathered keys (keys are distinct)
    int rank[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) rank[r] = 0;
    for (int f = 0; f < n; ++f) {
        const int kf = tab[f];
#pragma unroll
        for (int r = 0; r < PER; ++r) rank[r] += kf < kk[r];
    }
    const int64_t base = c_base(P, rptv, g);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        if (kk[r] != kEmptyKey && rank[r] < expect) {
            gst(P.colC + base + rank[r], kk[r]);
            gst(P.valC + base + rank[r], vv[r]);
        }
    }
}

template <int G, bool DEV, int TB, bool DONLY>
__global__ __launch_bounds__(TB) void k_num_group(const ProdDev *__restrict__ prods,
                                                   const uint64_t *__restrict__ items,
                                                   int64_t count, const int64_t *__restrict__ rptv,
                                                   int *__restrict__ err,
                                                   const int64_t *__restrict__ gstart, int gsel) {
    constexpr int R = TB / G;
    const int64_t blk = lin_block();
    if constexpr (DEV) {
        group_range(gstart, gsel, items, count);
        if (blk * R >= count) return;  // block-uniform
        if (*err & kErrCapacity) return;  // C does not fit its arena (block-uniform)
    }
    num_group_rows<G, TB, DONLY>(prods, items, count, rptv, err, blk);
}

// ---------------------------------------------------------------------------
// Block kernels: one row per workgroup.
// ---------------------------------------------------------------------------
template <int WG, int U, bool VALUES, typename F>
__device__ __forceinline__ void block_products(const ProdDev &P, int64_t i, int64_t *st_s,
                                               int *st_e, float *st_a, int *wsum, F &&f) {
    const int64_t a0 = gld(P.rptA + i), a1 = gld(P.rptA + i + 1);
    for (int64_t jb = a0; jb < a1; jb += WG) {
        const int64_t j = jb + threadIdx.x;
        int64_t s = 0;
        int len = 0;
        float a = 0.f;
        if (j < a1) {
            const int k = gld(P.colA + j);
            s = gld(P.rptB + k);
            len = (int)(gld(P.rptB + k + 1) - s);
            if (VALUES) a = gld(P.valA + j);
        }
        int total;
        const int excl = block_excl_scan<WG, int>(len, wsum, total);
        st_s[threadIdx.x] = s;
        st_e[threadIdx.x] = excl;
        if (threadIdx.x == 0) st_e[WG] = total;
        if (VALUES) st_a[threadIdx.x] = a;
        __syncthreads();
        const int nv = (int)((a1 - jb) < WG ? (a1 - jb) : WG);
        striped_products<WG, U, VALUES, int, int64_t>(st_s, st_e, st_a, nv, total, P.colB,
                                                      P.valB, f);
        __syncthreads();
    }
}

template <int WG, int TMAX>
__device__ __forceinline__ void sym_block_row(const ProdDev *__restrict__ prods,
                                              const uint64_t *__restrict__ items,
                                              const int64_t *__restrict__ ipv,
                                              int64_t *__restrict__ row_nnz,
                                              int *__restrict__ err, int64_t it) {
    __shared__ int keys[TMAX];
    __shared__ int64_t st_s[WG];
    __shared__ int st_e[WG + 1];
    __shared__ int wsum[WG / 64];
    const uint64_t e = items[it];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t g = P.row_base + i;
    const int64_t a0 = P.rptA[i];
    if (P.rptA[i + 1] - a0 == 1 && P.b_unique == 1) {
        // one A nonzero and strictly ascending B rows: the row's structure is
        // that B row's (block-uniform; no barrier has been reached)
        if (threadIdx.x == 0) {
            const int k = P.colA[a0];
            row_nnz[g] = P.rptB[k + 1] - P.rptB[k];
        }
        return;
    }
    int64_t bound = ipv[g] < P.n ? ipv[g] : P.n;
    // direct-mapped (slot = column) when B's columns fit the table
    const bool direct = P.n <= TMAX;
    int log2T = ceil_log2(direct ? P.n : 2 * bound);
    if (log2T < 8) log2T = 8;
    if (log2T > Log2<TMAX>::v) log2T = Log2<TMAX>::v;
    const int T = 1 << log2T;
    if (!direct && bound >= T) {  // cannot happen with validated bounds
        if (threadIdx.x == 0) atomicOr(err, kErrRow);
        return;
    }
    for (int s = threadIdx.x; s < T; s += WG) keys[s] = kEmptyKey;
    __syncthreads();
    int cnt = 0;
    block_products<WG, 8, false>(P, i, st_s, st_e, (float *)nullptr, wsum,
                                 [&](const int *cc, const float *, const float *, const bool *ok) {
                                     cnt += direct ? lds_mark_many<8>(keys, cc, ok)
                                                   : lds_insert_many<8>(keys, T - 1, log2T, cc,
                                                                        ok, err);
                                 });
    const int tot = block_sum<WG, int>(cnt, wsum);
    if (threadIdx.x == 0) row_nnz[g] = tot;
}

// One row per workgroup: row blockIdx.x, or (DEV) rows from the group's
// work counter until the group is exhausted (the rows are long, so the
// counter is touched rarely, while an upper bound of the group's rows would
// be a grid of all the batch's rows).
template <int WG, int TMAX, bool DEV>
__global__ __launch_bounds__(WG) void k_sym_block(const ProdDev *__restrict__ prods,
                                                   const uint64_t *__restrict__ items,
                                                   const int64_t *__restrict__ ipv,
                                                   int64_t *__restrict__ row_nnz,
                                                   int *__restrict__ err, int64_t count,
                                                   const int64_t *__restrict__ gstart, int gsel) {
    if constexpr (!DEV) {
        const int64_t it = lin_block();
        if (it >= count) return;  // a split grid covers its whole last row
        sym_block_row<WG, TMAX>(prods, items, ipv, row_nnz, err, it);
    } else {
        group_range(gstart, gsel, items, count);
        __shared__ int64_t next;
        if (threadIdx.x == 0) next = take_block(gstart, gsel);
        __syncthreads();
        for (int64_t it = next; it < count; it = next) {
            sym_block_row<WG, TMAX>(prods, items, ipv, row_nnz, err, it);
            __syncthreads();  // table free again, and every thread has read `next`
            if (threadIdx.x == 0) next = take_block(gstart, gsel);
            __syncthreads();
        }
    }
}

template <int WG, int TMAX>
__device__ __forceinline__ void num_block_row(const ProdDev *__restrict__ prods,
                                              const uint64_t *__restrict__ items,
                                              const int64_t *__restrict__ rptv,
                                              int *__restrict__ err, int64_t it) {
    __shared__ int keys[TMAX];
    __shared__ float vals[TMAX + 64];
    __shared__ int64_t st_s[WG];
    __shared__ int st_e[WG + 1];
    __shared__ float st_a[WG];
    __shared__ int wsum[WG / 64];
    __shared__ int fill;
    const uint64_t e = items[it];
    const ProdDev &P = prods[item_prod(e)];
    const int64_t i = item_row(e);
    const int64_t g = P.row_base + i;
    const int64_t expect = rptv[g + 1] - rptv[g];
    const int64_t a0 = P.rptA[i];
    if (P.rptA[i + 1] - a0 == 1 && P.b_unique == 1) {
        // one A nonzero and strictly ascending B rows: the row is that B row
        // scaled, already in column order; copied with coalesced accesses
        // (each value a single FP32 product, as the table would hold it)
        const int k = P.colA[a0];
        const float av = P.valA[a0];
        const int64_t b0 = P.rptB[k], len = P.rptB[k + 1] - b0;
        if (len != expect) {
            if (threadIdx.x == 0) atomicOr(err, kErrCount);
            return;
        }
        const int64_t base = c_base(P, rptv, g);
        for (int64_t q = threadIdx.x; q < len; q += WG) {
            gst(P.colC + base + q, gld(P.colB + b0 + q));
            gst(P.valC + base + q, av * gld(P.valB + b0 + q));
        }
        return;
    }
    // direct-mapped (slot = column) when B's columns fit the table
    const bool direct = P.n <= TMAX;
    int log2T = ceil_log2(direct ? P.n : 2 * expect);
    if (log2T < 8) log2T = 8;
    if (log2T > Log2<TMAX>::v) log2T = Log2<TMAX>::v;
    const int T = 1 << log2T;
    if (!direct && expect >= T) {
        if (threadIdx.x == 0) atomicOr(err, kErrRow);
        return;
    }
    for (int s = threadIdx.x; s < T; s += WG) { keys[s] = kEmptyKey; vals[s] = 0.f; }
    if (threadIdx.x < 64) vals[T + threadIdx.x] = 0.f;  // dummy slots of the batched adds
    if (threadIdx.x == 0) fill = 0;
    __syncthreads();
    const int dummy = T + (threadIdx.x & 63);
    block_products<WG, 8, true>(
        P, i, st_s, st_e, st_a, wsum,
        [&](const int *cc, const float *aa, const float *vb, const bool *ok) {
            float add[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) add[u] = aa[u] * vb[u];
            if (direct)
                lds_add_direct_many<8>(keys, vals, cc, add, ok, dummy);
            else
                lds_add_many<8>(keys, vals, T - 1, log2T, cc, add, ok, dummy, err);
        });
    if (direct) {
        // the occupied slots are the row's columns in order: a scan of the
        // occupancy places them, no compaction or sort
        const int64_t base = c_base(P, rptv, g);
        int done = 0;
        for (int r0 = 0; r0 < T; r0 += WG) {
            const int q = r0 + threadIdx.x;
            const bool occ = q < T && keys[q] != kEmptyKey;
            const float v = occ ? vals[q] : 0.f;
            int total;
            const int at = done + block_excl_scan<WG, int>(occ ? 1 : 0, wsum, total);
            if (occ && at < expect) {
                gst(P.colC + base + at, q);
                gst(P.valC + base + at, v);
            }
            done += total;
        }
        if (threadIdx.x == 0 && done != expect) atomicOr(err, kErrCount);
        return;
    }
    // gather occupied slots to the front, in place, one WG-wide round at a time
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int r0 = 0; r0 < T; r0 += WG) {
        const int q = r0 + threadIdx.x;
        int kk = kEmptyKey;
        float vv = 0.f;
        if (q < T) { kk = keys[q]; vv = vals[q]; }
        const bool occ = kk != kEmptyKey;
        __syncthreads();
        const unsigned long long m = __ballot(occ);
        int base = 0;
        if (lane == 0 && m) base = atomicAdd(&fill, __popcll(m));
        base = __shfl(base, 0, 64);
        if (occ) {
            const int pos = base + __popcll(m & lt);
            keys[pos] = kk;
            vals[pos] = vv;
        }
        __syncthreads();
    }
    const int n = fill;
    if (threadIdx.x == 0 && n != expect) atomicOr(err, kErrCount);
    int N = 1;
    while (N < n) N <<= 1;
    for (int q = n + threadIdx.x; q < N; q += WG) keys[q] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of the N (key, value) pairs
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = threadIdx.x; q < (N >> 1); q += WG) {
                const int lo = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                const int hi = lo + j;
                const bool asc = (lo & k) == 0;
                const int ka = keys[lo], kb = keys[hi];
                if ((ka > kb) == asc) {
                    keys[lo] = kb;
                    keys[hi] = ka;
                    const float va = vals[lo];
                    vals[lo] = vals[hi];
                    vals[hi] = va;
                }
            }
            __syncthreads();
        }
    }
    const int64_t base = c_base(P, rptv, g);
    const int nout = (int)(n < expect ? n : expect);
    for (int q = threadIdx.x; q < nout; q += WG) {
        gst(P.colC + base + q, keys[q]);
        gst(P.valC + base + q, vals[q]);
    }
}

template <int WG, int TMAX, bool DEV>
__global__ __launch_bounds__(WG) void k_num_block(const ProdDev *__restrict__ prods,
                                                   const uint64_t *__restrict__ items,
                                                   const int64_t *__restrict__ rptv,
                                                   int *__restrict__ err, int64_t count,
                                                   const int64_t *__restrict__ gstart, int gsel) {
    if constexpr (!DEV) {
        const int64_t it = lin_block();
        if (it >= count) return;  // a split grid covers its whole last row
        num_block_row<WG, TMAX>(prods, items, rptv, err, it);
    } else {
        group_range(gstart, gsel, items, count);
        if (*err & kErrCapacity) return;  // C does not fit its arena (block-uniform)
        __shared__ int64_t next;
        if (threadIdx.x == 0) next = take_block(gstart, gsel);
        __syncthreads();
        for (int64_t it = next; it < count; it = next) {
            num_block_row<WG, TMAX>(prods, items, rptv, err, it);
            __syncthreads();  // table free again, and every thread has read `next`
            if (threadIdx.x == 0) next = take_block(gstart, gsel);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.  Group g: 1..4 -> G = 8, 16, 32, 64; 5 -> 256-thread block,
// 6 -> 512-thread block.
// ---------------------------------------------------------------------------
// Host-sized launches cover the group exactly.  Device-sized ones (gstart)
// cover an upper bound: the group kernels every row of the batch, the block
// kernels a grid of kDeviceGridCap workgroups that take rows from the work
// counter.
constexpr int64_t kDeviceGridCap = 8192;  // 32 workgroups per compute unit

template <typename K, typename... Args>
static void launch_rows(K host, K dev, int64_t blocks, int64_t dev_blocks, int threads,
                        hipStream_t s, const int64_t *gstart, Args... args) {
    if (gstart)
        hipLaunchKernelGGL(dev, grid1d(dev_blocks, threads), dim3(threads), 0, s, args...);
    else
        hipLaunchKernelGGL(host, grid1d(blocks, threads), dim3(threads), 0, s, args...);
}

template <int G>
static void sym_group_launch(const ProdDev *prods, const uint64_t *items, int64_t count,
                             int64_t *row_nnz, int *err, hipStream_t s, const int64_t *gstart,
                             int gsel) {
    constexpr int R = 256 / G;
    const int64_t nb = (count + R - 1) / R;
    launch_rows(k_sym_group<G, false>, k_sym_group<G, true>, nb, nb, 256, s, gstart,
                prods, items, count, row_nnz, err, gstart, gsel);
}

void launch_sym_group(int g, const ProdDev *prods, const uint64_t *items, int64_t count,
                      int64_t *row_nnz, int *err, hipStream_t s, const int64_t *gstart,
                      int gsel) {
    if (count <= 0) return;
    switch (g) {
        case 1: sym_group_launch<8>(prods, items, count, row_nnz, err, s, gstart, gsel); break;
        case 2: sym_group_launch<16>(prods, items, count, row_nnz, err, s, gstart, gsel); break;
        case 3: sym_group_launch<32>(prods, items, count, row_nnz, err, s, gstart, gsel); break;
        case 4: sym_group_launch<64>(prods, items, count, row_nnz, err, s, gstart, gsel); break;
        default: break;
    }
}

// The 64-lane group runs one row per workgroup: its rows vary in length, and
// a workgroup of several rows waits at its barriers for the longest.
template <int G>
static void num_group_launch(const ProdDev *prods, const uint64_t *items, int64_t count,
                             const int64_t *rptv, int *err, hipStream_t s, const int64_t *gstart,
                             int gsel, int64_t max_ncols) {
    constexpr int TB = G == 64 ? 64 : 256;
    constexpr int R = TB / G;
    const int64_t nb = (count + R - 1) / R;
    if (max_ncols <= 8 * G)
        launch_rows(k_num_group<G, false, TB, true>, k_num_group<G, true, TB, true>, nb, nb, TB,
                    s, gstart, prods, items, count, rptv, err, gstart, gsel);
    else
        launch_rows(k_num_group<G, false, TB, false>, k_num_group<G, true, TB, false>, nb, nb,
                    TB, s, gstart, prods, items, count, rptv, err, gstart, gsel);
}

void launch_num_group(int g, const ProdDev *prods, const uint64_t *items, int64_t count,
                      const int64_t *rptv, int *err, hipStream_t s, const int64_t *gstart,
                      int gsel, int64_t max_ncols) {
    if (count <= 0) return;
    switch (g) {
        case 1: num_group_launch<8>(prods, items, count, rptv, err, s, gstart, gsel, max_ncols); break;
        case 2: num_group_launch<16>(prods, items, count, rptv, err, s, gstart, gsel, max_ncols); break;
        case 3: num_group_launch<32>(prods, items, count, rptv, err, s, gstart, gsel, max_ncols); break;
        case 4: num_group_launch<64>(prods, items, count, rptv, err, s, gstart, gsel, max_ncols); break;
        default: break;
    }
}

static int table_for(int64_t upper, int lo, int hi) {
    int t = lo;
    while (t < hi && (int64_t)t < 2 * upper) t <<= 1;
    return t;
}

template <int WG, int TMAX>
static void sym_block_launch(const ProdDev *prods, const uint64_t *items, const int64_t *ipv,
                             int64_t count, int64_t *row_nnz, int *err, hipStream_t s,
                             const int64_t *gstart, int gsel) {
    launch_rows(k_sym_block<WG, TMAX, false>, k_sym_block<WG, TMAX, true>, count,
                std::min(count, kDeviceGridCap), WG, s, gstart,
                prods, items, ipv, row_nnz, err, count, gstart, gsel);
}

template <int WG, int TMAX>
static void num_block_launch(const ProdDev *prods, const uint64_t *items, int64_t count,
                             const int64_t *rptv, int *err, hipStream_t s, const int64_t *gstart,
                             int gsel) {
    launch_rows(k_num_block<WG, TMAX, false>, k_num_block<WG, TMAX, true>, count,
                std::min(count, kDeviceGridCap), WG, s, gstart,
                prods, items, rptv, err, count, gstart, gsel);
}

// LDS tables are sized to the group's upper bound (twice the largest key,
// a power of two), so a group tuned to small rows keeps a high occupancy.
void launch_sym_block(int g, int64_t upper, const ProdDev *prods, const uint64_t *items,
                      const int64_t *ipv, int64_t count, int64_t *row_nnz, int *err,
                      hipStream_t s, const int64_t *gstart, int gsel) {
    if (count <= 0) return;
    if (g == 5) {
        switch (table_for(upper, 2048, 8192)) {
            case 2048: sym_block_launch<256, 2048>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
            case 4096: sym_block_launch<256, 4096>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
            default: sym_block_launch<256, 8192>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
        }
    } else {
        switch (table_for(upper, 8192, 32768)) {
            case 8192: sym_block_launch<512, 8192>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
            case 16384: sym_block_launch<512, 16384>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
            default: sym_block_launch<512, 32768>(prods, items, ipv, count, row_nnz, err, s, gstart, gsel); break;
        }
    }
}

void launch_num_block(int g, int64_t upper, const ProdDev *prods, const uint64_t *items,
                      int64_t count, const int64_t *rptv, int *err, hipStream_t s,
                      const int64_t *gstart, int gsel) {
    if (count <= 0) return;
    if (g == 5) {
        switch (table_for(upper, 1024, 4096)) {
            case 1024: num_block_launch<256, 1024>(prods, items, count, rptv, err, s, gstart, gsel); break;
            case 2048: num_block_launch<256, 2048>(prods, items, count, rptv, err, s, gstart, gsel); break;
            default: num_block_launch<256, 4096>(prods, items, count, rptv, err, s, gstart, gsel); break;
        }
    } else {
        switch (table_for(upper, 4096, 16384)) {
            case 4096: num_block_launch<512, 4096>(prods, items, count, rptv, err, s, gstart, gsel); break;
            case 8192: num_block_launch<512, 8192>(prods, items, count, rptv, err, s, gstart, gsel); break;
            default: num_block_launch<512, 16384>(prods, items, count, rptv, err, s, gstart, gsel); break;
        }
    }
}

}  // namespace spg
