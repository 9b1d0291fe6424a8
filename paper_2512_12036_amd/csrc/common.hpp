// Internal declarations shared by the HIP kernels and the host side of the
// library.  Wavefronts are 64 lanes wide (CDNA4); every kernel is written for
// that width.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

constexpr int kGroups = 8;           // row groups, see spgemm.h
constexpr int kChunkGroup = 7;       // column-chunked group
constexpr int64_t kIpPerLane = 16;   // numeric grouping: target products per lane
constexpr int64_t kDirectG4 = 512;   // table slots of group 4 (64 lanes x 8)
constexpr int64_t kBitmapCols = kDirectG4;  // B kept as row bitmaps up to this many columns
constexpr int kMaxChunkCols = 16384; // LDS: 64 KiB FP32 dense accumulator
constexpr int kMaxItemCols = 65536;  // widest merged item (8 KiB LDS bitmap)
constexpr int kSabsJ = 64;           // A nonzeros per workgroup of the sub-range tables
constexpr int kSabsC = 64;           // chunk bounds per LDS tile of them; rows of more
                                     // chunks are not merged
constexpr int kIpSlices = 32;        // most workgroups per row block in the IP count
constexpr int64_t kIpMinSlice = 4096; // fewest A nonzeros per IP-count workgroup
constexpr int kRowBlock = 256;       // rows per block in the grouping kernels
// Largest key each group can take (tables at most half full).
constexpr int64_t kSymCap[kGroups] = {0, 32, 64, 128, 256, 4096, 16384, 0};
constexpr int64_t kNumCap[kGroups] = {0, 32, 64, 128, 256, 2048, 8192, 0};
constexpr int kEmptyKey = -1;

// Error bits raised by kernels (OR-ed into the plan's device flag word).
constexpr int kErrProbe = 1;         // hash probe sequence exceeded the table
constexpr int kErrCount = 2;         // numeric count != symbolic count
constexpr int kErrChunk = 4;         // chunk count != symbolic chunk count
constexpr int kErrRow = 8;           // group-kernel row exceeds group capacity
constexpr int kErrCapacity = 16;     // C does not fit the caller's arena (nothing written)

// One product C = A * B as seen by the kernels.
struct ProdDev {
    const int64_t *rptA;
    const int32_t *colA;
    const float *valA;
    const int64_t *rptB;
    const int32_t *colB;
    const float *valB;
    int32_t *colC;
    float *valC;
    const int32_t *bsplit;  // chunk bounds per B row (group-7 rows, sorted B)
    int64_t m, k, n;
    int64_t row_base;   // first row of this product in the batch row space
    int32_t W;          // columns per chunk
    int32_t nch;        // chunks per row (multiple of 8)
    int32_t b_sorted;   // rows of B strictly ascending: 1 yes, 0 no, 2 detect
    int32_t c_arena;    // 1: colC / valC are one arena shared by the batch, indexed by
                        // the batch-wide row pointers (device-driven plans)
    int32_t b_unique;   // 1: B's rows strictly ascending, so no duplicate columns (B
                        // rows sorted by the plan may hold duplicates: 0)
    int32_t bmw;        // words per row of bmB (0: no bitmaps)
    const uint32_t *bmB;  // B's rows as column bitmaps (B with at most kBitmapCols
                          // columns), row k at bmB + k * bmw
    int64_t *rptC;        // device-driven plans: C's row pointers of this product
};

// One work item of group 7: the chunks q, q + Q, ... (K of them) of one row,
// or (K = 1) the `span` adjacent chunks q .. q + span - 1 taken as one.
struct ChunkDesc {
    int64_t a0;      // first A nonzero of the row
    int64_t out0;    // symbolic: batch row index; numeric: output offset of the row in C_p
    int64_t slot0;   // chunk-count slot of the row's chunk 0
    int64_t sb;      // start of the row's sub-range table (fast path), else -1
    int32_t alen;    // A nonzeros of the row
    int32_t q;       // first chunk of the item
    int32_t prod;    // product index
    int32_t pad;     // resolved numeric descriptors: the item's output count
    int32_t span;    // adjacent chunks taken as one (1 unless merged)
    int32_t pad2;
};

// One entry of the thread-per-row stream: the B range named by one A
// nonzero and that nonzero's value (numeric phase).
struct RangeEnt {
    int64_t b0;      // rpt_B[col]
    int32_t len;     // rpt_B[col + 1] - rpt_B[col]
    float a;         // A's value
};
constexpr int kRtSlots = 64;  // table slots per row of the thread-per-row kernels

// A block of up to kRowBlock consecutive rows of one product.
struct RowBlk {
    int32_t p;
    int32_t nrows;
    int64_t i0;
};

// Per-product figures accumulated on the device (one atomic per block).
struct ProdStats {
    unsigned long long ip_sum;
    unsigned long long ip_max;
    unsigned long long nnz_sum;
    unsigned long long nnz_max;
    unsigned long long h_rows;    // symbolic group-7 rows
    unsigned long long h_alen;    // their A nonzeros
    unsigned long long h_split;   // sum of alen * (nch + 1)
    unsigned long long h_items;   // sum of nch
    unsigned long long d_rows;    // numeric group-7 rows
    unsigned long long d_items;   // sum of nch over them
    unsigned long long h_tiles;   // sum of ceil(alen / kSabsJ) over symbolic group-7 rows
    unsigned long long pad[5];
};
static_assert(sizeof(ProdStats) % 8 == 0, "ProdStats is cleared in 8-byte words");

// First output slot of batch row g in its product's C arrays.
__device__ __forceinline__ int64_t c_base(const ProdDev &P, const int64_t *rptv, int64_t g) {
    return P.c_arena ? rptv[g] : rptv[g] - rptv[P.row_base];
}

// Launch geometry.  A dispatch packet holds each grid dimension's extent as
// a 32-bit count of work-items, so a 1-D grid of 2^32 work-items or more is
// laid out as rows of kGridRow workgroups over y (a wider x would wrap).
// Kernels take their workgroup's linear index from lin_block() and bound it
// themselves: a split grid covers its whole last row.
constexpr int64_t kGridRow = int64_t(1) << 16;
inline dim3 grid1d(int64_t blocks, int threads) {
    if (blocks * (int64_t)threads <= int64_t(0xFFFFFFFF)) return dim3((unsigned)blocks);
    return dim3((unsigned)kGridRow, (unsigned)((blocks + kGridRow - 1) / kGridRow));
}
__device__ __forceinline__ int64_t lin_block() {
    return (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
}

// Work order over the eight dies (XCDs) of the chip.  Workgroups go to the
// dies round-robin in order of their linear index, so work unit w of a
// walk (a workgroup's index, or index + k * grid for a grid walking its
// units) runs on die w % 8, and consecutive units would land on eight
// different L2 caches.  xcd_unit(w, n) renumbers [0, n) so that every die
// takes runs of kXcdRun consecutive units: the column chunks of one row then
// share that die's L2 (the row's A nonzeros and sub-range bounds, and the
// cache lines of B that straddle two chunks).  A bijection on [0, n): whole
// groups of 8 * kXcdRun units are interleaved, the tail keeps its order.
#ifndef SPG_XCD_RUN
#define SPG_XCD_RUN 4
#endif
constexpr int64_t kXcds = 8, kXcdRun = SPG_XCD_RUN;
__host__ __device__ __forceinline__ int64_t xcd_unit(int64_t w, int64_t n) {
    constexpr int64_t span = kXcds * kXcdRun;
    if (w >= n / span * span) return w;
    const int64_t r = w / kXcds;
    return r / kXcdRun * span + (w % kXcds) * kXcdRun + r % kXcdRun;
}

// Device-driven launches cover an upper bound of a group's rows and read the
// group's place in the row map from the device (gstart[gsel .. gsel + 1]).
__device__ __forceinline__ void group_range(const int64_t *gstart, int gsel,
                                            const uint64_t *__restrict__ &items, int64_t &count) {
    if (gstart) {
        const int64_t b = gstart[gsel];
        items += b;
        count = gstart[gsel + 1] - b;
    }
}

// Rows of a device-driven batch: its group launches cover every row.
constexpr int64_t kMaxDeviceRows = (int64_t(1) << 32) / 64 - 1;

// The block kernels' device-sized launches take rows one at a time from a
// work counter kWorkCtr entries after the group's start (zeroed before the
// launch), so a long row holds up no rows behind it.
constexpr int kWorkCtr = 2 * (kGroups + 1);
__device__ __forceinline__ int64_t take_block(const int64_t *gstart, int gsel) {
    return (int64_t)atomicAdd((unsigned long long *)(gstart + kWorkCtr + gsel), 1ull);
}

__device__ __forceinline__ uint64_t pack_item(int p, int64_t i) {
    return ((uint64_t)(uint32_t)p << 32) | (uint64_t)(uint32_t)i;
}
__device__ __forceinline__ int item_prod(uint64_t e) { return (int)(e >> 32); }
__device__ __forceinline__ int64_t item_row(uint64_t e) { return (int64_t)(uint32_t)e; }

// Multiplicative (Fibonacci) hashing: the top log2T bits of c * 2^32/phi.
__device__ __forceinline__ uint32_t hash_slot(int c, int log2T) {
    return ((uint32_t)c * 0x9E3779B1u) >> (32 - log2T);
}

// ---------------------------------------------------------------------------
// Host launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
// up[0] = 0, up[7] unused.  copy_group > 0: rows of a single A nonzero with
// strictly ascending B rows that would go past that group go to it instead
// (its kernels copy such rows); 0: no such rule.
struct GroupBounds {
    int64_t up[kGroups];
    int64_t copy_group;
};

size_t scan_temp_bytes(int64_t n);
// out[0..n] = exclusive prefix of in[0..n) (out[n] = total).  out != in.
void launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *temp,
                     hipStream_t s);

struct CsrCheck {
    const int64_t *rpt;
    const int32_t *col;
    int64_t m, nnz, ncols;
};
void launch_detect_sorted(ProdDev *prods, int nprod, const ProdDev *host_prods,
                          int *flags_out, hipStream_t s);
void launch_validate_rows(const CsrCheck &c, int *bad, hipStream_t s);
void launch_validate_cols(const CsrCheck &c, int *bad, hipStream_t s);

// ip[row] of every row (zeroed, then accumulated), then the symbolic group
// histograms and statistics.
void launch_ipcount(const ProdDev *prods, const RowBlk *blks, int nblk,
                    GroupBounds gb, int64_t *ip, int64_t *blkcnt, ProdStats *stats,
                    int64_t nrows, hipStream_t s);
// Numeric group histograms (key = output lengths).
void launch_count_groups(const ProdDev *prods, const RowBlk *blks, int nblk, GroupBounds gb,
                         const int64_t *key, const int64_t *ip, int64_t *blkcnt,
                         ProdStats *stats, hipStream_t s);
void launch_scatter(const ProdDev *prods, const RowBlk *blks, int nblk, GroupBounds gb,
                    const int64_t *key, const int64_t *off, uint64_t *map, int32_t *hslot,
                    const int64_t *ip, hipStream_t s);
void launch_group_starts(const int64_t *off, int nblk, int64_t *starts, hipStream_t s);

// Chunk preparation (group 7).
void launch_bsplit(const int64_t *rptB, const int32_t *colB, int64_t k_rows, int W, int nch,
                   int32_t *bsplit, hipStream_t s);
void launch_nch_of(const ProdDev *prods, const uint64_t *items, int64_t n, int div,
                   int64_t *nchv, hipStream_t s);
void launch_expand(const int64_t *base, int64_t n, int32_t *out, hipStream_t s);
void launch_row_splitlen(const ProdDev *prods, const uint64_t *items, int64_t nh, int64_t *len,
                         hipStream_t s);
// Sub-range tables of the group-7 rows (fast path), one workgroup per tile of
// kSabsJ A nonzeros: ntile / tbase / tile_row give the tiles of every row.
// With ipc (zeroed, one entry per chunk slot), the chunks' intermediate
// products are accumulated too, and launch_chunk_items then forms the merged
// work items of every row (mstart / nitem).
void launch_sabs_tiles(const ProdDev *prods, const uint64_t *items, int64_t nh, int64_t *ntile,
                       hipStream_t s);
void launch_sabs(const ProdDev *prods, const uint64_t *items, int64_t ntiles,
                 const int32_t *tile_row, const int64_t *tbase, const int64_t *sbase,
                 uint32_t *sabs, const int64_t *cbase, unsigned long long *ipc, hipStream_t s);
void launch_chunk_items(const ProdDev *prods, const uint64_t *items, int64_t nh, int merge,
                        int64_t cap, const int64_t *cbase, const unsigned long long *ipc,
                        int32_t *mstart, int64_t *nitem, hipStream_t s);
void launch_num_nitems(const ProdDev *prods, const uint64_t *ditems, int64_t n,
                       const int32_t *hslot, const int64_t *nitem, int64_t *dnch, hipStream_t s);
void launch_sym_desc(const ProdDev *prods, const uint64_t *items, const int32_t *item_of,
                     const int64_t *ibase, const int64_t *cbase, const int64_t *sbase,
                     int64_t nitems, int kper, const int32_t *mstart, const int64_t *nlim,
                     ChunkDesc *desc, hipStream_t s);
void launch_num_desc(const ProdDev *prods, const uint64_t *ditems, const int32_t *item_of,
                     const int64_t *dbase, int64_t nitems, int kper, const int32_t *hslot,
                     const int64_t *cbase, const int64_t *sbase, const int64_t *rptv,
                     const int32_t *mstart, const int64_t *nlim, ChunkDesc *desc, hipStream_t s);

// With gstart (device), `count` is an upper bound of the group's rows and
// the kernels take the group's range of the map from gstart[gsel .. gsel+1].
void launch_sym_group(int g, const ProdDev *prods, const uint64_t *items,
                      int64_t count, int64_t *row_nnz, int *err, hipStream_t s,
                      const int64_t *gstart = nullptr, int gsel = 0);
void launch_sym_block(int g, int64_t upper, const ProdDev *prods, const uint64_t *items,
                      const int64_t *ipv, int64_t count, int64_t *row_nnz, int *err,
                      hipStream_t s, const int64_t *gstart = nullptr, int gsel = 0);
void launch_sym_chunk(int wmax, bool fast, const ProdDev *prods, const ChunkDesc *desc,
                      const uint32_t *sabs, int64_t nitems, int kper, int64_t *chunk_cnt,
                      int64_t *row_nnz, uint32_t *sbits, int wpc, int wgs_per_cu, int threads,
                      int *err, hipStream_t s);
// max_ncols: the most columns of any product's B in the batch; when every B
// fits the group's direct-mapped table, a launch without a key table runs.
void launch_num_group(int g, const ProdDev *prods, const uint64_t *items,
                      int64_t count, const int64_t *rptv, int *err, hipStream_t s,
                      const int64_t *gstart = nullptr, int gsel = 0,
                      int64_t max_ncols = INT64_MAX);
void launch_num_block(int g, int64_t upper, const ProdDev *prods, const uint64_t *items,
                      int64_t count, const int64_t *rptv, int *err, hipStream_t s,
                      const int64_t *gstart = nullptr, int gsel = 0);
// Device-driven plans: kErrCapacity when the batch's nnz(C) exceeds the
// arena; each product's first slot in the arena (nprod + 1 entries).
void launch_arena_check(const int64_t *rptv, int64_t mtot, int64_t capacity, int *err,
                        const ProdDev *prods, int nprod, int64_t *offsets, hipStream_t s);
void launch_num_chunk(int wmax, bool fast, const ProdDev *prods, const ChunkDesc *desc,
                      const uint32_t *sabs, int64_t nitems, int kper, const int64_t *chunk_cnt,
                      const int64_t *chunk_pos, const uint32_t *sbits, int wpc, int wgs_per_cu,
                      int threads, int rank_cap, bool resolved, int *err, hipStream_t s);
// Numeric chunk items split by output count and span into five lists: more
// than cap outputs, single chunks above and at most cap / 2, merged items
// above and at most cap / 2.  fa/fb (and their scans) pack two counters each:
// fa = dense (low 32 bits) | small single (high), fb = large merged | small
// merged.
void launch_desc_flag(const ChunkDesc *desc, int64_t nitems, const int64_t *chunk_cnt,
                      int64_t cap, const int64_t *nlim, int64_t *fa, int64_t *fb, hipStream_t s);
void launch_desc_split(const ChunkDesc *desc, int64_t nitems, const int64_t *fa,
                       const int64_t *fapos, const int64_t *fb, const int64_t *fbpos,
                       const int64_t *chunk_cnt, const int64_t *chunk_pos, const int64_t *nlim,
                       ChunkDesc *out, hipStream_t s);
// Chunks with at most rank_cap outputs (fast path, one chunk per item only).
// f64: FP64 accumulation, for items of at most 2048 columns and a rank cap
// of 1024 or 2048; false (nothing launched) for any other shape.
bool num_chunk_rank_used(bool fast, int kper, int rank_cap);
bool launch_num_chunk_rank(int wmax, const ProdDev *prods, const ChunkDesc *desc,
                           const uint32_t *sabs, int64_t nitems, const int64_t *chunk_cnt,
                           const int64_t *chunk_pos, const uint32_t *sbits, int wpc, int rank_cap,
                           bool resolved, int *err, hipStream_t s, bool f64 = false);

// Algorithm 1 alone, aggregated into out[3] (device): sum of intermediate
// products, sum of min(ip, ncols), largest row.
// B's rows as column bitmaps (bmw = ceil(ncols / 32) words per row, at most
// kBitmapCols / 32): out[k * bmw + w] bit b set iff column 32 w + b is in row
// k.  Columns outside [0, ncols) are ignored.
void launch_brow_bitmap(const int64_t *rptB, const int32_t *colB, int64_t nrows, int64_t ncols,
                        int bmw, uint32_t *out, hipStream_t s);

// The same for every product of a batch whose descriptor has bitmaps, in
// one launch of row_blocks x nprod workgroups (each a stride over its
// product's B rows, 16 rows at a time); nprod <= 65535.
void launch_brow_bitmap_batch(const ProdDev *prods, int nprod, int64_t row_blocks,
                              hipStream_t s);
// Every product's own row pointers (prods[q].rptC, m + 1 entries) from the
// batch's (rptv), in one launch of row_blocks x nprod workgroups of 256
// threads; nprod <= 65535.
void launch_rows_local_batch(const ProdDev *prods, int nprod, int64_t row_blocks,
                             const int64_t *rptv, hipStream_t s);

void launch_ip_estimate(const int64_t *rptA, const int32_t *colA, const int64_t *rptB, int64_t m,
                        int64_t ncols, int64_t *out, hipStream_t s);
void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
void launch_rows_local(const int64_t *rptv, int64_t row_base, int64_t m,
                       int64_t *dst, hipStream_t s);

// Applications (k_apps.hip): transposed selector by counting sort; Markov
// clustering prune step (count pass, then write pass).
void launch_selector_t(const int32_t *labels, int64_t n, int64_t k, int64_t *rpt, int32_t *col,
                       float *val, int64_t *work, void *scan_tmp, int *err, hipStream_t s);
void launch_mcl_count(int64_t m, const int64_t *rpt, const float *val, float power, float theta,
                      int k, float *rowsum, int64_t *keep, int32_t *sel, hipStream_t s);
void launch_mcl_write(int64_t m, const int64_t *rpt, const int32_t *col, const float *val,
                      float power, float theta, const float *rowsum, const int32_t *sel,
                      const int64_t *out_rpt, int32_t *out_col, float *out_val, hipStream_t s);
void launch_mcl_change(int64_t m, const int64_t *rpt_a, const int32_t *col_a, const float *val_a,
                       int64_t nnz_a, const int64_t *rpt_b, const int32_t *col_b,
                       const float *val_b, int64_t nnz_b, double *out, hipStream_t s);
// Inverse transform sampling, s draws per row (bulk sampling).
void launch_its_sample(int64_t m, int s, const int64_t *rpt, const int32_t *col, const float *val,
                       const float *u, const int32_t *self, int32_t *out, hipStream_t st);
// Connected components (labels = smallest vertex of the component): init,
// then rounds of hook + compress until a round hooks nothing (*changed = 0).
void launch_cc_init(int64_t n, int32_t *lab, hipStream_t s);
void launch_cc_round(int64_t n, const int64_t *rpt, const int32_t *col, int64_t nnz, int32_t *lab,
                     int *changed, hipStream_t s);

// Thread-per-row kernels for the smallest group (k_rowthread.hip): per-row
// stream offsets (lens -> off, count + 1), the ranged gather and the two
// phases.
void launch_rt_offsets(const ProdDev *prods, const uint64_t *items, int64_t count, int64_t *lens,
                       int64_t *off, void *scan_tmp, hipStream_t s);
// Sorting B's rows at plan time (unsorted B with column-chunked rows): the
// scratch bytes of the sort, the sort of (column, position) pairs per row,
// and the numeric-time gather of B's values into the sorted order.
size_t bsort_temp_bytes(int64_t nnz, int64_t rows, int64_t ncols);
hipError_t launch_bsort(const int64_t *rpt, int64_t rows, int64_t ncols, const int32_t *col,
                        int64_t nnz, int32_t *col_out, int32_t *perm, void *tmp, size_t tmp_bytes,
                        hipStream_t s);
void launch_gather_f32(const float *val, const int32_t *perm, int64_t n, float *out,
                       hipStream_t s);
void launch_rt_gather(const ProdDev *prods, const uint64_t *items, int64_t count,
                      const int64_t *off, RangeEnt *stream, bool values, hipStream_t s);
void launch_sym_rowthread(const ProdDev *prods, const uint64_t *items, int64_t count,
                          const int64_t *off, const RangeEnt *stream, int64_t *row_nnz, int *err,
                          hipStream_t s);
void launch_num_rowthread(const ProdDev *prods, const uint64_t *items, int64_t count,
                          const int64_t *off, const RangeEnt *stream, const int64_t *rptv,
                          int *err, hipStream_t s);

// GNN layer pieces (k_gnn.hip).
void launch_rows_uniform(int64_t *rpt, int64_t n, int64_t k, hipStream_t s);
void launch_topk_rows(int64_t n, int64_t f, const float *x, int64_t ldx, int k, int32_t *col,
                      float *val, hipStream_t s);
void launch_csr_to_dense(int64_t m, int64_t n, const int64_t *rpt, const int32_t *col,
                         const float *val, float *d, int64_t ldd, hipStream_t s);
void launch_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t sar, int64_t sac,
                     const float *B, int64_t sbr, int64_t sbc, float *C, int64_t ldc,
                     hipStream_t s);
void launch_masked_spmm(int64_t m, const int64_t *rpt_t, const int32_t *col_t, const float *val_t,
                        const float *d, int64_t ldd, const int64_t *rpt_m, const int32_t *col_m,
                        float *out, hipStream_t s);
void launch_transpose(int64_t m, int64_t n, const int64_t *rpt, const int32_t *col,
                      const float *val, int64_t nnz, int64_t *rpt_t, int32_t *col_t,
                      float *val_t, int64_t *work, void *scan_tmp, hipStream_t s);

}  // namespace spg
