/*
 * spgemm.h -- C ABI of the MI355X (gfx950) hash-based multi-phase SpGEMM.
 *
 * Computes C = A * B for sparse A (m x k) and B (k x n) in compressed-row
 * storage (paper Section I states the problem; Section III the method).  The
 * work is split into the phases of paper Section III:
 *
 *   spgemm_plan_create   row-size estimation: intermediate products per row
 *                        (paper Algorithm 1) and row grouping by that count
 *                        (paper Section III-B, Table I).
 *   spgemm_symbolic      allocation phase: distinct output columns per row
 *                        with hash tables (paper Algorithms 2-4, keys only),
 *                        then the exclusive scan that yields C's row
 *                        pointers (paper Algorithms 2-3, last step).
 *   spgemm_numeric       accumulation phase: hash accumulation of the
 *                        products (paper Algorithms 4-5), gathering of the
 *                        occupied slots and ascending column sort of every
 *                        row (paper Section III-D).
 *   spgemm_free          releases a plan.
 *
 * Conventions for every entry point:
 *  - Pointers inside spgemm_csr and the output arrays are DEVICE pointers
 *    unless a parameter says "host".
 *  - Index types: row pointers int64, column indices int32, values FP32.
 *  - All work is enqueued on the HIP stream given at plan creation.  Only the
 *    calls documented as synchronising wait for the stream.
 *  - Errors are returned as spgemm_status; nothing aborts and no C++
 *    exception crosses the ABI.  After any failure the plan can still be
 *    freed.  A plan is not thread safe; distinct plans are independent.
 *  - Output contract: every row of C has strictly ascending columns, no
 *    duplicates, and keeps explicit zeros produced by cancellation (the
 *    structure of C is the boolean product of the stored patterns).
 *  - Values: each product a*b is rounded to FP32 and added in FP32 (paper
 *    Algorithm 4 adds valA x valB atomically); the order of the additions is
 *    not fixed, so values may differ in the last bits between runs while the
 *    structure is always identical.
 */
#ifndef SPGEMM_H
#define SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPGEMM_OK = 0,
    SPGEMM_EINVAL = 1,     /* NULL pointer, negative size, bad option value   */
    SPGEMM_EDIM = 2,       /* A.ncols != B.nrows, or a dimension out of range  */
    SPGEMM_EINDEX = 3,     /* device validation found a malformed CSR          */
    SPGEMM_EOVERFLOW = 4,  /* a count exceeds what the library's types hold    */
    SPGEMM_ENOMEM = 5,     /* the allocator returned NULL                      */
    SPGEMM_EHIP = 6,       /* a HIP runtime call failed                        */
    SPGEMM_ESTATE = 7,     /* calls made out of order                          */
    SPGEMM_EINTERNAL = 8   /* a kernel raised its error flag (probe limit,
                              symbolic / numeric count mismatch)               */
} spgemm_status;
/* With the environment variable SPGEMM_DEBUG set, a call that returns
 * SPGEMM_EHIP first prints the failing HIP call and its error name to
 * stderr. */

/* spgemm_csr.flags: every row stores strictly ascending columns. */
#define SPGEMM_ROWS_SORTED 1u

/* A sparse matrix in compressed-row storage.  All arrays are device memory
 * owned by the caller and borrowed by the library until the stream has
 * passed the last call that reads them. */
typedef struct {
    int64_t nrows;           /* >= 0, < 2^31                                   */
    int64_t ncols;           /* >= 0, < 2^31                                   */
    int64_t nnz;             /* == row_ptr[nrows]                              */
    const int64_t *row_ptr;  /* nrows + 1 entries, non-decreasing, [0] = 0     */
    const int32_t *col_idx;  /* nnz entries, 0 <= c < ncols; duplicates in a
                                row are summed                                 */
    const float *values;     /* nnz entries; may be NULL until spgemm_numeric  */
    uint32_t flags;          /* SPGEMM_ROWS_SORTED or 0 (then detected)        */
} spgemm_csr;

/* Device allocator used for all workspace (for example PyTorch's caching
 * allocator).  alloc returns NULL on failure.  Both may be NULL in
 * spgemm_plan_create, in which case hipMalloc / hipFree are used. */
typedef void *(*spgemm_alloc_fn)(void *ctx, size_t bytes, void *stream);
typedef void (*spgemm_free_fn)(void *ctx, void *ptr, void *stream);

/* Number of row groups.  Group 0 holds rows with nothing to do (no
 * intermediate products, or no output), groups 1-4 rows handled by 8, 16,
 * 32 or 64 lanes with a per-row LDS hash table of 8 slots per lane, groups
 * 5-6 rows handled by a 256- or 512-thread workgroup with an LDS hash table,
 * group 7 rows handled as column chunks with an LDS bitmap (symbolic) or an
 * LDS dense accumulator (numeric).  Paper Table I gives the four groups used
 * on the paper's GPU; these are the gfx950 equivalents. */
#define SPGEMM_NGROUPS 8

typedef struct {
    /* Inclusive upper bounds of groups 1..6 (index 0 unused, must be 0).
     * Symbolic groups are keyed by min(intermediate products of the row,
     * columns of B) -- both bound the row's distinct outputs; paper Table I
     * uses the first -- and numeric groups by the row's output length (paper
     * Section III-C: the table size is first set from the intermediate
     * products, then from the distinct count), raised to ceil(products / 16)
     * capped at B's columns, so rows with many products per output get more
     * lanes.  When B has at most 512 columns, a row whose key is at most 512
     * never goes past group 4: its table is then indexed by the column
     * itself (8 slots x 64 lanes = 512).  Non-decreasing.  Capacities (maximum legal bound):
     *   symbolic: 63, 127, 255, 511, 8191, 32767
     *   numeric : 63, 127, 255, 511, 2047, 8191
     * and sym_upper[6] <= num_upper[6] (a row handled as chunks in the
     * numeric phase must have been handled as chunks in the symbolic one). */
    int64_t sym_upper[SPGEMM_NGROUPS - 1];
    int64_t num_upper[SPGEMM_NGROUPS - 1];
    /* Maximum columns per chunk of group 7 (multiple of 64, 64 .. 16384).  The
     * number of chunks per row is a multiple of 8.  Chunk items are launched
     * in row order, so that the chunks of one row share its A nonzeros and
     * sub-range tables in cache. */
    int32_t chunk_cols;
    /* Validation level of A and B: 0 none (host-side argument checks only);
     * 1 cheap: row pointers checked on the device (row_ptr[0] = 0,
     * non-decreasing, row_ptr[nrows] = nnz; one pass over nrows + 1 values);
     * 2 full: also every column index in [0, ncols) (one pass over nnz
     * values).  A malformed input fails with SPGEMM_EINDEX. */
    int32_t validate;
    /* 1: record a HIP event pair around every kernel launch group on the
     * plan's stream (read back with spgemm_timing). */
    int32_t profile;
    /* Chunks of one group-7 row handled by one workgroup (1, 2, 4 or 8):
     * more amortises the row's staging, fewer gives more parallelism. */
    int32_t chunks_per_item;
    /* Launch shape of the group-7 kernels when chunks_per_item = 1 and B has
     * sorted rows: 0 = one workgroup per (row, chunk) item; k = 1..64 = k
     * resident workgroups per compute unit, each walking the items with the
     * next item's inputs loaded while the current one is processed. */
    int32_t chunk_wgs_per_cu;
    /* Threads per workgroup of the numeric group-7 kernel for dense chunks:
     * 0 = by chunk width (64 up to 2048 columns, 128 up to 4096, 256 up to
     * 8192, 512 wider), else 64, 128, 256 or 512. */
    int32_t chunk_threads;
    /* Same for the symbolic group-7 kernel (0 = 64). */
    int32_t sym_chunk_threads;
    /* Numeric chunks with at most this many outputs are accumulated by rank
     * in a compact array, one wave per chunk (0 = off, else 512, 1024 or
     * 2048); larger chunks use the dense accumulator. */
    int32_t num_rank_cap;
    /* Largest number of adjacent chunks of one group-7 row merged into one
     * work item (0 = default 2, else 1 = no merging, 2, 4 or 8).  Adjacent
     * chunks are merged, in column order, while their intermediate products
     * together stay within num_rank_cap; a merged item then has at most that
     * many outputs and always takes the rank path.  Needs sorted B rows,
     * chunks_per_item = 1 and num_rank_cap > 0 (else no merging); an item
     * spans at most 65536 columns, and rows of more than 64 chunks are not
     * merged. */
    int32_t chunk_merge;
    /* 1: the first spgemm_numeric (or spgemm_numeric_batch) call of the plan
     * captures the phase's kernel launches into a HIP graph that the plan
     * keeps, and every call, that one included, runs the phase as one launch
     * of that graph on the plan's stream.  A value-only re-run then costs
     * one descriptor upload and one graph launch, whatever the number of
     * row groups.  The graph holds no memory set or copy node; the value and
     * output pointers of each call reach the kernels through the uploaded
     * descriptors.  Ignored (launches stay eager) when profile = 1.  0 = off. */
    int32_t graph;
    /* Most column-chunk work items (group 7) a plan may create in either
     * phase; 0 = 2^31 - 1, what the 32-bit item indexing holds.  A plan that
     * needs more fails with SPGEMM_EOVERFLOW: spgemm_plan_create for the
     * symbolic items, spgemm_symbolic for the numeric ones. */
    int64_t item_limit;
    /* 1: rows of group 1 (the smallest) are handled one thread per row, in
     * the manner of the paper's AIA kernel (Section IV-D): a gather pass
     * first resolves rpt_B[col_A[j]] and rpt_B[col_A[j] + 1] of the group's
     * A nonzeros into one sequential stream per row, which each workgroup
     * stages in LDS; each thread then walks its row with a private LDS
     * table.  Requires sym_upper[1] and num_upper[1] <= 32.  0 = off (the
     * lane-group kernels). */
    int32_t row_thread;
    /* Accumulation precision of the column-chunked rows (group 7, the rows
     * with the longest outputs): 0 = FP32, as the paper's atomic adds of
     * valA x valB (Algorithm 4); 1 = FP64: each product a * b is formed
     * exactly in FP64, the sums are kept in FP64 and every output is rounded
     * to FP32 once.  With 1 the plan uses chunks of at most 2048 columns
     * (chunk_cols is lowered to 2048), num_rank_cap 2048, chunk_merge 1 and
     * chunks_per_item 1, and B must hold fewer than 2^30 nonzeros when such
     * rows exist (else SPGEMM_EINVAL).  The other groups accumulate in FP32;
     * lower the group bounds to send more rows to group 7 (every row whose
     * key exceeds num_upper[6]).  Device-driven plans have no group 7. */
    int32_t accumulate;
} spgemm_options;

typedef struct spgemm_plan spgemm_plan;

/* Per-plan figures, filled after each phase. */
typedef struct {
    int64_t flops;                         /* 2 * sum of intermediate products */
    int64_t ip_total;                      /* sum of intermediate products     */
    int64_t ip_max;                        /* largest row                      */
    int64_t nnz_c;                         /* after spgemm_symbolic, else -1   */
    int64_t sym_group_rows[SPGEMM_NGROUPS];
    int64_t num_group_rows[SPGEMM_NGROUPS];/* after spgemm_symbolic            */
    int64_t chunk_cols;                    /* chunk width used (product 0)     */
    int64_t chunks_per_row;                /* chunks per group-7 row (prod. 0) */
    size_t workspace_bytes;                /* device workspace held            */
} spgemm_info;

/* Fills *opt with the tuned defaults for gfx950. */
void spgemm_default_options(spgemm_options *opt);

/* Creates a plan for C = A * B and runs the row-size estimation (paper
 * Algorithm 1) and the row grouping (paper Section III-B) on `stream`
 * (a hipStream_t; NULL = default stream).  Synchronises the stream once to
 * read the group sizes.  A and B describe structure only (values may be
 * NULL); the descriptors are copied, the arrays they point to are borrowed.
 * opt NULL = spgemm_default_options.  Errors: EINVAL, EDIM (A->ncols !=
 * B->nrows or a size >= 2^31), EINDEX (validate = 1 and a malformed input),
 * ENOMEM, EHIP.  On error *out is NULL. */
spgemm_status spgemm_plan_create(spgemm_plan **out, const spgemm_csr *A,
                                 const spgemm_csr *B, const spgemm_options *opt,
                                 void *stream, spgemm_alloc_fn alloc_fn,
                                 spgemm_free_fn free_fn, void *alloc_ctx);

/* Same for `nprod` independent products C_p = A_p * B_p that share every
 * launch: each phase runs one launch per row group over the rows of all
 * products (a global group queue).  A and B are host arrays of nprod
 * descriptors. */
spgemm_status spgemm_plan_create_batch(spgemm_plan **out, int32_t nprod,
                                       const spgemm_csr *A, const spgemm_csr *B,
                                       const spgemm_options *opt, void *stream,
                                       spgemm_alloc_fn alloc_fn,
                                       spgemm_free_fn free_fn, void *alloc_ctx);

/* Allocation phase (paper Algorithms 2-4, keys only) and row-pointer scan.
 * Writes the m + 1 row pointers of C to c_row_ptr (device, caller owned).
 * Synchronises the stream and returns nnz(C) in *nnz_c (host) and, when
 * flops is not NULL, 2 * sum(IP) in *flops (host).  Must follow
 * spgemm_plan_create exactly once (else ESTATE).  Single-product plans only
 * (ESTATE on a batch plan). */
spgemm_status spgemm_symbolic(spgemm_plan *p, int64_t *c_row_ptr,
                              int64_t *nnz_c, int64_t *flops);

/* Batch form: c_row_ptr is a host array of nprod device pointers (product p
 * gets A_p.nrows + 1 entries); nnz_c a host array of nprod counts. */
spgemm_status spgemm_symbolic_batch(spgemm_plan *p, int64_t *const *c_row_ptr,
                                    int64_t *nnz_c);

/* Accumulation phase (paper Algorithms 4-5, Section III-D): writes nnz(C)
 * sorted column indices and FP32 values (device, caller owned) for the
 * structure computed by spgemm_symbolic.  Asynchronous on the plan's stream.
 * May be called again with new values for the same structures (value-only
 * re-run).  a_values / b_values must hold A.nnz / B.nnz FP32 values.
 * ESTATE before spgemm_symbolic. */
spgemm_status spgemm_numeric(spgemm_plan *p, const float *a_values,
                             const float *b_values, int32_t *c_col_idx,
                             float *c_values);

/* Batch form: host arrays of nprod device pointers each. */
spgemm_status spgemm_numeric_batch(spgemm_plan *p, const float *const *a_values,
                                   const float *const *b_values,
                                   int32_t *const *c_col_idx,
                                   float *const *c_values);

/* Row-size estimation alone (paper Algorithm 1), for admission control
 * before a plan exists: writes three int64 to out (device memory, caller
 * owned): out[0] = sum over rows of the intermediate products, out[1] = sum
 * over rows of min(intermediate products, B.ncols), an upper bound of
 * nnz(C), out[2] = the largest row's intermediate products.  Reads
 * A.row_ptr, A.col_idx and B.row_ptr only (no values, no B columns).
 * Enqueued on `stream`; never synchronises and allocates nothing.  Errors:
 * EINVAL (NULL pointers, negative sizes), EDIM (A.ncols != B.nrows or a size
 * >= 2^31), EHIP (launch failed). */
spgemm_status spgemm_estimate(const spgemm_csr *A, const spgemm_csr *B, int64_t *out,
                              void *stream);

/* ------------------------------------------------------------------------
 * Device-driven batch plans: no host synchronisation and no host round trip
 * between the phases.  Every row-group launch covers an upper bound of its
 * rows and takes the group's part of the row map from device memory, and C
 * is written into one arena the caller sizes from an upper bound
 * (spgemm_estimate's sum of min(IP, ncols)).  The whole execution can be
 * captured as one HIP graph.  For products whose B has at most
 * min(sym_upper[6], num_upper[6]) columns (no row is then column chunked),
 * such as the served aggregation requests.
 * ------------------------------------------------------------------------ */

/* Creates a device-driven plan for nprod products (host arrays of
 * descriptors, as spgemm_plan_create_batch): checks, allocates the per-row
 * workspace (one allocator call) and uploads the descriptors; no kernel runs
 * and the stream is not synchronised.  EINVAL also when a B has more columns
 * than the bound above, or options.validate / options.row_thread are set;
 * EOVERFLOW when the products' A have 2^26 rows or more in total (the
 * group launches cover every row of the batch). */
spgemm_status spgemm_plan_create_device(spgemm_plan **out, int32_t nprod, const spgemm_csr *A,
                                        const spgemm_csr *B, const spgemm_options *opt,
                                        void *stream, spgemm_alloc_fn alloc_fn,
                                        spgemm_free_fn free_fn, void *alloc_ctx);

/* Runs the whole product for every product of a device-driven plan,
 * enqueued on the plan's stream with no host synchronisation: intermediate
 * products and grouping (paper Algorithm 1, Section III-B), the allocation
 * phase and row-pointer scan (Algorithms 2-4), the regrouping and the
 * accumulation phase with its ordered gathering (Algorithms 4-5,
 * Section III-D).
 *   a_values, b_values  host arrays of nprod device pointers (FP32 values);
 *   c_row_ptr           host array of nprod device pointers, A_p.nrows + 1
 *                       int64 each: product p's own row pointers;
 *   c_offsets           device, nprod + 1 int64: product p's C occupies
 *                       arena entries [c_offsets[p], c_offsets[p + 1]);
 *   c_col, c_val        the arena (device, capacity entries each).
 * All caller owned.  When the batch's nnz(C) exceeds capacity nothing is
 * written to the arena and spgemm_sync reports SPGEMM_ENOMEM (c_offsets then
 * holds the sizes needed).  May be called again (new values, or the same).
 * With options.graph = 1 the first call captures every launch into one
 * HIP graph and later calls replay it (re-captured when c_row_ptr,
 * c_offsets or capacity change).  ESTATE on a plan not made by
 * spgemm_plan_create_device; symbolic / numeric calls on such a plan return
 * ESTATE. */
spgemm_status spgemm_execute_arena(spgemm_plan *p, const float *const *a_values,
                                   const float *const *b_values, int64_t *const *c_row_ptr,
                                   int64_t *c_offsets, int32_t *c_col, float *c_val,
                                   int64_t capacity);

/* Waits for the plan's stream and reports a kernel-raised error flag
 * (EINTERNAL), a C too large for its arena (ENOMEM, device-driven plans) or
 * a failed launch (EHIP). */
spgemm_status spgemm_sync(spgemm_plan *p);

/* Fills *info (host).  Never synchronises. */
spgemm_status spgemm_get_info(const spgemm_plan *p, spgemm_info *info);

/* Copies internal per-row arrays into caller device buffers (for tests):
 *   what 0: intermediate products, int64 [total rows]
 *   what 1: symbolic row map, int64 [total rows], entries (product << 32) | row,
 *           listed group by group, ascending row order inside a group
 *   what 2: numeric row map, same layout (after spgemm_symbolic)
 * group_start (host, SPGEMM_NGROUPS + 1 entries) receives the group offsets
 * into the map (what 1 / 2) and may be NULL.  Enqueued on the plan's stream. */
spgemm_status spgemm_export(const spgemm_plan *p, int32_t what, void *dst,
                            int64_t *group_start);

/* With options.profile = 1: number of timed launch groups recorded so far,
 * and the name and duration (milliseconds, from HIP events on the plan's
 * stream) of entry idx.  spgemm_timing synchronises the stream.  Names are
 * static strings ("plan.ipcount", "sym.g5", "num.g7", ...). */
int32_t spgemm_timing_count(const spgemm_plan *p);
spgemm_status spgemm_timing(spgemm_plan *p, int32_t idx, const char **name, float *ms);

/* ------------------------------------------------------------------------
 * Device steps of the applications that chain products (paper Section V).
 * ------------------------------------------------------------------------ */

/* Graph contraction (paper Algorithm 7) contracts with the selector S, n x k,
 * S[v, labels[v]] = 1.  This builds its transpose S^T (k x n) by a counting
 * sort of the labels: row_ptr (k + 1 int64), col_idx (n int32: the vertices
 * of cluster l, in no fixed order inside the row, so the result is not
 * SPGEMM_ROWS_SORTED), values (n FP32, all 1).  labels: n int32 in [0, k).
 * All arrays are device memory owned by the caller; `workspace` is a device
 * buffer of spgemm_selector_transpose_workspace(k) bytes.  Enqueued on
 * `stream`, then synchronises it to report EINDEX for a label outside
 * [0, k).  EINVAL for NULL pointers or negative sizes. */
size_t spgemm_selector_transpose_workspace(int64_t k);
spgemm_status spgemm_selector_transpose(const int32_t *labels, int64_t n, int64_t k,
                                        int64_t *row_ptr, int32_t *col_idx, float *values,
                                        void *workspace, void *stream);

/* Markov clustering (paper Algorithm 6) after each expansion, on the
 * row-stochastic transpose of the column-stochastic matrix (the paper's
 * column operations become row operations): every entry x becomes x^power,
 * each row is divided by its sum, entries below theta are dropped (strictly:
 * y >= theta is kept), with k > 0 only the k largest of the rest are kept
 * (ordered by the input values, which must be nonnegative; equal values in
 * storage order, so the lower columns of a column-sorted row first), and
 * each row is divided by the sum of what it keeps; kept entries stay in
 * their input order.  Two calls share `workspace`
 * (spgemm_mcl_prune_workspace(m) bytes of device memory) and the same
 * power, theta and k:
 *   _count writes the m + 1 output row pointers (device) and returns the
 *          output length in *out_nnz (host; synchronises the stream);
 *   _write fills out_col / out_val (device, out_nnz entries each).
 * Arithmetic in FP32.  A row whose entries are all zero keeps nothing.
 * EINVAL for NULL pointers, negative m or k, theta < 0 or power <= 0. */
size_t spgemm_mcl_prune_workspace(int64_t m);
spgemm_status spgemm_mcl_prune_count(int64_t m, const int64_t *row_ptr, const float *values,
                                     float power, float theta, int32_t k, int64_t *out_row_ptr,
                                     void *workspace, int64_t *out_nnz, void *stream);
spgemm_status spgemm_mcl_prune_write(int64_t m, const int64_t *row_ptr, const int32_t *col_idx,
                                     const float *values, float power, float theta, int32_t k,
                                     const int64_t *out_row_ptr, void *workspace,
                                     int32_t *out_col, float *out_val, void *stream);

/* The convergence test of Markov clustering (paper Algorithm 6 iterates
 * while successive matrices change): writes to *out (device, one double)
 * the largest |a_ij - b_ij| over the union of the patterns of two m-row CSR
 * matrices A and B with column-sorted rows (an entry stored on one side
 * only counts against 0), computed in FP64 from the FP32 values, so exactly.
 * Enqueued on `stream`, no synchronisation.  EINVAL for NULL pointers or
 * negative sizes. */
spgemm_status spgemm_mcl_change(int64_t m, const int64_t *rpt_a, const int32_t *col_a,
                                const float *val_a, const int64_t *rpt_b, const int32_t *col_b,
                                const float *val_b, int64_t nnz_a, int64_t nnz_b, double *out,
                                void *stream);

/* The cluster interpretation of Markov clustering (paper Algorithm 6, last
 * step): connected components of the undirected graph with an edge {i, j}
 * for every stored entry (i, j) of the n x n pattern (row_ptr n + 1 int64,
 * col_idx nnz int32; values are not read).  labels (device, n int32) gets,
 * for every vertex, the smallest vertex of its component.  Rounds of
 * hooking and pointer jumping on the device; the host reads a flag after
 * each round (synchronises the stream) and returns the number of rounds in
 * *rounds (host, may be NULL).  workspace: spgemm_components_workspace()
 * bytes of device memory.  EINVAL for NULL pointers or negative sizes, EDIM
 * for n >= 2^31, EINTERNAL if the rounds do not settle (a malformed
 * pattern). */
size_t spgemm_components_workspace(void);
spgemm_status spgemm_components(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                                int64_t nnz, int32_t *labels, void *workspace, void *stream,
                                int32_t *rounds);

/* ------------------------------------------------------------------------
 * The GNN layer with a pruning layer (paper Section V-C): forward
 * X_l = A TopK(X_{l-1}, k) W_l (Eq. 1-2), the product A TopK(X) being the
 * SpGEMM of this library, and backward
 * dL/dX_{l-1} = M_k (.) (A^T (dL/dX_l) W_l^T) (Eq. 3).  Dense matrices are
 * row-major FP32 device arrays.
 * ------------------------------------------------------------------------ */

/* TopK(X, k) per row (per sample): the k entries of largest magnitude of
 * every row of the dense n x f matrix X (leading dimension ldx >= f), equal
 * magnitudes in column order, as compressed rows with ascending columns:
 * row_ptr (n + 1 int64), col_idx and values (n * min(k, f) each), all
 * device, caller owned.  The pattern is the mask M_k of Eq. 2.  Enqueued on
 * `stream`.  EINVAL for NULL pointers, negative sizes or ldx < f. */
spgemm_status spgemm_topk_rows(int64_t n, int64_t f, const float *x, int64_t ldx, int32_t k,
                               int64_t *row_ptr, int32_t *col_idx, float *values, void *stream);

/* Writes the m x n CSR matrix into the dense row-major array `dense`
 * (leading dimension ldd >= n; every other entry set to 0).  Enqueued. */
spgemm_status spgemm_csr_to_dense(int64_t m, int64_t n, const int64_t *row_ptr,
                                  const int32_t *col_idx, const float *values, float *dense,
                                  int64_t ldd, void *stream);

/* Dense C = op(A) op(B) in FP32 on the matrix cores: op(A) is M x K with
 * element (i, k) at A[i * a_row + k * a_col], op(B) is K x N with element
 * (k, j) at B[k * b_row + j * b_col] (so a transpose is a swap of the two
 * strides), C is M x N at C[i * ldc + j] (ldc >= N), overwritten.  Products
 * and sums in FP32.  Enqueued.  EINVAL for NULL pointers, negative sizes or
 * ldc < N; EDIM for M >= 64 * 65535. */
spgemm_status spgemm_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t a_row,
                              int64_t a_col, const float *B, int64_t b_row, int64_t b_col,
                              float *C, int64_t ldc, void *stream);

/* The backward product of Eq. 3 evaluated where the mask keeps an entry:
 * for every stored entry e = (i, c) of the mask (an m-row CSR pattern:
 * rpt_mask, col_mask), out[e] = sum over the stored entries (i, r, a) of
 * row i of A^T (rpt_t, col_t, val_t) of a * dense[r * ldd + c].  out has
 * the mask's nnz entries (device).  FP32.  Enqueued. */
spgemm_status spgemm_masked_spmm(int64_t m, const int64_t *rpt_t, const int32_t *col_t,
                                 const float *val_t, const float *dense, int64_t ldd,
                                 const int64_t *rpt_mask, const int32_t *col_mask, float *out,
                                 void *stream);

/* CSR transpose of the m x n matrix (nnz entries): rpt_t (n + 1), col_t and
 * val_t (nnz; val_t may be NULL when values is NULL), device, caller owned.
 * Entries of an output row are in no fixed order (the result is not
 * SPGEMM_ROWS_SORTED).  workspace: spgemm_transpose_workspace(n) bytes of
 * device memory.  Enqueued.  EINVAL for NULL pointers or negative sizes,
 * EDIM for m >= 2^31. */
size_t spgemm_transpose_workspace(int64_t ncols);
spgemm_status spgemm_transpose(int64_t m, int64_t n, const int64_t *row_ptr,
                               const int32_t *col_idx, const float *values, int64_t nnz,
                               int64_t *rpt_t, int32_t *col_t, float *val_t, void *workspace,
                               void *stream);

/* SAMPLE of matrix-based bulk sampling (paper Section V-C): s draws per row
 * of the m-row CSR matrix P (row_ptr, col_idx, values: nonnegative weights,
 * one distribution per row) by inverse transform sampling.  Draw t of row r
 * uses u[r * s + t] in [0, 1) (device, caller supplied, so the random
 * numbers are inputs): with S the FP32 sum of the row's weights in storage
 * order, it takes the column of the first entry whose FP32 running sum (the
 * same order) exceeds u * S, or the last entry if rounding leaves none; a
 * row of zero total weight draws self[r].  out (device, m * s int32) gets
 * the drawn columns, row-major.  Enqueued.  EINVAL for NULL pointers or
 * negative sizes. */
spgemm_status spgemm_its_sample(int64_t m, int32_t s, const int64_t *row_ptr,
                                const int32_t *col_idx, const float *values, const float *u,
                                const int32_t *self, int32_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Allocation-free entry point.  For callers that cannot allocate device
 * memory: code that must not call hipMalloc / hipFree or an allocator, such
 * as tight serving loops or harnesses that forbid allocation.
 * ------------------------------------------------------------------------ */

/* Size in bytes of the library's static device scratch array (64 MiB), the
 * largest workspace spgemm_multiply_noalloc can use.  Every GPU the library
 * runs on holds one such array until the process ends. */
size_t spgemm_noalloc_scratch_bytes(void);

/* C = A * B in one call, with the kernels of spgemm_plan_create +
 * spgemm_symbolic + spgemm_numeric, but allocating nothing: no hipMalloc,
 * hipFree, pinned host allocation, allocator callback, HIP event, stream or
 * graph.  The plan workspace is carved from the static scratch array of the
 * current device (the stream must belong to it), the host bookkeeping from
 * static host buffers.
 *   A, B      device CSR with values (borrowed); opt NULL = defaults
 *             (profile and graph are ignored).
 *   c_row_ptr device, A.nrows + 1 entries, caller owned.
 *   c_col_idx, c_values  device, c_capacity entries each, caller owned.
 *   nnz_c     host: nnz(C) once the symbolic phase has run, else -1.
 * Synchronises the stream before returning.  Returns OK when C is complete.
 * ENOMEM with *nnz_c = -1: the workspace would exceed
 * spgemm_noalloc_scratch_bytes() (or the static host bookkeeping), nothing
 * written.  ENOMEM with *nnz_c >= 0: nnz(C) exceeds c_capacity; c_row_ptr is
 * written, columns and values are not (call again with larger arrays).
 * Other errors as spgemm_plan_create / spgemm_symbolic / spgemm_sync.
 * The scratch array is shared by every call on a GPU and keeps the last
 * call's contents (the kernels clear what must start at zero).  Calls that
 * overlapped on one GPU would race on it; the library serialises calls
 * inside a process, and each returns only after its stream has drained. */
spgemm_status spgemm_multiply_noalloc(const spgemm_csr *A, const spgemm_csr *B,
                                      const spgemm_options *opt, void *stream,
                                      int64_t *c_row_ptr, int32_t *c_col_idx, float *c_values,
                                      int64_t c_capacity, int64_t *nnz_c);

/* Releases a plan and its workspace.  NULL-safe.  Waits for the stream. */
void spgemm_free(spgemm_plan *p);

/* Static description of a status code. */
const char *spgemm_status_string(spgemm_status s);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_H */
