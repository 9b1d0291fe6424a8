// Rows of a B stored out of column order, sorted once at plan time when the
// product has column-chunked rows.  The chunk kernels then find each chunk's
// part of a B row by the tabulated chunk bounds (one binary search per B row
// and bound) instead of scanning the whole row for every chunk, which would
// cost a factor of the chunk count in gathers.
//
// The sort is rocPRIM's segmented radix sort of (column, original position)
// pairs, one segment per B row, over just the bits the column count needs.
// The permutation is kept: every numeric call gathers B's values into the
// sorted order first (B's values may change between calls, its structure
// may not).
#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "common.hpp"

namespace spg {

static int key_bits(int64_t ncols) {
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < ncols) ++bits;
    return bits;
}

size_t bsort_temp_bytes(int64_t nnz, int64_t rows, int64_t ncols) {
    size_t bytes = 0;
    rocprim::counting_iterator<int32_t> idx(0);
    const hipError_t e = rocprim::segmented_radix_sort_pairs(
        nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr, idx, (int32_t *)nullptr,
        (unsigned)nnz, (unsigned)rows, (const int64_t *)nullptr, (const int64_t *)nullptr, 0,
        (unsigned)key_bits(ncols), (hipStream_t)0);
    return e == hipSuccess ? bytes : 0;
}

hipError_t launch_bsort(const int64_t *rpt, int64_t rows, int64_t ncols, const int32_t *col,
                        int64_t nnz, int32_t *col_out, int32_t *perm, void *tmp, size_t tmp_bytes,
                        hipStream_t s) {
    if (nnz <= 0 || rows <= 0) return hipSuccess;
    rocprim::counting_iterator<int32_t> idx(0);
    size_t bytes = tmp_bytes;
    return rocprim::segmented_radix_sort_pairs(tmp, bytes, col, col_out, idx, perm,
                                               (unsigned)nnz, (unsigned)rows, rpt, rpt + 1, 0,
                                               (unsigned)key_bits(ncols), s);
}

// out[j] = val[perm[j]]: B's values in the sorted order.
__global__ void k_gather_f32(const float *__restrict__ val, const int32_t *__restrict__ perm,
                             int64_t n, float *__restrict__ out) {
    const int64_t j = lin_block() * blockDim.x + threadIdx.x;
    if (j < n) out[j] = val[perm[j]];
}

void launch_gather_f32(const float *val, const int32_t *perm, int64_t n, float *out,
                       hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_f32, grid1d((n + 255) / 256, 256), dim3(256), 0, s, val, perm, n,
                       out);
}

}  // namespace spg
