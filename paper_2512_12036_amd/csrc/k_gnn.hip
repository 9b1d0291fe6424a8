// The GNN layer with a pruning layer (paper Section V-C, Eq. 1-3), around
// the SpGEMM path:
//
//  * k_topk_rows: TopK(X, k) of a dense row-major feature matrix, per row
//    (per sample): the k entries of largest magnitude, ties in column order,
//    written as compressed rows with ascending columns -- the sparse X (.) M_k
//    of Eq. 2 and, through its pattern, the mask M_k itself.  Radix
//    selection on the magnitude bits, 8 bits per pass, one wave per row.
//  * k_csr_to_dense: the SpGEMM result A TopK(X) scattered into a dense
//    row-major matrix for the product with W.
//  * k_gemm_f32: dense C = op(A) op(B) in FP32 on the matrix cores
//    (v_mfma_f32_16x16x4f32): 64 x 64 output tiles per 256-thread
//    workgroup, 32 x 32 per wave as 2 x 2 MFMA tiles, operands staged
//    through LDS 16 deep in k.  Strided operands, so transposed views
//    (W^T, H^T) need no copy.  Used for X_l = (A TopK(X)) W, for the
//    backward G W^T and for the weight gradient H^T G.
//  * k_masked_spmm: the backward product of Eq. 3 evaluated only where the
//    mask keeps an entry: out[i, c] = sum_r A^T[i, r] D[r, c] for the kept
//    columns c of row i (one wave per row, a lane per kept column).
//  * k_transpose_*: CSR transpose by a counting sort of the columns (row
//    order inside an output row not fixed).
#include "common.hpp"
#include "dev.hpp"

namespace spg {

// ---------------------------------------------------------------------------
// TopK per row
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_topk_rows(int64_t n, int64_t f, const float *__restrict__ x,
                                                  int64_t ldx, int k,
                                                  int32_t *__restrict__ col,
                                                  float *__restrict__ val) {
    __shared__ uint32_t hist[256];
    const int64_t i = lin_block();
    const int lane = threadIdx.x;
    if (i >= n) return;
    const float *row = x + i * ldx;
    const int kk = (int64_t)k < f ? k : (int)f;
    int32_t *oc = col + i * kk;
    float *ov = val + i * kk;
    uint32_t thr = 0;
    int ties = kk;  // keep every entry when k >= f
    if (kk < f) {
        uint32_t prefix = 0, mask = 0;
        int need = kk;
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int b = lane; b < 256; b += 64) hist[b] = 0;
            __syncthreads();
            for (int64_t j = lane; j < f; j += 64) {
                const uint32_t key = __float_as_uint(row[j]) & 0x7fffffffu;
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
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
    // emit in column order: magnitude above thr, or equal to it among the
    // first `ties` such entries
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int o = 0, tie_seen = 0;
    for (int64_t jb = 0; jb < f; jb += 64) {
        const int64_t j = jb + lane;
        bool keep = false, tie = false;
        float v = 0.f;
        if (j < f) {
            v = row[j];
            const uint32_t key = __float_as_uint(v) & 0x7fffffffu;
            if (kk < f) {
                keep = key > thr;
                tie = key == thr;
            } else {
                keep = true;
            }
        }
        const unsigned long long tb = __ballot(tie);
        if (tie && tie_seen + __popcll(tb & lt) < ties) keep = true;
        tie_seen += __popcll(tb);
        const unsigned long long bal = __ballot(keep);
        const int at = o + __popcll(bal & lt);
        if (keep && at < kk) {
            oc[at] = (int32_t)j;
            ov[at] = v;
        }
        o += __popcll(bal);
    }
}

// ---------------------------------------------------------------------------
// CSR -> dense (zero-filled first)
// ---------------------------------------------------------------------------
__global__ void k_fill_f32(float *__restrict__ p, int64_t n, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = lin_block() * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_rows(int64_t m, int64_t n, float *__restrict__ c,
                                                   int64_t ldc) {
    const int64_t r = lin_block() * 4 + (threadIdx.x >> 6);
    if (r >= m) return;
    for (int64_t j = threadIdx.x & 63; j < n; j += 64) c[r * ldc + j] = 0.f;
}

__global__ __launch_bounds__(256) void k_csr_to_dense(int64_t m, const int64_t *__restrict__ rpt,
                                                      const int32_t *__restrict__ col,
                                                      const float *__restrict__ val,
                                                      float *__restrict__ d, int64_t ldd) {
    const int64_t r = lin_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    for (int64_t j = rpt[r] + lane; j < rpt[r + 1]; j += 64) d[r * ldd + col[j]] = val[j];
}

// ---------------------------------------------------------------------------
// FP32 GEMM on MFMA.  op(A)[i, k] = A[i * sar + k * sac], op(B)[k, j] =
// B[k * sbr + j * sbc], C[i, j] at C[i * ldc + j].
//
// v_mfma_f32_16x16x4f32 (one wave): D[16 x 16] += A[16 x 4] B[4 x 16]; lane
// l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + r][l % 16] in its r-th accumulator, r = 0..3.
//
// Split k: when the output has too few tiles to fill the chip (the weight
// gradient H^T G is 512 x 256 over k = the graph's rows), blockIdx.z takes
// its own range of k and adds its partial tile into C (zeroed first) with
// FP32 atomics; the sum's order is then not fixed, its error bound the same.
// ---------------------------------------------------------------------------
constexpr int GT = 64;   // output tile edge per workgroup
constexpr int GK = 16;   // k depth staged per step

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_f32(int64_t M, int64_t N, int64_t K,
                                                  const float *__restrict__ A, int64_t sar,
                                                  int64_t sac, const float *__restrict__ B,
                                                  int64_t sbr, int64_t sbc,
                                                  float *__restrict__ C, int64_t ldc,
                                                  int64_t kslice) {
    __shared__ float sA[GK][GT + 4];  // [k][i]
    __shared__ float sB[GK][GT + 4];  // [k][j]
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.y * GT, j0 = (int64_t)blockIdx.x * GT;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    // loader mapping: 1024 elements per operand tile, 4 per thread; walk
    // along whichever index is contiguous in memory so the loads coalesce
    const bool a_kfast = sac == 1;
    const bool b_jfast = sbc == 1;
    int ai[4], ak[4], bj[4], bk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;  // 0..1023
        if (a_kfast) { ak[q] = e & 15; ai[q] = e >> 4; } else { ai[q] = e & 63; ak[q] = e >> 6; }
        if (b_jfast) { bj[q] = e & 63; bk[q] = e >> 6; } else { bk[q] = e & 15; bj[q] = e >> 4; }
    }
    const int64_t kbeg = (int64_t)blockIdx.z * kslice;
    const int64_t kend = kbeg + kslice < K ? kbeg + kslice : K;
    // the next k step's elements are loaded into registers while the MFMAs
    // of the current one run
    float ra[4], rb[4];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gi = i0 + ai[q], gk = k0 + ak[q];
            ra[q] = (gi < M && gk < kend) ? A[gi * sar + gk * sac] : 0.f;
            const int64_t gj = j0 + bj[q], gkb = k0 + bk[q];
            rb[q] = (gj < N && gkb < kend) ? B[gkb * sbr + gj * sbc] : 0.f;
        }
    };
    fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sA[ak[q]][ai[q]] = ra[q];
            sB[bk[q]][bj[q]] = rb[q];
        }
        __syncthreads();
        if (k0 + GK < kend) fetch(k0 + GK);
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const int kr = ks + (lane >> 4);
            float av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sA[kr][wr + 16 * a + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sB[kr][wc + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0,
                                                                      0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = i0 + wr + 16 * a + 4 * (lane >> 4) + r;
                const int64_t gj = j0 + wc + 16 * b + (lane & 15);
                if (gi < M && gj < N) {
                    if (gridDim.z > 1)
                        atomicAdd(&C[gi * ldc + gj], acc[a][b][r]);
                    else
                        C[gi * ldc + gj] = acc[a][b][r];
                }
            }
}

// ---------------------------------------------------------------------------
// Masked SpMM (Eq. 3): out[e] for every kept entry e = (i, c) of the mask
// (row i, column c) = sum over the nonzeros (r, a) of row i of A^T of
// a * D[r, c].  One wave per row, one lane per kept entry (rows keep at
// most a few dozen); the A^T entries are read once per wave.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_masked_spmm(int64_t m, const int64_t *__restrict__ rpt_t,
                                                     const int32_t *__restrict__ col_t,
                                                     const float *__restrict__ val_t,
                                                     const float *__restrict__ d, int64_t ldd,
                                                     const int64_t *__restrict__ rpt_m,
                                                     const int32_t *__restrict__ col_m,
                                                     float *__restrict__ out) {
    const int64_t i = lin_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    const int64_t m0 = rpt_m[i], m1 = rpt_m[i + 1];
    const int64_t a0 = rpt_t[i], a1 = rpt_t[i + 1];
    for (int64_t eb = m0; eb < m1; eb += 64) {
        const int64_t e = eb + lane;
        const bool act = e < m1;
        const int32_t c = act ? col_m[e] : 0;
        float s = 0.f;
        for (int64_t j = a0; j < a1; ++j) {
            const int32_t r = col_t[j];
            const float a = val_t[j];
            if (act) s += a * d[(int64_t)r * ldd + c];
        }
        if (act) out[e] = s;
    }
}

// ---------------------------------------------------------------------------
// CSR transpose (counting sort by column).
// ---------------------------------------------------------------------------
__global__ void k_col_count(const int32_t *__restrict__ col, int64_t nnz,
                            unsigned long long *__restrict__ cnt) {
    const int64_t j = lin_block() * blockDim.x + threadIdx.x;
    if (j < nnz) atomicAdd(&cnt[col[j]], 1ull);
}

__global__ __launch_bounds__(256) void k_transpose_scatter(int64_t m, const int64_t *__restrict__ rpt,
                                                           const int32_t *__restrict__ col,
                                                           const float *__restrict__ val,
                                                           unsigned long long *__restrict__ cursor,
                                                           int32_t *__restrict__ col_t,
                                                           float *__restrict__ val_t) {
    const int64_t r = lin_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    for (int64_t j = rpt[r] + lane; j < rpt[r + 1]; j += 64) {
        const int64_t pos = (int64_t)atomicAdd(&cursor[col[j]], 1ull);
        col_t[pos] = (int32_t)r;
        if (val) val_t[pos] = val[j];
    }
}

__global__ void k_rows_uniform(int64_t *__restrict__ rpt, int64_t n, int64_t k) {
    const int64_t i = lin_block() * blockDim.x + threadIdx.x;
    if (i <= n) rpt[i] = i * k;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_rows_uniform(int64_t *rpt, int64_t n, int64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_uniform, grid1d(((n + 256) / 256), 256), dim3(256), 0, s, rpt, n,
                       k);
}

void launch_topk_rows(int64_t n, int64_t f, const float *x, int64_t ldx, int k, int32_t *col,
                      float *val, hipStream_t s) {
    if (n <= 0 || f <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_topk_rows, grid1d(n, 64), dim3(64), 0, s, n, f, x, ldx, k, col, val);
}

void launch_csr_to_dense(int64_t m, int64_t n, const int64_t *rpt, const int32_t *col,
                         const float *val, float *d, int64_t ldd, hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    const int64_t total = (m - 1) * ldd + n;
    int64_t nb = (total + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)nb), dim3(256), 0, s, d, total, 0.f);
    hipLaunchKernelGGL(k_csr_to_dense, grid1d(((m + 3) / 4), 256), dim3(256), 0, s, m, rpt, col,
                       val, d, ldd);
}

void launch_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t sar, int64_t sac,
                     const float *B, int64_t sbr, int64_t sbc, float *C, int64_t ldc,
                     hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    if (K <= 0) {  // empty sum: C = 0
        hipLaunchKernelGGL(k_fill_rows, grid1d(((M + 3) / 4), 256), dim3(256), 0, s, M, N, C,
                           ldc);
        return;
    }
    // split k until the grid has about four workgroups per compute unit,
    // keeping at least 256 of k per slice
    const int64_t tiles = ((N + GT - 1) / GT) * ((M + GT - 1) / GT);
    int64_t split = 1;
    while (tiles * split < 1024 && K / (2 * split) >= 256 && split < 64) split *= 2;
    const int64_t kslice = ((K + split - 1) / split + GK - 1) / GK * GK;
    split = (K + kslice - 1) / kslice;
    if (split > 1)
        hipLaunchKernelGGL(k_fill_rows, grid1d(((M + 3) / 4), 256), dim3(256), 0, s, M, N, C,
                           ldc);
    dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)split);
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, s, M, N, K, A, sar, sac, B, sbr, sbc, C,
                       ldc, kslice);
}

void launch_masked_spmm(int64_t m, const int64_t *rpt_t, const int32_t *col_t, const float *val_t,
                        const float *d, int64_t ldd, const int64_t *rpt_m, const int32_t *col_m,
                        float *out, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_masked_spmm, grid1d(((m + 3) / 4), 256), dim3(256), 0, s, m, rpt_t,
                       col_t, val_t, d, ldd, rpt_m, col_m, out);
}

void launch_transpose(int64_t m, int64_t n, const int64_t *rpt, const int32_t *col,
                      const float *val, int64_t nnz, int64_t *rpt_t, int32_t *col_t,
                      float *val_t, int64_t *work, void *scan_tmp, hipStream_t s) {
    launch_fill_i64(work, n, 0, s);
    if (nnz > 0)
        hipLaunchKernelGGL(k_col_count, grid1d(((nnz + 255) / 256), 256), dim3(256), 0, s, col,
                           nnz, (unsigned long long *)work);
    launch_scan_i64(work, rpt_t, n, scan_tmp, s);
    (void)hipMemcpyAsync(work, rpt_t, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s);
    if (m > 0 && nnz > 0)
        hipLaunchKernelGGL(k_transpose_scatter, grid1d(((m + 3) / 4), 256), dim3(256), 0, s, m,
                           rpt, col, val, (unsigned long long *)work, col_t, val_t);
}

}  // namespace spg
