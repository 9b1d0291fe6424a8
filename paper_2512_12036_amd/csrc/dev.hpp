// Device-side helpers shared by the hash and chunk kernels.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace spg {

// Loads through the global address space: the pointers the kernels read come
// from descriptors in device memory, so the compiler cannot infer the address
// space and would otherwise emit flat loads (which also wait on LDS traffic).
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

template <typename T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// A pointer that every lane of the wave holds, moved to scalar registers so
// that loads can use the scalar-base + 32-bit-offset addressing form.
template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const T *)(((uint64_t)hi << 32) | lo);
}

// The value at a 32-bit byte offset from a uniform base (one global load
// with a scalar base and a vector offset).
template <typename T>
__device__ __forceinline__ T gld_boff(const T *base, uint32_t byte) {
    return *(const __attribute__((address_space(1))) T *)((const char *)base + byte);
}

// Element idx of a uniform base, addressed the same way (requires
// idx * sizeof(T) < 2^32).
template <typename T>
__device__ __forceinline__ T gld_off(const T *base, uint32_t idx) {
    return gld_boff(base, idx * (uint32_t)sizeof(T));
}

// Largest o in [lo, hi) with e[o] <= q (e non-decreasing, e[lo] <= q).
template <typename T>
__device__ __forceinline__ int lds_owner(const T *e, int lo, int hi, T q) {
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (e[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

// FP32 add into LDS through a compare-and-swap loop.  On gfx950 the LDS
// float atomic add (ds_add_f32) retires about a third of a lane per clock per
// CU -- some 16x below the integer LDS atomics the loop is built from -- so
// the loop is far faster whenever retries are rare (distinct addresses in a
// wave, the common case of hash and dense accumulators).
__device__ __forceinline__ void lds_fadd(float *p, float v) {
    uint32_t *q = reinterpret_cast<uint32_t *>(p);
    uint32_t cur = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const uint32_t next = __float_as_uint(__uint_as_float(cur) + v);
        const uint32_t prev = atomicCAS(q, cur, next);
        if (prev == cur) return;
        cur = prev;
    }
}

// Inclusive prefix sum over the 64 lanes of a wave (every lane active).
// 32-bit integers go through DPP: row shifts of 1, 2, 4 and 8 lanes give
// each 16-lane row its own prefix, then the broadcasts of lane 15 (into rows
// 1 and 3) and of lane 31 (into rows 2 and 3) add the earlier rows' totals.
// That is six ALU steps with no LDS traffic, where a shuffle (ds_bpermute)
// costs an LDS round trip per step.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    if constexpr (sizeof(T) == 4 && std::is_integral<T>::value) {
        int v = (int)x;
        v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
        v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
        v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
        v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
        v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
        v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
        return (T)v;
    } else {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            T o = __shfl_up(x, off, 64);
            if (lane >= off) x += o;
        }
        return x;
    }
}

// Inclusive prefix sum over aligned segments of G lanes (G = 8, 16, 32 or
// 64; every lane of the segment active, other segments may be idle).  The
// DPP steps only ever read lanes of the same segment: shifts inside a
// 16-lane row, masked at segment starts when G < 16, then for G >= 32 the
// broadcast of lane 15 into the next row and for G = 64 that of lane 31.
template <int G>
__device__ __forceinline__ int seg_incl_scan(int v) {
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "segment width");
    const int l = (int)threadIdx.x & (G - 1);
    int t = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (G >= 16 || l >= 1) ? t : 0;
    t = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (G >= 16 || l >= 2) ? t : 0;
    t = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (G >= 16 || l >= 4) ? t : 0;
    if constexpr (G >= 16) v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    if constexpr (G >= 32) v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    if constexpr (G >= 64) v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

// The value of the last lane of each lane's G-lane segment (its total after
// seg_incl_scan), by readlanes: those of other segments are read but unused.
template <int G>
__device__ __forceinline__ int seg_last(int v) {
    if constexpr (G == 64) {
        return __builtin_amdgcn_readlane(v, 63);
    } else {
        const int seg = ((int)threadIdx.x & 63) / G;
        int r = 0;
#pragma unroll
        for (int s = 0; s < 64 / G; ++s) {
            const int x = __builtin_amdgcn_readlane(v, s * G + G - 1);
            if (seg == s) r = x;
        }
        return r;
    }
}

// Lane 63's value, in every lane (the wave total after wave_incl_scan).
template <typename T>
__device__ __forceinline__ T wave_last(T x) {
    if constexpr (sizeof(T) == 4 && std::is_integral<T>::value)
        return (T)__builtin_amdgcn_readlane((int)x, 63);
    else
        return __shfl(x, 63, 64);
}

template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *wsum, T &total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T incl = wave_incl_scan(v);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T x = wsum[i];
        if (i < w) before += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return before + incl - v;
}

// Sum over the 64 lanes of a wave, valid in lane 0 (in every lane for
// 32-bit integers).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    if constexpr (sizeof(T) == 4 && std::is_integral<T>::value) {
        return wave_last(wave_incl_scan(v));
    } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        return v;
    }
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += wsum[i];
    __syncthreads();
    return tot;
}

// Workgroup barrier that orders LDS traffic only: waits for this wave's LDS
// operations, then meets the other waves.  Unlike __syncthreads it does not
// drain outstanding global loads, so loads issued ahead of time (the next
// item's inputs) stay in flight across it.  Only for code whose cross-thread
// communication goes entirely through LDS.
__device__ __forceinline__ void lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Orders the LDS traffic of one wave (its LDS operations complete in issue
// order; this waits for them and keeps the compiler from moving memory
// accesses across).  For waves that work independently of the rest of their
// workgroup.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// block_excl_scan / block_sum with LDS-only barriers (see lds_sync); a
// single-wave workgroup needs no barrier at all.
template <int NT, typename T>
__device__ __forceinline__ T wg_excl_scan(T v, T *wsum, T &total) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T incl = wave_incl_scan(v);
    if (NW == 1) {
        total = wave_last(incl);
        return incl - v;
    }
    if (lane == 63) wsum[w] = incl;
    lds_sync();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T x = wsum[i];
        if (i < w) before += x;
        tot += x;
    }
    lds_sync();
    total = tot;
    return before + incl - v;
}

template <int NT, typename T>
__device__ __forceinline__ T wg_sum(T v, T *wsum) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if constexpr (NW == 1) {
        if constexpr (sizeof(T) == 4 && std::is_integral<T>::value) return v;
        else return __shfl(v, 0, 64);
    }
    if (lane == 0) wsum[w] = v;
    lds_sync();
    T tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) tot += wsum[i];
    lds_sync();
    return tot;
}

// 64-bit value of lane l (l uniform), in scalar registers.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Enumerates the products of one staged batch of A nonzeros, flat over the
// workgroup: product q belongs to the staged entry o with st_e[o] <= q <
// st_e[o+1] (st_e[nv] = total) and reads B entry st_s[o] + q - st_e[o].
// Each thread takes runs of VT consecutive products (merge-path style): one
// binary search per run, then a sequential walk that crosses B-row
// boundaries with one LDS read each (sub-ranges are often only a few entries
// long), and all VT gathers of a run are issued before any is consumed.
// S is the type of the staged B-row starts: uint32_t when every B of the
// plan has fewer than 2^30 entries (gathers then use 32-bit offsets from a
// scalar base, one address register per load), int64_t otherwise.
// f(col, a_value, b_value).
template <int WG, int VT, bool VALUES, typename E, typename S, typename F>
__device__ __forceinline__ void staged_products(const S *st_s, const E *st_e, const float *st_a,
                                                int nv, E total, const int32_t *colB,
                                                const float *valB, F &&f) {
    constexpr bool kOff32 = sizeof(S) == 4;
    const int32_t *ucol = uniform_ptr(colB);
    const float *uval = VALUES ? uniform_ptr(valB) : valB;
    for (E r0 = (E)threadIdx.x * VT; r0 < total; r0 += (E)WG * VT) {
        int o = lds_owner<E>(st_e, 0, nv, r0);
        E enext = st_e[o + 1];
        S t = st_s[o] + (S)(r0 - st_e[o]);
        float a = VALUES ? st_a[o] : 0.f;
        int cc[VT];
        float aa[VT], vv[VT];
        bool ok[VT];
#pragma unroll
        for (int v = 0; v < VT; ++v) {
            const E q = r0 + v;
            ok[v] = q < total;
            cc[v] = 0;
            aa[v] = 0.f;
            vv[v] = 0.f;
            if (ok[v]) {
                while (q >= enext) {
                    ++o;
                    t = st_s[o];
                    enext = st_e[o + 1];
                    if (VALUES) a = st_a[o];
                }
                if (kOff32) {
                    cc[v] = gld_off(ucol, (uint32_t)t);
                    if (VALUES) vv[v] = gld_off(uval, (uint32_t)t);
                } else {
                    cc[v] = gld(colB + t);
                    if (VALUES) vv[v] = gld(valB + t);
                }
                aa[v] = a;
                ++t;
            }
        }
#pragma unroll
        for (int v = 0; v < VT; ++v)
            if (ok[v]) f(cc[v], aa[v], vv[v]);
    }
}

// Lane groups of striped_products (see there).
#ifndef SPG_STRIPE_GROUPS
#define SPG_STRIPE_GROUPS 8
#endif
constexpr int kStripeGroups = SPG_STRIPE_GROUPS;

// Same contract as staged_products, but striped.  A wave takes a contiguous
// range of the batch's products and splits it between G groups of 64 / G
// lanes; each group takes a contiguous sub-range in steps of 64 / G
// products, lane k of the group handling product k of each step.  So one
// load instruction reads G runs of consecutive B entries (a few cache lines
// instead of one per lane), and a lane's successive products are only 64 / G
// apart: the owner of each product is found by walking forward from the
// lane's previous owner (one LDS round trip per B-row slice boundary
// crossed), and short slices make long walks when the steps are wide.  The
// owner of each group's first product comes from one binary search per
// staged batch (in a single-wave workgroup, a ballot over my_e, each lane's
// own st_e entry).  f receives VT products per lane at a time (arrays +
// valid flags).  CLAMP: a lane past its group's end reads the group's last
// product again (a real one, at or after the lane's previous product), so
// the loads need no branch, and f gets that product with its flag false;
// this pays where most lanes are busy and costs redundant loads where items
// are short.  Without CLAMP, an entry whose flag is false holds zeros.
template <int WG, int VT, bool VALUES, typename E, typename S, bool CLAMP = true, typename F>
__device__ __forceinline__ void striped_products(const S *st_s, const E *st_e, const float *st_a,
                                                 int nv, E total, const int32_t *colB,
                                                 const float *valB, F &&f,
                                                 int tid = threadIdx.x, E my_e = 0) {
    constexpr bool kOff32 = sizeof(S) == 4;
    constexpr int G = kStripeGroups;
    constexpr int GL = 64 / G;  // lanes per group
    static_assert(G >= 1 && G <= 64 && 64 % G == 0, "lane groups");
    const int32_t *ucol = uniform_ptr(colB);
    const float *uval = VALUES ? uniform_ptr(valB) : valB;
    constexpr int NW = WG / 64;
    const int lane = tid & 63, w = tid >> 6;
    const int g = lane / GL, k = lane % GL;
    // wave w takes a contiguous range of 64-product rows, group g a
    // contiguous part of it, so lanes only ever walk forward
    const E nrow = (total + 63) >> 6;
    const E r0 = nrow * w / NW, r1 = nrow * (w + 1) / NW;
    if (r0 >= r1) return;
    const E p0 = r0 * 64, p1 = r1 * 64 < total ? r1 * 64 : total;
    const E sub = ((p1 - p0 + G - 1) / G + GL - 1) / GL * GL;  // per group, whole steps
    const E g0 = p0 + (E)g * sub;
    const E g1 = g0 + sub < p1 ? g0 + sub : p1;
    int o = 0;
    if constexpr (NW == 1 && G > 1) {
        // A single-wave workgroup: lane j holds st_e[j] in my_e (not
        // decreasing over the lanes, lanes past nv at total), so the owner of
        // each group's first product is a ballot count, without a search
        // through LDS; taken before any lane leaves, so that every lane votes.
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            E qg = p0 + (E)gg * sub;
            if (qg > total - 1) qg = total - 1;
            const int og = __popcll(__ballot(my_e <= qg)) - 1;
            if (g == gg) o = og;
        }
    }
    // a group past the end of the wave's range has nothing to do (f holds no
    // wave-wide operation, so its lanes may leave)
    if (CLAMP && G > 1 && g0 >= g1) return;
    if constexpr (!(NW == 1 && G > 1))
        o = G == 1 ? __builtin_amdgcn_readfirstlane(lds_owner<E>(st_e, 0, nv, p0))
                   : lds_owner<E>(st_e, 0, nv, g0 < total ? g0 : total - 1);
    E e0 = st_e[o], e1 = st_e[o + 1];
    S base = st_s[o];
    float a = VALUES ? st_a[o] : 0.f;
    if constexpr (CLAMP && kOff32) {
        // Byte units (4 q, 4 e1, 4 (base - e0)), so that a product's address
        // is one add; B offsets are below 2^32 bytes here, and products of a
        // batch far fewer.
        uint32_t e1b = (uint32_t)e1 * 4u;
        uint32_t bob = ((uint32_t)base - (uint32_t)e0) * 4u;
        const uint32_t lastb = (uint32_t)(g1 - 1) * 4u;
        for (E s = 0; s < sub; s += (E)VT * GL) {
            int cc[VT];
            float aa[VT], vv[VT];
            bool ok[VT];
            const uint32_t qs = (uint32_t)(g0 + s + k) * 4u;
#pragma unroll
            for (int v = 0; v < VT; ++v) {
                const uint32_t qb = qs + (uint32_t)(v * GL * 4);
                ok[v] = qb <= lastb;
                const uint32_t qcb = qb < lastb ? qb : lastb;
                while (qcb >= e1b) {
                    ++o;
                    bob = ((uint32_t)st_s[o] - (uint32_t)e1) * 4u;  // e1 is o's first product
                    e1 = st_e[o + 1];
                    e1b = (uint32_t)e1 * 4u;
                    if (VALUES) a = st_a[o];
                }
                const uint32_t tb = bob + qcb;
                cc[v] = gld_boff(ucol, tb);
                vv[v] = VALUES ? gld_boff(uval, tb) : 0.f;
                aa[v] = a;
            }
            f(cc, aa, vv, ok);
        }
        return;
    }
    for (E s = 0; s < sub; s += (E)VT * GL) {
        int cc[VT];
        float aa[VT], vv[VT];
        bool ok[VT];
#pragma unroll
        for (int v = 0; v < VT; ++v) {
            const E q = g0 + s + (E)(v * GL + k);
            ok[v] = q < g1;
            if (CLAMP) {
                const E qc = ok[v] ? q : g1 - 1;
                while (qc >= e1) {
                    ++o;
                    e0 = e1;
                    e1 = st_e[o + 1];
                    base = st_s[o];
                    if (VALUES) a = st_a[o];
                }
                const S t = base + (S)(qc - e0);
                if (kOff32) {
                    cc[v] = gld_off(ucol, (uint32_t)t);
                    vv[v] = VALUES ? gld_off(uval, (uint32_t)t) : 0.f;
                } else {
                    cc[v] = gld(colB + t);
                    vv[v] = VALUES ? gld(valB + t) : 0.f;
                }
                aa[v] = a;
            } else {
                cc[v] = 0;
                aa[v] = 0.f;
                vv[v] = 0.f;
                if (ok[v]) {
                    while (q >= e1) {
                        ++o;
                        e0 = e1;
                        e1 = st_e[o + 1];
                        base = st_s[o];
                        if (VALUES) a = st_a[o];
                    }
                    const S t = base + (S)(q - e0);
                    if (kOff32) {
                        cc[v] = gld_off(ucol, (uint32_t)t);
                        if (VALUES) vv[v] = gld_off(uval, (uint32_t)t);
                    } else {
                        cc[v] = gld(colB + t);
                        if (VALUES) vv[v] = gld(valB + t);
                    }
                    aa[v] = a;
                }
            }
        }
        f(cc, aa, vv, ok);
    }
}

// Adds add[v] to acc[idx[v]] (LDS) for VT entries at once with the
// compare-and-swap scheme of lds_fadd, but batched: all loads, then all
// compare-and-swaps are issued before any result is waited for, so one
// wave pays two LDS round trips per VT products instead of 2 * VT.  Entries
// whose swap lost a race (another lane or step updated the same slot) retry
// one by one.  idx[v] must be a valid slot for every v: callers point the
// unused entries at a private dummy slot per lane with add = 0.
template <int VT>
__device__ __forceinline__ void lds_fadd_many(float *acc, const int *idx, const float *add) {
    uint32_t *q = reinterpret_cast<uint32_t *>(acc);
    uint32_t cur[VT], prev[VT];
#pragma unroll
    for (int v = 0; v < VT; ++v)
        cur[v] = __hip_atomic_load(q + idx[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int v = 0; v < VT; ++v)
        prev[v] = atomicCAS(q + idx[v], cur[v], __float_as_uint(__uint_as_float(cur[v]) + add[v]));
#pragma unroll
    for (int v = 0; v < VT; ++v) {
        uint32_t c = prev[v];
        bool pending = prev[v] != cur[v];
        while (pending) {
            const uint32_t p = atomicCAS(q + idx[v], c, __float_as_uint(__uint_as_float(c) + add[v]));
            pending = p != c;
            c = p;
        }
    }
}

}  // namespace spg
