// Host side of the C ABI declared in include/spgemm.h: plan state, workspace
// management and the launch sequence of the three phases of paper Section III
// (row grouping, allocation, accumulation).  All kernels are enqueued on the
// plan's stream; the only host synchronisations are the two documented ones
// (group sizes after planning, nnz(C) after the symbolic phase).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory_resource>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "spgemm.h"

using namespace spg;

namespace {
#include "tuned_defaults.inc"
}  // namespace

namespace {

constexpr int kDescSlots = 4;  // pinned descriptor staging buffers (ring)

// Process-wide pools of pinned host buffers and of events, per device.
// Pinned allocation and event creation are driver calls of tens of
// microseconds (a pinned free can wait on the device), which a stream of
// plans (a server, a benchmark loop) would otherwise pay per plan.  Plans
// take from the pools and give back in spgemm_free, after synchronising
// their stream; the pools keep everything until the process ends.
constexpr int kPoolDevices = 64;

class HostPools {
  public:
    // a pinned buffer of at least `bytes` (a power of two from 4 KB);
    // *got = its size; null if the allocation fails
    void *pinned(size_t bytes, size_t *got) {
        const int d = device();
        std::lock_guard<std::mutex> g(mu_);
        auto &fl = pinned_[d];
        size_t best = SIZE_MAX;
        for (size_t i = 0; i < fl.size(); ++i)
            if (fl[i].first >= bytes && (best == SIZE_MAX || fl[i].first < fl[best].first))
                best = i;
        if (best != SIZE_MAX) {
            const auto e = fl[best];
            fl.erase(fl.begin() + (std::ptrdiff_t)best);
            *got = e.first;
            return e.second;
        }
        size_t cap = 4096;
        while (cap < bytes) cap <<= 1;
        void *h = nullptr;
        if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        *got = cap;
        return h;
    }
    void give_pinned(void *h, size_t bytes) {
        if (!h) return;
        const int d = device();
        std::lock_guard<std::mutex> g(mu_);
        pinned_[d].emplace_back(bytes, h);
    }
    // an event; timing: false -> created with hipEventDisableTiming
    hipError_t event(hipEvent_t *e, bool timing) {
        const int d = device();
        {
            std::lock_guard<std::mutex> g(mu_);
            auto &fl = events_[timing][d];
            if (!fl.empty()) {
                *e = fl.back();
                fl.pop_back();
                return hipSuccess;
            }
        }
        return timing ? hipEventCreate(e) : hipEventCreateWithFlags(e, hipEventDisableTiming);
    }
    void give_event(hipEvent_t e, bool timing) {
        if (!e) return;
        const int d = device();
        std::lock_guard<std::mutex> g(mu_);
        events_[timing][d].push_back(e);
    }

  private:
    static int device() {
        int d = 0;
        if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kPoolDevices) d = 0;
        return d;
    }
    std::mutex mu_;
    std::vector<std::pair<size_t, void *>> pinned_[kPoolDevices];
    std::vector<hipEvent_t> events_[2][kPoolDevices];
};

// never destroyed: it may be used until the runtime shuts down
HostPools &pools() {
    static HostPools *p = new HostPools;
    return *p;
}

struct HostStats {
    int64_t ip_sum = 0, ip_max = 0, nnz_sum = 0, nnz_max = 0;
};

}  // namespace

struct spgemm_plan {
    // Host containers draw from `mr`: the heap for ordinary plans, a static
    // host buffer for the allocation-free entry point.
    explicit spgemm_plan(std::pmr::memory_resource *r = std::pmr::new_delete_resource())
        : A(r), B(r), hprods(r), hblks(r), hstats(r), nnz_c(r), timed(r), dev_rpt(r),
          bs_perm(r), bs_val(r), allocs(r) {}
    hipStream_t stream = nullptr;
    spgemm_alloc_fn afn = nullptr;
    spgemm_free_fn ffn = nullptr;
    void *actx = nullptr;
    spgemm_options opt{};
    bool batch = false;
    int nprod = 0;
    std::pmr::vector<spgemm_csr> A, B;
    std::pmr::vector<ProdDev> hprods;
    ProdDev *dprods = nullptr;
    ProdDev *pinned = nullptr;  // kDescSlots * nprod descriptors
    size_t pinned_bytes = 0;
    hipEvent_t desc_ev[kDescSlots] = {};
    bool desc_ev_used[kDescSlots] = {};
    int desc_next = 0;
    std::pmr::vector<RowBlk> hblks;
    RowBlk *dblks = nullptr;
    int nblk = 0;
    int64_t Mtot = 0;

    int64_t *ip = nullptr, *row_nnz = nullptr, *rptv = nullptr;
    uint64_t *map_sym = nullptr, *map_num = nullptr;
    int32_t *hslot = nullptr;
    int64_t *blkcnt = nullptr, *blkoff = nullptr, *starts = nullptr;
    ProdStats *stats = nullptr;
    int *flags = nullptr;  // [0] kernel error bits, [1..2] validation, [3..] unsorted per product
    void *scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;

    // chunk group (symbolic group 7)
    int64_t nh = 0, h_items = 0, h_split = 0, h_tiles = 0;
    int64_t *nchv = nullptr, *ibase = nullptr, *cbase = nullptr, *chunk_cnt = nullptr;
    int64_t *chunk_pos = nullptr;
    int32_t *hitem_row = nullptr;
    ChunkDesc *sdesc = nullptr;
    int64_t *slen = nullptr, *sbase = nullptr;  // sub-range tables (fast path)
    uint32_t *sabs = nullptr;
    uint32_t *sbits = nullptr;  // per-chunk structure bitmaps from the symbolic phase
    int wpc = 0;                // bitmap words per chunk
    // merging of adjacent light chunks into one item (merge > 1)
    int merge = 1;
    int wmax_item = 0;          // widest item: wmax * merge
    int32_t *mstart = nullptr;  // per chunk slot: first chunk of each item of the row
    int64_t s_items = 0;        // symbolic items
    // numeric group 7
    int64_t nd = 0, d_items = 0;
    int64_t *dnchv = nullptr, *dbase = nullptr;
    int32_t *ditem_row = nullptr;
    ChunkDesc *ndesc = nullptr;
    // numeric items split by output count: dense ones first (n_dense of them)
    ChunkDesc *ndesc_split = nullptr;
    int64_t *dflag = nullptr, *dfpos = nullptr;
    int64_t n_dense = -1;  // -1: not split
    int64_t n_items = 0;   // numeric items (exact)
    // the split list: dense | large single | small single | large merged |
    // small merged (small: at most half the rank cap outputs)
    int64_t n_s1 = 0, n_s0 = 0, n_m1 = 0, n_m0 = 0;
    int64_t *dflag2 = nullptr, *dfpos2 = nullptr;
    // thread-per-row group 1 (opt.row_thread): per-row stream offsets and
    // the streams of both phases
    int64_t *rt_lens = nullptr, *rt_off_sym = nullptr, *rt_off_num = nullptr;
    RangeEnt *rt_stream = nullptr;
    int wmax = 0;       // widest chunk over the products
    bool fast = true;   // every B sorted with < 2^30 entries (32-bit chunk indexing)

    // pinned host readback
    int64_t *hread = nullptr;
    size_t hread_bytes = 0;

    int64_t sym_start[kGroups + 1] = {};
    int64_t num_start[kGroups + 1] = {};
    std::pmr::vector<HostStats> hstats;
    int64_t ip_total = 0, ip_max = 0, nnz_total = -1;
    std::pmr::vector<int64_t> nnz_c;

    struct Timed { const char *name; hipEvent_t a, b; };
    std::pmr::vector<Timed> timed;

    int state = 0;  // 1 planned, 2 symbolic done
    // device-driven plans (spgemm_plan_create_device): every phase sized
    // from device-side counts, C in a caller's arena; the whole execution
    // optionally captured as one graph
    bool device_driven = false;
    int sym_hi = 0, num_hi = 0;          // last row group that can hold rows
    hipGraphExec_t dev_graph = nullptr;  // captured execution (opt.graph)
    std::pmr::vector<int64_t *> dev_rpt; // the row-pointer arrays it was captured with
    int64_t *dev_off = nullptr;
    int64_t dev_cap = -1;
    // B sorted at plan time (unsorted B with column-chunked rows): the sort's
    // permutation and the sorted values, gathered at every numeric call
    std::pmr::vector<int32_t *> bs_perm;
    std::pmr::vector<float *> bs_val;
    hipGraphExec_t num_graph = nullptr;  // the numeric launches, captured (opt.graph)
    bool num_graph_empty = false;        // captured, with nothing to launch
    std::pmr::vector<void *> allocs;
    size_t ws_bytes = 0;
    // Workspace pooling: the buffers of one planning stage are carved from a
    // single reservation, so a stage costs one allocator call.  `measuring`
    // makes dalloc only add up the sizes (a dry run of the stage).
    bool measuring = false;
    size_t measured = 0;
    char *res = nullptr;
    size_t res_cap = 0, res_used = 0;

    // Allocation-free mode: every workspace buffer is carved from this
    // device arena (the library's static scratch array), host read-backs and
    // descriptor staging use static host buffers, and no event is created.
    bool noalloc = false;
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    int64_t *host_read = nullptr;
    size_t host_read_bytes = 0;
};

namespace {

// With SPGEMM_DEBUG set in the environment, every HIP failure that turns
// into SPGEMM_EHIP is reported on stderr with the call and its error name.
void report_hip(const char *what, hipError_t e, int line) {
    static const bool on = std::getenv("SPGEMM_DEBUG") != nullptr;
    if (on) std::fprintf(stderr, "spgemm: %s -> %s (api.cpp:%d)\n", what, hipGetErrorName(e), line);
}

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e__ = (expr);                          \
        if (e__ != hipSuccess) {                          \
            report_hip(#expr, e__, __LINE__);             \
            return SPGEMM_EHIP;                           \
        }                                                 \
    } while (0)

#define ST_TRY(expr)                                      \
    do {                                                  \
        spgemm_status s__ = (expr);                       \
        if (s__ != SPGEMM_OK) return s__;                 \
    } while (0)

spgemm_status launch_check(int line = __builtin_LINE()) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return SPGEMM_OK;
    report_hip("kernel launch", e, line);
    return SPGEMM_EHIP;
}

// Event pair around a launch group when profiling is on.
struct TimeScope {
    spgemm_plan *p;
    size_t idx = SIZE_MAX;
    TimeScope(spgemm_plan *plan, const char *name) : p(plan) {
        if (!p->opt.profile) return;
        spgemm_plan::Timed t{name, nullptr, nullptr};
        if (pools().event(&t.a, true) != hipSuccess) return;
        if (pools().event(&t.b, true) != hipSuccess) {
            pools().give_event(t.a, true);
            return;
        }
        (void)hipEventRecord(t.a, p->stream);
        idx = p->timed.size();
        p->timed.push_back(t);
    }
    ~TimeScope() {
        if (idx != SIZE_MAX) (void)hipEventRecord(p->timed[idx].b, p->stream);
    }
};

template <typename T>
spgemm_status dalloc(spgemm_plan *p, T **out, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    bytes = (bytes + 255) & ~size_t(255);
    void *ptr = nullptr;
    if (p->measuring) {
        p->measured += bytes;
        *out = nullptr;
        return SPGEMM_OK;
    }
    if (p->noalloc) {
        if (bytes > p->arena_cap - p->arena_used) return SPGEMM_ENOMEM;
        *out = (T *)(p->arena + p->arena_used);
        p->arena_used += bytes;
        p->ws_bytes += bytes;
        return SPGEMM_OK;
    }
    if (p->res && bytes <= p->res_cap - p->res_used) {
        *out = (T *)(p->res + p->res_used);
        p->res_used += bytes;
        return SPGEMM_OK;
    }
    if (p->afn) {
        ptr = p->afn(p->actx, bytes, (void *)p->stream);
        if (!ptr) return SPGEMM_ENOMEM;
    } else {
        if (hipMalloc(&ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return SPGEMM_ENOMEM;
        }
    }
    p->allocs.push_back(ptr);
    p->ws_bytes += bytes;
    *out = (T *)ptr;
    return SPGEMM_OK;
}

spgemm_status ensure_scan_tmp(spgemm_plan *p, int64_t n) {
    size_t need = scan_temp_bytes(n);
    if (need <= p->scan_tmp_bytes) return SPGEMM_OK;
    char *t = nullptr;
    ST_TRY(dalloc(p, &t, need));
    if (p->measuring) return SPGEMM_OK;
    p->scan_tmp = t;
    p->scan_tmp_bytes = need;
    return SPGEMM_OK;
}

// One allocation of `bytes` that the following dallocs are carved from.
spgemm_status reserve(spgemm_plan *p, size_t bytes) {
    p->res = nullptr;
    p->res_cap = p->res_used = 0;
    if (p->noalloc || bytes == 0) return SPGEMM_OK;
    void *ptr = nullptr;
    if (p->afn) {
        ptr = p->afn(p->actx, bytes, (void *)p->stream);
        if (!ptr) return SPGEMM_ENOMEM;
    } else {
        if (hipMalloc(&ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return SPGEMM_ENOMEM;
        }
    }
    p->allocs.push_back(ptr);
    p->ws_bytes += bytes;
    p->res = (char *)ptr;
    p->res_cap = bytes;
    return SPGEMM_OK;
}

// Runs the allocations of a planning stage twice: a dry run adds up their
// sizes, one reservation of that total follows, and the real run carves
// every buffer from it.  `stage` may only allocate.
template <typename F>
spgemm_status alloc_stage(spgemm_plan *p, F &&stage) {
    p->measuring = true;
    p->measured = 0;
    spgemm_status s = stage();
    p->measuring = false;
    if (s != SPGEMM_OK) return s;
    ST_TRY(reserve(p, p->measured));
    s = stage();
    p->res = nullptr;
    p->res_cap = p->res_used = 0;
    return s;
}

spgemm_status scan(spgemm_plan *p, const int64_t *in, int64_t *out, int64_t n) {
    ST_TRY(ensure_scan_tmp(p, n));
    launch_scan_i64(in, out, n, p->scan_tmp, p->stream);
    return launch_check();
}

spgemm_status ensure_hread(spgemm_plan *p, size_t bytes) {
    if (bytes <= p->hread_bytes) return SPGEMM_OK;
    if (p->noalloc) {
        if (bytes > p->host_read_bytes) return SPGEMM_ENOMEM;
        p->hread = p->host_read;
        p->hread_bytes = p->host_read_bytes;
        return SPGEMM_OK;
    }
    // the old buffer holds nothing still in flight: every read into it was
    // waited for
    pools().give_pinned(p->hread, p->hread_bytes);
    p->hread = nullptr;
    p->hread_bytes = 0;
    size_t got = 0;
    void *h = pools().pinned(bytes, &got);
    if (!h) return SPGEMM_EHIP;
    p->hread = (int64_t *)h;
    p->hread_bytes = got;
    return SPGEMM_OK;
}

// Copies the host descriptors to the device through a pinned ring slot.
spgemm_status upload_descriptors(spgemm_plan *p) {
    if (p->noalloc) {
        // one static staging slot: wait until the copy has left it
        std::memcpy(p->pinned, p->hprods.data(), sizeof(ProdDev) * p->nprod);
        HIP_TRY(hipMemcpyAsync(p->dprods, p->pinned, sizeof(ProdDev) * p->nprod,
                               hipMemcpyHostToDevice, p->stream));
        HIP_TRY(hipStreamSynchronize(p->stream));
        return SPGEMM_OK;
    }
    const int slot = p->desc_next;
    p->desc_next = (p->desc_next + 1) % kDescSlots;
    if (p->desc_ev_used[slot]) HIP_TRY(hipEventSynchronize(p->desc_ev[slot]));
    ProdDev *src = p->pinned + (size_t)slot * p->nprod;
    std::memcpy(src, p->hprods.data(), sizeof(ProdDev) * p->nprod);
    HIP_TRY(hipMemcpyAsync(p->dprods, src, sizeof(ProdDev) * p->nprod, hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipEventRecord(p->desc_ev[slot], p->stream));
    p->desc_ev_used[slot] = true;
    return SPGEMM_OK;
}

spgemm_status check_options(const spgemm_options &o) {
    if (o.sym_upper[0] != 0 || o.num_upper[0] != 0) return SPGEMM_EINVAL;
    for (int g = 1; g < kGroups - 1; ++g) {
        if (o.sym_upper[g] < o.sym_upper[g - 1] || o.num_upper[g] < o.num_upper[g - 1])
            return SPGEMM_EINVAL;
        if (o.sym_upper[g] > kSymCap[g] || o.num_upper[g] > kNumCap[g]) return SPGEMM_EINVAL;
    }
    if (o.sym_upper[kGroups - 2] > o.num_upper[kGroups - 2]) return SPGEMM_EINVAL;
    if (o.chunk_cols < 64 || o.chunk_cols > kMaxChunkCols || (o.chunk_cols % 64) != 0)
        return SPGEMM_EINVAL;
    if (o.validate < 0 || o.validate > 2) return SPGEMM_EINVAL;
    if (o.item_limit < 0) return SPGEMM_EINVAL;
    if (o.row_thread < 0 || o.row_thread > 1) return SPGEMM_EINVAL;
    if (o.accumulate < 0 || o.accumulate > 1) return SPGEMM_EINVAL;
    if (o.row_thread && (o.sym_upper[1] > kRtSlots / 2 || o.num_upper[1] > kRtSlots / 2))
        return SPGEMM_EINVAL;
    if (o.profile < 0 || o.profile > 1) return SPGEMM_EINVAL;
    if (o.chunks_per_item != 1 && o.chunks_per_item != 2 && o.chunks_per_item != 4 &&
        o.chunks_per_item != 8)
        return SPGEMM_EINVAL;
    if (o.chunk_wgs_per_cu < 0 || o.chunk_wgs_per_cu > 64) return SPGEMM_EINVAL;
    for (int t : {o.chunk_threads, o.sym_chunk_threads})
        if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512) return SPGEMM_EINVAL;
    if (o.num_rank_cap != 0 && o.num_rank_cap != 512 && o.num_rank_cap != 1024 &&
        o.num_rank_cap != 2048)
        return SPGEMM_EINVAL;
    if (o.chunk_merge != 0 && o.chunk_merge != 1 && o.chunk_merge != 2 && o.chunk_merge != 4 &&
        o.chunk_merge != 8)
        return SPGEMM_EINVAL;
    if (o.graph < 0 || o.graph > 1) return SPGEMM_EINVAL;
    return SPGEMM_OK;
}

// FP64 accumulation (accumulate = 1) takes every column chunk through the
// rank kernel's FP64 form: chunks of at most 2048 columns, a rank cap of
// 2048 (so no chunk is dense), no merging, one chunk per item.
void apply_accumulate(spgemm_options &o) {
    if (o.accumulate != 1) return;
    if (o.chunk_cols > 2048) o.chunk_cols = 2048;
    o.num_rank_cap = 2048;
    o.chunk_merge = 1;
    o.chunks_per_item = 1;
}

spgemm_status check_csr(const spgemm_csr &m, bool need_values) {
    if (m.nrows < 0 || m.ncols < 0 || m.nnz < 0) return SPGEMM_EINVAL;
    if (m.nrows >= (int64_t(1) << 31) || m.ncols >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    if (!m.row_ptr) return SPGEMM_EINVAL;
    if (m.nnz > 0 && !m.col_idx) return SPGEMM_EINVAL;
    if (need_values && m.nnz > 0 && !m.values) return SPGEMM_EINVAL;
    return SPGEMM_OK;
}

int64_t item_limit(const spgemm_options &o) {
    const int64_t cap = (int64_t(1) << 31) - 1;
    return (o.item_limit > 0 && o.item_limit < cap) ? o.item_limit : cap;
}

// copy_group: the block group whose kernels copy single-nonzero rows (0:
// none, for device-driven plans that do not launch it)
GroupBounds bounds_of(const int64_t *up, int copy_group = 5) {
    GroupBounds gb{};
    for (int g = 0; g < kGroups - 1; ++g) gb.up[g] = up[g];
    gb.up[kGroups - 1] = INT64_MAX;
    gb.copy_group = copy_group;
    return gb;
}

spgemm_status read_flags(spgemm_plan *p, int *out, int n) {
    ST_TRY(ensure_hread(p, sizeof(int) * n + 64));
    HIP_TRY(hipMemcpyAsync(p->hread, p->flags, sizeof(int) * n, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    std::memcpy(out, p->hread, sizeof(int) * n);
    return SPGEMM_OK;
}

// Sorts the rows of every B that is stored out of column order and meets
// column-chunked rows (fewer than 2^30 entries): the sorted columns replace
// B's in the descriptor, and the permutation gathers B's values at every
// numeric call.
spgemm_status sort_b_rows(spgemm_plan *p, const ProdStats *ps) {
    size_t tmp_bytes = 0;
    bool any = false;
    for (int q = 0; q < p->nprod; ++q) {
        const spgemm_csr &b = p->B[q];
        if (ps[q].h_rows == 0 || p->hprods[q].b_sorted != 0 || b.nnz <= 0 ||
            b.nnz >= (int64_t(1) << 30))
            continue;
        const size_t t = bsort_temp_bytes(b.nnz, b.nrows, b.ncols);
        if (t == 0) return SPGEMM_EHIP;
        tmp_bytes = std::max(tmp_bytes, t);
        any = true;
    }
    if (!any) return SPGEMM_OK;
    std::pmr::vector<int32_t *> cols(p->nprod, nullptr, p->hblks.get_allocator());
    uint8_t *tmp = nullptr;
    ST_TRY(alloc_stage(p, [&]() -> spgemm_status {
        for (int q = 0; q < p->nprod; ++q) {
            const spgemm_csr &b = p->B[q];
            if (ps[q].h_rows == 0 || p->hprods[q].b_sorted != 0 || b.nnz <= 0 ||
                b.nnz >= (int64_t(1) << 30))
                continue;
            ST_TRY(dalloc(p, &cols[q], (size_t)b.nnz));
            ST_TRY(dalloc(p, &p->bs_perm[q], (size_t)b.nnz));
            ST_TRY(dalloc(p, &p->bs_val[q], (size_t)b.nnz));
        }
        return dalloc(p, &tmp, tmp_bytes);
    }));
    TimeScope ts(p, "plan.bsort");
    for (int q = 0; q < p->nprod; ++q) {
        if (!cols[q]) continue;
        ProdDev &P = p->hprods[q];
        const spgemm_csr &b = p->B[q];
        HIP_TRY(launch_bsort(b.row_ptr, b.nrows, b.ncols, b.col_idx, b.nnz, cols[q],
                             p->bs_perm[q], tmp, tmp_bytes, p->stream));
        P.colB = cols[q];
        P.b_sorted = 1;
    }
    return upload_descriptors(p);
}

// Host side of plan creation: descriptors, row blocks, the per-row
// workspace, the pinned staging; the descriptors and row blocks are
// uploaded.  No kernel runs yet.
spgemm_status plan_setup(spgemm_plan *p, int nprod, const spgemm_csr *A, const spgemm_csr *B) {
    p->nprod = nprod;
    p->A.assign(A, A + nprod);
    p->B.assign(B, B + nprod);
    p->hprods.resize(nprod);
    p->hstats.resize(nprod);
    p->nnz_c.assign(nprod, -1);
    p->bs_perm.assign(nprod, nullptr);
    p->bs_val.assign(nprod, nullptr);
    int64_t row_base = 0;
    {
        size_t nb = 0;
        for (int q = 0; q < nprod; ++q)
            if (A[q].nrows > 0) nb += (size_t)((A[q].nrows + kRowBlock - 1) / kRowBlock);
        p->hblks.reserve(nb);
    }
    for (int q = 0; q < nprod; ++q) {
        const spgemm_csr &a = A[q], &b = B[q];
        ST_TRY(check_csr(a, false));
        ST_TRY(check_csr(b, false));
        if (a.ncols != b.nrows) return SPGEMM_EDIM;
        ProdDev &P = p->hprods[q];
        std::memset(&P, 0, sizeof(P));
        P.rptA = a.row_ptr;
        P.colA = a.col_idx;
        P.valA = a.values;
        P.rptB = b.row_ptr;
        P.colB = b.col_idx;
        P.valB = b.values;
        P.m = a.nrows;
        P.k = a.ncols;
        P.n = b.ncols;
        P.row_base = row_base;
        const int64_t wmax = p->opt.chunk_cols;
        int64_t qn = (P.n + 8 * wmax - 1) / (8 * wmax);
        if (qn < 1) qn = 1;
        P.nch = (int32_t)(8 * qn);
        int64_t w = (P.n + P.nch - 1) / P.nch;
        w = (w + 63) / 64 * 64;
        if (w < 64) w = 64;
        P.W = (int32_t)w;
        p->wmax = std::max<int>(p->wmax, P.W);
        P.b_sorted = (b.flags & SPGEMM_ROWS_SORTED) ? 1 : 2;
        P.b_unique = (b.flags & SPGEMM_ROWS_SORTED) ? 1 : 0;
        // a B of few columns is also kept as row bitmaps, from which the
        // symbolic phase of direct-mapped rows takes its counts
        if (b.ncols > 0 && b.ncols <= kBitmapCols && b.nnz > 0 && b.nrows > 0)
            P.bmw = (int32_t)((b.ncols + 31) / 32);
        for (int64_t i0 = 0; i0 < a.nrows; i0 += kRowBlock) {
            RowBlk rb;
            rb.p = q;
            rb.nrows = (int32_t)std::min<int64_t>(kRowBlock, a.nrows - i0);
            rb.i0 = i0;
            p->hblks.push_back(rb);
        }
        row_base += a.nrows;
    }
    p->Mtot = row_base;
    p->nblk = (int)p->hblks.size();
    if ((int64_t)p->hblks.size() >= (int64_t(1) << 31)) return SPGEMM_EOVERFLOW;

    const int64_t M = p->Mtot;
    ST_TRY(alloc_stage(p, [&]() -> spgemm_status {
        ST_TRY(dalloc(p, &p->dprods, nprod));
        ST_TRY(dalloc(p, &p->dblks, p->hblks.size()));
        ST_TRY(dalloc(p, &p->ip, M));
        ST_TRY(dalloc(p, &p->row_nnz, M));
        ST_TRY(dalloc(p, &p->rptv, M + 1));
        ST_TRY(dalloc(p, &p->map_sym, M));
        ST_TRY(dalloc(p, &p->map_num, M));
        ST_TRY(dalloc(p, &p->hslot, M));
        ST_TRY(dalloc(p, &p->blkcnt, (size_t)kGroups * p->nblk));
        ST_TRY(dalloc(p, &p->blkoff, (size_t)kGroups * p->nblk + 1));
        // group starts (symbolic, numeric), then the device-sized launches'
        // work counters (symbolic, numeric)
        ST_TRY(dalloc(p, &p->starts, 4 * (kGroups + 1)));
        ST_TRY(dalloc(p, &p->stats, nprod));
        ST_TRY(dalloc(p, &p->flags, 3 + nprod));
        for (int q = 0; q < nprod; ++q) {
            ProdDev &P = p->hprods[q];
            if (P.bmw == 0) continue;
            uint32_t *bm = nullptr;
            ST_TRY(dalloc(p, &bm, (size_t)B[q].nrows * P.bmw));
            P.bmB = bm;
        }
        return ensure_scan_tmp(p, std::max<int64_t>(M, (int64_t)kGroups * p->nblk));
    }));
    if (!p->noalloc) {
        size_t got = 0;
        void *h = pools().pinned(sizeof(ProdDev) * nprod * kDescSlots, &got);
        if (!h) return SPGEMM_EHIP;
        p->pinned = (ProdDev *)h;
        p->pinned_bytes = got;
        for (int s = 0; s < kDescSlots; ++s) HIP_TRY(pools().event(&p->desc_ev[s], false));
    }
    // cleared by fill kernels, not memsets, so that a caller may capture the
    // plan's work in a graph (device allocations are padded to 256 bytes, so
    // the flags' last 8-byte word is in bounds)
    launch_fill_i64((int64_t *)p->stats, (int64_t)(sizeof(ProdStats) / 8) * nprod, 0, p->stream);
    launch_fill_i64((int64_t *)p->flags, (3 + nprod + 1) / 2, 0, p->stream);
    ST_TRY(upload_descriptors(p));
    if (!p->hblks.empty())
        HIP_TRY(hipMemcpyAsync(p->dblks, p->hblks.data(), sizeof(RowBlk) * p->hblks.size(),
                               hipMemcpyHostToDevice, p->stream));
    // B's row bitmaps: one launch for the batch (its workgroup rows are the
    // products), as wide as the mean product needs
    {
        int64_t rows = 0;
        int nbm = 0;
        for (int q = 0; q < nprod; ++q)
            if (p->hprods[q].bmw > 0) {
                rows += B[q].nrows;
                ++nbm;
            }
        if (nbm > 0) {
            const int64_t blocks = std::max<int64_t>(1, (rows / nbm + 15) / 16);
            if (nprod <= 65535) {
                launch_brow_bitmap_batch(p->dprods, nprod, blocks, p->stream);
            } else {
                for (int q = 0; q < nprod; ++q) {
                    const ProdDev &P = p->hprods[q];
                    if (P.bmw > 0)
                        launch_brow_bitmap(B[q].row_ptr, B[q].col_idx, B[q].nrows, B[q].ncols,
                                           P.bmw, const_cast<uint32_t *>(P.bmB), p->stream);
                }
            }
        }
    }

    return SPGEMM_OK;
}

spgemm_status plan_create_impl(spgemm_plan *p, int nprod, const spgemm_csr *A,
                               const spgemm_csr *B) {
    ST_TRY(plan_setup(p, nprod, A, B));
    const int64_t M = p->Mtot;
    if (p->opt.validate) {
        int f[3];
        for (int q = 0; q < nprod; ++q) {
            CsrCheck ca{A[q].row_ptr, A[q].col_idx, A[q].nrows, A[q].nnz, A[q].ncols};
            CsrCheck cb{B[q].row_ptr, B[q].col_idx, B[q].nrows, B[q].nnz, B[q].ncols};
            launch_validate_rows(ca, p->flags + 1, p->stream);
            launch_validate_rows(cb, p->flags + 2, p->stream);
        }
        ST_TRY(launch_check());
        ST_TRY(read_flags(p, f, 3));
        if (f[1] || f[2]) return SPGEMM_EINDEX;
    }
    if (p->opt.validate >= 2) {
        int f[3];
        for (int q = 0; q < nprod; ++q) {
            CsrCheck ca{A[q].row_ptr, A[q].col_idx, A[q].nrows, A[q].nnz, A[q].ncols};
            CsrCheck cb{B[q].row_ptr, B[q].col_idx, B[q].nrows, B[q].nnz, B[q].ncols};
            launch_validate_cols(ca, p->flags + 1, p->stream);
            launch_validate_cols(cb, p->flags + 2, p->stream);
        }
        ST_TRY(launch_check());
        ST_TRY(read_flags(p, f, 3));
        if (f[1] || f[2]) return SPGEMM_EINDEX;
    }

    launch_detect_sorted(p->dprods, nprod, p->hprods.data(), p->flags + 3, p->stream);
    const GroupBounds gb = bounds_of(p->opt.sym_upper);
    {
        TimeScope ts(p, "plan.ipcount");
        launch_ipcount(p->dprods, p->dblks, p->nblk, gb, p->ip, p->blkcnt, p->stats, M,
                       p->stream);
    }
    ST_TRY(launch_check());
    {
        TimeScope ts(p, "plan.group");
        ST_TRY(scan(p, p->blkcnt, p->blkoff, (int64_t)kGroups * p->nblk));
        launch_scatter(p->dprods, p->dblks, p->nblk, gb, p->ip, p->blkoff, p->map_sym, p->hslot,
                       nullptr, p->stream);
        launch_group_starts(p->blkoff, p->nblk, p->starts, p->stream);
    }
    ST_TRY(launch_check());

    // one synchronisation: group sizes and per-product figures
    const size_t sbytes = sizeof(int64_t) * (kGroups + 1);
    const size_t pbytes = sizeof(ProdStats) * nprod;
    ST_TRY(ensure_hread(p, sbytes + pbytes + sizeof(int) * (3 + nprod)));
    char *hb = (char *)p->hread;
    HIP_TRY(hipMemcpyAsync(hb, p->starts, sbytes, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipMemcpyAsync(hb + sbytes, p->stats, pbytes, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipMemcpyAsync(hb + sbytes + pbytes, p->flags + 3, sizeof(int) * nprod,
                           hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    std::memcpy(p->sym_start, hb, sbytes);
    const ProdStats *ps = (const ProdStats *)(hb + sbytes);
    const int *unsorted = (const int *)(hb + sbytes + pbytes);
    p->ip_total = 0;
    p->ip_max = 0;
    for (int q = 0; q < nprod; ++q) {
        p->hstats[q].ip_sum = (int64_t)ps[q].ip_sum;
        p->hstats[q].ip_max = (int64_t)ps[q].ip_max;
        p->ip_total += (int64_t)ps[q].ip_sum;
        p->ip_max = std::max<int64_t>(p->ip_max, (int64_t)ps[q].ip_max);
        p->nh += (int64_t)ps[q].h_rows;
        p->h_split += (int64_t)ps[q].h_split;
        p->h_items += (int64_t)ps[q].h_items;
        p->h_tiles += (int64_t)ps[q].h_tiles;
        if (p->hprods[q].b_sorted == 2) {
            p->hprods[q].b_sorted = unsorted[q] ? 0 : 1;
            p->hprods[q].b_unique = unsorted[q] ? 0 : 1;
        }
    }
    // B stored out of order, with column-chunked rows: sort its rows once
    // (the chunk kernels then take each chunk's part of a B row directly)
    ST_TRY(sort_b_rows(p, ps));
    for (int q = 0; q < nprod; ++q)
        if (p->hprods[q].b_sorted != 1 || p->B[q].nnz >= (int64_t(1) << 30)) p->fast = false;
    // FP64 accumulation runs on the rank kernel, which needs the fast path
    if (p->opt.accumulate == 1 && p->nh > 0 && !p->fast) return SPGEMM_EINVAL;
    if (p->nh != p->sym_start[kGroups] - p->sym_start[kGroups - 1]) return SPGEMM_EINTERNAL;
    if (p->h_items > item_limit(p->opt)) return SPGEMM_EOVERFLOW;

    // chunk-group preparation: chunk bases, item -> row map, chunk bounds of
    // every B row, item descriptors
    // merging of adjacent light chunks: fast path with one chunk per item and
    // the rank accumulator only (a merged item never exceeds the rank cap)
    p->merge = 1;
    if (num_chunk_rank_used(p->fast, p->opt.chunks_per_item, p->opt.num_rank_cap)) {
        p->merge = p->opt.chunk_merge ? p->opt.chunk_merge : 2;
        while (p->merge > 1 && (int64_t)p->wmax * p->merge > kMaxItemCols) p->merge >>= 1;
    }
    p->wmax_item = p->wmax * p->merge;
    p->s_items = p->h_items / p->opt.chunks_per_item;
    if (p->nh > 0) {
        const int64_t nh = p->nh;
        const uint64_t *hitems = p->map_sym + p->sym_start[kGroups - 1];
        const int64_t nitems = p->h_items / p->opt.chunks_per_item;  // upper bound when merging
        p->wpc = (p->wmax + 31) / 32;
        // every buffer of the chunk preparation, in one reservation
        int64_t *ntile = nullptr, *tbase = nullptr;
        int32_t *tile_row = nullptr;
        unsigned long long *ipc = nullptr;
        std::pmr::vector<int32_t *> bsv(nprod, nullptr, p->hblks.get_allocator());
        ST_TRY(alloc_stage(p, [&]() -> spgemm_status {
            ST_TRY(dalloc(p, &p->nchv, nh));
            ST_TRY(dalloc(p, &p->ibase, nh + 1));
            ST_TRY(dalloc(p, &p->cbase, nh + 1));
            ST_TRY(dalloc(p, &p->chunk_cnt, p->h_items));
            ST_TRY(dalloc(p, &p->chunk_pos, p->h_items + 1));
            ST_TRY(dalloc(p, &p->hitem_row, nitems));
            ST_TRY(dalloc(p, &p->sdesc, nitems));
            ST_TRY(dalloc(p, &p->sbits, (size_t)p->h_items * p->wpc));
            for (int q = 0; q < nprod; ++q) {
                const ProdDev &P = p->hprods[q];
                if (ps[q].h_rows == 0 || P.b_sorted != 1) continue;
                ST_TRY(dalloc(p, &bsv[q], (size_t)P.k * (P.nch + 1)));
            }
            if (p->merge > 1) ST_TRY(dalloc(p, &p->mstart, p->h_items));
            if (p->fast) {
                ST_TRY(dalloc(p, &p->slen, nh));
                ST_TRY(dalloc(p, &p->sbase, nh + 1));
                ST_TRY(dalloc(p, &p->sabs, p->h_split));
                ST_TRY(dalloc(p, &ntile, nh));
                ST_TRY(dalloc(p, &tbase, nh + 1));
                ST_TRY(dalloc(p, &tile_row, p->h_tiles));
                if (p->merge > 1) ST_TRY(dalloc(p, &ipc, p->h_items));
            }
            return ensure_scan_tmp(p, std::max(nh, p->h_items));
        }));
        TimeScope ts(p, "plan.split");
        bool reupload = false;
        for (int q = 0; q < nprod; ++q) {
            ProdDev &P = p->hprods[q];
            if (!bsv[q]) continue;
            launch_bsplit(P.rptB, P.colB, P.k, P.W, P.nch, bsv[q], p->stream);
            P.bsplit = bsv[q];
            reupload = true;
        }
        if (reupload) ST_TRY(upload_descriptors(p));
        launch_nch_of(p->dprods, hitems, nh, 1, p->nchv, p->stream);
        ST_TRY(launch_check());
        ST_TRY(scan(p, p->nchv, p->cbase, nh));
        if (p->fast) {
            launch_row_splitlen(p->dprods, hitems, nh, p->slen, p->stream);
            ST_TRY(launch_check());
            ST_TRY(scan(p, p->slen, p->sbase, nh));
            // one workgroup per tile of A nonzeros of every row
            launch_sabs_tiles(p->dprods, hitems, nh, ntile, p->stream);
            ST_TRY(launch_check());
            ST_TRY(scan(p, ntile, tbase, nh));
            launch_expand(tbase, nh, tile_row, p->stream);
            if (p->merge > 1) launch_fill_i64((int64_t *)ipc, p->h_items, 0, p->stream);
            launch_sabs(p->dprods, hitems, p->h_tiles, tile_row, tbase, p->sbase, p->sabs,
                        p->cbase, ipc, p->stream);
            ST_TRY(launch_check());
            if (p->merge > 1) {  // the items of every row (nchv = items per row)
                launch_chunk_items(p->dprods, hitems, nh, p->merge, p->opt.num_rank_cap,
                                   p->cbase, ipc, p->mstart, p->nchv, p->stream);
                ST_TRY(launch_check());
            }
        }
        if (p->merge == 1) {
            launch_nch_of(p->dprods, hitems, nh, p->opt.chunks_per_item, p->nchv, p->stream);
            ST_TRY(launch_check());
        }
        ST_TRY(scan(p, p->nchv, p->ibase, nh));
        launch_expand(p->ibase, nh, p->hitem_row, p->stream);
        launch_sym_desc(p->dprods, hitems, p->hitem_row, p->ibase, p->cbase, p->sbase, nitems,
                        p->opt.chunks_per_item, p->mstart,
                        p->merge > 1 ? p->ibase + nh : nullptr, p->sdesc, p->stream);
        ST_TRY(launch_check());
        if (p->merge > 1) {  // the item count is data-dependent: read it back
            HIP_TRY(hipMemcpyAsync(p->hread, p->ibase + nh, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, p->stream));
            HIP_TRY(hipStreamSynchronize(p->stream));
            p->s_items = p->hread[0];
            if (p->s_items < 0 || p->s_items > nitems) return SPGEMM_EINTERNAL;
        }
    }
    p->state = 1;
    return SPGEMM_OK;
}

// ---------------------------------------------------------------------------
// Device-driven plans: no host synchronisation anywhere.  Every launch of a
// row group covers an upper bound of its rows (all rows of the batch) and
// takes the group's range of the row map from the device; C is written into
// one arena at the batch-wide row pointers.  Restricted to products whose B
// has no more columns than the block groups take, so that no row is column
// chunked (that path sizes its work items on the host).
// ---------------------------------------------------------------------------
int last_group(const int64_t *upper, int64_t max_ncols) {
    // keys never exceed B's columns; B of at most 512 columns keeps its rows
    // in the 64-lane group (direct-mapped tables)
    int hi = 0;
    for (int g = 1; g <= 6; ++g)
        if (upper[g - 1] < max_ncols) hi = g;
    if (max_ncols <= kDirectG4 && hi > 4) hi = 4;
    return hi;
}

// The most columns of any product's B in the plan (the group kernels hold no
// key table when every B fits their direct-mapped table).
int64_t max_b_cols(const spgemm_plan *p) {
    int64_t m = 0;
    for (int q = 0; q < p->nprod; ++q) m = std::max(m, p->hprods[q].n);
    return m;
}

spgemm_status device_plan_setup(spgemm_plan *p, int nprod, const spgemm_csr *A,
                                const spgemm_csr *B) {
    if (p->opt.validate || p->opt.row_thread) return SPGEMM_EINVAL;
    int64_t max_ncols = 0;
    for (int q = 0; q < nprod; ++q) max_ncols = std::max(max_ncols, B[q].ncols);
    if (max_ncols > p->opt.sym_upper[kGroups - 2] || max_ncols > p->opt.num_upper[kGroups - 2])
        return SPGEMM_EINVAL;  // rows could need the column-chunked path
    int64_t rows = 0;
    for (int q = 0; q < nprod; ++q) rows += A[q].nrows;
    // the group launches cover every row of the batch: 64 threads per row
    // in the widest group, within a grid's 2^32 work-items
    if (rows > kMaxDeviceRows) return SPGEMM_EOVERFLOW;
    ST_TRY(plan_setup(p, nprod, A, B));
    p->sym_hi = last_group(p->opt.sym_upper, max_ncols);
    p->num_hi = last_group(p->opt.num_upper, max_ncols);
    p->device_driven = true;
    p->dev_rpt.assign(nprod, nullptr);
    p->state = 1;
    return SPGEMM_OK;
}

// Every kernel of a device-driven execution, in order, on `st`.
spgemm_status device_launch_all(spgemm_plan *p, hipStream_t st, int64_t *const *c_row_ptr,
                                int64_t *c_offsets, int64_t capacity) {
    const int64_t M = p->Mtot;
    const int nprod = p->nprod;
    // the flag and statistics words start at zero (fill kernels, no memset)
    launch_fill_i64((int64_t *)p->stats, (int64_t)(sizeof(ProdStats) / 8) * nprod, 0, st);
    launch_fill_i64((int64_t *)p->flags, (3 + nprod + 1) / 2, 0, st);
    launch_fill_i64(p->starts + kWorkCtr, 2 * (kGroups + 1), 0, st);
    // Algorithm 1 and the symbolic grouping
    const GroupBounds gs = bounds_of(p->opt.sym_upper, p->sym_hi >= 5 ? 5 : 0);
    launch_ipcount(p->dprods, p->dblks, p->nblk, gs, p->ip, p->blkcnt, p->stats, M, st);
    launch_scan_i64(p->blkcnt, p->blkoff, (int64_t)kGroups * p->nblk, p->scan_tmp, st);
    launch_scatter(p->dprods, p->dblks, p->nblk, gs, p->ip, p->blkoff, p->map_sym, p->hslot,
                   nullptr, st);
    launch_group_starts(p->blkoff, p->nblk, p->starts, st);
    // allocation phase and row pointers
    launch_fill_i64(p->row_nnz, M, 0, st);
    for (int g = 1; g <= std::min(p->sym_hi, 4); ++g)
        launch_sym_group(g, p->dprods, p->map_sym, M, p->row_nnz, p->flags, st, p->starts, g);
    for (int g = 5; g <= p->sym_hi; ++g)
        launch_sym_block(g, p->opt.sym_upper[g], p->dprods, p->map_sym, p->ip, M, p->row_nnz,
                         p->flags, st, p->starts, g);
    launch_scan_i64(p->row_nnz, p->rptv, M, p->scan_tmp, st);
    // numeric grouping by output length
    const GroupBounds gn = bounds_of(p->opt.num_upper, p->num_hi >= 5 ? 5 : 0);
    launch_count_groups(p->dprods, p->dblks, p->nblk, gn, p->row_nnz, p->ip, p->blkcnt, p->stats,
                        st);
    launch_scan_i64(p->blkcnt, p->blkoff, (int64_t)kGroups * p->nblk, p->scan_tmp, st);
    launch_scatter(p->dprods, p->dblks, p->nblk, gn, p->row_nnz, p->blkoff, p->map_num, nullptr,
                   p->ip, st);
    launch_group_starts(p->blkoff, p->nblk, p->starts + (kGroups + 1), st);
    // the arena: capacity check (kErrCapacity stops the numeric kernels),
    // each product's offset and its own row pointers
    launch_arena_check(p->rptv, M, capacity, p->flags, p->dprods, nprod, c_offsets, st);
    // every product's own row pointers (the descriptors carry c_row_ptr),
    // one launch for the batch
    if (nprod <= 65535) {
        launch_rows_local_batch(p->dprods, nprod, std::max<int64_t>(1, (M / nprod + 256) / 256),
                                p->rptv, st);
    } else {
        for (int q = 0; q < nprod; ++q)
            launch_rows_local(p->rptv, p->hprods[q].row_base, p->hprods[q].m, c_row_ptr[q], st);
    }
    // accumulation phase
    const int64_t *ns = p->starts + (kGroups + 1);
    for (int g = 1; g <= std::min(p->num_hi, 4); ++g)
        launch_num_group(g, p->dprods, p->map_num, M, p->rptv, p->flags, st, ns, g,
                         max_b_cols(p));
    for (int g = 5; g <= p->num_hi; ++g)
        launch_num_block(g, p->opt.num_upper[g], p->dprods, p->map_num, M, p->rptv, p->flags, st,
                         ns, g);
    return launch_check();
}

spgemm_status capture_device(spgemm_plan *p, int64_t *const *c_row_ptr, int64_t *c_offsets,
                             int64_t capacity) {
    if (p->dev_graph) (void)hipGraphExecDestroy(p->dev_graph);
    p->dev_graph = nullptr;
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    spgemm_status s = SPGEMM_OK;
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
        s = device_launch_all(p, cs, c_row_ptr, c_offsets, capacity);
        e = hipStreamEndCapture(cs, &g);  // always ends the capture
    }
    if (s == SPGEMM_OK && e == hipSuccess) e = hipGraphInstantiate(&p->dev_graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (s != SPGEMM_OK) return s;
    if (e != hipSuccess) {
        report_hip("device plan capture", e, __LINE__);
        p->dev_graph = nullptr;
        (void)hipGetLastError();
        return SPGEMM_EHIP;
    }
    for (int q = 0; q < p->nprod; ++q) p->dev_rpt[q] = c_row_ptr[q];
    p->dev_off = c_offsets;
    p->dev_cap = capacity;
    return SPGEMM_OK;
}

spgemm_status create_common(spgemm_plan **out, int32_t nprod, const spgemm_csr *A,
                            const spgemm_csr *B, const spgemm_options *opt, void *stream,
                            spgemm_alloc_fn afn, spgemm_free_fn ffn, void *actx, bool batch) {
    if (!out) return SPGEMM_EINVAL;
    *out = nullptr;
    if (nprod <= 0 || !A || !B) return SPGEMM_EINVAL;
    if ((afn == nullptr) != (ffn == nullptr)) return SPGEMM_EINVAL;
    spgemm_options o;
    if (opt) o = *opt; else spgemm_default_options(&o);
    ST_TRY(check_options(o));
    apply_accumulate(o);
    spgemm_plan *p = new (std::nothrow) spgemm_plan();
    if (!p) return SPGEMM_ENOMEM;
    p->stream = (hipStream_t)stream;
    p->afn = afn;
    p->ffn = ffn;
    p->actx = actx;
    p->opt = o;
    p->batch = batch;
    spgemm_status s;
    try {
        s = plan_create_impl(p, nprod, A, B);
    } catch (...) {
        s = SPGEMM_ENOMEM;
    }
    if (s != SPGEMM_OK) {
        spgemm_free(p);
        return s;
    }
    *out = p;
    return SPGEMM_OK;
}

// Workspace of the thread-per-row group: offsets for the rows of group 1 in
// either phase and one stream with room for every A nonzero of the plan.
spgemm_status rt_prepare(spgemm_plan *p) {
    if (p->rt_stream) return SPGEMM_OK;
    int64_t nnz_a = 0;
    for (int q = 0; q < p->nprod; ++q) nnz_a += p->A[q].nnz;
    const int64_t rows = std::max(p->sym_start[2] - p->sym_start[1], int64_t(1));
    return alloc_stage(p, [&]() -> spgemm_status {
        ST_TRY(dalloc(p, &p->rt_lens, p->Mtot + 1));
        ST_TRY(dalloc(p, &p->rt_off_sym, rows + 1));
        ST_TRY(dalloc(p, &p->rt_off_num, p->Mtot + 1));
        ST_TRY(dalloc(p, &p->rt_stream, std::max<int64_t>(nnz_a, 1)));
        return ensure_scan_tmp(p, p->Mtot);
    });
}

spgemm_status symbolic_impl(spgemm_plan *p) {
    if (p->state != 1) return SPGEMM_ESTATE;
    const int64_t M = p->Mtot;
    hipStream_t st = p->stream;
    static const char *const sym_names[kGroups] = {"sym.g0", "sym.g1", "sym.g2", "sym.g3",
                                                   "sym.g4", "sym.g5", "sym.g6", "sym.g7"};
    launch_fill_i64(p->row_nnz, M, 0, st);
    if (p->opt.row_thread) ST_TRY(rt_prepare(p));
    for (int g = 1; g <= 4; ++g) {
        if (p->sym_start[g + 1] == p->sym_start[g]) continue;
        TimeScope ts(p, sym_names[g]);
        if (g == 1 && p->opt.row_thread) {
            const int64_t cnt = p->sym_start[2] - p->sym_start[1];
            const uint64_t *items = p->map_sym + p->sym_start[1];
            ST_TRY(ensure_scan_tmp(p, cnt));
            launch_rt_offsets(p->dprods, items, cnt, p->rt_lens, p->rt_off_sym, p->scan_tmp, st);
            launch_rt_gather(p->dprods, items, cnt, p->rt_off_sym, p->rt_stream, false, st);
            launch_sym_rowthread(p->dprods, items, cnt, p->rt_off_sym, p->rt_stream,
                                 p->row_nnz, p->flags, st);
            continue;
        }
        launch_sym_group(g, p->dprods, p->map_sym + p->sym_start[g],
                         p->sym_start[g + 1] - p->sym_start[g], p->row_nnz, p->flags, st);
    }
    for (int g = 5; g <= 6; ++g) {
        if (p->sym_start[g + 1] == p->sym_start[g]) continue;
        TimeScope ts(p, sym_names[g]);
        launch_sym_block(g, p->opt.sym_upper[g], p->dprods, p->map_sym + p->sym_start[g], p->ip,
                         p->sym_start[g + 1] - p->sym_start[g], p->row_nnz, p->flags, st);
    }
    if (p->nh > 0) {
        TimeScope ts(p, sym_names[7]);
        launch_sym_chunk(p->wmax_item, p->fast, p->dprods, p->sdesc, p->sabs, p->s_items,
                         p->opt.chunks_per_item, p->chunk_cnt, p->row_nnz, p->sbits, p->wpc,
                         p->opt.chunk_wgs_per_cu,
                         p->opt.sym_chunk_threads ? p->opt.sym_chunk_threads : 64, p->flags, st);
    }
    ST_TRY(launch_check());
    {
        TimeScope ts(p, "sym.scan");
        ST_TRY(scan(p, p->row_nnz, p->rptv, M));
        if (p->nh > 0) ST_TRY(scan(p, p->chunk_cnt, p->chunk_pos, p->h_items));
    }

    // numeric grouping by output length (paper Section III-C)
    const GroupBounds gb = bounds_of(p->opt.num_upper);
    {
        TimeScope ts(p, "sym.regroup");
        launch_count_groups(p->dprods, p->dblks, p->nblk, gb, p->row_nnz, p->ip, p->blkcnt, p->stats,
                            st);
        ST_TRY(launch_check());
        ST_TRY(scan(p, p->blkcnt, p->blkoff, (int64_t)kGroups * p->nblk));
        launch_scatter(p->dprods, p->dblks, p->nblk, gb, p->row_nnz, p->blkoff, p->map_num,
                       nullptr, p->ip, st);
        launch_group_starts(p->blkoff, p->nblk, p->starts + (kGroups + 1), st);
    }
    ST_TRY(launch_check());

    const size_t sbytes = sizeof(int64_t) * (kGroups + 1);
    const size_t pbytes = sizeof(ProdStats) * p->nprod;
    ST_TRY(ensure_hread(p, sbytes + pbytes + 64));
    char *hb = (char *)p->hread;
    HIP_TRY(hipMemcpyAsync(hb, p->starts + (kGroups + 1), sbytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hb + sbytes, p->stats, pbytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hb + sbytes + pbytes, p->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(p->num_start, hb, sbytes);
    const ProdStats *ps = (const ProdStats *)(hb + sbytes);
    const int err = *(const int *)(hb + sbytes + pbytes);
    if (err) return SPGEMM_EINTERNAL;
    p->nnz_total = 0;
    p->nd = 0;
    p->d_items = 0;
    for (int q = 0; q < p->nprod; ++q) {
        p->hstats[q].nnz_sum = (int64_t)ps[q].nnz_sum;
        p->hstats[q].nnz_max = (int64_t)ps[q].nnz_max;
        p->nnz_c[q] = (int64_t)ps[q].nnz_sum;
        p->nnz_total += (int64_t)ps[q].nnz_sum;
        p->nd += (int64_t)ps[q].d_rows;
        p->d_items += (int64_t)ps[q].d_items;
    }
    if (p->nd != p->num_start[kGroups] - p->num_start[kGroups - 1]) return SPGEMM_EINTERNAL;
    if (p->d_items > item_limit(p->opt)) return SPGEMM_EOVERFLOW;
    p->n_items = p->d_items / p->opt.chunks_per_item;
    p->n_s1 = p->n_s0 = p->n_m1 = p->n_m0 = 0;
    if (p->nd > 0) {
        const uint64_t *ditems = p->map_num + p->num_start[kGroups - 1];
        // with merging an upper bound; the exact count is dbase[nd]
        const int64_t nitems = p->d_items / p->opt.chunks_per_item;
        const bool split_lists = num_chunk_rank_used(p->fast, p->opt.chunks_per_item,
                                                     p->opt.num_rank_cap);
        ST_TRY(alloc_stage(p, [&]() -> spgemm_status {
            ST_TRY(dalloc(p, &p->dnchv, p->nd));
            ST_TRY(dalloc(p, &p->dbase, p->nd + 1));
            ST_TRY(dalloc(p, &p->ditem_row, nitems));
            ST_TRY(dalloc(p, &p->ndesc, nitems));
            if (split_lists) {
                ST_TRY(dalloc(p, &p->ndesc_split, nitems));
                ST_TRY(dalloc(p, &p->dflag, nitems));
                ST_TRY(dalloc(p, &p->dfpos, nitems + 1));
                ST_TRY(dalloc(p, &p->dflag2, nitems));
                ST_TRY(dalloc(p, &p->dfpos2, nitems + 1));
            }
            return ensure_scan_tmp(p, std::max(p->nd, nitems));
        }));
        const int64_t *nlim = p->merge > 1 ? p->dbase + p->nd : nullptr;
        if (p->merge > 1)
            launch_num_nitems(p->dprods, ditems, p->nd, p->hslot, p->nchv, p->dnchv, st);
        else
            launch_nch_of(p->dprods, ditems, p->nd, p->opt.chunks_per_item, p->dnchv, st);
        ST_TRY(launch_check());
        ST_TRY(scan(p, p->dnchv, p->dbase, p->nd));
        launch_expand(p->dbase, p->nd, p->ditem_row, st);
        launch_num_desc(p->dprods, ditems, p->ditem_row, p->dbase, nitems,
                        p->opt.chunks_per_item, p->hslot, p->cbase, p->sbase, p->rptv, p->mstart,
                        nlim, p->ndesc, st);
        ST_TRY(launch_check());
        p->n_dense = -1;
        if (num_chunk_rank_used(p->fast, p->opt.chunks_per_item, p->opt.num_rank_cap)) {
            // dense chunks first, then the rank-accumulated items by kind and
            // size, so that each launch covers its own items only
            launch_desc_flag(p->ndesc, nitems, p->chunk_cnt, p->opt.num_rank_cap, nlim, p->dflag,
                             p->dflag2, st);
            ST_TRY(launch_check());
            ST_TRY(scan(p, p->dflag, p->dfpos, nitems));
            ST_TRY(scan(p, p->dflag2, p->dfpos2, nitems));
            launch_desc_split(p->ndesc, nitems, p->dflag, p->dfpos, p->dflag2, p->dfpos2,
                              p->chunk_cnt, p->chunk_pos, nlim, p->ndesc_split, st);
            ST_TRY(launch_check());
            HIP_TRY(hipMemcpyAsync(p->hread, p->dfpos + nitems, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(p->hread + 1, p->dfpos2 + nitems, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(p->hread + 2, p->dbase + p->nd, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            p->n_dense = p->hread[0] & 0xffffffffll;
            p->n_s0 = p->hread[0] >> 32;
            p->n_m1 = p->hread[1] & 0xffffffffll;
            p->n_m0 = p->hread[1] >> 32;
            p->n_items = p->hread[2];
            p->n_s1 = p->n_items - p->n_dense - p->n_s0 - p->n_m1 - p->n_m0;
            if (p->n_items < 0 || p->n_items > nitems || p->n_s1 < 0) return SPGEMM_EINTERNAL;
        }
    }
    if (p->opt.row_thread && p->num_start[2] > p->num_start[1]) {
        const int64_t cnt = p->num_start[2] - p->num_start[1];
        ST_TRY(ensure_scan_tmp(p, cnt));
        launch_rt_offsets(p->dprods, p->map_num + p->num_start[1], cnt, p->rt_lens,
                          p->rt_off_num, p->scan_tmp, st);
        ST_TRY(launch_check());
    }
    p->state = 2;
    return SPGEMM_OK;
}

// Enqueues every kernel of the numeric phase on `st`.  Each kernel reads the
// value and output pointers from the device descriptors; every other argument
// is fixed once the symbolic phase is done, so the same launches can be
// captured once and replayed.
spgemm_status numeric_launch(spgemm_plan *p, hipStream_t st) {
    static const char *const num_names[kGroups] = {"num.g0", "num.g1", "num.g2", "num.g3",
                                                   "num.g4", "num.g5", "num.g6", "num.g7"};
    for (int g = 1; g <= 4; ++g) {
        if (p->num_start[g + 1] == p->num_start[g]) continue;
        TimeScope ts(p, num_names[g]);
        if (g == 1 && p->opt.row_thread) {
            const int64_t cnt = p->num_start[2] - p->num_start[1];
            const uint64_t *items = p->map_num + p->num_start[1];
            launch_rt_gather(p->dprods, items, cnt, p->rt_off_num, p->rt_stream, true, st);
            launch_num_rowthread(p->dprods, items, cnt, p->rt_off_num, p->rt_stream, p->rptv,
                                 p->flags, st);
            continue;
        }
        launch_num_group(g, p->dprods, p->map_num + p->num_start[g],
                         p->num_start[g + 1] - p->num_start[g], p->rptv, p->flags, st, nullptr,
                         0, max_b_cols(p));
    }
    for (int g = 5; g <= 6; ++g) {
        if (p->num_start[g + 1] == p->num_start[g]) continue;
        TimeScope ts(p, num_names[g]);
        launch_num_block(g, p->opt.num_upper[g], p->dprods, p->map_num + p->num_start[g],
                         p->num_start[g + 1] - p->num_start[g], p->rptv, p->flags, st);
    }
    if (p->nd > 0) {
        const int kper = p->opt.chunks_per_item;
        const bool rank = num_chunk_rank_used(p->fast, kper, p->opt.num_rank_cap);
        const bool split = rank && p->n_dense >= 0;
        const ChunkDesc *dense_desc = split ? p->ndesc_split : p->ndesc;
        const int64_t n_dense = split ? p->n_dense : p->d_items / kper;
        if (n_dense > 0) {
            TimeScope ts(p, num_names[7]);
            launch_num_chunk(p->wmax, p->fast, p->dprods, dense_desc, p->sabs, n_dense, kper,
                             p->chunk_cnt, p->chunk_pos, p->sbits, p->wpc,
                             p->opt.chunk_wgs_per_cu, p->opt.chunk_threads,
                             rank ? p->opt.num_rank_cap : 0, split, p->flags, st);
        }
        if (rank) {
            // large and small single chunks, then large and small merged items
            // (merged items have a wider structure; small items a half-size
            // accumulator)
            TimeScope ts(p, "num.g7r");
            const int cap = p->opt.num_rank_cap;
            const bool f64 = p->opt.accumulate == 1;
            if (!split) {
                if (!launch_num_chunk_rank(p->wmax, p->dprods, p->ndesc, p->sabs, p->d_items,
                                           p->chunk_cnt, p->chunk_pos, p->sbits, p->wpc, cap,
                                           false, p->flags, st, f64))
                    return SPGEMM_EINTERNAL;
            } else {
                const ChunkDesc *r = p->ndesc_split + p->n_dense;
                const struct { int64_t n; int w, cap; } parts[4] = {
                    {p->n_s1, p->wmax, cap},
                    {p->n_s0, p->wmax, cap / 2},
                    {p->n_m1, p->wmax_item, cap},
                    {p->n_m0, p->wmax_item, cap / 2}};
                for (const auto &q : parts) {
                    if (q.n > 0 &&
                        !launch_num_chunk_rank(q.w, p->dprods, r, p->sabs, q.n, p->chunk_cnt,
                                               p->chunk_pos, p->sbits, p->wpc, q.cap, true,
                                               p->flags, st, f64))
                        return SPGEMM_EINTERNAL;
                    r += q.n;
                }
            }
        }
    }
    return launch_check();
}

// Captures numeric_launch into p->num_graph, on a private stream (the
// plan's stream may be the null stream, which cannot be captured).
spgemm_status capture_numeric(spgemm_plan *p) {
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    spgemm_status s = SPGEMM_OK;
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
        s = numeric_launch(p, cs);
        e = hipStreamEndCapture(cs, &g);  // always ends the capture
    }
    size_t nodes = 0;
    if (s == SPGEMM_OK && e == hipSuccess) e = hipGraphGetNodes(g, nullptr, &nodes);
    if (s == SPGEMM_OK && e == hipSuccess) {
        if (nodes == 0)
            p->num_graph_empty = true;  // an empty product: nothing to replay
        else
            e = hipGraphInstantiate(&p->num_graph, g, nullptr, nullptr, 0);
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (s != SPGEMM_OK) return s;
    if (e != hipSuccess) {
        report_hip("numeric graph capture", e, __LINE__);
        p->num_graph = nullptr;
        (void)hipGetLastError();
        return SPGEMM_EHIP;
    }
    return SPGEMM_OK;
}

spgemm_status numeric_impl(spgemm_plan *p) {
    if (p->state != 2) return SPGEMM_ESTATE;
    for (int q = 0; q < p->nprod; ++q) {  // B sorted at plan time: its values too
        if (!p->bs_perm[q]) continue;
        TimeScope ts(p, "num.bgather");
        launch_gather_f32(p->hprods[q].valB, p->bs_perm[q], p->B[q].nnz, p->bs_val[q],
                          p->stream);
        p->hprods[q].valB = p->bs_val[q];
    }
    ST_TRY(upload_descriptors(p));
    if (!p->opt.graph || p->opt.profile) return numeric_launch(p, p->stream);
    if (!p->num_graph && !p->num_graph_empty) ST_TRY(capture_numeric(p));
    if (p->num_graph) HIP_TRY(hipGraphLaunch(p->num_graph, p->stream));
    return SPGEMM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free entry point: the workspace lives in `scratch`, a static
// device array (one copy per GPU, held until the process ends).  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, fetched once per device.  Host bookkeeping uses static
// buffers.  Calls are serialised by g_noalloc_mu and synchronise their
// stream before returning, so a call never finds the array in use.
// ---------------------------------------------------------------------------
constexpr size_t kNoallocScratch = size_t(64) << 20;
constexpr int kNoallocMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocScratch];

namespace {

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoallocMaxDevices];
alignas(64) unsigned char g_noalloc_host[1 << 20];
alignas(64) int64_t g_noalloc_read[8192];
ProdDev g_noalloc_desc[1];
alignas(spgemm_plan) unsigned char g_noalloc_plan[sizeof(spgemm_plan)];

// Device address of the scratch array on the current device (held lock).
spgemm_status noalloc_scratch(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) return SPGEMM_EINVAL;
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return SPGEMM_EHIP;
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SPGEMM_OK;
}

spgemm_status noalloc_run(spgemm_plan *p, const spgemm_csr *A, const spgemm_csr *B,
                          int64_t *c_row_ptr, int32_t *c_col_idx, float *c_values,
                          int64_t c_capacity, int64_t *nnz_c) {
    ST_TRY(plan_create_impl(p, 1, A, B));
    ST_TRY(symbolic_impl(p));
    *nnz_c = p->nnz_total;
    HIP_TRY(hipMemcpyAsync(c_row_ptr, p->rptv, sizeof(int64_t) * (p->Mtot + 1),
                           hipMemcpyDeviceToDevice, p->stream));
    if (p->nnz_total > c_capacity) return SPGEMM_ENOMEM;
    if (p->nnz_total > 0 && (!c_col_idx || !c_values)) return SPGEMM_EINVAL;
    p->hprods[0].valA = A->values;
    p->hprods[0].valB = B->values;
    p->hprods[0].colC = c_col_idx;
    p->hprods[0].valC = c_values;
    ST_TRY(numeric_impl(p));
    HIP_TRY(hipGetLastError());
    int f[1];
    ST_TRY(read_flags(p, f, 1));
    return f[0] ? SPGEMM_EINTERNAL : SPGEMM_OK;
}

}  // namespace

extern "C" {

void spgemm_default_options(spgemm_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    // the autotuner's result for this architecture (tuned/<arch>.json,
    // compiled in by the build)
    for (int g = 0; g < kGroups - 1; ++g) {
        opt->sym_upper[g] = kTunedSym[g];
        opt->num_upper[g] = kTunedNum[g];
    }
    opt->chunk_cols = kTuned_chunk_cols;
    opt->chunks_per_item = kTuned_chunks_per_item;
    opt->chunk_wgs_per_cu = kTuned_chunk_wgs_per_cu;
    opt->chunk_threads = kTuned_chunk_threads;
    opt->sym_chunk_threads = kTuned_sym_chunk_threads;
    opt->num_rank_cap = kTuned_num_rank_cap;
    opt->chunk_merge = kTuned_chunk_merge;
    opt->row_thread = kTuned_row_thread;
    opt->validate = 0;
}

spgemm_status spgemm_plan_create(spgemm_plan **out, const spgemm_csr *A, const spgemm_csr *B,
                                 const spgemm_options *opt, void *stream,
                                 spgemm_alloc_fn alloc_fn, spgemm_free_fn free_fn,
                                 void *alloc_ctx) {
    return create_common(out, 1, A, B, opt, stream, alloc_fn, free_fn, alloc_ctx, false);
}

spgemm_status spgemm_plan_create_batch(spgemm_plan **out, int32_t nprod, const spgemm_csr *A,
                                       const spgemm_csr *B, const spgemm_options *opt,
                                       void *stream, spgemm_alloc_fn alloc_fn,
                                       spgemm_free_fn free_fn, void *alloc_ctx) {
    return create_common(out, nprod, A, B, opt, stream, alloc_fn, free_fn, alloc_ctx, true);
}

spgemm_status spgemm_symbolic(spgemm_plan *p, int64_t *c_row_ptr, int64_t *nnz_c,
                              int64_t *flops) {
    if (!p || !c_row_ptr || !nnz_c) return SPGEMM_EINVAL;
    if (p->batch) return SPGEMM_ESTATE;
    spgemm_status s;
    try { s = symbolic_impl(p); } catch (...) { s = SPGEMM_ENOMEM; }
    if (s != SPGEMM_OK) return s;
    HIP_TRY(hipMemcpyAsync(c_row_ptr, p->rptv, sizeof(int64_t) * (p->Mtot + 1),
                           hipMemcpyDeviceToDevice, p->stream));
    *nnz_c = p->nnz_total;
    if (flops) *flops = 2 * p->ip_total;
    return SPGEMM_OK;
}

spgemm_status spgemm_symbolic_batch(spgemm_plan *p, int64_t *const *c_row_ptr, int64_t *nnz_c) {
    if (!p || !c_row_ptr || !nnz_c) return SPGEMM_EINVAL;
    if (p->device_driven) return SPGEMM_ESTATE;
    for (int q = 0; q < p->nprod; ++q)
        if (!c_row_ptr[q]) return SPGEMM_EINVAL;
    spgemm_status s;
    try { s = symbolic_impl(p); } catch (...) { s = SPGEMM_ENOMEM; }
    if (s != SPGEMM_OK) return s;
    if (p->nprod > 1 && p->nprod <= 65535) {
        // every product's row pointers in one launch (the descriptors carry
        // c_row_ptr)
        for (int q = 0; q < p->nprod; ++q) p->hprods[q].rptC = c_row_ptr[q];
        ST_TRY(upload_descriptors(p));
        launch_rows_local_batch(p->dprods, p->nprod,
                                std::max<int64_t>(1, (p->Mtot / p->nprod + 256) / 256), p->rptv,
                                p->stream);
    } else {
        for (int q = 0; q < p->nprod; ++q)
            launch_rows_local(p->rptv, p->hprods[q].row_base, p->hprods[q].m, c_row_ptr[q],
                              p->stream);
    }
    for (int q = 0; q < p->nprod; ++q) nnz_c[q] = p->nnz_c[q];
    return launch_check();
}

spgemm_status spgemm_numeric(spgemm_plan *p, const float *a_values, const float *b_values,
                             int32_t *c_col_idx, float *c_values) {
    if (!p) return SPGEMM_EINVAL;
    if (p->batch) return SPGEMM_ESTATE;
    if (p->state != 2) return SPGEMM_ESTATE;
    if ((p->A[0].nnz > 0 && !a_values) || (p->B[0].nnz > 0 && !b_values)) return SPGEMM_EINVAL;
    if (p->nnz_total > 0 && (!c_col_idx || !c_values)) return SPGEMM_EINVAL;
    p->hprods[0].valA = a_values;
    p->hprods[0].valB = b_values;
    p->hprods[0].colC = c_col_idx;
    p->hprods[0].valC = c_values;
    return numeric_impl(p);
}

spgemm_status spgemm_numeric_batch(spgemm_plan *p, const float *const *a_values,
                                   const float *const *b_values, int32_t *const *c_col_idx,
                                   float *const *c_values) {
    if (!p || !a_values || !b_values || !c_col_idx || !c_values) return SPGEMM_EINVAL;
    if (p->state != 2 || p->device_driven) return SPGEMM_ESTATE;
    for (int q = 0; q < p->nprod; ++q) {
        if ((p->A[q].nnz > 0 && !a_values[q]) || (p->B[q].nnz > 0 && !b_values[q]))
            return SPGEMM_EINVAL;
        if (p->nnz_c[q] > 0 && (!c_col_idx[q] || !c_values[q])) return SPGEMM_EINVAL;
        p->hprods[q].valA = a_values[q];
        p->hprods[q].valB = b_values[q];
        p->hprods[q].colC = c_col_idx[q];
        p->hprods[q].valC = c_values[q];
    }
    return numeric_impl(p);
}

spgemm_status spgemm_estimate(const spgemm_csr *A, const spgemm_csr *B, int64_t *out,
                              void *stream) {
    if (!A || !B || !out) return SPGEMM_EINVAL;
    if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0 || B->nrows < 0 || B->ncols < 0)
        return SPGEMM_EINVAL;
    if (A->nrows >= (int64_t(1) << 31) || B->ncols >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    if (A->ncols != B->nrows) return SPGEMM_EDIM;
    if (!A->row_ptr || !B->row_ptr || (A->nnz > 0 && !A->col_idx)) return SPGEMM_EINVAL;
    launch_ip_estimate(A->row_ptr, A->col_idx, B->row_ptr, A->nrows, B->ncols, out,
                       (hipStream_t)stream);
    return launch_check();
}

spgemm_status spgemm_plan_create_device(spgemm_plan **out, int32_t nprod, const spgemm_csr *A,
                                        const spgemm_csr *B, const spgemm_options *opt,
                                        void *stream, spgemm_alloc_fn alloc_fn,
                                        spgemm_free_fn free_fn, void *alloc_ctx) {
    if (!out) return SPGEMM_EINVAL;
    *out = nullptr;
    if (nprod <= 0 || !A || !B) return SPGEMM_EINVAL;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return SPGEMM_EINVAL;
    spgemm_options o;
    if (opt) o = *opt; else spgemm_default_options(&o);
    ST_TRY(check_options(o));
    apply_accumulate(o);
    spgemm_plan *p = new (std::nothrow) spgemm_plan();
    if (!p) return SPGEMM_ENOMEM;
    p->stream = (hipStream_t)stream;
    p->afn = alloc_fn;
    p->ffn = free_fn;
    p->actx = alloc_ctx;
    p->opt = o;
    p->batch = true;
    spgemm_status s;
    try {
        s = device_plan_setup(p, nprod, A, B);
    } catch (...) {
        s = SPGEMM_ENOMEM;
    }
    if (s != SPGEMM_OK) {
        spgemm_free(p);
        return s;
    }
    *out = p;
    return SPGEMM_OK;
}

spgemm_status spgemm_execute_arena(spgemm_plan *p, const float *const *a_values,
                                   const float *const *b_values, int64_t *const *c_row_ptr,
                                   int64_t *c_offsets, int32_t *c_col, float *c_val,
                                   int64_t capacity) {
    if (!p || !a_values || !b_values || !c_row_ptr || !c_offsets || capacity < 0)
        return SPGEMM_EINVAL;
    if (!p->device_driven) return SPGEMM_ESTATE;
    if (capacity > 0 && (!c_col || !c_val)) return SPGEMM_EINVAL;
    for (int q = 0; q < p->nprod; ++q) {
        if (!c_row_ptr[q]) return SPGEMM_EINVAL;
        if ((p->A[q].nnz > 0 && !a_values[q]) || (p->B[q].nnz > 0 && !b_values[q]))
            return SPGEMM_EINVAL;
        p->hprods[q].valA = a_values[q];
        p->hprods[q].valB = b_values[q];
        p->hprods[q].colC = c_col;
        p->hprods[q].valC = c_val;
        p->hprods[q].rptC = c_row_ptr[q];
        p->hprods[q].c_arena = 1;
    }
    ST_TRY(upload_descriptors(p));
    if (!p->opt.graph || p->opt.profile) {
        TimeScope ts(p, "device.all");
        return device_launch_all(p, p->stream, c_row_ptr, c_offsets, capacity);
    }
    bool same = p->dev_graph && p->dev_off == c_offsets && p->dev_cap == capacity;
    for (int q = 0; same && q < p->nprod; ++q) same = p->dev_rpt[q] == c_row_ptr[q];
    if (!same) ST_TRY(capture_device(p, c_row_ptr, c_offsets, capacity));
    HIP_TRY(hipGraphLaunch(p->dev_graph, p->stream));
    return SPGEMM_OK;
}

spgemm_status spgemm_sync(spgemm_plan *p) {
    if (!p) return SPGEMM_EINVAL;
    HIP_TRY(hipGetLastError());
    int f[1];
    ST_TRY(read_flags(p, f, 1));
    static const bool debug = std::getenv("SPGEMM_DEBUG") != nullptr;
    if (debug && f[0]) std::fprintf(stderr, "spgemm: kernel error flags 0x%x\n", f[0]);
    if (f[0] == kErrCapacity) return SPGEMM_ENOMEM;  // C did not fit the arena
    return f[0] ? SPGEMM_EINTERNAL : SPGEMM_OK;
}

spgemm_status spgemm_get_info(const spgemm_plan *p, spgemm_info *info) {
    if (!p || !info) return SPGEMM_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->flops = 2 * p->ip_total;
    info->ip_total = p->ip_total;
    info->ip_max = p->ip_max;
    info->nnz_c = p->state >= 2 ? p->nnz_total : -1;
    for (int g = 0; g < kGroups; ++g) {
        info->sym_group_rows[g] = p->sym_start[g + 1] - p->sym_start[g];
        info->num_group_rows[g] = p->state >= 2 ? p->num_start[g + 1] - p->num_start[g] : 0;
    }
    info->chunk_cols = p->hprods.empty() ? 0 : p->hprods[0].W;
    info->chunks_per_row = p->hprods.empty() ? 0 : p->hprods[0].nch;
    info->workspace_bytes = p->ws_bytes;
    return SPGEMM_OK;
}

spgemm_status spgemm_export(const spgemm_plan *p, int32_t what, void *dst, int64_t *group_start) {
    if (!p || !dst) return SPGEMM_EINVAL;
    const void *src = nullptr;
    const int64_t *gs = nullptr;
    if (what == 0) src = p->ip;
    else if (what == 1) { src = p->map_sym; gs = p->sym_start; }
    else if (what == 2) {
        if (p->state < 2) return SPGEMM_ESTATE;
        src = p->map_num;
        gs = p->num_start;
    } else return SPGEMM_EINVAL;
    if (p->Mtot > 0)
        HIP_TRY(hipMemcpyAsync(dst, src, sizeof(int64_t) * p->Mtot, hipMemcpyDeviceToDevice,
                               p->stream));
    if (group_start && gs) std::memcpy(group_start, gs, sizeof(int64_t) * (kGroups + 1));
    return SPGEMM_OK;
}

void spgemm_free(spgemm_plan *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    if (p->num_graph) (void)hipGraphExecDestroy(p->num_graph);
    if (p->dev_graph) (void)hipGraphExecDestroy(p->dev_graph);
    for (void *ptr : p->allocs) {
        if (p->ffn) p->ffn(p->actx, ptr, (void *)p->stream);
        else (void)hipFree(ptr);
    }
    p->allocs.clear();
    // the stream is idle: the pinned buffers and events go back to the pools
    for (auto &t : p->timed) {
        pools().give_event(t.a, true);
        pools().give_event(t.b, true);
    }
    if (!p->noalloc) {
        pools().give_pinned(p->pinned, p->pinned_bytes);
        pools().give_pinned(p->hread, p->hread_bytes);
    }
    for (int s = 0; s < kDescSlots; ++s) pools().give_event(p->desc_ev[s], false);
    delete p;
}

int32_t spgemm_timing_count(const spgemm_plan *p) { return p ? (int32_t)p->timed.size() : 0; }

spgemm_status spgemm_timing(spgemm_plan *p, int32_t idx, const char **name, float *ms) {
    if (!p || !name || !ms || idx < 0 || idx >= (int32_t)p->timed.size()) return SPGEMM_EINVAL;
    HIP_TRY(hipEventSynchronize(p->timed[idx].b));
    HIP_TRY(hipEventElapsedTime(ms, p->timed[idx].a, p->timed[idx].b));
    *name = p->timed[idx].name;
    return SPGEMM_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t spgemm_selector_transpose_workspace(int64_t k) {
    if (k < 0) return 0;
    return 256 + align256(sizeof(int64_t) * (size_t)(k + 1)) + align256(scan_temp_bytes(k));
}

spgemm_status spgemm_selector_transpose(const int32_t *labels, int64_t n, int64_t k,
                                        int64_t *row_ptr, int32_t *col_idx, float *values,
                                        void *workspace, void *stream) {
    if (n < 0 || k < 0 || !row_ptr || !workspace) return SPGEMM_EINVAL;
    if (n > 0 && (!labels || !col_idx || !values)) return SPGEMM_EINVAL;
    if (n >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)workspace;
    int *flag = (int *)w;
    int64_t *work = (int64_t *)(w + 256);
    void *tmp = w + 256 + align256(sizeof(int64_t) * (size_t)(k + 1));
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
    launch_selector_t(labels, n, k, row_ptr, col_idx, values, work, tmp, flag, st);
    ST_TRY(launch_check());
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return h ? SPGEMM_EINDEX : SPGEMM_OK;
}

// MCL prune workspace: rowsum (2 m floats), sel (2 m int32), keep (m + 1
// int64), scan tiles.
size_t spgemm_mcl_prune_workspace(int64_t m) {
    if (m < 0) return 0;
    return align256(sizeof(float) * 2 * (size_t)m) + align256(sizeof(int32_t) * 2 * (size_t)m) +
           align256(sizeof(int64_t) * (size_t)(m + 1)) + align256(scan_temp_bytes(m));
}

namespace {
struct MclWs {
    float *rowsum;
    int32_t *sel;
    int64_t *keep;
    void *tmp;
};
MclWs mcl_ws(void *workspace, int64_t m) {
    char *w = (char *)workspace;
    MclWs r;
    r.rowsum = (float *)w;
    w += align256(sizeof(float) * 2 * (size_t)m);
    r.sel = (int32_t *)w;
    w += align256(sizeof(int32_t) * 2 * (size_t)m);
    r.keep = (int64_t *)w;
    w += align256(sizeof(int64_t) * (size_t)(m + 1));
    r.tmp = w;
    return r;
}
}  // namespace

spgemm_status spgemm_mcl_prune_count(int64_t m, const int64_t *row_ptr, const float *values,
                                     float power, float theta, int32_t k, int64_t *out_row_ptr,
                                     void *workspace, int64_t *out_nnz, void *stream) {
    if (m < 0 || !row_ptr || !out_row_ptr || !workspace || !out_nnz) return SPGEMM_EINVAL;
    if (!(power > 0.f) || !(theta >= 0.f) || k < 0) return SPGEMM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const MclWs w = mcl_ws(workspace, m);
    launch_mcl_count(m, row_ptr, values, power, theta, k, w.rowsum, w.keep, w.sel, st);
    launch_scan_i64(w.keep, out_row_ptr, m, w.tmp, st);
    ST_TRY(launch_check());
    int64_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, out_row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out_nnz = nnz;
    return SPGEMM_OK;
}

spgemm_status spgemm_mcl_prune_write(int64_t m, const int64_t *row_ptr, const int32_t *col_idx,
                                     const float *values, float power, float theta, int32_t k,
                                     const int64_t *out_row_ptr, void *workspace,
                                     int32_t *out_col, float *out_val, void *stream) {
    if (m < 0 || !row_ptr || !out_row_ptr || !workspace) return SPGEMM_EINVAL;
    if (!(power > 0.f) || !(theta >= 0.f) || k < 0) return SPGEMM_EINVAL;
    const MclWs w = mcl_ws(workspace, m);
    launch_mcl_write(m, row_ptr, col_idx, values, power, theta, w.rowsum, w.sel, out_row_ptr,
                     out_col, out_val, (hipStream_t)stream);
    return launch_check();
}

spgemm_status spgemm_mcl_change(int64_t m, const int64_t *rpt_a, const int32_t *col_a,
                                const float *val_a, const int64_t *rpt_b, const int32_t *col_b,
                                const float *val_b, int64_t nnz_a, int64_t nnz_b, double *out,
                                void *stream) {
    if (m < 0 || nnz_a < 0 || nnz_b < 0 || !rpt_a || !rpt_b || !out) return SPGEMM_EINVAL;
    if ((nnz_a > 0 && (!col_a || !val_a)) || (nnz_b > 0 && (!col_b || !val_b)))
        return SPGEMM_EINVAL;
    launch_mcl_change(m, rpt_a, col_a, val_a, nnz_a, rpt_b, col_b, val_b, nnz_b, out,
                      (hipStream_t)stream);
    return launch_check();
}

size_t spgemm_components_workspace(void) { return 256; }

spgemm_status spgemm_components(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                                int64_t nnz, int32_t *labels, void *workspace, void *stream,
                                int32_t *rounds) {
    if (n < 0 || nnz < 0 || !row_ptr || !labels || !workspace) return SPGEMM_EINVAL;
    if (nnz > 0 && !col_idx) return SPGEMM_EINVAL;
    if (n >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    hipStream_t st = (hipStream_t)stream;
    int *changed = (int *)workspace;
    launch_cc_init(n, labels, st);
    // every round lowers at least one parent, and parents are vertex
    // indices: the loop ends; the bound only guards against a broken input
    const int max_rounds = 64 + 2 * 31;
    int r = 0;
    for (; r < max_rounds; ++r) {
        launch_cc_round(n, row_ptr, col_idx, nnz, labels, changed, st);
        ST_TRY(launch_check());
        int h = 0;
        HIP_TRY(hipMemcpyAsync(&h, changed, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (!h) break;
    }
    if (rounds) *rounds = r + 1;
    return r < max_rounds ? SPGEMM_OK : SPGEMM_EINTERNAL;
}

spgemm_status spgemm_topk_rows(int64_t n, int64_t f, const float *x, int64_t ldx, int32_t k,
                               int64_t *row_ptr, int32_t *col_idx, float *values, void *stream) {
    if (n < 0 || f < 0 || k < 0 || ldx < f || !row_ptr) return SPGEMM_EINVAL;
    const int64_t kk = std::min<int64_t>(k, f);
    if (n > 0 && kk > 0 && (!x || !col_idx || !values)) return SPGEMM_EINVAL;
    if (f >= (int64_t(1) << 31) || n >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    hipStream_t st = (hipStream_t)stream;
    launch_rows_uniform(row_ptr, n, kk, st);
    launch_topk_rows(n, f, x, ldx, (int)kk, col_idx, values, st);
    return launch_check();
}

spgemm_status spgemm_csr_to_dense(int64_t m, int64_t n, const int64_t *row_ptr,
                                  const int32_t *col_idx, const float *values, float *dense,
                                  int64_t ldd, void *stream) {
    if (m < 0 || n < 0 || ldd < n || !row_ptr || (m > 0 && n > 0 && !dense)) return SPGEMM_EINVAL;
    launch_csr_to_dense(m, n, row_ptr, col_idx, values, dense, ldd, (hipStream_t)stream);
    return launch_check();
}

spgemm_status spgemm_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t a_row,
                              int64_t a_col, const float *B, int64_t b_row, int64_t b_col,
                              float *C, int64_t ldc, void *stream) {
    if (M < 0 || N < 0 || K < 0 || ldc < N) return SPGEMM_EINVAL;
    if (M > 0 && N > 0 && (!C || (K > 0 && (!A || !B)))) return SPGEMM_EINVAL;
    if (M / 64 >= 65535) return SPGEMM_EDIM;
    launch_gemm_f32(M, N, K, A, a_row, a_col, B, b_row, b_col, C, ldc, (hipStream_t)stream);
    return launch_check();
}

spgemm_status spgemm_masked_spmm(int64_t m, const int64_t *rpt_t, const int32_t *col_t,
                                 const float *val_t, const float *dense, int64_t ldd,
                                 const int64_t *rpt_mask, const int32_t *col_mask, float *out,
                                 void *stream) {
    if (m < 0 || !rpt_t || !rpt_mask) return SPGEMM_EINVAL;
    launch_masked_spmm(m, rpt_t, col_t, val_t, dense, ldd, rpt_mask, col_mask, out,
                       (hipStream_t)stream);
    return launch_check();
}

size_t spgemm_transpose_workspace(int64_t ncols) {
    if (ncols < 0) return 0;
    return align256(sizeof(int64_t) * (size_t)(ncols + 1)) + align256(scan_temp_bytes(ncols));
}

spgemm_status spgemm_transpose(int64_t m, int64_t n, const int64_t *row_ptr,
                               const int32_t *col_idx, const float *values, int64_t nnz,
                               int64_t *rpt_t, int32_t *col_t, float *val_t, void *workspace,
                               void *stream) {
    if (m < 0 || n < 0 || nnz < 0 || !row_ptr || !rpt_t || !workspace) return SPGEMM_EINVAL;
    if (nnz > 0 && (!col_idx || !col_t || (values && !val_t))) return SPGEMM_EINVAL;
    if (m >= (int64_t(1) << 31)) return SPGEMM_EDIM;
    char *w = (char *)workspace;
    int64_t *work = (int64_t *)w;
    void *tmp = w + align256(sizeof(int64_t) * (size_t)(n + 1));
    launch_transpose(m, n, row_ptr, col_idx, values, nnz, rpt_t, col_t, val_t, work, tmp,
                     (hipStream_t)stream);
    return launch_check();
}

spgemm_status spgemm_its_sample(int64_t m, int32_t s, const int64_t *row_ptr,
                                const int32_t *col_idx, const float *values, const float *u,
                                const int32_t *self, int32_t *out, void *stream) {
    if (m < 0 || s < 0 || !row_ptr) return SPGEMM_EINVAL;
    if (m > 0 && s > 0 && (!u || !self || !out)) return SPGEMM_EINVAL;
    launch_its_sample(m, s, row_ptr, col_idx, values, u, self, out, (hipStream_t)stream);
    return launch_check();
}

size_t spgemm_noalloc_scratch_bytes(void) { return kNoallocScratch; }

spgemm_status spgemm_multiply_noalloc(const spgemm_csr *A, const spgemm_csr *B,
                                      const spgemm_options *opt, void *stream,
                                      int64_t *c_row_ptr, int32_t *c_col_idx, float *c_values,
                                      int64_t c_capacity, int64_t *nnz_c) {
    if (!A || !B || !c_row_ptr || !nnz_c || c_capacity < 0) return SPGEMM_EINVAL;
    *nnz_c = -1;
    ST_TRY(check_csr(*A, true));
    ST_TRY(check_csr(*B, true));
    if (A->ncols != B->nrows) return SPGEMM_EDIM;
    spgemm_options o;
    if (opt) o = *opt; else spgemm_default_options(&o);
    ST_TRY(check_options(o));
    apply_accumulate(o);
    o.profile = 0;  // no timing events
    o.graph = 0;    // no graph objects
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    void *arena = nullptr;
    ST_TRY(noalloc_scratch(&arena));
    std::pmr::monotonic_buffer_resource mr(g_noalloc_host, sizeof(g_noalloc_host),
                                           std::pmr::null_memory_resource());
    spgemm_plan *p = new (g_noalloc_plan) spgemm_plan(&mr);
    p->noalloc = true;
    p->arena = (char *)arena;
    p->arena_cap = kNoallocScratch;
    p->host_read = g_noalloc_read;
    p->host_read_bytes = sizeof(g_noalloc_read);
    p->pinned = g_noalloc_desc;
    p->stream = (hipStream_t)stream;
    p->opt = o;
    spgemm_status s;
    try {
        s = noalloc_run(p, A, B, c_row_ptr, c_col_idx, c_values, c_capacity, nnz_c);
    } catch (...) {
        s = SPGEMM_ENOMEM;  // the static host buffer of the bookkeeping is full
    }
    // nothing may still use the scratch array when the next call starts
    if (hipStreamSynchronize(p->stream) != hipSuccess && s == SPGEMM_OK) s = SPGEMM_EHIP;
    p->~spgemm_plan();
    return s;
}

const char *spgemm_status_string(spgemm_status s) {
    switch (s) {
        case SPGEMM_OK: return "ok";
        case SPGEMM_EINVAL: return "invalid argument";
        case SPGEMM_EDIM: return "dimension mismatch or out of range";
        case SPGEMM_EINDEX: return "malformed CSR input";
        case SPGEMM_EOVERFLOW: return "count overflow";
        case SPGEMM_ENOMEM: return "out of device memory";
        case SPGEMM_EHIP: return "HIP runtime error";
        case SPGEMM_ESTATE: return "call out of order";
        case SPGEMM_EINTERNAL: return "kernel error flag raised";
        default: return "unknown status";
    }
}

}  // extern "C"
