// C-ABI entry points of the fpts library: argument checks, workspace layout
// and the enqueue order of the kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "fpts_internal.hpp"
#include "fpts_lpt.h"

using namespace fpts;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Cursor {
    size_t at = 0;
    size_t take(size_t bytes)
    {
        size_t o = at;
        at = align_up(at + std::max<size_t>(bytes, 1));
        return o;
    }
};

bool sticky_error()
{
    hipError_t e = hipGetLastError();
    return e != hipSuccess;
}

// Fixed scratch of fpts_find_eval_noalloc: one copy per device, held until
// the process ends.  Host code never uses the array's name as an address:
// the device address of each device's copy is looked up once, with that
// device current (fpts_setup on it), and kept in noalloc_ptr[device].
constexpr int kMaxDevices = 64;
void *noalloc_ptr[kMaxDevices] = {nullptr};
std::mutex noalloc_mu;

}  // namespace

static __device__ __align__(256) char scratch[FPTS_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of this device's scratch copy (device `dev` current);
// nullptr when the lookup failed.
void *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        noalloc_ptr[dev] = p;
    }
    return noalloc_ptr[dev];
}

template <class T>
T *at(void *base, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

constexpr int kCounters = 64;   // ints: 0 the second search's list count, 2 to 5 below;
                                 // from 16 on the Newton passes' element-queue counters
constexpr int kNewtonCounters = 16;   // each Newton pass owns 16 counters from here on
static_assert(3 * kNewtonCounters <= kCounters, "the two Newton passes need disjoint counters");
constexpr int kStats = 16;      // unsigned long long: Newton counters per pass
constexpr int kParkCount = 2;   // int counter of the parked pairs
constexpr int kOverflowCount = 3;   // int counter of the overflowed points
constexpr int kSlotTotal = 4;   // 64-bit running total of the second search's slots (ints 4, 5)
constexpr int kHintPasses = 8;  // Newton passes of the hinted search

void clear_events(fpts_mesh *m)
{
    for (auto &v : m->ev) {
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        v.clear();
    }
    m->prof_find = m->prof_eval = m->prof_lpt = 0;
}

// Records an event pair around a kernel group when profiling is on.
struct Span {
    fpts_mesh *m;
    int k;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    Span(fpts_mesh *m_, int k_, hipStream_t s_) : m(m_), k(k_), s(s_)
    {
        if (!m->profiling) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            (void)hipGetLastError();
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~Span()
    {
        if (!a) return;
        (void)hipEventRecord(b, s);
        m->ev[k].emplace_back(a, b);
    }
};

void free_mesh(fpts_mesh *m)
{
    if (!m) return;
    clear_events(m);
    (void)hipFree(m->d_nodes);
    (void)hipFree(m->d_nodes32);
    (void)hipFree(m->d_near);
    (void)hipFree(m->d_xc);
    (void)hipFree(m->d_box);
    (void)hipFree(m->d_cell_off);
    (void)hipFree(m->d_cell_el);
    delete m;
}

}  // namespace

namespace fpts {

FindWs find_ws_layout(const fpts_mesh *m, int64_t n)
{
    FindWs w;
    Cursor c;
    int64_t ncell = 1;
    for (int d = 0; d < m->D; ++d) ncell *= m->NL;
    w.ncell = ncell;
    // slots for the other candidates of unsettled points: one per point (a
    // few per cent of the points are unsettled on volume meshes, about a
    // quarter of a slot per point on surfaces); points beyond the capacity
    // are searched one per wavefront (overflow path).  Line meshes keep the
    // exact bound (their kernel has no overflow path).
    const int64_t cmax = n * (int64_t)std::max(m->max_cell - 1, 1);
    w.cap2 = std::max<int64_t>(1, m->R == 1 ? cmax : std::min<int64_t>(cmax, n));
    w.bin_shift = bin_shift(ncell);
    w.bin_hist_n = w.bin_shift < 0 ? 0
                                    : ((ncell + (1ll << w.bin_shift) - 1) >> w.bin_shift) *
                                          bin_tiles(n);
    w.scan_blocks = scan_tmp_blocks(
        std::max<int64_t>(std::max<int64_t>(std::max<int64_t>(n, m->nel), ncell), w.bin_hist_n));
    const size_t I = sizeof(int);
    w.cell_cnt = c.take(I * ncell);
    w.cell_poff = c.take(I * (ncell + 1));
    w.cell_choff = c.take(I * (ncell + 1));
    w.cellpt = c.take(I * n);
    w.pbin = c.take(I * n);
    w.cand = c.take(sizeof(int2) * n);
    w.rank = c.take(I * n);
    w.bin_prim = c.take(I * n);
    w.elem_cnt = c.take(I * m->nel);
    w.elem_off = c.take(I * (m->nel + 1));
    w.chunk_off = c.take(I * (m->nel + 1));
    w.sorted = c.take(I * n);
    w.ulist = c.take(I * n);
    w.uoff = c.take(I * n);
    w.ucnt = c.take(I * n);
    w.elem_cnt2 = c.take(I * m->nel);
    w.elem_fill2 = c.take(I * m->nel);
    w.elem_off2 = c.take(I * (m->nel + 1));
    w.chunk_off2 = c.take(I * (m->nel + 1));
    w.slot_pt = c.take(I * w.cap2);
    w.slot_elem = c.take(I * w.cap2);
    w.sorted2 = c.take(I * w.cap2);
    w.res_r = c.take(sizeof(double) * m->R * w.cap2);
    w.res_dist = c.take(sizeof(double) * w.cap2);
    w.res_code = c.take(I * w.cap2);
    w.tb_cell = task_bound(n, ncell);
    w.tb_elem = task_bound(n, m->nel);
    w.tb_elem2 = task_bound(w.cap2, m->nel);
    w.task_cell = c.take(I * w.tb_cell);
    w.task_elem = c.take(I * w.tb_elem);
    w.task_elem2 = c.take(I * w.tb_elem2);
    w.scan_tmp = c.take(I * w.scan_blocks);
    w.pts4 = c.take(m->R >= 2 ? sizeof(double) * pt_stride(m->D) * n : 1);
    w.start = c.take(sizeof(double) * m->R * n);
    // parked pairs of the primary pass (at most one per point)
    w.park_meta = c.take(sizeof(int4) * n);
    w.park_r = c.take(sizeof(double) * (m->R + 1) * n);
    // saved iteration states: a few per cent of the pairs park on volume
    // meshes; those beyond the capacity are re-evaluated by the face kernel
    w.park_state_cap = std::min<int64_t>(n, n / 8 + 1024);
    w.park_state = c.take(sizeof(double) * kParkState * w.park_state_cap);
    w.park_cnt = c.take(I * m->nel);
    w.park_off = c.take(I * (m->nel + 1));
    w.park_choff = c.take(I * (m->nel + 1));
    w.park_rank = c.take(I * n);
    w.park_sorted = c.take(I * n);
    w.tb_park = task_bound(n, m->nel);
    w.park_task = c.take(I * w.tb_park);
    w.olist = c.take(I * n);
    w.ov_grid = (int64_t)m->cus * 4;
    w.ov_int = c.take(I * 3 * w.ov_grid);
    w.ov_dbl = c.take(sizeof(double) * (m->R + 1) * w.ov_grid);
    w.bin_hist = c.take(I * (w.bin_hist_n + 1));
    w.bin_pairs = c.take(w.bin_shift < 0 ? 1 : sizeof(int2) * n);
    w.counters = c.take(I * kCounters);
    w.stats = c.take(sizeof(unsigned long long) * 3 * kStats);
    w.total = c.at;
    return w;
}

EvalWs eval_ws_layout(const fpts_mesh *m, int64_t n)
{
    EvalWs w;
    Cursor c;
    w.elem_cnt = c.take(sizeof(int) * m->nel);
    w.elem_off = c.take(sizeof(int) * (m->nel + 1));
    w.rank = c.take(sizeof(int) * std::max<int64_t>(n, 1));
    w.chunk_off = c.take(sizeof(int) * (m->nel + 1));
    w.scan_tmp = c.take(sizeof(int) * scan_tmp_blocks(m->nel));
    w.sorted = c.take(sizeof(int) * std::max<int64_t>(n, 1));
    w.tb_elem = task_bound(n, m->nel);
    w.task_elem = c.take(sizeof(int) * w.tb_elem);
    w.slist = c.take(sizeof(int) * std::max<int64_t>(n, 1));
    w.scount = c.take(sizeof(int));
    w.total = c.at;
    return w;
}

hipError_t launch_newton(const fpts_mesh *m, int precision, int64_t n, const double *pts,
                         const NewtonIO &io, int which, hipStream_t s)
{
    const bool mixed = precision == FPTS_MIXED;
    if (m->D == 3 && m->R == 3) return launch_newton_hex(m, mixed, n, pts, io, which, s);
    if (m->D == 2 && m->R == 2) return launch_newton_quad(m, mixed, n, pts, io, which, s);
    if (m->R == 1) return launch_newton_line(m, n, pts, io, which, s);
    return launch_newton_surf(m, mixed, n, pts, io, which, s);
}

}  // namespace fpts

namespace fpts {

// fpts_find with an optional keep mask: points with keep[p] != 0 hold final
// results on entry and are not searched; with rs the primary pass also
// writes its settling results in list order (NewtonIO::rs).
int find_impl(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code, int32_t *d_elem,
              double *d_r, double *d_dist, int precision, void *d_ws, size_t ws_bytes,
              void *stream, const int *keep, double *rs, const EvalRest *rest)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return FPTS_EINVAL;
    if (precision != FPTS_FP64 && precision != FPTS_MIXED) return FPTS_EINVAL;
    if (n == 0) return FPTS_OK;
    if (!d_pts || !d_code || !d_elem || !d_r || !d_dist || !d_ws) return FPTS_EINVAL;
    if (((uintptr_t)d_ws & 255) != 0) return FPTS_EINVAL;
    const FindWs w = find_ws_layout(m, n);
    if (w.cap2 > INT32_MAX || ws_bytes < w.total) return FPTS_EINVAL;
    if (sticky_error()) return FPTS_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    int *cell_cnt = at<int>(d_ws, w.cell_cnt), *rank = at<int>(d_ws, w.rank);
    int *bin_prim = at<int>(d_ws, w.bin_prim);
    int *cell_poff = at<int>(d_ws, w.cell_poff), *cell_choff = at<int>(d_ws, w.cell_choff);
    int *cellpt = at<int>(d_ws, w.cellpt), *pbin = at<int>(d_ws, w.pbin);
    int2 *cand = at<int2>(d_ws, w.cand);
    int *elem_cnt = at<int>(d_ws, w.elem_cnt);
    int *elem_off = at<int>(d_ws, w.elem_off), *chunk_off = at<int>(d_ws, w.chunk_off);
    int *sorted = at<int>(d_ws, w.sorted), *ulist = at<int>(d_ws, w.ulist);
    int *uoff = at<int>(d_ws, w.uoff), *ucnt = at<int>(d_ws, w.ucnt);
    int *elem_cnt2 = at<int>(d_ws, w.elem_cnt2), *elem_fill2 = at<int>(d_ws, w.elem_fill2);
    int *elem_off2 = at<int>(d_ws, w.elem_off2), *chunk_off2 = at<int>(d_ws, w.chunk_off2);
    int *slot_pt = at<int>(d_ws, w.slot_pt), *slot_elem = at<int>(d_ws, w.slot_elem);
    int *sorted2 = at<int>(d_ws, w.sorted2);
    double *res_r = at<double>(d_ws, w.res_r), *res_dist = at<double>(d_ws, w.res_dist);
    int *res_code = at<int>(d_ws, w.res_code), *tmp = at<int>(d_ws, w.scan_tmp);
    int *counters = at<int>(d_ws, w.counters);
    int *task_cell = at<int>(d_ws, w.task_cell), *task_elem = at<int>(d_ws, w.task_elem);
    int *task_elem2 = at<int>(d_ws, w.task_elem2);
    // the packed copy of the points: volume and surface meshes (the line
    // kernel reads the [D][n] coordinates)
    double *pts4 = m->R >= 2 ? at<double>(d_ws, w.pts4) : nullptr;
    double *start = at<double>(d_ws, w.start);
    int4 *park_meta = at<int4>(d_ws, w.park_meta);
    double *park_r = at<double>(d_ws, w.park_r);
    double *park_state = at<double>(d_ws, w.park_state);
    int *park_cnt = at<int>(d_ws, w.park_cnt), *park_off = at<int>(d_ws, w.park_off);
    int *park_choff = at<int>(d_ws, w.park_choff), *park_rank = at<int>(d_ws, w.park_rank);
    int *park_sorted = at<int>(d_ws, w.park_sorted), *park_task = at<int>(d_ws, w.park_task);
    int *olist = at<int>(d_ws, w.olist), *ov_int = at<int>(d_ws, w.ov_int);
    double *ov_dbl = at<double>(d_ws, w.ov_dbl);
    unsigned long long *stats = at<unsigned long long>(d_ws, w.stats);
    const int64_t nel = m->nel, ncell = w.ncell, tb = w.scan_blocks;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    {   // phases A and B: bin points by cell, candidates and primaries
        Span sp(m, 0, s);
        chk(launch_fill_i32(cell_cnt, ncell, 0, s));
        chk(launch_fill_i32(elem_cnt, nel, 0, s));
        chk(launch_fill_i32(elem_cnt2, nel, 0, s));
        chk(launch_fill_i32(elem_fill2, nel, 0, s));
        chk(launch_fill_i32(park_cnt, nel, 0, s));
        chk(launch_fill_i32(counters, kCounters, 0, s));
        if (rest) chk(launch_fill_i32(rest->count, 1, 0, s));
        chk(launch_fill_i32(reinterpret_cast<int *>(stats), 6 * kStats, 0, s));
        if (w.bin_shift >= 0) {
            int *bh = at<int>(d_ws, w.bin_hist);
            int2 *pairs = at<int2>(d_ws, w.bin_pairs);
            const int *npairs = bh + w.bin_hist_n;   // the scan's total
            chk(launch_bin_tiles(m, n, d_pts, pts4, keep, cellpt, cand, d_code, d_elem, d_r,
                                 d_dist, w.bin_shift, bh, s));
            chk(launch_exclusive_scan(bh, bh, w.bin_hist_n, 1, tmp, tb, s));
            chk(launch_bin_coarse(m, n, cellpt, w.bin_shift, bh, pairs, s));
            chk(launch_bin_rank(n, npairs, w.bin_shift, pairs, cell_cnt, rank, s));
            chk(launch_exclusive_scan(cell_cnt, cell_poff, ncell, 1, tmp, tb, s));
            chk(launch_exclusive_scan(cell_cnt, cell_choff, ncell, kChunk, tmp, tb, s));
            chk(launch_task_map(cell_choff, ncell, task_cell, s));
            chk(launch_bin_scatter(n, npairs, pairs, rank, cell_poff, pbin, m->cus, s));
        } else {
            chk(launch_cell_bin(m, 0, n, d_pts, pts4, keep, cellpt, cell_cnt, nullptr, rank,
                                nullptr, cand, d_code, d_elem, d_r, d_dist, s));
            chk(launch_exclusive_scan(cell_cnt, cell_poff, ncell, 1, tmp, tb, s));
            chk(launch_exclusive_scan(cell_cnt, cell_choff, ncell, kChunk, tmp, tb, s));
            chk(launch_task_map(cell_choff, ncell, task_cell, s));
            chk(launch_cell_bin(m, 1, n, d_pts, nullptr, keep, cellpt, nullptr, cell_poff, rank,
                                pbin, nullptr, d_code, d_elem, d_r, d_dist, s));
        }
        chk(launch_locate_cells(m, n, d_pts, pts4, pbin, cell_poff, cell_choff, ncell, task_cell,
                                w.tb_cell, cand, elem_cnt, rank, bin_prim, d_code,
                                d_elem, d_r, d_dist, s));
        chk(launch_exclusive_scan(elem_cnt, elem_off, nel, 1, tmp, tb, s));
        chk(launch_exclusive_scan(elem_cnt, chunk_off, nel, kChunk, tmp, tb, s));
        chk(launch_task_map(chunk_off, nel, task_elem, s));
        // the binned points number cell_poff[ncell]
        chk(launch_primary_scatter_bins(n, cell_poff + ncell, pbin, bin_prim, rank, elem_off,
                                        sorted, s));
    }
    {   // phase C: Newton on the primary candidates, results straight to the outputs
        NewtonIO io{sorted, elem_off, chunk_off, nullptr, d_code, d_elem, d_r, n, d_dist,
                    counters + kNewtonCounters, stats, task_elem, w.tb_elem, rs, n};
        io.pts4 = pts4;
        if (m->R >= 2) {
            io.start = start;
            io.start_stride = n;
            // pairs that reach a face leave the primary kernel's waves
            io.park_meta = park_meta;
            io.park_r = park_r;
            io.park_cap = n;
            io.park_count = counters + kParkCount;
            io.park_state = park_state;
            io.park_state_cap = w.park_state_cap;
            io.polish = precision == FPTS_MIXED && m->R == m->D;
        }
        {
            Span sp(m, 1, s);
            chk(launch_newton(m, precision, n, d_pts, io, 1, s));
        }
        {
            Span sp(m, 2, s);
            chk(launch_newton(m, precision, n, d_pts, io, 2, s));
        }
        if (m->R >= 2) {
            // the parked pairs, binned by element, go on in the face kernel
            Span sp(m, 7, s);
            chk(launch_park_bin(0, park_meta, counters + kParkCount, n, park_cnt, nullptr,
                                park_rank, nullptr, m->cus, s));
            chk(launch_exclusive_scan(park_cnt, park_off, nel, 1, tmp, tb, s));
            chk(launch_exclusive_scan(park_cnt, park_choff, nel, kChunk, tmp, tb, s));
            chk(launch_task_map(park_choff, nel, park_task, s));
            chk(launch_park_bin(1, park_meta, counters + kParkCount, n, nullptr, park_off,
                                park_rank, park_sorted, m->cus, s));
            NewtonIO fio{park_sorted, park_off, park_choff, nullptr, d_code, d_elem, d_r, n,
                         d_dist, nullptr, stats + 2 * kStats, park_task, w.tb_park, rs, n};
            fio.pts4 = pts4;
            fio.park_meta = park_meta;
            fio.park_r = park_r;
            fio.park_cap = n;
            fio.park_state = park_state;
            fio.park_state_cap = w.park_state_cap;
            chk(launch_newton(m, FPTS_FP64, n, d_pts, fio, 4, s));
        }
    }
    {   // phase D: other candidates of unsettled points, then the selection rule
        Span sp(m, 3, s);
        // counters[0]: listed points, counters[1]: slots handed out
        const EvalRest none{nullptr, nullptr, nullptr, 0};
        chk(launch_unsettled(m, n, cellpt, cand, d_code, d_r, ulist, counters,
                             rest ? *rest : none, s));
        unsigned long long *slot_total =
            reinterpret_cast<unsigned long long *>(counters + kSlotTotal);
        chk(launch_resolve(m, 0, n, d_pts, cellpt, cand, ulist, counters, uoff, ucnt,
                           slot_total, elem_cnt2, nullptr, nullptr, nullptr, nullptr, nullptr,
                           w.cap2, olist, counters + kOverflowCount, s));
        chk(launch_exclusive_scan(elem_cnt2, elem_off2, nel, 1, tmp, tb, s));
        chk(launch_exclusive_scan(elem_cnt2, chunk_off2, nel, kChunk, tmp, tb, s));
        chk(launch_task_map(chunk_off2, nel, task_elem2, s));
        chk(launch_resolve(m, 1, n, d_pts, cellpt, cand, ulist, counters, uoff, ucnt,
                           nullptr, nullptr, elem_off2, elem_fill2, slot_pt, slot_elem, sorted2,
                           w.cap2, nullptr, nullptr, s));
        NewtonIO io{sorted2, elem_off2, chunk_off2, slot_pt, res_code, nullptr, res_r, w.cap2,
                    res_dist, counters + 2 * kNewtonCounters, stats + kStats, task_elem2,
                    w.tb_elem2};
        io.pts4 = pts4;
        // the other candidates are few and near element faces: plain FP64
        // in both modes (an FP32 phase would not pay for its launches)
        chk(launch_newton(m, FPTS_FP64, n, d_pts, io, 3, s));
        chk(launch_select2(m, n, ulist, counters, uoff, ucnt, cand, slot_elem, w.cap2, res_r,
                           res_dist, res_code, d_code, d_elem, d_r, d_dist, s));
        if (m->R >= 2) {
            // points whose other candidates did not fit the slots (none in
            // the common case: the kernel reads the count and returns)
            NewtonIO oio{olist, nullptr, nullptr, nullptr, d_code, d_elem, d_r, n, d_dist,
                         nullptr, stats + kStats, nullptr, w.ov_grid};
            oio.pts4 = pts4;
            oio.ocount = counters + kOverflowCount;
            oio.cellpt = cellpt;
            oio.cand = cand;
            oio.ov_int = ov_int;
            oio.ov_dbl = ov_dbl;
            chk(launch_newton(m, FPTS_FP64, n, d_pts, oio, 8, s));
        }
    }
    if (m->profiling) m->prof_find++;
    return e == hipSuccess ? FPTS_OK : FPTS_EDEVICE;
}

}  // namespace fpts

extern "C" {

void fpts_params_default(fpts_params *p, int dim, int ref_dim, int nodes_1d, int64_t n_elem)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dim = dim;
    p->ref_dim = ref_dim;
    p->nodes_1d = nodes_1d;
    p->n_elem = n_elem;
    p->hash_n = 0;
    p->bbox_tol = 0.1;
    p->surf_eps_d = 1e-10;
    p->max_iter = 50;
    p->newton_tol = 1e-10;
    p->mixed_max_iter = 10;
    p->mixed_tol = 1e-3;
}

const char *fpts_status_string(int s)
{
    switch (s) {
    case FPTS_OK: return "ok";
    case FPTS_EINVAL: return "invalid argument";
    case FPTS_ENOMEM: return "out of memory";
    case FPTS_EDEVICE: return "HIP device error";
    case FPTS_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

int fpts_setup(const fpts_params *p, const double *h_nodes, void *stream, fpts_mesh **out)
{
    if (!p || !h_nodes || !out) return FPTS_EINVAL;
    *out = nullptr;
    const bool vol = p->ref_dim == p->dim && (p->dim == 2 || p->dim == 3);
    const bool surf = p->dim == 3 && p->ref_dim == 2;
    const bool line = p->ref_dim == 1 && (p->dim == 2 || p->dim == 3);
    if (!(vol || surf || line)) return FPTS_EINVAL;
    if (p->nodes_1d < 2 || p->nodes_1d > kMaxN) return FPTS_EINVAL;
    if (p->n_elem < 1 || p->n_elem > INT32_MAX / 2) return FPTS_EINVAL;
    if (!(p->bbox_tol >= 0.0) || !(p->newton_tol > 0.0) || p->max_iter < 1 ||
        p->max_iter > 1000 || !(p->surf_eps_d >= 0.0) || p->hash_n < 0 ||
        p->mixed_max_iter < 1 || p->mixed_max_iter > 1000 || !(p->mixed_tol > 0.0))
        return FPTS_EINVAL;
    if (sticky_error()) return FPTS_EDEVICE;
    fpts_mesh *m = new (std::nothrow) fpts_mesh();
    if (!m) return FPTS_ENOMEM;
    m->p = *p;
    m->D = p->dim;
    m->R = p->ref_dim;
    m->N = p->nodes_1d;
    m->NP = m->R == 3 ? m->N * m->N * m->N : m->R == 2 ? m->N * m->N : m->N;
    m->nel = p->n_elem;
    if (hipGetDevice(&m->device) != hipSuccess ||
        hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, m->device) !=
            hipSuccess) {
        delete m;
        return FPTS_EDEVICE;
    }
    // set-up of the allocation-free entry point: this device's scratch
    // address, looked up once with the device current
    if (!noalloc_scratch(m->device)) {
        delete m;
        return FPTS_EDEVICE;
    }
    int st;
    try {
        st = host_setup(m, h_nodes);
    } catch (const std::bad_alloc &) {
        st = FPTS_ENOMEM;
    }
    if (st != FPTS_OK) {
        delete m;
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nn = (size_t)m->nel * m->D * m->NP;
    const size_t nb = m->box.size(), nx = m->xc.size();
    m->near_npad = (m->NP + 31) / 32 * 32;
    const size_t nr = (size_t)m->nel * 4 * m->near_npad;
    bool ok = hipMalloc(&m->d_nodes, sizeof(double) * nn) == hipSuccess &&
              hipMalloc(&m->d_nodes32, sizeof(float) * nn) == hipSuccess &&
              hipMalloc(&m->d_near, sizeof(double) * nr) == hipSuccess &&
              hipMalloc(&m->d_xc, sizeof(double) * nx) == hipSuccess &&
              hipMalloc(&m->d_box, sizeof(double) * nb) == hipSuccess &&
              hipMalloc(&m->d_cell_off, sizeof(int) * m->cell_off.size()) == hipSuccess &&
              hipMalloc(&m->d_cell_el, sizeof(int) * m->cell_el.size()) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_mesh(m);
        return FPTS_ENOMEM;
    }
    ok = hipMemcpyAsync(m->d_nodes, h_nodes, sizeof(double) * nn, hipMemcpyHostToDevice, s) ==
             hipSuccess &&
         hipMemcpyAsync(m->d_xc, m->xc.data(), sizeof(double) * nx, hipMemcpyHostToDevice, s) ==
             hipSuccess &&
         hipMemcpyAsync(m->d_box, m->box.data(), sizeof(double) * nb, hipMemcpyHostToDevice,
                        s) == hipSuccess &&
         hipMemcpyAsync(m->d_cell_off, m->cell_off.data(), sizeof(int) * m->cell_off.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess &&
         hipMemcpyAsync(m->d_cell_el, m->cell_el.data(), sizeof(int) * m->cell_el.size(),
                        hipMemcpyHostToDevice, s) == hipSuccess &&
         launch_nodes32(m, s) == hipSuccess && launch_near_rows(m, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_mesh(m);
        return FPTS_EDEVICE;
    }
    *out = m;
    return FPTS_OK;
}

int fpts_destroy(fpts_mesh *m)
{
    if (!m) return FPTS_OK;
    (void)hipDeviceSynchronize();
    free_mesh(m);
    return FPTS_OK;
}

size_t fpts_find_workspace_size(const fpts_mesh *m, int64_t n)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return 0;
    FindWs w = find_ws_layout(m, n);
    if (w.cap2 > INT32_MAX) return 0;
    return w.total;
}

int fpts_find(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code, int32_t *d_elem,
              double *d_r, double *d_dist, int precision, void *d_ws, size_t ws_bytes,
              void *stream)
{
    return find_impl(m, n, d_pts, d_code, d_elem, d_r, d_dist, precision, d_ws, ws_bytes,
                     stream, nullptr, nullptr);
}

size_t fpts_eval_workspace_size(const fpts_mesh *m, int64_t n)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return 0;
    return eval_ws_layout(m, n).total;
}

int fpts_eval(fpts_mesh *m, int64_t n, const int32_t *d_code, const int32_t *d_elem,
              const double *d_r, int n_fields, const double *d_field, double *d_out, void *d_ws,
              size_t ws_bytes, void *stream)
{
    if (!m) return FPTS_EINVAL;
    return fpts_eval_order(m, n, d_code, d_elem, d_r, n_fields, m->N, d_field, d_out, d_ws,
                           ws_bytes, stream);
}

int fpts_eval_order(fpts_mesh *m, int64_t n, const int32_t *d_code, const int32_t *d_elem,
                    const double *d_r, int n_fields, int field_nodes_1d, const double *d_field,
                    double *d_out, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!m || n < 0 || n > INT32_MAX - 1 || n_fields < 1) return FPTS_EINVAL;
    if (field_nodes_1d < 2 || field_nodes_1d > kMaxN) return FPTS_EINVAL;
    if (n == 0) return FPTS_OK;
    if (!d_code || !d_elem || !d_r || !d_field || !d_out || !d_ws) return FPTS_EINVAL;
    if (((uintptr_t)d_ws & 255) != 0) return FPTS_EINVAL;
    const EvalWs w = eval_ws_layout(m, n);
    if (ws_bytes < w.total) return FPTS_EINVAL;
    if (sticky_error()) return FPTS_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    int *elem_cnt = at<int>(d_ws, w.elem_cnt);
    int *elem_off = at<int>(d_ws, w.elem_off);
    int *rank = at<int>(d_ws, w.rank);
    int *chunk_off = at<int>(d_ws, w.chunk_off);
    int *tmp = at<int>(d_ws, w.scan_tmp);
    int *sorted = at<int>(d_ws, w.sorted);
    int *task_elem = at<int>(d_ws, w.task_elem);
    const int64_t tb = scan_tmp_blocks(m->nel);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    {
        Span sp(m, 4, s);
        chk(launch_fill_i32(elem_cnt, m->nel, 0, s));
        chk(launch_eval_bin(m, 0, n, d_code, d_elem, nullptr, nullptr, n_fields, d_out, elem_cnt,
                            nullptr, rank, nullptr, s));
        chk(launch_exclusive_scan(elem_cnt, elem_off, m->nel, 1, tmp, tb, s));
        chk(launch_exclusive_scan(elem_cnt, chunk_off, m->nel, kChunk, tmp, tb, s));
        chk(launch_task_map(chunk_off, m->nel, task_elem, s));
        chk(launch_eval_bin(m, 1, n, d_code, d_elem, nullptr, nullptr, n_fields, d_out, nullptr,
                            elem_off,
                            rank, sorted, s));
    }
    {
        Span sp(m, 5, s);
        chk(launch_eval(m, n, d_r, n_fields, field_nodes_1d, d_field, d_out, sorted, elem_off,
                        chunk_off, task_elem, w.tb_elem, s));
    }
    if (m->profiling) m->prof_eval++;
    return e == hipSuccess ? FPTS_OK : FPTS_EDEVICE;
}

int fpts_find_stats_get(const fpts_mesh *m, int64_t n, const void *d_ws, int pass,
                        fpts_find_stats *out, void *stream)
{
    if (!m || !d_ws || !out || n < 0 || pass < 0 || pass > 3) return FPTS_EINVAL;
    const FindWs w = find_ws_layout(m, n);
    unsigned long long all[3 * kStats] = {0}, v[kStats] = {0};
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(all, static_cast<const char *>(d_ws) + w.stats, sizeof(all),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    int ctr[kCounters] = {0};
    if (hipMemcpyAsync(ctr, static_cast<const char *>(d_ws) + w.counters, sizeof(ctr),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    for (int k = 0; k < kStats; ++k)
        for (int q = 0; q < 3; ++q)
            if (pass == 0 || pass == q + 1) v[k] += all[q * kStats + k];
    out->overflow_points = ctr[kOverflowCount];
    out->parked_pairs = ctr[kParkCount];
    out->listed_points = ctr[0];
    out->pairs = (int64_t)v[0];
    out->passes = (int64_t)v[1];
    out->evals = (int64_t)v[2];
    out->evals_h2 = (int64_t)v[3];
    out->passes_fp32 = (int64_t)v[4];
    out->evals_fp32 = (int64_t)v[5];
    out->evals_h2_exec = (int64_t)v[6];
    out->sweeps = (int64_t)v[7];
    out->sweeps_h2 = (int64_t)v[8];
    out->sweeps_fp32 = (int64_t)v[9];
    out->evals_fp32_node = (int64_t)v[10];
    return FPTS_OK;
}

int fpts_profile(fpts_mesh *m, int enable)
{
    if (!m) return FPTS_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return FPTS_EDEVICE;
    clear_events(m);
    m->profiling = enable != 0;
    return FPTS_OK;
}

int fpts_profile_read(fpts_mesh *m, fpts_kernel_times *out)
{
    if (!m || !out) return FPTS_EINVAL;
    double ms[kSpans] = {0};
    for (int k = 0; k < kSpans; ++k)
        for (auto &pr : m->ev[k]) {
            float t = 0.0f;
            if (hipEventSynchronize(pr.second) != hipSuccess ||
                hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess)
                return FPTS_EDEVICE;
            ms[k] += t;
        }
    out->locate_ms = ms[0];
    out->nearest_ms = ms[1];
    out->newton_ms = ms[2];
    out->select_ms = ms[3];
    out->eval_bin_ms = ms[4];
    out->eval_ms = ms[5];
    out->advance_ms = ms[6];
    out->face_ms = ms[7];
    out->find_calls = m->prof_find;
    out->eval_calls = m->prof_eval;
    out->lpt_calls = m->prof_lpt;
    const bool on = m->profiling;
    clear_events(m);
    m->profiling = on;
    return FPTS_OK;
}

int fpts_update_nodes(fpts_mesh *m, const double *d_nodes, void *stream)
{
    if (!m || !d_nodes) return FPTS_EINVAL;
    if (sticky_error()) return FPTS_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const size_t nn = (size_t)m->nel * m->D * m->NP;
    if (d_nodes != m->d_nodes &&
        hipMemcpyAsync(m->d_nodes, d_nodes, sizeof(double) * nn, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
        return FPTS_EDEVICE;
    const int st = device_setup(m, s);
    if (st != FPTS_OK) return st;
    if (launch_nodes32(m, s) != hipSuccess || launch_near_rows(m, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    return FPTS_OK;
}

int fpts_get_boxes(const fpts_mesh *m, double *h_aabb, double *h_obb_A, double *h_obb_c)
{
    if (!m) return FPTS_EINVAL;
    const int D = m->D, W = box_words(D);
    for (int64_t e = 0; e < m->nel; ++e) {
        const double *rec = &m->box[(size_t)e * W];
        for (int d = 0; d < D; ++d) {
            if (h_aabb) {
                h_aabb[((size_t)e * D + d) * 2] = rec[d];
                h_aabb[((size_t)e * D + d) * 2 + 1] = rec[D + d];
            }
            if (h_obb_c) h_obb_c[(size_t)e * D + d] = rec[2 * D + d];
        }
        if (h_obb_A)
            for (int a = 0; a < D * D; ++a) h_obb_A[(size_t)e * D * D + a] = rec[3 * D + a];
    }
    return FPTS_OK;
}

int fpts_get_hash(const fpts_mesh *m, double *h_lo, double *h_hi, double *h_delta, int *hash_n,
                  int64_t *nnz, int *max_cell)
{
    if (!m) return FPTS_EINVAL;
    for (int d = 0; d < m->D; ++d) {
        if (h_lo) h_lo[d] = m->hlo[d];
        if (h_hi) h_hi[d] = m->hhi[d];
        if (h_delta) h_delta[d] = m->hdel[d];
    }
    if (hash_n) *hash_n = m->NL;
    if (nnz) *nnz = (int64_t)m->cell_off.back();
    if (max_cell) *max_cell = m->max_cell;
    return FPTS_OK;
}

int fpts_get_cells(const fpts_mesh *m, int32_t *h_cell_off, int32_t *h_cell_el)
{
    if (!m) return FPTS_EINVAL;
    if (h_cell_off)
        std::copy(m->cell_off.begin(), m->cell_off.end(), h_cell_off);
    if (h_cell_el)
        std::copy(m->cell_el.begin(), m->cell_el.begin() + m->cell_off.back(), h_cell_el);
    return FPTS_OK;
}


size_t fpts_lpt_workspace_size(const fpts_mesh *m, int64_t n)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return 0;
    const size_t fw = fpts_find_workspace_size(m, n);
    if (fw == 0) return 0;
    const size_t ew = eval_ws_layout(m, n).total;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    return align_up(sizeof(double) * (size_t)m->D * nn) + align_up(sizeof(int) * nn) +
           std::max(fw, ew);
}

int fpts_lpt_step(fpts_mesh *m, const fpts_lpt_params *p, int64_t n, int first, double *d_x,
                  double *d_v, double *d_hist, const double *d_field, int32_t *d_code,
                  int32_t *d_elem, double *d_r, double *d_dist, int precision, void *d_ws,
                  size_t ws_bytes, void *stream)
{
    if (!m || !p || n < 0 || n > INT32_MAX - 1 || m->R != m->D) return FPTS_EINVAL;
    if (!(std::isfinite(p->tau) && p->tau > 0) || !(std::isfinite(p->dt) && p->dt > 0))
        return FPTS_EINVAL;
    for (int d = 0; d < m->D; ++d)
        if (!(std::isfinite(p->lo[d]) && std::isfinite(p->hi[d]) && p->lo[d] < p->hi[d]) ||
            (p->periodic[d] != 0 && p->periodic[d] != 1))
            return FPTS_EINVAL;
    if (precision != FPTS_FP64 && precision != FPTS_MIXED) return FPTS_EINVAL;
    if (n == 0) return FPTS_OK;
    if (!d_x || !d_v || !d_hist || !d_field || !d_code || !d_elem || !d_r || !d_dist || !d_ws)
        return FPTS_EINVAL;
    if (((uintptr_t)d_ws & 255) != 0) return FPTS_EINVAL;
    const size_t need = fpts_lpt_workspace_size(m, n);
    if (need == 0 || ws_bytes < need) return FPTS_EINVAL;
    if (sticky_error()) return FPTS_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    // [D][n] interpolated fluid velocity, [n] keep flags of the hinted
    // search, then the Find / Interpolate space
    const size_t u_bytes = align_up(sizeof(double) * (size_t)m->D * (size_t)n);
    const size_t k_bytes = align_up(sizeof(int) * (size_t)n);
    double *u = static_cast<double *>(d_ws);
    int *keep = at<int>(d_ws, u_bytes);
    void *sub = static_cast<char *>(d_ws) + u_bytes + k_bytes;
    const size_t sub_bytes = ws_bytes - u_bytes - k_bytes;
    int st = fpts_eval(m, n, d_code, d_elem, d_r, m->D, d_field, u, sub, sub_bytes, stream);
    if (st != FPTS_OK) return st;
    LptArgs a;
    a.x = d_x;
    a.v = d_v;
    a.hist_v = d_hist;
    a.hist_a = d_hist + (size_t)m->D * (size_t)n;
    a.u = u;
    a.code = d_code;
    a.n = n;
    a.tau = p->tau;
    a.dt = p->dt;
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = d < m->D ? p->lo[d] : 0.0;
        a.hi[d] = d < m->D ? p->hi[d] : 1.0;
        a.periodic[d] = d < m->D ? p->periodic[d] : 0;
    }
    a.first = first != 0;
    hipError_t e;
    {
        Span sp(m, 6, s);
        e = launch_lpt_advance(m, a, s);
    }
    if (e != hipSuccess) return FPTS_EDEVICE;
    if (m->profiling) m->prof_lpt++;
    if (!p->hint)
        return find_impl(m, n, d_x, d_code, d_elem, d_r, d_dist, precision, sub, sub_bytes,
                         stream, nullptr, nullptr);
    // Hinted search: a particle whose last code was INTERIOR is first searched
    // in its previous element from its previous r; the full search then
    // skips the particles that this settled.
    const FindWs w = find_ws_layout(m, n);
    int2 *cand = at<int2>(sub, w.cand);
    int *elem_cnt = at<int>(sub, w.elem_cnt);
    int *rank = at<int>(sub, w.rank), *elem_off = at<int>(sub, w.elem_off);
    int *chunk_off = at<int>(sub, w.chunk_off), *sorted = at<int>(sub, w.sorted);
    int *task_elem = at<int>(sub, w.task_elem), *tmp = at<int>(sub, w.scan_tmp);
    int *counters = at<int>(sub, w.counters);
    unsigned long long *stats = at<unsigned long long>(sub, w.stats);
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    {
        Span sp(m, 0, s);
        chk(launch_fill_i32(elem_cnt, m->nel, 0, s));
        chk(launch_fill_i32(counters, kCounters, 0, s));
        chk(launch_fill_i32(reinterpret_cast<int *>(stats), 6 * kStats, 0, s));
        chk(launch_hint(m, 0, n, d_code, d_elem, d_r, cand, elem_cnt, rank, nullptr, s));
        chk(launch_exclusive_scan(elem_cnt, elem_off, m->nel, 1, tmp, w.scan_blocks, s));
        chk(launch_exclusive_scan(elem_cnt, chunk_off, m->nel, kChunk, tmp, w.scan_blocks, s));
        chk(launch_task_map(chunk_off, m->nel, task_elem, s));
        chk(launch_primary_scatter(n, m->nel, cand, elem_off, rank, sorted, s));
    }
    {
        Span sp(m, 2, s);
        // a particle that left its element walks to the face and on: a few
        // passes tell, and the full Find takes it (kHintPasses; a warm
        // start converges in three or four)
        NewtonIO io{sorted, elem_off, chunk_off, nullptr, d_code, d_elem, d_r, n, d_dist,
                    counters + kNewtonCounters, stats, task_elem, w.tb_elem, nullptr, 0,
                    keep, kHintPasses};
        chk(launch_newton(m, precision, n, d_x, io, 2, s));
        chk(launch_hint(m, 1, n, d_code, d_elem, d_r, cand, nullptr, nullptr, keep, s));
    }
    if (e != hipSuccess) return FPTS_EDEVICE;
    return find_impl(m, n, d_x, d_code, d_elem, d_r, d_dist, precision, sub, sub_bytes, stream,
                     keep, nullptr);
}

size_t fpts_find_eval_workspace_size(const fpts_mesh *m, int64_t n)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return 0;
    const size_t fw = fpts_find_workspace_size(m, n);
    if (fw == 0) return 0;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    return fw + align_up(eval_ws_layout(m, n).total) +
           align_up(sizeof(double) * (size_t)m->R * nn);
}

int fpts_find_eval(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code,
                   int32_t *d_elem, double *d_r, double *d_dist, int precision, int n_fields,
                   int field_nodes_1d, const double *d_field, double *d_out, void *d_ws,
                   size_t ws_bytes, void *stream)
{
    if (!m || n < 0 || n > INT32_MAX - 1 || n_fields < 1) return FPTS_EINVAL;
    if (field_nodes_1d < 2 || field_nodes_1d > kMaxN) return FPTS_EINVAL;
    if (precision != FPTS_FP64 && precision != FPTS_MIXED) return FPTS_EINVAL;
    if (n == 0) return FPTS_OK;
    if (!d_pts || !d_code || !d_elem || !d_r || !d_dist || !d_field || !d_out || !d_ws)
        return FPTS_EINVAL;
    if (((uintptr_t)d_ws & 255) != 0) return FPTS_EINVAL;
    const size_t need = fpts_find_eval_workspace_size(m, n);
    if (need == 0 || ws_bytes < need) return FPTS_EINVAL;
    // [find workspace][interpolation workspace][R][n] results in list order
    const FindWs w = find_ws_layout(m, n);
    const EvalWs v = eval_ws_layout(m, n);
    void *ews = static_cast<char *>(d_ws) + w.total;
    double *rs = at<double>(d_ws, w.total + align_up(v.total));
    // volume and surface meshes: the points left for the second
    // interpolation pass are listed by the find's marking pass (in slist,
    // which only the line-mesh path uses otherwise)
    const bool listed = m->R >= 2;
    const EvalRest rest{at<int>(ews, v.slist), at<int>(ews, v.scount), d_out, n_fields};
    int st = find_impl(m, n, d_pts, d_code, d_elem, d_r, d_dist, precision, d_ws, w.total,
                       stream, nullptr, rs, listed ? &rest : nullptr);
    if (st != FPTS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int2 *cand = at<int2>(d_ws, w.cand);
    const int *sorted = at<int>(d_ws, w.sorted);
    const int *elem_off = at<int>(d_ws, w.elem_off), *chunk_off = at<int>(d_ws, w.chunk_off);
    const int *task_elem = at<int>(d_ws, w.task_elem);
    int *elem_cnt = at<int>(ews, v.elem_cnt), *erank = at<int>(ews, v.rank);
    int *eoff = at<int>(ews, v.elem_off), *choff = at<int>(ews, v.chunk_off);
    int *tmp = at<int>(ews, v.scan_tmp), *esorted = at<int>(ews, v.sorted);
    int *etask = at<int>(ews, v.task_elem);
    int *slist = at<int>(ews, v.slist), *scount = at<int>(ews, v.scount);
    const int64_t tb = scan_tmp_blocks(m->nel);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    {
        // points the primary pass settled: Find's own element buckets, r in
        // list order (no re-binning, no gather of r)
        Span sp(m, 5, s);
        chk(launch_eval(m, n, nullptr, n_fields, field_nodes_1d, d_field, d_out, sorted,
                        elem_off, chunk_off, task_elem, w.tb_elem, s, rs));
    }
    {
        // the rest (settled by the second search, BORDER, NOT_FOUND): the
        // plain interpolation path restricted to them.  They are few and
        // scattered; on line meshes, elements holding at most a few of them
        // have their points interpolated one lane per point (the per-lane
        // arithmetic of the element tasks); the other meshes interpolate
        // every point on the matrix cores, as fpts_eval does, so both calls
        // give the same bits
        const bool split = m->R == 1;
        Span sp(m, 4, s);
        chk(launch_fill_i32(elem_cnt, m->nel, 0, s));
        if (listed) {
            chk(launch_eval_bin_list(m, 0, slist, scount, n, d_elem, elem_cnt, nullptr, erank,
                                     nullptr, s));
        } else {
            chk(launch_fill_i32(scount, 1, 0, s));
            chk(launch_eval_bin(m, 0, n, d_code, d_elem, d_r, cand, n_fields, d_out, elem_cnt,
                                nullptr, erank, nullptr, s));
        }
        if (split)
            chk(launch_eval_split(m, n, d_elem, erank, elem_cnt, nullptr, nullptr, nullptr,
                                  nullptr, 0, s));
        chk(launch_exclusive_scan(elem_cnt, eoff, m->nel, 1, tmp, tb, s));
        chk(launch_exclusive_scan(elem_cnt, choff, m->nel, kChunk, tmp, tb, s));
        chk(launch_task_map(choff, m->nel, etask, s));
        if (split)
            chk(launch_eval_split(m, n, d_elem, erank, elem_cnt, eoff, esorted, slist, scount, 1,
                                  s));
        else if (listed)
            chk(launch_eval_bin_list(m, 1, slist, scount, n, d_elem, nullptr, eoff, erank,
                                     esorted, s));
        else
            chk(launch_eval_bin(m, 1, n, d_code, d_elem, d_r, cand, n_fields, d_out, nullptr,
                                eoff, erank, esorted, s));
    }
    {
        Span sp(m, 5, s);
        chk(launch_eval(m, n, d_r, n_fields, field_nodes_1d, d_field, d_out, esorted, eoff,
                        choff, etask, v.tb_elem, s));
        if (m->R == 1)
            chk(launch_eval_sparse(m, n, d_r, n_fields, field_nodes_1d, d_field, d_out, d_elem,
                                   slist, scount, s));
    }
    if (m->profiling) m->prof_eval++;
    return e == hipSuccess ? FPTS_OK : FPTS_EDEVICE;
}

int fpts_find_eval_noalloc(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code,
                           int32_t *d_elem, double *d_r, double *d_dist, int precision,
                           int n_fields, int field_nodes_1d, const double *d_field,
                           double *d_out, void *stream)
{
    if (!m || n < 0 || n > INT32_MAX - 1) return FPTS_EINVAL;
    const size_t need = fpts_find_eval_workspace_size(m, n);
    if (need == 0) return FPTS_EINVAL;
    if (need > (size_t)FPTS_NOALLOC_SCRATCH_BYTES) return FPTS_ENOMEM;
    void *ws = m->device >= 0 && m->device < kMaxDevices ? noalloc_ptr[m->device] : nullptr;
    if (!ws) return FPTS_EDEVICE;
    return fpts_find_eval(m, n, d_pts, d_code, d_elem, d_r, d_dist, precision, n_fields,
                          field_nodes_1d, d_field, d_out, ws, need, stream);
}

}  // extern "C"
