// Find, outside Newton (Section 3.2): points are binned by cell of the local
// map (Section 3.1.3); each cell's candidates are tested with the AABB and
// OBB tests (eqs. eq_AABB_test, eq_OBB_test); the primary candidate of each
// point is bucketed by element for Newton; points the primary does not
// settle get their other candidates in a second pass and the selection rule
// of Section 3.2.  Also the int32 exclusive scan and fill kernels used by
// find and eval.
#include "fpts_internal.hpp"

namespace fpts {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_fill_i32(int *p, int64_t count, int value)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

__device__ inline int scan_in(const int *in, int64_t i, int64_t n, int ceil_div)
{
    if (i >= n) return 0;
    int v = in[i];
    return ceil_div > 1 ? (v + ceil_div - 1) / ceil_div : v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ inline int block_exclusive(int v, int &excl)
{
    __shared__ int warp_tot[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) warp_tot[wid] = incl;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        int t = warp_tot[w];
        if (w < wid) base += t;
        total += t;
    }
    __syncthreads();
    excl = base + incl - v;
    return total;
}

// Pass 1: per tile, local exclusive scan into out and the tile total.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int *in, int *out, int64_t n,
                                                            int ceil_div, int *tile_sum)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = scan_in(in, base + k, n, ceil_div);
        s += v[k];
    }
    int excl;
    int tot = block_exclusive(s, excl);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = excl;
        excl += v[k];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Pass 2: one block scans the tile totals (exclusive) and writes the grand
// total to out[n].
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int *tile_sum, int64_t tiles, int *out,
                                                           int64_t n)
{
    int carry = 0;
    for (int64_t b = 0; b < tiles; b += kScanThreads) {
        int64_t i = b + threadIdx.x;
        int v = i < tiles ? tile_sum[i] : 0;
        int excl;
        int tot = block_exclusive(v, excl);
        if (i < tiles) tile_sum[i] = carry + excl;
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

// Pass 3: add the tile offsets.
__global__ __launch_bounds__(kScanThreads) void k_scan_add(int *out, int64_t n, const int *tile_sum)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int add = tile_sum[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads) {
        int64_t i = base + k;
        if (i < n) out[i] += add;
    }
}

// Cell of x in the local map, or -1 when x is not finite or outside the
// union of the boxes.  Same operations as the host registration of element
// boxes (subtract, divide, floor, clamp), so a point inside an element's AABB
// always lands in a cell that lists the element.
template <int D>
__device__ inline int cell_of(const HashView &h, const double *x)
{
    int cell = 0, mul = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (!__builtin_isfinite(x[d]) || !(x[d] >= h.lo[d] && x[d] <= h.hi[d])) return -1;
        double t = floor((x[d] - h.lo[d]) / h.del[d]);
        t = fmin(fmax(t, 0.0), (double)(h.NL - 1));
        cell += mul * (int)t;
        mul *= h.NL;
    }
    return cell;
}

typedef const __attribute__((address_space(4))) double cdouble;

__device__ inline void write_not_found(int p, int n, int R, int32_t *code, int32_t *elem,
                                       double *r, double *dist)
{
    code[p] = FPTS_NOT_FOUND;
    elem[p] = -1;
    dist[p] = __builtin_huge_val();
    for (int a = 0; a < R; ++a) r[(size_t)a * n + p] = 0.0;
}

// Phase A for one point: its cell (-1 for a kept point, whose result is
// already final, and for a point outside the map), the packed copy of its
// coordinates (pts4 not null), defined candidate data, and NOT_FOUND for a
// point outside the map.
template <int D>
__device__ inline int bin_point(const HashView &h, int p, int n, int R, const double *pts,
                                double *pts4, const int *keep, int *cellpt, int2 *cand,
                                int32_t *code, int32_t *elem, double *r, double *dist)
{
    int c = -1;
    const bool kept = keep && keep[p];
    if (!kept) {
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = pts[(size_t)d * n + p];
        c = cell_of<D>(h, x);
        if (pts4) {
            // the packed copy (one cache line per point for the kernels that
            // visit points in bucket order)
            typedef double v2 __attribute__((ext_vector_type(2)));
            v2 *o = reinterpret_cast<v2 *>(pts4 + (size_t)p * pt_stride(D));
            o[0] = v2{x[0], x[1]};
            if (D == 3) o[1] = v2{x[D - 1], 0.0};
        }
    }
    cellpt[p] = c;
    cand[p] = make_int2(0, -1);
    if (c < 0 && !kept) write_not_found(p, n, R, code, elem, r, dist);
    return c;
}

// Phase A with one atomic per point (meshes with more than kBinMaxCells
// cells).  pass 0: bin_point and the count per cell; pass 1: scatter point
// ids into their cell's bucket.
template <int D>
__global__ __launch_bounds__(256) void k_cell_bin(HashView h, int pass, int n, int R,
                                                 const double *pts, double *pts4, const int *keep,
                                                 int *cellpt, int *cell_cnt,
                                                 const int *cell_poff, int *rank,
                                                 int *pbin, int2 *cand, int32_t *code,
                                                 int32_t *elem, double *r, double *dist)
{
    // no early exit: wave_inc needs every lane
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < n;
    if (pass == 0) {
        const int c =
            in ? bin_point<D>(h, p, n, R, pts, pts4, keep, cellpt, cand, code, elem, r, dist) : -1;
        const int k = wave_inc(cell_cnt, c, c >= 0);
        if (c >= 0) rank[p] = k;
    } else {
        const int c = in ? cellpt[p] : -1;
        if (c >= 0) pbin[cell_poff[c] + rank[p]] = p;
    }
}

// Phase A without per-point atomics.  Points arrive in any order (uniformly
// random in the benchmarks), so a count per cell by atomics costs one
// device atomic per point (about 26 G/s on this GPU) and the scatter into
// cell buckets one write at a random place per point.  Instead the cells
// are grouped into coarse buckets of 2^shift consecutive cells (at most
// kBinMaxBuckets buckets):
//  tiles:   per tile of kBinTile points, bin_point and the tile's histogram
//           over the buckets (LDS atomics), stored bucket-major in bh; an
//           exclusive scan of bh gives each (bucket, tile) its range;
//  coarse:  each tile writes its points as (cell, id) pairs into those
//           ranges: pairs sorted by bucket, one short run per (tile, bucket);
//  rank:    windows of kBinTile consecutive pairs (cells of at most two
//           buckets, unless the buckets are sparse) count their cells in LDS
//           and take one atomic per cell on cell_cnt for a block of ranks;
//  scatter: after the scan of cell_cnt, pbin[cell_poff[c] + rank] = id in
//           pair order, so a window's writes fall in the cells of one or two
//           buckets.
// The scatter's ranges go to the XCDs in contiguous blocks (task_of_block),
// so that an XCD's writes stay within a few buckets and partly written cache
// lines meet in one L2 (the same mapping for the tiles measured slower).
constexpr int kBinThreads = 256;
constexpr int kBinItems = 32;
constexpr int kBinTile = kBinThreads * kBinItems;

template <int D>
__global__ __launch_bounds__(kBinThreads) void k_bin_tiles(HashView h, int n, int R,
                                                          const double *pts, double *pts4,
                                                          const int *keep, int *cellpt,
                                                          int2 *cand,
                                                          int32_t *code, int32_t *elem, double *r,
                                                          double *dist, int shift, int nb,
                                                          int ntile, int *bh)
{
    extern __shared__ int hist[];   // [nb]
    const int tile = blockIdx.x;
    for (int i = threadIdx.x; i < nb; i += kBinThreads) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)tile * kBinTile;
    for (int k = 0; k < kBinItems; ++k) {
        const int64_t q = base + (int64_t)k * kBinThreads + threadIdx.x;
        if (q < n) {
            const int c = bin_point<D>(h, (int)q, n, R, pts, pts4, keep, cellpt, cand, code,
                                       elem, r, dist);
            if (c >= 0) atomicAdd(&hist[c >> shift], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kBinThreads)
        bh[(int64_t)i * ntile + tile] = hist[i];
}

__global__ __launch_bounds__(kBinThreads) void k_bin_coarse(int n, const int *cellpt, int shift,
                                                           int nb, int ntile, const int *boff,
                                                           int2 *pairs)
{
    extern __shared__ int off[];   // [nb] next free place of each bucket's range
    const int tile = blockIdx.x;
    for (int i = threadIdx.x; i < nb; i += kBinThreads)
        off[i] = boff[(int64_t)i * ntile + tile];
    __syncthreads();
    const int64_t base = (int64_t)tile * kBinTile;
    for (int k = 0; k < kBinItems; ++k) {
        const int64_t q = base + (int64_t)k * kBinThreads + threadIdx.x;
        if (q < n) {
            const int c = cellpt[q];
            if (c >= 0) pairs[atomicAdd(&off[c >> shift], 1)] = make_int2(c, (int)q);
        }
    }
}

__global__ __launch_bounds__(kBinThreads) void k_bin_rank(const int *total_p, int shift,
                                                         const int2 *pairs, int *cell_cnt,
                                                         int *rank)
{
    extern __shared__ int cnt[];   // [2 << shift] cells of buckets hA, hA + 1
    const int total = *total_p;
    const int64_t w0 = (int64_t)task_of_block() * kBinTile;
    if (w0 >= total) return;   // the whole block
    const int w1 = (int)(w0 + kBinTile < total ? w0 + kBinTile : total);
    const int hA = pairs[w0].x >> shift, hB = pairs[w1 - 1].x >> shift;
    if (hB - hA > 1) {
        // sparse buckets: few pairs per cell, one atomic each
        for (int64_t i = w0 + threadIdx.x; i < w1; i += kBinThreads)
            rank[i] = atomicAdd(&cell_cnt[pairs[i].x], 1);
        return;
    }
    const int c0 = hA << shift, nbin = 2 << shift;
    for (int i = threadIdx.x; i < nbin; i += kBinThreads) cnt[i] = 0;
    __syncthreads();
    int bin[kBinItems], lr[kBinItems];
#pragma unroll
    for (int k = 0; k < kBinItems; ++k) {
        const int64_t i = w0 + (int64_t)k * kBinThreads + threadIdx.x;
        bin[k] = 0;
        lr[k] = 0;
        if (i < w1) {
            bin[k] = pairs[i].x - c0;
            lr[k] = atomicAdd(&cnt[bin[k]], 1);
        }
    }
    __syncthreads();
    // the window's block of ranks in each of its cells
    for (int j = threadIdx.x; j < nbin; j += kBinThreads) {
        const int v = cnt[j];
        if (v > 0) cnt[j] = atomicAdd(&cell_cnt[c0 + j], v);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBinItems; ++k) {
        const int64_t i = w0 + (int64_t)k * kBinThreads + threadIdx.x;
        if (i < w1) rank[i] = cnt[bin[k]] + lr[k];
    }
}

__global__ __launch_bounds__(kBinThreads) void k_bin_scatter(const int *total_p, const int2 *pairs,
                                                            const int *rank,
                                                            const int *cell_poff, int *pbin)
{
    const int64_t total = *total_p;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;   // pairs per block
    const int64_t b0 = task_of_block() * per, b1 = b0 + per < total ? b0 + per : total;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kBinThreads) {
        const int2 cp = pairs[i];
        pbin[cell_poff[cp.x] + rank[i]] = cp.y;
    }
}

// task -> unit map: the tasks of unit u are chunk_off[u] .. chunk_off[u+1]-1
__global__ __launch_bounds__(256) void k_task_map(const int *chunk_off, int nunit,
                                                 int *task_unit)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nunit) return;
    for (int t = chunk_off[u]; t < chunk_off[u + 1]; ++t) task_unit[t] = u;
}

// Phase B: one wavefront per task of up to 64 points of one cell (task
// grid); every lane tests its own point against the cell's candidates.  The
// candidates' box records are loaded into registers with vector loads, up to
// kLocChunk at a time (lane j holds the first half of candidate j's record,
// lane 32 + j the second), and each candidate's record is then broadcast to
// scalar registers with lane reads.  A task's inputs come through dependent
// loads (task -> cell -> point ids and candidate ids -> coordinates and
// records): those of the wave's next task are issued while the current one
// is tested, level by level, so that their latency hides behind the tests.
// Per point: number of candidates, primary candidate (smallest OBB depth,
// lowest id on ties), and the primary's bucket count.
constexpr int kLocChunk = 32;

__device__ __forceinline__ double read_lane(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

template <int D, bool PACKED>
__global__ __launch_bounds__(64) void k_locate_cells(HashView h, int n, int R, const double *pts,
                                                    const double *pts4,
                                                    const int *pbin, const int *cell_poff,
                                                    const int *cell_choff, int ncell,
                                                    const int *task_cell, int2 *cand,
                                                    int *elem_cnt, int *rank,
                                                    int *bin_prim, int32_t *code, int32_t *elem,
                                                    double *r, double *dist)
{
    constexpr int RS = 3 * D + D * D;   // doubles per box record
    constexpr int HR = (RS + 1) / 2;    // record doubles per lane (half a record)
    const int lane = threadIdx.x;
    const int total = cell_choff[ncell];
    const int G = gridDim.x;
    struct Task {
        int c, beg, end, q0, q1;
    };
    // level 1: the task's cell, its points' range and its candidates' range
    auto task_of = [&](int t) __attribute__((always_inline)) {
        Task k;
        k.c = __builtin_amdgcn_readfirstlane(task_cell[t]);
        k.beg = cell_poff[k.c] + (t - cell_choff[k.c]) * kChunk;
        k.end = min(cell_poff[k.c + 1], k.beg + kChunk);
        k.q0 = __builtin_amdgcn_readfirstlane(h.cell_off[k.c]);
        k.q1 = __builtin_amdgcn_readfirstlane(h.cell_off[k.c + 1]);
        return k;
    };
    // level 2: this lane's point id and candidate id (candidate qb + lane % 32)
    auto ids_of = [&](const Task &k, int qb, int &p, int &mine) __attribute__((always_inline)) {
        p = k.beg + lane < k.end ? pbin[k.beg + lane] : 0;
        const int j = lane & (kLocChunk - 1);
        mine = j < min(kLocChunk, k.q1 - qb) ? h.cell_el[qb + j] : 0;
    };
    // level 3: the point's coordinates and this lane's half record
    auto data_of = [&](const Task &k, int qb, int p, int mine, double (&x)[D],
                       double (&rv)[HR]) __attribute__((always_inline)) {
        const bool has = k.beg + lane < k.end;
#pragma unroll
        for (int d = 0; d < D; ++d)
            x[d] = !has    ? 0.0
                   : PACKED ? pts4[(size_t)p * pt_stride(D) + d]
                            : pts[(size_t)d * n + p];
        const bool live = (lane & (kLocChunk - 1)) < min(kLocChunk, k.q1 - qb);
        const int f0 = (lane >> 5) * HR;
        const double *src = h.box + (size_t)mine * RS + f0;
#pragma unroll
        for (int u = 0; u < HR; ++u) rv[u] = (live && f0 + u < RS) ? src[u] : 0.0;
    };
    int t = task_of_block();
    if (t >= total) return;
    Task cur = task_of(t);
    int p, mine;
    double x[D], rv[HR];
    ids_of(cur, cur.q0, p, mine);
    data_of(cur, cur.q0, p, mine, x, rv);
    for (;;) {
        const int tn = t + G;
        const bool more = tn < total;
        Task nxt = cur;
        if (more) nxt = task_of(tn);   // next task, level 1
        int pn = 0, minen = 0;
        double xn[D], rvn[HR];
        bool l2 = !more, l3 = !more;
        const bool has = cur.beg + lane < cur.end;
        int cnt = 0, prim = -1;
        double best = __builtin_huge_val();
        for (int qb = cur.q0; qb < cur.q1; qb += kLocChunk) {
            const int nb = min(kLocChunk, cur.q1 - qb);
            if (qb != cur.q0) {
                // more candidates than one chunk: the next chunk, loaded now
                int pq;
                double xq[D];
                ids_of(cur, qb, pq, mine);
                data_of(cur, qb, pq, mine, xq, rv);
            }
            if (!l2) {
                ids_of(nxt, nxt.q0, pn, minen);   // next task, level 2
                l2 = true;
            }
            for (int j = 0; j < nb; ++j) {
                if (!l3 && j == nb / 2) {
                    data_of(nxt, nxt.q0, pn, minen, xn, rvn);   // next task, level 3
                    l3 = true;
                }
                // candidate j's record, broadcast to scalar registers: the
                // AABB first; when no point of the wave lies inside it (a
                // box that only grazes the cell) the OBB part is neither
                // read nor tested
                double rec[RS];
#pragma unroll
                for (int f = 0; f < 2 * D; ++f) rec[f] = read_lane(rv[f % HR], j + 32 * (f / HR));
                const bool in = has && aabb_in<D>(rec, x);
                if (!__ballot(in)) continue;
#pragma unroll
                for (int f = 2 * D; f < RS; ++f) rec[f] = read_lane(rv[f % HR], j + 32 * (f / HR));
                const int e = __builtin_amdgcn_readlane(mine, j);
                const double depth = obb_depth<D>(rec, x);
                if (in && depth <= 1.0) {
                    ++cnt;
                    if (depth < best) {
                        best = depth;
                        prim = e;
                    }
                }
            }
        }
        if (!l2) ids_of(nxt, nxt.q0, pn, minen);   // a cell without candidates
        if (!l3) data_of(nxt, nxt.q0, pn, minen, xn, rvn);
        if (has) {
            cand[p] = make_int2(cnt, prim);   // one scattered write per point
            if (prim < 0) write_not_found(p, n, R, code, elem, r, dist);
        }
        const int k = wave_inc(elem_cnt, prim, has && prim >= 0);
        // primary and rank in bin order (coalesced), for the scatter by bins
        if (has) {
            bin_prim[cur.beg + lane] = prim;
            rank[cur.beg + lane] = k;
        }
        if (!more) break;
        t = tn;
        cur = nxt;
        p = pn;
        mine = minen;
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = xn[d];
#pragma unroll
        for (int u = 0; u < HR; ++u) rv[u] = rvn[u];
    }
}

__global__ __launch_bounds__(256) void k_primary_scatter(int n, int nel, const int2 *cand,
                                                        const int *elem_off, const int *rank,
                                                        int *sorted)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = p < n ? cand[p].y : -1;
    if (e >= 0 && e < nel) sorted[elem_off[e] + rank[p]] = p;
}

// Primary buckets from the bin-ordered output of k_locate_cells: the point
// at bin position i goes to sorted[elem_off[bin_prim[i]] + rank[i]].
__global__ __launch_bounds__(256) void k_primary_scatter_bins(int n, const int *nbinned,
                                                             const int *pbin,
                                                             const int *bin_prim,
                                                             const int *rank,
                                                             const int *elem_off, int *sorted)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || i >= *nbinned) return;
    const int e = bin_prim[i];
    if (e >= 0) sorted[elem_off[e] + rank[i]] = pbin[i];
}

// A primary result settles the point when it is INTERIOR at least `guard`
// inside the reference box: no other element can then hold the point in its
// interior (it would overlap the primary), so the paper's rule -- first
// INTERIOR candidate in ascending id order -- picks the same element.

__device__ inline bool deep_interior(int32_t cd, const double (&rr)[3], int R)
{
    if (cd != FPTS_INTERIOR) return false;
    double m = 1.0;
    for (int a = 0; a < R; ++a) m = fmin(m, 1.0 - fabs(rr[a]));
    return m > kSettleGuard;
}

__device__ inline bool settled(int nc, int32_t cd, const double (&rr)[3], int R)
{
    return nc <= 1 || deep_interior(cd, rr, R);
}

// Phase D, marking: every point whose primary result leaves the search open
// (a cell, a primary and not settled) is appended to ulist, in no particular
// order, *ucount of them.  The other candidates of the few listed points are
// then handled by dense wavefronts: tested where they lie among all points,
// their candidate loops (dependent loads) kept whole wavefronts waiting.
// A block marks kMarkChunk consecutive points, gathers its listed points in
// LDS and reserves their places with one atomic: device-scope atomics on one
// address serialise (several ns each), so one per wavefront with a listed
// point would take longer than the loads.  All of a point's loads are
// issued at once.
constexpr int kMarkChunk = 4096;

// With rest.list (fused find + interpolate, volume and surface meshes) the
// same pass also lists the points the interpolation over the primary list
// leaves out -- found, but not INTERIOR at least kSettleGuard inside by the
// primary result (the listed points among them) -- and writes NaN to the
// interpolated values of NOT_FOUND points, so that the interpolation needs
// no pass over all points of its own.
__device__ inline void list_append(bool take, int p, int lane, int *lst, int &lcnt)
{
    const unsigned long long m = __ballot(take);
    if (m) {
        int at = 0;
        if (lane == 0) at = atomicAdd(&lcnt, __popcll(m));
        at = __shfl(at, 0, 64);
        if (take) lst[at + __popcll(m & ((1ull << lane) - 1))] = p;
    }
}

__global__ __launch_bounds__(256) void k_unsettled(int n, int R, const int *cellpt,
                                                  const int2 *cand,
                                                  const int32_t *code, const double *r,
                                                  int *ulist, int *ucount, EvalRest rest)
{
    __shared__ int lst[kMarkChunk], elst[kMarkChunk];
    __shared__ int lcnt, ecnt, gbase, ebase;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        lcnt = 0;
        ecnt = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kMarkChunk;
    for (int it = 0; it < kMarkChunk / 256; ++it) {
        const int64_t q = base + it * 256 + threadIdx.x;
        const int p = (int)q;
        bool todo = false, other = false;
        if (q < n) {
            const int c = cellpt[p];
            const int2 cd2 = cand[p];
            const int prim = cd2.y, nc = cd2.x;
            const int32_t cd = code[p];
            double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < R) rr[a] = r[(size_t)a * n + p];
            todo = c >= 0 && prim >= 0 && !settled(nc, cd, rr, R);
            if (rest.list) {
                const bool found = cd != FPTS_NOT_FOUND;
                other = found && !deep_interior(cd, rr, R);
                if (!found)
                    for (int f = 0; f < rest.n_fields; ++f)
                        rest.out[(size_t)f * n + p] = __builtin_nan("");
            }
        }
        list_append(todo, p, lane, lst, lcnt);
        if (rest.list) list_append(other, p, lane, elst, ecnt);
    }
    __syncthreads();
    const int cnt = lcnt, ec = ecnt;
    if (threadIdx.x == 0) {
        if (cnt) gbase = atomicAdd(ucount, cnt);
        if (ec) ebase = atomicAdd(rest.count, ec);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 256) ulist[gbase + i] = lst[i];
    for (int i = threadIdx.x; i < ec; i += 256) rest.list[ebase + i] = elst[i];
}

// Exclusive prefix sum of v over the lanes of a wavefront; total = the sum.
__device__ __forceinline__ int wave_excl_sum(int v, int &total)
{
    const int lane = __lane_id();
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

// Phase D over the listed points (grid-stride).  pass 0: count each point's
// other candidates and give the point a block of that many slots, uoff[i] ..
// uoff[i] + ucnt[i] - 1 (one atomic per wavefront on *slot_total), and count
// them per element; a point whose block would end beyond the slot capacity
// cap2 gets none (ucnt[i] = 0) and goes to the overflow list instead
// (olist, *ocount: searched one point per wavefront).  pass 1: write the
// slots (k-th other candidate in ascending id at uoff[i] + k) and bucket them
// by element.
template <int D>
__global__ __launch_bounds__(256) void k_resolve(HashView h, int pass, int n, const double *pts,
                                                const int *cellpt, const int2 *cand,
                                                const int *ulist, const int *ucount,
                                                int *uoff, int *ucnt,
                                                unsigned long long *slot_total,
                                                int *elem_cnt2, const int *elem_off2,
                                                int *elem_fill2, int *slot_pt, int *slot_elem,
                                                int *sorted2, int64_t cap2, int *olist,
                                                int *ocount)
{
    const int cnt = *ucount;
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    // the loop condition is wave-uniform (the stride is a multiple of 64)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i - lane < cnt; i += stride) {
        const bool act = i < cnt;
        int k = 0, p = 0, prim = -1, c = 0;
        double x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = 0.0;
        if (act) {
            p = ulist[i];
            prim = cand[p].y;
            c = cellpt[p];
#pragma unroll
            for (int d = 0; d < D; ++d) x[d] = pts[(size_t)d * n + p];
        }
        if (pass == 0) {
            if (act) {
                for (int q = h.cell_off[c]; q < h.cell_off[c + 1]; ++q) {
                    const int e = h.cell_el[q];
                    double depth;
                    if (e != prim && box_pass<D>(h.box + (size_t)e * (3 * D + D * D), x, depth))
                        ++k;
                }
            }
            int tot;
            const int ex = wave_excl_sum(k, tot);
            unsigned long long base = 0;
            if (lane == 0 && tot > 0) base = atomicAdd(slot_total, (unsigned long long)tot);
            base = __shfl(base, 0, 64);
            const bool fits = base + (unsigned long long)(ex + k) <= (unsigned long long)cap2;
            if (act) {
                uoff[i] = fits ? (int)(base + ex) : 0;
                ucnt[i] = fits ? k : 0;
            }
            if (act && k > 0) {
                if (fits) {
                    for (int q = h.cell_off[c]; q < h.cell_off[c + 1]; ++q) {
                        const int e = h.cell_el[q];
                        double depth;
                        if (e != prim &&
                            box_pass<D>(h.box + (size_t)e * (3 * D + D * D), x, depth))
                            atomicAdd(&elem_cnt2[e], 1);
                    }
                } else {
                    olist[atomicAdd(ocount, 1)] = p;
                }
            }
        } else if (act && ucnt[i] > 0) {
            const int s0 = uoff[i];
            for (int q = h.cell_off[c]; q < h.cell_off[c + 1]; ++q) {
                const int e = h.cell_el[q];
                double depth;
                if (e == prim || !box_pass<D>(h.box + (size_t)e * (3 * D + D * D), x, depth))
                    continue;
                const int sl = s0 + k;
                slot_pt[sl] = p;
                slot_elem[sl] = e;
                sorted2[elem_off2[e] + atomicAdd(&elem_fill2[e], 1)] = sl;
                ++k;
            }
        }
    }
}

// Section 3.2 selection over the primary and the other candidates of a
// listed point: the lowest-id INTERIOR candidate, else the smallest
// distance (lowest id on ties).
__global__ __launch_bounds__(256) void k_select2(int n, int R, const int *ulist,
                                                const int *ucount, const int *uoff,
                                                const int *ucnt, const int2 *cand,
                                                const int *slot_elem, int64_t cap2,
                                                const double *res_r, const double *res_dist,
                                                const int *res_code, int32_t *code,
                                                int32_t *elem, double *r, double *dist)
{
    const int cnt = *ucount;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const int p = ulist[i];
        const int s0 = uoff[i], s1 = s0 + ucnt[i];
        if (s0 == s1) continue;
        // best so far: the primary (slot -1)
        int best = -1;
        int bcode = code[p], belem = cand[p].y;
        double bdist = dist[p];
        for (int s = s0; s < s1; ++s) {
            const int e = slot_elem[s], cd = res_code[s];
            const double dd = res_dist[s];
            bool take;
            if (bcode == FPTS_INTERIOR) take = cd == FPTS_INTERIOR && e < belem;
            else if (cd == FPTS_INTERIOR) take = true;
            else take = dd < bdist || (dd == bdist && e < belem);
            if (take) {
                best = s;
                bcode = cd;
                belem = e;
                bdist = dd;
            }
        }
        if (best < 0) continue;
        code[p] = bcode;
        elem[p] = belem;
        dist[p] = bdist;
        for (int a = 0; a < R; ++a) r[(size_t)a * n + p] = res_r[(size_t)a * cap2 + best];
    }
}

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }


// Search hints (points that move a little between searches): pass 0 takes
// the previous element of every point whose previous code was INTERIOR as
// its only candidate and counts it per element; pass 1 marks the points
// whose hinted search converged (keep[p] holds the Newton convergence flag
// on entry) INTERIOR at least kSettleGuard inside the reference box: no
// other element can hold them in its interior, so that result is the one
// the full search gives, and they are kept.
__global__ __launch_bounds__(256) void k_hint(int pass, int n, int nel, int R,
                                             const int32_t *code, const int32_t *elem,
                                             const double *r, int2 *cand, int *elem_cnt,
                                             int *rank, int *keep)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < n;
    if (pass == 0) {
        const int e = in && code[p] == FPTS_INTERIOR ? elem[p] : -1;
        const bool ok = e >= 0 && e < nel;
        if (in) cand[p] = make_int2(ok ? 1 : 0, ok ? e : -1);
        const int k = wave_inc(elem_cnt, e, ok);
        if (ok) rank[p] = k;
    } else if (in) {
        bool k = cand[p].y >= 0 && code[p] == FPTS_INTERIOR && keep[p] == 1;
        double mg = 1.0;
        for (int a = 0; a < R; ++a) mg = fmin(mg, 1.0 - fabs(r[(size_t)a * n + p]));
        keep[p] = k && mg > kSettleGuard;
    }
}

// Parked pairs of the primary Newton pass, binned by element (their queue
// for the face kernel).  A fixed grid strides over the *count records; the
// loop bound is uniform per wavefront, as wave_inc needs.
__global__ __launch_bounds__(256) void k_park_bin(int pass, const int4 *meta, const int *count,
                                                 int cap, int *elem_cnt, const int *elem_off,
                                                 int *rank, int *sorted)
{
    const int total = min(*count, cap);
    const int lane = threadIdx.x & 63;
    for (int k0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63); k0 < total;
         k0 += gridDim.x * blockDim.x) {
        const int k = k0 + lane;
        const bool active = k < total;
        const int e = active ? meta[k].z : 0;
        if (pass == 0) {
            const int rk = wave_inc(elem_cnt, e, active);
            if (active) rank[k] = rk;
        } else if (active) {
            sorted[elem_off[e] + rank[k]] = k;
        }
    }
}

}  // namespace

hipError_t launch_fill_i32(int *p, int64_t count, int value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>(grid_for(count, 256), 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

int64_t scan_tmp_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// out[0..n] = exclusive scan of in[0..n) (optionally ceil(in/ceil_div)),
// out[n] = total.  `out` may alias `in` only when ceil_div <= 1.
hipError_t launch_exclusive_scan(const int *in, int *out, int64_t n, int ceil_div, int *tmp,
                                 int64_t tmp_blocks, hipStream_t s)
{
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles + 1 > tmp_blocks) return hipErrorInvalidValue;
    if (tiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out,
                           n, ceil_div, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, tiles, out, n);
    if (tiles > 0)
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, out, n,
                           tmp);
    return hipGetLastError();
}

hipError_t launch_park_bin(int pass, const int4 *meta, const int *count, int64_t cap,
                           int *elem_cnt, const int *elem_off, int *rank, int *sorted, int cus,
                           hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(grid_for(cap, 256), (int64_t)cus * 4);
    hipLaunchKernelGGL(k_park_bin, dim3(grid), dim3(256), 0, s, pass, meta, count, (int)cap,
                       elem_cnt, elem_off, rank, sorted);
    return hipGetLastError();
}

hipError_t launch_cell_bin(const fpts_mesh *m, int pass, int64_t n, const double *pts,
                           double *pts4, const int *keep, int *cellpt, int *cell_cnt,
                           const int *cell_poff, int *rank, int *pbin, int2 *cand,
                           int32_t *code, int32_t *elem, double *r, double *dist, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    HashView h = hash_view(m);
    const int grid = grid_for(n, 256);
    auto k = m->D == 2 ? k_cell_bin<2> : k_cell_bin<3>;
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, h, pass, (int)n, m->R, pts, pts4, keep,
                       cellpt, cell_cnt, cell_poff, rank, pbin, cand, code, elem, r, dist);
    return hipGetLastError();
}

int bin_shift(int64_t ncell)
{
    if (ncell > kBinMaxCells) return -1;
    // buckets of at least 512 cells: a tile's run per bucket is then tens
    // of pairs long (whole cache lines) at a few points per cell
    int shift = 9;
    while ((ncell + (1ll << shift) - 1) >> shift > kBinMaxBuckets) ++shift;
    return shift;
}

int64_t bin_tiles(int64_t n) { return (n + kBinTile - 1) / kBinTile; }

// a grid of at least `blocks` blocks, a multiple of the XCD count
static unsigned xcd_grid(int64_t blocks)
{
    return (unsigned)((std::max<int64_t>(blocks, 1) + kXcd - 1) / kXcd * kXcd);
}

hipError_t launch_bin_tiles(const fpts_mesh *m, int64_t n, const double *pts, double *pts4,
                            const int *keep, int *cellpt, int2 *cand,
                            int32_t *code, int32_t *elem, double *r, double *dist, int shift,
                            int *bh, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    HashView h = hash_view(m);
    const int64_t ncell = bin_cells(m);
    const int nb = (int)((ncell + (1ll << shift) - 1) >> shift), ntile = (int)bin_tiles(n);
    auto k = m->D == 2 ? k_bin_tiles<2> : k_bin_tiles<3>;
    hipLaunchKernelGGL(k, dim3(ntile), dim3(kBinThreads), sizeof(int) * nb, s, h, (int)n, m->R,
                       pts, pts4, keep, cellpt, cand, code, elem, r, dist, shift, nb,
                       ntile, bh);
    return hipGetLastError();
}

hipError_t launch_bin_coarse(const fpts_mesh *m, int64_t n, const int *cellpt, int shift,
                             const int *boff, int2 *pairs, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t ncell = bin_cells(m);
    const int nb = (int)((ncell + (1ll << shift) - 1) >> shift), ntile = (int)bin_tiles(n);
    hipLaunchKernelGGL(k_bin_coarse, dim3(ntile), dim3(kBinThreads), sizeof(int) * nb, s, (int)n,
                       cellpt, shift, nb, ntile, boff, pairs);
    return hipGetLastError();
}

hipError_t launch_bin_rank(int64_t n, const int *total, int shift, const int2 *pairs,
                           int *cell_cnt, int *rank, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_rank, dim3(xcd_grid(bin_tiles(n))), dim3(kBinThreads),
                       sizeof(int) * (2 << shift), s, total, shift, pairs, cell_cnt, rank);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(int64_t n, const int *total, const int2 *pairs, const int *rank,
                              const int *cell_poff, int *pbin, int cus, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = xcd_grid(std::min<int64_t>(grid_for(n, kBinThreads), (int64_t)cus * 16));
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid), dim3(kBinThreads), 0, s, total, pairs, rank,
                       cell_poff, pbin);
    return hipGetLastError();
}

hipError_t launch_task_map(const int *chunk_off, int64_t nunit, int *task_unit, hipStream_t s)
{
    if (nunit <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_task_map, dim3(grid_for(nunit, 256)), dim3(256), 0, s, chunk_off,
                       (int)nunit, task_unit);
    return hipGetLastError();
}

hipError_t launch_locate_cells(const fpts_mesh *m, int64_t n, const double *pts,
                               const double *pts4,
                               const int *pbin, const int *cell_poff, const int *cell_choff,
                               int64_t ncell, const int *task_cell, int64_t task_bound,
                               int2 *cand, int *elem_cnt, int *rank,
                               int *bin_prim, int32_t *code, int32_t *elem, double *r,
                               double *dist, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    HashView h = hash_view(m);
    auto k = m->D == 2 ? (pts4 ? k_locate_cells<2, true> : k_locate_cells<2, false>)
                       : (pts4 ? k_locate_cells<3, true> : k_locate_cells<3, false>);
    hipLaunchKernelGGL(k, dim3(task_grid(task_bound, m->cus)), dim3(64), 0, s, h, (int)n, m->R,
                       pts, pts4, pbin, cell_poff, cell_choff, (int)ncell, task_cell, cand,
                       elem_cnt, rank, bin_prim, code, elem, r, dist);
    return hipGetLastError();
}

hipError_t launch_primary_scatter_bins(int64_t n, const int *nbinned, const int *pbin,
                                       const int *bin_prim, const int *rank,
                                       const int *elem_off, int *sorted, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_primary_scatter_bins, dim3(grid_for(n, 256)), dim3(256), 0, s, (int)n,
                       nbinned, pbin, bin_prim, rank, elem_off, sorted);
    return hipGetLastError();
}

hipError_t launch_primary_scatter(int64_t n, int64_t nel, const int2 *cand,
                                  const int *elem_off, const int *rank, int *sorted,
                                  hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_primary_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, (int)n,
                       (int)nel, cand, elem_off, rank, sorted);
    return hipGetLastError();
}

hipError_t launch_unsettled(const fpts_mesh *m, int64_t n, const int *cellpt, const int2 *cand,
                            const int32_t *code, const double *r, int *ulist,
                            int *ucount, const EvalRest &rest, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unsettled, dim3(grid_for(n, kMarkChunk)), dim3(256), 0, s, (int)n, m->R,
                       cellpt, cand, code, r, ulist, ucount, rest);
    return hipGetLastError();
}

// grid-stride kernels over the unsettled list: enough blocks to fill the
// chip when the list is long, few to launch when it is short
static int list_grid(const fpts_mesh *m, int64_t n)
{
    return std::max(1, (int)std::min<int64_t>(grid_for(n, 256), (int64_t)m->cus * 16));
}

hipError_t launch_resolve(const fpts_mesh *m, int pass, int64_t n, const double *pts,
                          const int *cellpt, const int2 *cand, const int *ulist,
                          const int *ucount, int *uoff, int *ucnt, unsigned long long *slot_total,
                          int *elem_cnt2, const int *elem_off2, int *elem_fill2, int *slot_pt,
                          int *slot_elem, int *sorted2, int64_t cap2, int *olist, int *ocount,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    HashView h = hash_view(m);
    auto k = m->D == 2 ? k_resolve<2> : k_resolve<3>;
    hipLaunchKernelGGL(k, dim3(list_grid(m, n)), dim3(256), 0, s, h, pass, (int)n, pts, cellpt,
                       cand, ulist, ucount, uoff, ucnt, slot_total, elem_cnt2, elem_off2,
                       elem_fill2, slot_pt, slot_elem, sorted2, cap2, olist, ocount);
    return hipGetLastError();
}

hipError_t launch_select2(const fpts_mesh *m, int64_t n, const int *ulist, const int *ucount,
                          const int *uoff, const int *ucnt, const int2 *cand,
                          const int *slot_elem, int64_t cap2, const double *res_r,
                          const double *res_dist, const int *res_code, int32_t *code,
                          int32_t *elem, double *r, double *dist, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select2, dim3(list_grid(m, n)), dim3(256), 0, s, (int)n, m->R, ulist,
                       ucount, uoff, ucnt, cand, slot_elem, cap2, res_r, res_dist, res_code,
                       code, elem, r, dist);
    return hipGetLastError();
}

}  // namespace fpts

namespace fpts {

hipError_t launch_hint(const fpts_mesh *m, int pass, int64_t n, const int32_t *code,
                       const int32_t *elem, const double *r, int2 *cand, int *elem_cnt,
                       int *rank, int *keep, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hint, dim3(grid_for(n, 256)), dim3(256), 0, s, pass, (int)n,
                       (int)m->nel, m->R, code, elem, r, cand, elem_cnt, rank, keep);
    return hipGetLastError();
}

}  // namespace fpts
