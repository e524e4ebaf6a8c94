// Find, outside Newton (Section 3.2): candidate lookup in the local map
// (Section 3.1.3) with the AABB and OBB tests (eqs. eq_AABB_test,
// eq_OBB_test), grouping of (point, element) pairs by element, and the
// per-point selection of the result.  Also the int32 exclusive scan and
// fill kernels used by find and eval.
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
__device__ inline int64_t cell_of(const HashView &h, const double *x)
{
    int64_t cell = 0, mul = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (!__builtin_isfinite(x[d]) || !(x[d] >= h.lo[d] && x[d] <= h.hi[d])) return -1;
        double t = floor((x[d] - h.lo[d]) / h.del[d]);
        t = fmin(fmax(t, 0.0), (double)(h.NL - 1));
        cell += mul * (int64_t)t;
        mul *= h.NL;
    }
    return cell;
}

// Box filter of element e (eq. eq_AABB_test, then eq. eq_OBB_test).
template <int D>
__device__ inline bool box_pass(const HashView &h, int e, const double *x)
{
    const double *rec = h.box + (size_t)e * (3 * D + D * D);
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (!((x[d] - rec[d]) * (rec[D + d] - x[d]) >= 0.0)) return false;
    double y[D];
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] - rec[2 * D + d];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) t += rec[3 * D + a * D + b] * y[b];
        if (!(fabs(t) <= 1.0)) return false;
    }
    return true;
}

// pass 0: count candidates per point and per element.
// pass 1: write the pairs: slot s = pt_off[p] + k for the k-th candidate
// (ascending element id), and scatter s into its element's bucket.
template <int D>
__global__ __launch_bounds__(256) void k_locate(HashView h, int pass, int n, const double *pts,
                                               int *pt_cnt_or_off, int *elem_cnt,
                                               const int *elem_off, int *elem_fill,
                                               int *slot_pt, int *slot_elem, int *sorted)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double x[D];
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = pts[(size_t)d * n + p];
    const int64_t cell = cell_of<D>(h, x);
    int k = 0;
    int s0 = pass ? pt_cnt_or_off[p] : 0;
    if (cell >= 0) {
        const int q0 = h.cell_off[cell], q1 = h.cell_off[cell + 1];
        for (int q = q0; q < q1; ++q) {
            const int e = h.cell_el[q];
            if (!box_pass<D>(h, e, x)) continue;
            if (pass == 0) {
                atomicAdd(&elem_cnt[e], 1);
            } else {
                const int s = s0 + k;
                slot_pt[s] = p;
                slot_elem[s] = e;
                sorted[elem_off[e] + atomicAdd(&elem_fill[e], 1)] = s;
            }
            ++k;
        }
    }
    if (pass == 0) pt_cnt_or_off[p] = k;
}

// Section 3.2 selection: the first INTERIOR candidate in ascending element
// order, else the smallest distance (first on ties); NOT_FOUND without
// candidates.
__global__ __launch_bounds__(256) void k_select(int n, int R, const int *pt_off,
                                               const int *slot_elem, int64_t cap,
                                               const double *res_r, const double *res_dist,
                                               const int *res_code, int32_t *code, int32_t *elem,
                                               double *r, double *dist)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int s0 = pt_off[p], s1 = pt_off[p + 1];
    int best = -1;
    for (int s = s0; s < s1; ++s) {
        if (res_code[s] == FPTS_INTERIOR) { best = s; break; }
        if (best < 0 || res_dist[s] < res_dist[best]) best = s;
    }
    if (best < 0) {
        code[p] = FPTS_NOT_FOUND;
        elem[p] = -1;
        dist[p] = __builtin_huge_val();
        for (int a = 0; a < R; ++a) r[(size_t)a * n + p] = 0.0;
        return;
    }
    code[p] = res_code[best];
    elem[p] = slot_elem[best];
    dist[p] = res_dist[best];
    for (int a = 0; a < R; ++a) r[(size_t)a * n + p] = res_r[(size_t)a * cap + best];
}

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

HashView hash_view(const fpts_mesh *m)
{
    HashView h;
    for (int d = 0; d < 3; ++d) {
        h.lo[d] = d < m->D ? m->hlo[d] : 0.0;
        h.hi[d] = d < m->D ? m->hhi[d] : 0.0;
        h.del[d] = d < m->D ? m->hdel[d] : 1.0;
    }
    h.NL = m->NL;
    h.cell_off = m->d_cell_off;
    h.cell_el = m->d_cell_el;
    h.box = m->d_box;
    return h;
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

hipError_t launch_locate(const fpts_mesh *m, int pass, int64_t n, const double *pts,
                         int *pt_cnt_or_off, int *elem_cnt, const int *elem_off, int *elem_fill,
                         int *slot_pt, int *slot_elem, int *sorted, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    HashView h = hash_view(m);
    const int grid = grid_for(n, 256);
    if (m->D == 2)
        hipLaunchKernelGGL(k_locate<2>, dim3(grid), dim3(256), 0, s, h, pass, (int)n, pts,
                           pt_cnt_or_off, elem_cnt, elem_off, elem_fill, slot_pt, slot_elem,
                           sorted);
    else
        hipLaunchKernelGGL(k_locate<3>, dim3(grid), dim3(256), 0, s, h, pass, (int)n, pts,
                           pt_cnt_or_off, elem_cnt, elem_off, elem_fill, slot_pt, slot_elem,
                           sorted);
    return hipGetLastError();
}

hipError_t launch_select(const fpts_mesh *m, int64_t n, const int *pt_off, const int *slot_elem,
                         int64_t cap, const double *res_r, const double *res_dist,
                         const int *res_code, int32_t *code, int32_t *elem, double *r,
                         double *dist, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(grid_for(n, 256)), dim3(256), 0, s, (int)n, m->R, pt_off,
                       slot_elem, cap, res_r, res_dist, res_code, code, elem, r, dist);
    return hipGetLastError();
}

}  // namespace fpts
