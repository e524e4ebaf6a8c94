// Internal declarations of the fpts library (host setup, kernel launchers).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "fpts.h"

namespace fpts {

constexpr int kMaxN = 10;        // nodes per direction with compiled kernels
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kChunk = 64;       // (point, element) pairs per wave task
// doubles per point in the packed copy of the points (x, y, z, 0 / x, y)
constexpr int pt_stride(int D) { return D == 3 ? 4 : 2; }

// GLL nodes z_i and product-form weights w_i = 1 / prod_{m != i}(z_i - z_m):
// phi_i(r) = w_i prod_{m != i}(r - z_m).
struct Basis {
    double z[16];
    double w[16];
};

// Packed box record of one element: AABB lo[D], hi[D]; OBB centre c[D] and
// inverse transform A[D][D] (all zero when the centre Jacobian is singular,
// which makes the OBB test pass).
inline int box_words(int D) { return 3 * D + D * D; }

// Local map on the device: implicit Cartesian grid + CSR cell lists.
struct HashView {
    double lo[3], hi[3], del[3];
    int NL;
    const int *cell_off;   // [NL^D + 1]
    const int *cell_el;    // [nnz], ascending element id per cell
    const double *box;     // [nel][box_words(D)]
};

// Byte offsets of the find workspace for n points (every array 256-aligned).
// Phase A bins points by cell of the local map, phase B tests each cell's
// candidates and picks a primary candidate per point, phase C runs Newton on
// the primaries, phase D runs the remaining candidates of the points the
// primary did not settle.
// Task grids.  Items (points or pairs) bucketed by unit (cell or element)
// are processed in tasks of up to kChunk items of one unit, one 64-lane
// workgroup per task.  Workgroups go to the 8 XCDs round-robin, so block b
// runs task (b mod 8) * (G / 8) + b / 8 of a grid of G blocks (G a multiple
// of 8): each XCD works through a contiguous range of tasks and the tasks of
// one unit share its L2; a block continues with tasks t + G, t + 2G, ...
// Task -> unit comes from a map filled after the task offsets are scanned
// (launch_task_map).
constexpr int kXcd = 8;
// a primary result settles its point when INTERIOR at least this far inside
// the reference box (no other element can then hold the point inside)
constexpr double kSettleGuard = 1e-9;

// Upper bound on the tasks of n items over nunit units.
inline int64_t task_bound(int64_t n, int64_t nunit)
{
    return n / kChunk + std::min<int64_t>(n, nunit) + 1;
}

// Grid size (blocks) for a task bound: a multiple of the XCD count, at most
// 64 blocks per CU; blocks loop over tasks t, t + G, ...
inline int64_t task_grid(int64_t bound, int cus)
{
    const int64_t g = std::min<int64_t>(bound, (int64_t)cus * 64);
    return (std::max<int64_t>(g, 1) + kXcd - 1) / kXcd * kXcd;
}

__device__ __forceinline__ int task_of_block()
{
    const int b = blockIdx.x, G = gridDim.x;
    return (b % kXcd) * (G / kXcd) + b / kXcd;
}

// OBB frame of a line element (Section 4.2): J_c = Q^T for the rotation Q
// that takes the unit centre tangent u = t/|t| to e1, by Rodrigues' formula
// about k = u x e1 with cos = u.e1 and sin = |u x e1|; u = -e1 takes the half
// turn about e3.  Left all zero when t = 0.  Host and device setup share it,
// so both round alike (the device file is built without contraction).
__host__ __device__ inline void rodrigues_frame(int D, double tx, double ty, double tz,
                                                double *Jc)
{
    const double tn = sqrt(tx * tx + ty * ty + tz * tz);
    if (!(tn > 0.0)) return;
    const double u[3] = {tx / tn, ty / tn, tz / tn};
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    const double sn = sqrt(u[1] * u[1] + u[2] * u[2]), cs = u[0];
    if (sn > 0.0) {
        const double k[3] = {0.0, u[2] / sn, -u[1] / sn};
        const double K[3][3] = {{0.0, -k[2], k[1]}, {k[2], 0.0, -k[0]}, {-k[1], k[0], 0.0}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double kk = 0.0;
                for (int q = 0; q < 3; ++q) kk += K[i][q] * K[q][j];
                Q[i][j] = (i == j ? 1.0 : 0.0) + sn * K[i][j] + (1.0 - cs) * kk;
            }
    } else if (cs < 0.0) {
        Q[0][0] = -1.0;
        Q[1][1] = -1.0;
    }
    for (int c = 0; c < D; ++c)
        for (int q = 0; q < D; ++q) Jc[c * D + q] = Q[q][c];
}

// ctr[key]++ for every active lane, returning the lane's old value, with one
// atomic per group of lanes that share a key: the group of the lowest pending
// lane is peeled off with a ballot and takes a block of consecutive values.
// Points that arrive clustered (along a curve, in a lattice, element by
// element) otherwise pile thousands of atomics onto one address, and
// device-scope atomics on one address serialise.  Peeling stops once a group
// has fewer than 4 lanes (scattered keys); the rest use one atomic each.
// Every lane of the wavefront must call it (it ballots).
__device__ __forceinline__ int wave_inc(int *ctr, int key, bool active)
{
    const int lane = __lane_id();
    const unsigned long long bit = 1ull << lane;
    unsigned long long pend = __ballot(active);
    int out = 0;
    for (int round = 0; round < 16 && pend; ++round) {
        const int leader = __builtin_ctzll(pend);
        const int k = __shfl(key, leader, 64);
        const unsigned long long grp = __ballot(key == k) & pend;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], __popcll(grp));
        base = __shfl(base, leader, 64);
        if (grp & bit) out = base + __popcll(grp & (bit - 1));
        pend &= ~grp;
        if (__popcll(grp) < 4) break;
    }
    if (pend & bit) out = atomicAdd(&ctr[key], 1);
    return out;
}

// Box filter of one element record: the AABB test (eq. eq_AABB_test,
// inclusive) and the point's OBB depth ||A(x - c)||_inf (eq. eq_OBB_test:
// inside when <= 1; smaller = deeper).
template <int D, typename P>
__device__ inline bool aabb_in(P rec, const double *x)
{
    bool in = true;
#pragma unroll
    for (int d = 0; d < D; ++d) in = in && ((x[d] - rec[d]) * (rec[D + d] - x[d]) >= 0.0);
    return in;
}
template <int D, typename P>
__device__ inline double obb_depth(P rec, const double *x)
{
    double y[D];
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] - rec[2 * D + d];
    double mx = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) t += rec[3 * D + a * D + b] * y[b];
        mx = fmax(mx, fabs(t));
    }
    return mx;
}
// Both tests; `depth` receives the OBB depth.
template <int D, typename P>
__device__ inline bool box_pass(P rec, const double *x, double &depth)
{
    const bool in = aabb_in<D>(rec, x);
    depth = obb_depth<D>(rec, x);
    return in && (depth <= 1.0);
}

// fused find + interpolate (list null otherwise): the points the pass over
// the primary list does not interpolate (list, *count of them; count zeroed
// by the find), and NaN values for NOT_FOUND points
struct EvalRest {
    int *list;
    int *count;
    double *out;
    int n_fields;
};

// cand[p] (find workspace): (number of candidates that pass the box tests,
// primary element or -1) of point p
struct FindWs {
    size_t cell_cnt, cell_poff, cell_choff, cellpt, pbin, cand, rank, bin_prim,
        elem_cnt, elem_off, chunk_off, sorted, ulist, uoff, ucnt, elem_cnt2, elem_fill2,
        elem_off2, chunk_off2, slot_pt, slot_elem, sorted2, res_r, res_dist, res_code,
        task_cell, task_elem, task_elem2, scan_tmp, counters, stats, pts4, start, park_meta,
        park_r, park_state, park_cnt, park_off, park_choff, park_rank, park_sorted, park_task,
        olist, ov_int, ov_dbl, bin_hist, bin_pairs, total;
    int64_t cap2;           // capacity for second-pass (point, candidate) pairs
    int64_t scan_blocks;
    int64_t ncell;
    int64_t tb_cell, tb_elem, tb_elem2, tb_park;   // task bounds
    int64_t park_state_cap;  // parked pairs whose iteration state is saved
    int64_t ov_grid;        // blocks of the overflow search (its scratch)
    int bin_shift;          // phase A without per-point atomics: bucket shift, or -1
    int64_t bin_hist_n;     // entries of its bucket histograms (nb * ntile)
};

struct EvalWs {
    size_t elem_cnt, elem_off, rank, chunk_off, scan_tmp, sorted, task_elem, slist, scount,
        total;
    int64_t tb_elem;
};

// Where one Newton launch reads its work and writes its results.
struct NewtonIO {
    const int *list;        // bucketed item ids, element-major
    const int *elem_off;    // [nel+1] bucket offsets into list
    const int *chunk_off;   // [nel+1] offsets of 64-item tasks
    const int *slot_pt;     // item -> point (nullptr: the item is the point)
    int32_t *code;          // [item]
    int32_t *elem;          // [item] or nullptr
    double *r;              // [R][ostride]
    int64_t ostride;
    double *dist;           // [item]
    int *counter;           // element-queue counters (zeroed before the launch)
    unsigned long long *stats;
    const int *task_elem;   // task -> element of the nearest-node task grid
    int64_t task_bound;     // tasks of that grid at most
    // optional (fused find + interpolate, primary pass): results that settle
    // their point -- INTERIOR at least kSettleGuard inside -- also go to
    // rs[k * rs_stride + q] at the pair's position q in `list`; NaN marks
    // the other positions
    double *rs;
    int64_t rs_stride;
    // optional: conv[item] = 1 when the step test ended the iteration, 0 when
    // the pass limit did; max_iter > 0 replaces the mesh's pass limit
    int *conv;
    int max_iter;
    // optional: the points packed per point, [n][pt_stride(D)] (read instead
    // of the [D][n] coordinates: one cache line per gathered point)
    const double *pts4;
    // optional: the starts of the Newton kernel (nearest node, or the FP32
    // phase's result in mixed mode) at the pair's position q in `list`,
    // start[k * start_stride + q], instead of in r: written and read in list
    // order, without a gather
    double *start;
    int64_t start_stride;
    // optional (primary FP64 pass): a pair whose next pass needs second
    // derivatives (a pass on a face, eq. eq_newton_hessian) leaves its wave
    // and is parked: park_meta[k] = {item, list position, element, passes
    // so far}, park_r[j * park_cap + k] = r_j (j < R) and the trust-region
    // radius alpha (j = R); *park_count counts the parked pairs (at most
    // park_cap, one per pair of the pass).  The face kernel resumes them,
    // binned by element, with list = park indices.
    int4 *park_meta;
    double *park_r;
    int64_t park_cap;
    int *park_count;
    // optional: the iteration state at r of parked pair k < park_state_cap,
    // park_state[k * kParkState + j] (j: f, g[R], the Gauss-Newton Hessian
    // [kSym<R>], dx[D]), so that the face kernel resumes without evaluating
    // the map at r again; pairs parked beyond the capacity are re-evaluated
    double *park_state;
    int64_t park_state_cap;
    // mixed mode, FP64 phase of a volume mesh: when the first FP64 Newton
    // step from the FP32 result is below kPolishTol and off the faces, that
    // step ends the iteration (one FP64 evaluation per pair)
    int polish;
    // overflow search (which & 8): list = overflowed points, *ocount of
    // them; their cells and primaries; per-block scratch ov_int [3][grid]
    // and ov_dbl [R + 1][grid]; code/elem/r/dist are the final outputs
    const int *ocount;
    const int *cellpt;
    const int2 *cand;
    int *ov_int;
    double *ov_dbl;
};

// Largest first FP64 step from the FP32 result that ends the iteration in
// mixed mode.  Newton converges quadratically: from a point within 1e-6 of
// the solution one step leaves an error of order kappa * 1e-12, kappa the
// element map's relative curvature (<< 1 for elements of a valid mesh).
constexpr double kPolishTol = 1e-6;

// Doubles per saved park state (at most 1 + 3 + 6 + 3 used), one 128-byte
// record per parked pair.
constexpr int kParkState = 16;

}  // namespace fpts

// profiling spans: locate, nearest-node start, Newton (primary pass), select
// (other candidates + selection), eval binning, eval, particle update, face
// kernel (parked pairs, with their binning)
constexpr int kSpans = 8;

struct fpts_mesh {
    fpts_params p;
    int D, R, N, NP;
    int64_t nel;
    int device;
    int cus;                 // compute units of the device
    fpts::Basis basis;
    // host copies of setup products
    std::vector<double> box;      // [nel][box_words]
    std::vector<double> xc;       // [nel][D] element centre x(0)
    std::vector<int> cell_off, cell_el;
    double hlo[3], hhi[3], hdel[3];
    int NL;
    int max_cell;
    // profiling: event pairs per kernel group
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kSpans];
    int64_t prof_find = 0, prof_eval = 0, prof_lpt = 0;
    // device copies
    double *d_nodes = nullptr;    // [nel][D][NP]
    float *d_nodes32 = nullptr;   // [nel][D][NP] x - x_c in FP32 (mixed mode)
    double *d_near = nullptr;     // [nel][4][near_npad] nearest-node score rows (FP64)
    int near_npad = 0;
    double *d_xc = nullptr;       // [nel][D]
    double *d_box = nullptr;
    int *d_cell_off = nullptr, *d_cell_el = nullptr;
};

namespace fpts {

// The local map and box records of a mesh as kernels read them.
inline HashView hash_view(const fpts_mesh *m)
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

// host setup (setup.cpp)
int host_setup(fpts_mesh *m, const double *h_nodes);

// Basis-bound tables of Section 3.1.1 (built on the host, M = 2N Chebyshev
// points), the Legendre moments of the bases and the bases at r = 0, as the
// device setup reads them.
struct BoundTables {
    int N, M;
    double eta[2 * kMaxN];
    double vlo[kMaxN * 2 * kMaxN], vhi[kMaxN * 2 * kMaxN];   // [N][M]
    double mom0[kMaxN], mom1[kMaxN];
    double z[kMaxN];
    double v0[kMaxN], d0[kMaxN];
};
void bound_tables(const fpts_mesh *m, BoundTables *t);

// Device setup (setup_device.hip): boxes and centres of every element from
// m->d_nodes into m->d_box / m->d_xc, then the local map, with the same
// arithmetic in the same order as host_setup; updates the host copies.
int device_setup(fpts_mesh *m, hipStream_t s);

// fpts_find; points with keep[p] != 0 (keep may be null) hold final results
// and are not searched (api.cpp)
int find_impl(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code, int32_t *d_elem,
              double *d_r, double *d_dist, int precision, void *d_ws, size_t ws_bytes,
              void *stream, const int *keep, double *rs, const EvalRest *rest = nullptr);

// workspace layouts (api.cpp)
FindWs find_ws_layout(const fpts_mesh *m, int64_t n);
EvalWs eval_ws_layout(const fpts_mesh *m, int64_t n);

// launchers (kernels_*.hip); all return hipError_t of the last launch
hipError_t launch_fill_i32(int *p, int64_t count, int value, hipStream_t s);
hipError_t launch_exclusive_scan(const int *in, int *out, int64_t n, int ceil_div,
                                 int *tmp, int64_t tmp_blocks, hipStream_t s);
int64_t scan_tmp_blocks(int64_t n);
// phase A: pass 0 counts points per cell (and writes NOT_FOUND for points
// outside the map), keeping each point's rank among its cell's points; pass 1
// puts point ids into cell buckets at those ranks; points with keep[p] != 0
// (keep may be null) are left out and keep their results; pass 0 also
// writes the coordinates packed per point to pts4 unless it is null
hipError_t launch_cell_bin(const fpts_mesh *m, int pass, int64_t n, const double *pts,
                           double *pts4, const int *keep, int *cellpt, int *cell_cnt,
                           const int *cell_poff, int *rank, int *pbin, int2 *cand,
                           int32_t *code, int32_t *elem, double *r, double *dist, hipStream_t s);
// Phase A without per-point atomics (meshes with at most kBinMaxCells
// cells; bin_shift returns -1 beyond): cells grouped into buckets of
// 2^shift cells, at most kBinMaxBuckets of them.  tiles: as pass 0 of
// launch_cell_bin, and each tile's bucket histogram into bh[bucket * ntile
// + tile] (ntile = bin_tiles(n); bh is then scanned in place, its total at
// bh[nb * ntile]); coarse: (cell, id) pairs sorted by bucket from the
// scanned bh; rank: each pair's rank in its cell (cell_cnt zeroed before,
// complete after), *total pairs; scatter: pbin[cell_poff[c] + rank[i]] =
// id of pair i.
constexpr int64_t kBinMaxCells = (int64_t)1 << 24;
constexpr int kBinMaxBuckets = 4096;
int bin_shift(int64_t ncell);
int64_t bin_tiles(int64_t n);
inline int64_t bin_cells(const fpts_mesh *m)
{
    int64_t c = 1;
    for (int d = 0; d < m->D; ++d) c *= m->NL;
    return c;
}
hipError_t launch_bin_tiles(const fpts_mesh *m, int64_t n, const double *pts, double *pts4,
                            const int *keep, int *cellpt, int2 *cand,
                            int32_t *code, int32_t *elem, double *r, double *dist, int shift,
                            int *bh, hipStream_t s);
hipError_t launch_bin_coarse(const fpts_mesh *m, int64_t n, const int *cellpt, int shift,
                             const int *boff, int2 *pairs, hipStream_t s);
hipError_t launch_bin_rank(int64_t n, const int *total, int shift, const int2 *pairs,
                           int *cell_cnt, int *rank, hipStream_t s);
hipError_t launch_bin_scatter(int64_t n, const int *total, const int2 *pairs, const int *rank,
                              const int *cell_poff, int *pbin, int cus, hipStream_t s);
// search hints: pass 0 makes the previous element of each previously
// INTERIOR point its primary (counted per element); pass 1 sets keep[p] for
// points the hinted search settled
hipError_t launch_hint(const fpts_mesh *m, int pass, int64_t n, const int32_t *code,
                       const int32_t *elem, const double *r, int2 *cand, int *elem_cnt,
                       int *rank, int *keep, hipStream_t s);
// phase B: candidates of each point from its cell's list (one wave per 64
// points of one cell), primary = deepest inside its OBB
// task -> unit map of a task grid over nunit units with task offsets chunk_off
hipError_t launch_task_map(const int *chunk_off, int64_t nunit, int *task_unit, hipStream_t s);
// Parked pairs binned by element: pass 0 counts them per element (elem_cnt,
// zeroed before) and keeps each one's rank, pass 1 writes park index k at
// sorted[elem_off[elem] + rank[k]]; *count pairs (at most cap).
hipError_t launch_park_bin(int pass, const int4 *meta, const int *count, int64_t cap,
                           int *elem_cnt, const int *elem_off, int *rank, int *sorted, int cus,
                           hipStream_t s);
// (counts primaries per element; in bin order, bin_prim[i] and rank[i] are
// the primary of the point at bin position i and its rank in that bucket)
hipError_t launch_locate_cells(const fpts_mesh *m, int64_t n, const double *pts,
                               const double *pts4,
                               const int *pbin, const int *cell_poff, const int *cell_choff,
                               int64_t ncell, const int *task_cell, int64_t task_bound,
                               int2 *cand, int *elem_cnt, int *rank,
                               int *bin_prim, int32_t *code, int32_t *elem, double *r,
                               double *dist, hipStream_t s);
// sorted[elem_off[bin_prim[i]] + rank[i]] = pbin[i] for i < *nbinned
hipError_t launch_primary_scatter_bins(int64_t n, const int *nbinned, const int *pbin,
                                       const int *bin_prim, const int *rank,
                                       const int *elem_off, int *sorted, hipStream_t s);
// sorted[elem_off[cand[p].y] + rank[p]] = p
hipError_t launch_primary_scatter(int64_t n, int64_t nel, const int2 *cand,
                                  const int *elem_off, const int *rank, int *sorted,
                                  hipStream_t s);
// phase D: list the points whose primary result does not settle them
// (ulist, *ucount of them); pass 0 counts their other candidates and gives
// each point a block of slots (uoff, ucnt, running total *slot_total), pass
// 1 writes the (point, element) slots into element buckets; select2 applies
// the selection rule to every listed point
hipError_t launch_unsettled(const fpts_mesh *m, int64_t n, const int *cellpt, const int2 *cand,
                            const int32_t *code, const double *r, int *ulist,
                            int *ucount, const EvalRest &rest, hipStream_t s);
hipError_t launch_resolve(const fpts_mesh *m, int pass, int64_t n, const double *pts,
                          const int *cellpt, const int2 *cand, const int *ulist,
                          const int *ucount, int *uoff, int *ucnt, unsigned long long *slot_total,
                          int *elem_cnt2, const int *elem_off2, int *elem_fill2, int *slot_pt,
                          int *slot_elem, int *sorted2, int64_t cap2, int *olist, int *ocount,
                          hipStream_t s);
hipError_t launch_select2(const fpts_mesh *m, int64_t n, const int *ulist, const int *ucount,
                          const int *uoff, const int *ucnt, const int2 *cand,
                          const int *slot_elem, int64_t cap2, const double *res_r,
                          const double *res_dist, const int *res_code, int32_t *code,
                          int32_t *elem, double *r, double *dist, hipStream_t s);
// which: 1 = nearest-node start, 2 = Newton, 3 = both
hipError_t launch_newton(const fpts_mesh *m, int precision, int64_t n, const double *pts,
                         const NewtonIO &io, int which, hipStream_t s);
// fused rest, split into element buckets and a per-point list: phase 0
// zeroes the counts of elements with few points, phase 1 places every binned
// point (bucket at its rank, or the list, *count entries)
hipError_t launch_eval_split(const fpts_mesh *m, int64_t n, const int32_t *elem, const int *rank,
                             int *elem_cnt, const int *elem_off, int *sorted, int *list,
                             int *count, int phase, hipStream_t s);
// interpolation of the listed points, one lane per point
hipError_t launch_eval_sparse(const fpts_mesh *m, int64_t n, const double *r, int n_fields,
                              int field_n, const double *field, double *out,
                              const int32_t *elem, const int *list, const int *count,
                              hipStream_t s);
// interpolation binning; with `cand` (fused find + interpolate) the
// points their primary result settled are left out (r is read for that)
// (pass 0 keeps each point's rank in its element's bucket, pass 1 uses it)
// the same over a list of points (*count of them) whose results are final
// and found (no NaN writes): pass 0 counts per element and keeps each entry's
// rank, pass 1 places the points
hipError_t launch_eval_bin_list(const fpts_mesh *m, int pass, const int *list, const int *count,
                                int64_t cap, const int32_t *elem, int *elem_cnt,
                                const int *elem_off, int *rank, int *sorted, hipStream_t s);
hipError_t launch_eval_bin(const fpts_mesh *m, int pass, int64_t n, const int32_t *code,
                           const int32_t *elem, const double *r, const int2 *cand,
                           int n_fields, double *out, int *elem_cnt, const int *elem_off,
                           int *rank, int *sorted, hipStream_t s);
// field_n: GLL nodes per direction of the field (its own order, 2..kMaxN)
hipError_t launch_eval(const fpts_mesh *m, int64_t n, const double *r, int n_fields, int field_n,
                       const double *field, double *out, const int *sorted,
                       const int *elem_off, const int *chunk_off, const int *task_elem,
                       int64_t task_bound, hipStream_t s, const double *rs = nullptr);
hipError_t launch_nodes32(const fpts_mesh *m, hipStream_t s);
// score rows of the nearest-node contraction: per element and node j,
// (-2 x_j, -2 y_j, -2 z_j, |x_j|^2) element-local (D = 2: (-2x, -2y, |x|^2, 0)),
// padding columns j >= N^R score 1e300
hipError_t launch_near_rows(const fpts_mesh *m, hipStream_t s);

// Newton launchers per element kind (kernels_newton.hip; lines:
// kernels_newton_line.hip)
hipError_t launch_newton_hex(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                             const NewtonIO &io, int which, hipStream_t s);
hipError_t launch_newton_quad(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s);
hipError_t launch_newton_surf(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s);
// line elements (kernels_newton_line.hip): FP64 in every mode
hipError_t launch_newton_line(const fpts_mesh *m, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s);

// particle transport step (lpt.hip): drag, Adams-Bashforth 2 / Euler, box
// boundary; all arrays [D][n]
struct LptArgs {
    double *x, *v, *hist_v, *hist_a;
    const double *u;
    const int32_t *code;
    int64_t n;
    double tau, dt;
    double lo[3], hi[3];
    int periodic[3];
    int first;
};
hipError_t launch_lpt_advance(const fpts_mesh *m, const LptArgs &a, hipStream_t s);

}  // namespace fpts
