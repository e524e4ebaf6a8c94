// Interpolate (Section 3.3): u_f(r*) = sum_ijk u_f,ijk phi_i(r) phi_j(s)
// phi_k(t) (eq. eq_u_tensor) at the computational coordinates from Find.
//
// Points are first counted and scattered into per-element buckets (the
// grouping by element the paper's CPU code uses, Section 5 remark), then a
// wavefront takes up to 64 points of ONE element, stages the element's nodal
// values in LDS (once per wave, not once per point) and each lane contracts
// them sum-factorised: N^3 + N^2 + N FMAs per field and point.  On quad, hex
// and surface meshes the first contraction runs on the matrix cores, 16
// points at a time (k_eval_mfma): every lane reading the same staged value
// (a broadcast, 64 copies per read) left the per-lane form bound by LDS
// bandwidth.  Line meshes keep the per-lane form.
// Also: the FP32 element-local node copy used by mixed-precision Newton.
#include "fpts_internal.hpp"
#include "gll_table.hpp"
#include "newton_mfma.hpp"

namespace fpts {
namespace {

// fused find + interpolate: elements holding at most this many of the
// remaining points have them interpolated one lane per point
constexpr int kSparseMax = 4;

// pass 0: count points per element, keep each point's rank in its bucket
// (-1 for points not binned) and write NaN for NOT_FOUND points; pass 1:
// place point ids at their ranks in their element's bucket.  With `cand`
// (fused find + interpolate) the points that their primary result settled
// are left out: the fused pass over Find's primary list has them.
__global__ __launch_bounds__(256) void k_eval_bin(int pass, int n, int nel, int R,
                                                 const int32_t *code, const int32_t *elem,
                                                 const double *r, const int2 *cand,
                                                 int n_fields, double *out, int *elem_cnt,
                                                 const int *elem_off, int *rank,
                                                 int *sorted)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < n;
    if (pass == 1) {
        // rank[p] < 0: not binned
        if (!in) return;
        const int k = rank[p], e = elem[p];
        if (k >= 0) sorted[elem_off[e] + k] = p;
        return;
    }
    // pass 0, no early exit (wave_inc needs every lane); all of a point's
    // loads are issued at once
    int e = -1, pr = -1;
    int32_t cd = FPTS_NOT_FOUND;
    double rr[3] = {0.0, 0.0, 0.0};
    if (in) {
        e = elem[p];
        cd = code[p];
        if (cand) {
            pr = cand[p].y;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < R) rr[k] = r[(size_t)k * n + p];
        }
    }
    const bool found = in && cd != FPTS_NOT_FOUND && e >= 0 && e < nel;
    bool done = false;
    if (cand && found && cd == FPTS_INTERIOR && pr == e) {
        double mg = 1.0;
        for (int k = 0; k < R; ++k) mg = fmin(mg, 1.0 - fabs(rr[k]));
        done = mg > kSettleGuard;
    }
    const bool bin = found && !done;
    const int k = wave_inc(elem_cnt, e, bin);
    if (in) rank[p] = bin ? k : -1;
    if (in && !found)
        for (int f = 0; f < n_fields; ++f) out[(size_t)f * n + p] = __builtin_nan("");
}

// k_eval_bin over a list of found points (grid-stride; the loop bound is
// uniform per wavefront, as wave_inc needs)
__global__ __launch_bounds__(256) void k_eval_bin_list(int pass, const int *list,
                                                      const int *count, int nel,
                                                      const int32_t *elem, int *elem_cnt,
                                                      const int *elem_off, int *rank,
                                                      int *sorted)
{
    const int cnt = *count;
    const int lane = threadIdx.x & 63;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i - lane < cnt;
         i += gridDim.x * blockDim.x) {
        const bool act = i < cnt;
        const int p = act ? list[i] : 0;
        const int e = act ? elem[p] : -1;
        const bool ok = act && e >= 0 && e < nel;
        if (pass == 0) {
            const int k = wave_inc(elem_cnt, e, ok);
            if (act) rank[i] = ok ? k : -1;
        } else if (ok && rank[i] >= 0) {
            sorted[elem_off[e] + rank[i]] = p;
        }
    }
}

template <int N>
__device__ __forceinline__ void basis_v(double r, const double *z, const double *w, double (&v)[N])
{
    double pv[N];
    pv[0] = 1.0;
#pragma unroll
    for (int i = 1; i < N; ++i) pv[i] = pv[i - 1] * (r - z[i - 1]);
    double sv = 1.0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        v[i] = w[i] * (pv[i] * sv);
        sv *= r - z[i];
    }
}

struct EvalArgs {
    const double *r;        // [R][n]
    int n;
    int nel;
    int n_fields;
    const double *field;    // [n_fields][nel][NP]
    double *out;            // [n_fields][n]
    const int *sorted;
    const int *elem_off;
    const int *chunk_off;
    const int *task_elem;   // task -> element (task grid)
    Basis basis;
    // fused mode (rs != null): `sorted` is the primary list of Find and
    // r comes from rs[k * n + list position]; NaN there skips the point
    const double *rs;
    int f0;                 // first field of this launch (k_eval_mfma)
    // k_eval_mfma: walk the elements (every wave at most a few of them)
    // instead of the task grid
    int by_elem;
};

typedef const __attribute__((address_space(4))) double cdouble;

// sum over the element's nodal values u of one field times the tensor bases
template <int R, int N, typename P>
__device__ __forceinline__ double contract(P u, const double (&v0)[N], const double (&v1)[N],
                                           const double (&v2)[N])
{
    double acc = 0.0;
    if constexpr (R == 3) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double B = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                double A = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) A = fma(u[i + N * (j + N * k)], v0[i], A);
                B = fma(A, v1[j], B);
            }
            acc = fma(B, v2[k], acc);
        }
    } else if constexpr (R == 2) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double A = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) A = fma(u[i + N * j], v0[i], A);
            acc = fma(A, v1[j], acc);
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) acc = fma(u[i], v0[i], acc);
    }
    return acc;
}

// LDS: the element's nodal values of each field are staged in LDS with
// coalesced loads and read by every lane at the same address (broadcast);
// otherwise they are read with scalar loads.  Staging wins when an element
// holds few points (its values are cold, and scalar loads of them stall on
// latency); when many tasks share an element its values stay in the scalar
// cache and the scalar operands save the LDS reads.  The staged loads are
// software-pipelined: the values of the next field (or of the next task's
// first field) are loaded into registers while the current field is
// contracted, so their latency hides behind the arithmetic.
template <int R, int N, bool LDS>
__global__ __launch_bounds__(64) void k_eval(EvalArgs a)
{
    constexpr int NP = (R == 3) ? N * N * N : (R == 2) ? N * N : N;
    constexpr int PER = (NP + 63) / 64;   // staged values per lane
    extern __shared__ double ldsu[];   // [NP] (LDS staging)
    const int lane = threadIdx.x;
    const int total = a.chunk_off[a.nel];
    const int G = gridDim.x;
    double pre[PER];
    // the nodal values of field f of element e into pre
    auto fetch = [&](int e, int f) {
        const double *src = a.field + ((size_t)f * a.nel + e) * NP;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int j = lane + 64 * k;
            pre[k] = (NP % 64 == 0 || j < NP) ? src[j] : 0.0;
        }
    };
    int t = task_of_block();
    if (LDS && t < total && a.n_fields > 0)
        fetch(__builtin_amdgcn_readfirstlane(a.task_elem[t]), 0);
    for (; t < total; t += G) {
        const int e = __builtin_amdgcn_readfirstlane(a.task_elem[t]);
        const int beg = a.elem_off[e] + (t - a.chunk_off[e]) * kChunk;
        const int end = min(a.elem_off[e + 1], beg + kChunk);
        const int idx = beg + lane;
        bool has = idx < end;
        const int p = has ? a.sorted[idx] : 0;
        double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (has) rr[k] = a.rs ? a.rs[(size_t)k * a.n + idx] : a.r[(size_t)k * a.n + p];
        if (a.rs) has = has && !__builtin_isnan(rr[0]);
        double v0[N], v1[N], v2[N];
        basis_v<N>(has ? rr[0] : 0.0, a.basis.z, a.basis.w, v0);
        if (R >= 2) basis_v<N>(has ? rr[1] : 0.0, a.basis.z, a.basis.w, v1);
        if (R == 3) basis_v<N>(has ? rr[2] : 0.0, a.basis.z, a.basis.w, v2);
        for (int f = 0; f < a.n_fields; ++f) {
            double acc;
            if constexpr (LDS) {
                __syncthreads();   // the previous field's reads come first
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int j = lane + 64 * k;
                    if (NP % 64 == 0 || j < NP) ldsu[j] = pre[k];
                }
                __syncthreads();
                if (f + 1 < a.n_fields) fetch(e, f + 1);
                else if (t + G < total) fetch(__builtin_amdgcn_readfirstlane(a.task_elem[t + G]), 0);
                acc = contract<R, N>((const double *)ldsu, v0, v1, v2);
            } else {
                acc = contract<R, N>((cdouble *)(a.field + ((size_t)f * a.nel + e) * NP), v0, v1,
                                     v2);
            }
            if (has) a.out[(size_t)f * a.n + p] = acc;
        }
    }
}

// Interpolation with the first contraction on the matrix cores (quad, hex
// and surface meshes; FC fields a0.f0 .. a.f0 + FC - 1 per launch).  One
// wavefront per element (the first of its 64-point tasks in the task grid;
// the element's other tasks are skipped): the FC fields of the element are
// staged in LDS once (layout of the Newton kernels' node block, one field
// per coordinate slot), and its points are taken 64 and then 16 at a time,
// one per slot of four lanes (slot = lane % 16, quarter g = lane /
// 16).  Quarter g builds the bases of direction g of its slot's point; then
// C_f[row][s] = sum_i u_f[i][row] phi_i(r_s) by v_mfma_f64_16x16x4 (A = the
// element's values, row = (j, k) or j; B = the slots' phi_i), each lane
// weights its four rows of each tile with phi_j(s) phi_k(t) of its slot
// (hexes with N = 4, 8: summed over k first, then weighted per j), and the
// four lanes of a slot are summed.  A point's value depends on its own
// coordinates and element only, not on the group it lands in.
// The wave walks the elements e, e + G, ... (G = grid size; each XCD a
// contiguous range per round) and skips those without points; the fields
// of its next element are loaded into registers while the current one is
// contracted, and the bucket offsets of the one after are loaded then too,
// so that an element's staging does not wait on memory.  (Two waves per
// SIMD: the prefetched fields take 48 VGPRs; the LDS footprint, 15 KiB per
// wave for three fields of N = 8, allowed at most ten waves per CU anyway.)
template <int R, int N, int FC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void
k_eval_mfma(EvalArgs a)
{
    typedef newton::Shape<3, R, N> S;
    typedef newton::NodeLds<double, FC, R, N> L;
    typedef newton::Factor<R, N> F;
    typedef newton::V4<double>::type v4;
    constexpr int NP = S::NP, MT = S::MT, KS = S::KS, ROWS = S::ROWS;
    constexpr int PER = (NP + 63) / 64;
    constexpr bool kFullA = (N % 4 == 0) && (ROWS % 16 == 0);
    extern __shared__ double lds_eval[];
    double *xl = lds_eval;        // the FC fields, NodeLds layout
    double *tab = xl + L::SIZE;   // [R][N][16] bases of the group's points
    const int lane = threadIdx.x, slot = lane & 15, g = lane >> 4;
    const int G = gridDim.x, nel = a.nel;
    double v[FC][PER];
    auto load_fields = [&](int en) __attribute__((always_inline)) {
#pragma unroll
        for (int f = 0; f < FC; ++f) {
            const double *src = a.field + ((size_t)(a.f0 + f) * nel + en) * NP;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int j = lane + 64 * k;
                v[f][k] = (NP % 64 == 0 || j < NP) ? src[j] : 0.0;
            }
        }
    };
    // the element's FC fields, from v into LDS
    auto stage_fields = [&]() __attribute__((always_inline)) {
        __syncthreads();   // the previous element's reads come first
#pragma unroll
        for (int f = 0; f < FC; ++f)
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int j = lane + 64 * k;
                if (NP % 64 == 0 || j < NP) xl[L::at(f, j / N, j % N)] = v[f][k];
            }
        __syncthreads();
    };
    // the points of the staged element: list positions [ebeg, eend)
    auto points = [&](int ebeg, int eend) __attribute__((always_inline)) {
        for (int beg = ebeg; beg < eend; beg += kChunk) {
        const int end = min(eend, beg + kChunk);
        const int idx = beg + lane;
        bool has = idx < end;
        const int p = has ? a.sorted[idx] : 0;
        double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (has) rr[k] = a.rs ? a.rs[(size_t)k * a.n + idx] : a.r[(size_t)k * a.n + p];
        if (a.rs) has = has && !__builtin_isnan(rr[0]);
        const int ngrp = (end - beg + 15) >> 4;
        for (int grp = 0; grp < ngrp; ++grp) {
            const int pl = 16 * grp + slot;   // task position of this slot's point
            // coordinate g of that point (each coordinate shuffled, then the
            // quarter's one selected)
            const double c0 = __shfl(rr[0], pl);
            const double c1 = R >= 2 ? __shfl(rr[1], pl) : 0.0;
            const double c2 = R == 3 ? __shfl(rr[2], pl) : 0.0;
            const double x = g == 0 ? c0 : g == 1 ? c1 : c2;
            newton::wave_lds_sync();   // the previous group's table reads come first
            if (g < R) {
                double pv[N];
                pv[0] = 1.0;
#pragma unroll
                for (int i = 1; i < N; ++i) pv[i] = pv[i - 1] * (x - a.basis.z[i - 1]);
                double sv = 1.0;
#pragma unroll
                for (int i = N - 1; i >= 0; --i) {
                    tab[(g * N + i) * 16 + slot] = a.basis.w[i] * (pv[i] * sv);
                    sv *= x - a.basis.z[i];
                }
            }
            newton::wave_lds_sync();
            const double *ts = tab + N * 16, *tt = tab + 2 * N * 16;
            double b0[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int i = 4 * ks + g;
                b0[ks] = i < N ? tab[i * 16 + slot] : 0.0;
            }
            double X[FC], Z[F::NJ][FC];
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                X[f] = 0.0;
#pragma unroll
                for (int js = 0; js < F::NJ; ++js) Z[js][f] = 0.0;
            }
#pragma unroll(MT <= 4 ? MT : 1)
            for (int m = 0; m < MT; ++m) {
                v4 acc[FC];
#pragma unroll
                for (int f = 0; f < FC; ++f) acc[f] = v4{0, 0, 0, 0};
                const int arow = 16 * m + slot;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int ai = 4 * ks + g;
                    const bool aok = kFullA || (arow < ROWS && ai < N);
#pragma unroll
                    for (int f = 0; f < FC; ++f)
                        acc[f] = newton::mfma16(xl[aok ? L::at(f, arow, ai) : 0], b0[ks], acc[f]);
                }
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int row = newton::out_row(m, g, qq);
                    if (ROWS % 16 != 0 && row >= ROWS) continue;
                    if constexpr (F::ON) {
                        const int k = (16 * m + 4 * qq) / N, js = qq % F::NJ;
                        const double tv = tt[k * 16 + slot];
#pragma unroll
                        for (int f = 0; f < FC; ++f) Z[js][f] = fma(acc[f][qq], tv, Z[js][f]);
                    } else {
                        const double w = R == 3 ? ts[(row % N) * 16 + slot] * tt[(row / N) * 16 + slot]
                                                : ts[row * 16 + slot];
#pragma unroll
                        for (int f = 0; f < FC; ++f) X[f] = fma(acc[f][qq], w, X[f]);
                    }
                }
            }
            if constexpr (F::ON) {
#pragma unroll
                for (int js = 0; js < F::NJ; ++js) {
                    const double sv = ts[(g + 4 * js) * 16 + slot];
#pragma unroll
                    for (int f = 0; f < FC; ++f) X[f] = fma(Z[js][f], sv, X[f]);
                }
            }
            newton::slot_sum_all(X);
            const bool hp = __shfl((int)has, pl) != 0;
            const int pp = __shfl(p, pl);
            // quarter g writes field g of its slot's point
#pragma unroll
            for (int f = 0; f < FC; ++f)
                if (hp && g == f) a.out[(size_t)(a.f0 + f) * a.n + pp] = X[f];
        }
        }
    };
    if (!a.by_elem) {
        // task grid: the element's first task takes all its points, so that
        // its fields are staged once (its other tasks have nothing to do)
        const int total = a.chunk_off[nel];
        for (int t = task_of_block(); t < total; t += G) {
            const int e = __builtin_amdgcn_readfirstlane(a.task_elem[t]);
            if (t != a.chunk_off[e]) continue;
            load_fields(e);
            stage_fields();
            points(a.elem_off[e], a.elem_off[e + 1]);
        }
        return;
    }
    // element walk: the wave's first element with points from e0 on, in
    // steps of G (nel when none), its bucket range in o0, o1
    auto busy_from = [&](int e0, int &o0, int &o1) __attribute__((always_inline)) {
        int en = e0;
        for (; en < nel; en += G) {
            o0 = a.elem_off[en];
            o1 = a.elem_off[en + 1];
            if (o1 > o0) break;
        }
        return en;
    };
    int ebeg = 0, eend = 0;
    int e = busy_from(task_of_block(), ebeg, eend);
    if (e < nel) load_fields(e);
    // offsets of the element after the next, loaded one element ahead
    int nb = 0, nnb = 0;
    int en = e + G;
    if (en < nel) {
        nb = a.elem_off[en];
        nnb = a.elem_off[en + 1];
    }
    while (e < nel) {
        stage_fields();   // fields loaded during the previous element
        // the next element with points: en, whose offsets arrived meanwhile
        // (past an empty one the search goes on from there)
        if (en < nel && !(nnb > nb)) en = busy_from(en + G, nb, nnb);
        const int n0 = nb, n1 = nnb;
        if (en < nel) {
            load_fields(en);
            if (en + G < nel) {
                nb = a.elem_off[en + G];
                nnb = a.elem_off[en + G + 1];
            }
        }
        points(ebeg, eend);
        e = en;
        ebeg = n0;
        eend = n1;
        en = e + G;
    }
}

// Line meshes: points of elements that hold at most kSparseMax of the
// points to interpolate, one lane per point: a wavefront per element task
// would run the whole element's contraction for one or two points.  Each
// lane reads its own element's nodal values (global loads), with the
// arithmetic of k_eval, so both give the same bits.  Grid-stride over the
// list.
template <int R, int N>
__global__ __launch_bounds__(256) void k_eval_sparse(EvalArgs a, const int32_t *elem,
                                                    const int *list, const int *count)
{
    constexpr int NP = (R == 3) ? N * N * N : (R == 2) ? N * N : N;
    const int cnt = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const int p = list[i];
        const int e = elem[p];
        double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k) rr[k] = a.r[(size_t)k * a.n + p];
        double v0[N], v1[N], v2[N];
        basis_v<N>(rr[0], a.basis.z, a.basis.w, v0);
        if (R >= 2) basis_v<N>(rr[1], a.basis.z, a.basis.w, v1);
        if (R == 3) basis_v<N>(rr[2], a.basis.z, a.basis.w, v2);
        for (int f = 0; f < a.n_fields; ++f) {
            const double *src = a.field + ((size_t)f * a.nel + e) * NP;
            a.out[(size_t)f * a.n + p] = contract<R, N>(src, v0, v1, v2);
        }
    }
}

// Elements with at most kSparseMax binned points drop out of the bucket
// counts (their points go to the per-point list).
__global__ __launch_bounds__(256) void k_eval_dense(int nel, int *elem_cnt)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nel && elem_cnt[e] <= kSparseMax) elem_cnt[e] = 0;
}

// Pass 1 with the split: a binned point (rank >= 0) of a dense element goes
// to its bucket, one of a sparse element to the list.  A block takes
// kSplitChunk consecutive points, gathers its listed points in LDS and
// reserves their places with one atomic (same-address device atomics
// serialise).
constexpr int kSplitChunk = 4096;

__global__ __launch_bounds__(256) void k_eval_split(int n, const int32_t *elem, const int *rank,
                                                   const int *dense_cnt, const int *elem_off,
                                                   int *sorted, int *list, int *count)
{
    __shared__ int lst[kSplitChunk];
    __shared__ int lcnt, gbase;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) lcnt = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSplitChunk;
    for (int it = 0; it < kSplitChunk / 256; ++it) {
        const int64_t q = base + it * 256 + threadIdx.x;
        const int p = (int)q;
        bool sp = false;
        if (q < n) {
            const int k = rank[p], e = elem[p];
            if (k >= 0) {
                if (dense_cnt[e] > 0) sorted[elem_off[e] + k] = p;
                else sp = true;
            }
        }
        const unsigned long long m = __ballot(sp);
        if (m) {
            int at = 0;
            if (lane == 0) at = atomicAdd(&lcnt, __popcll(m));
            at = __shfl(at, 0, 64);
            if (sp) lst[at + __popcll(m & ((1ull << lane) - 1))] = p;
        }
    }
    __syncthreads();
    const int cnt = lcnt;
    if (cnt == 0) return;
    if (threadIdx.x == 0) gbase = atomicAdd(count, cnt);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 256) list[gbase + i] = lst[i];
}

__global__ void k_nodes32(const double *nodes, const double *xc, float *out, int64_t nel, int D,
                          int NP)
{
    const int64_t total = nel * D * NP;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / ((int64_t)D * NP);
        const int c = (int)((i / NP) % D);
        out[i] = (float)(nodes[i] - xc[e * D + c]);
    }
}

__global__ void k_near_rows(const double *nodes, const double *xc, double *rows, int64_t nel,
                            int D, int NP, int npad)
{
    const int64_t total = nel * npad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / npad;
        const int j = (int)(i % npad);
        double b[4] = {0.0, 0.0, 0.0, 0.0};
        if (j < NP) {
            double n2 = 0.0;
            for (int c = 0; c < D; ++c) {
                const double v = nodes[(e * D + c) * NP + j] - xc[e * D + c];
                b[c] = -2.0 * v;
                n2 = fma(v, v, n2);
            }
            b[D] = n2;
        } else {
            b[D] = 1e300;
        }
        for (int k = 0; k < 4; ++k) rows[(e * 4 + k) * npad + j] = b[k];
    }
}

typedef void (*EvalFn)(EvalArgs);

template <int R, bool LDS>
EvalFn pick_eval(int N)
{
    switch (N) {
    case 2: return k_eval<R, 2, LDS>;
    case 3: return k_eval<R, 3, LDS>;
    case 4: return k_eval<R, 4, LDS>;
    case 5: return k_eval<R, 5, LDS>;
    case 6: return k_eval<R, 6, LDS>;
    case 7: return k_eval<R, 7, LDS>;
    case 8: return k_eval<R, 8, LDS>;
    case 9: return k_eval<R, 9, LDS>;
    case 10: return k_eval<R, 10, LDS>;
    default: return nullptr;
    }
}

typedef void (*SparseFn)(EvalArgs, const int32_t *, const int *, const int *);

template <int R>
SparseFn pick_sparse(int N)
{
    switch (N) {
    case 2: return k_eval_sparse<R, 2>;
    case 3: return k_eval_sparse<R, 3>;
    case 4: return k_eval_sparse<R, 4>;
    case 5: return k_eval_sparse<R, 5>;
    case 6: return k_eval_sparse<R, 6>;
    case 7: return k_eval_sparse<R, 7>;
    case 8: return k_eval_sparse<R, 8>;
    case 9: return k_eval_sparse<R, 9>;
    case 10: return k_eval_sparse<R, 10>;
    default: return nullptr;
    }
}

template <int R, int FC>
EvalFn pick_eval_mfma(int N, size_t *lds)
{
    switch (N) {
#define FPTS_CASE(NN)                                                                      \
    case NN:                                                                               \
        *lds = sizeof(double) * (newton::NodeLds<double, FC, R, NN>::SIZE + R * NN * 16);  \
        return k_eval_mfma<R, NN, FC>;
        FPTS_CASE(2)
        FPTS_CASE(3)
        FPTS_CASE(4)
        FPTS_CASE(5)
        FPTS_CASE(6)
        FPTS_CASE(7)
        FPTS_CASE(8)
        FPTS_CASE(9)
        FPTS_CASE(10)
#undef FPTS_CASE
    default: return nullptr;
    }
}

template <int R>
EvalFn pick_eval_mfma_fc(int N, int fc, size_t *lds)
{
    return fc == 3 ? pick_eval_mfma<R, 3>(N, lds)
                   : fc == 2 ? pick_eval_mfma<R, 2>(N, lds) : pick_eval_mfma<R, 1>(N, lds);
}

template <bool LDS>
EvalFn pick_eval_r(int R, int N)
{
    return R == 1 ? pick_eval<1, LDS>(N) : nullptr;   // line meshes
}

}  // namespace

hipError_t launch_eval_bin_list(const fpts_mesh *m, int pass, const int *list, const int *count,
                                int64_t cap, const int32_t *elem, int *elem_cnt,
                                const int *elem_off, int *rank, int *sorted, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((cap + 255) / 256,
                                                                 (int64_t)m->cus * 16));
    hipLaunchKernelGGL(k_eval_bin_list, dim3(grid), dim3(256), 0, s, pass, list, count,
                       (int)m->nel, elem, elem_cnt, elem_off, rank, sorted);
    return hipGetLastError();
}

hipError_t launch_eval_bin(const fpts_mesh *m, int pass, int64_t n, const int32_t *code,
                           const int32_t *elem, const double *r, const int2 *cand,
                           int n_fields, double *out, int *elem_cnt, const int *elem_off,
                           int *rank, int *sorted, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_bin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pass,
                       (int)n, (int)m->nel, m->R, code, elem, r, cand, n_fields, out,
                       elem_cnt, elem_off, rank, sorted);
    return hipGetLastError();
}

hipError_t launch_eval(const fpts_mesh *m, int64_t n, const double *r, int n_fields, int field_n,
                       const double *field, double *out, const int *sorted, const int *elem_off,
                       const int *chunk_off, const int *task_elem, int64_t task_bound,
                       hipStream_t s, const double *rs)
{
    EvalArgs a;
    a.r = r;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.n_fields = n_fields;
    a.field = field;
    a.out = out;
    a.sorted = sorted;
    a.elem_off = elem_off;
    a.chunk_off = chunk_off;
    a.task_elem = task_elem;
    a.rs = rs;
    a.f0 = 0;
    if (field_n == m->N) a.basis = m->basis;
    else gll::fill(field_n, a.basis.z, a.basis.w);
    const dim3 grid(task_grid(task_bound, m->cus));
    // the matrix-core kernel walks the elements when every wave has at most
    // eight of them to visit (many points); else it follows the task grid
    a.by_elem = (int64_t)grid.x * 8 >= m->nel;
    if (m->R >= 2) {
        // matrix cores, up to three fields per launch
        for (int f0 = 0; f0 < n_fields; f0 += 3) {
            size_t lds = 0;
            const int fc = std::min(3, n_fields - f0);
            EvalFn fn = m->R == 3 ? pick_eval_mfma_fc<3>(field_n, fc, &lds)
                                  : pick_eval_mfma_fc<2>(field_n, fc, &lds);
            if (!fn) return hipErrorInvalidValue;
            a.f0 = f0;
            hipLaunchKernelGGL(fn, grid, dim3(64), lds, s, a);
        }
        return hipGetLastError();
    }
    // line meshes: stage in LDS unless elements hold many points (several
    // tasks each)
    const bool lds = n <= (int64_t)4 * kChunk * m->nel;
    EvalFn fn = lds ? pick_eval_r<true>(m->R, field_n) : pick_eval_r<false>(m->R, field_n);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, grid, dim3(64), lds ? sizeof(double) * field_n : 0, s, a);
    return hipGetLastError();
}

hipError_t launch_eval_split(const fpts_mesh *m, int64_t n, const int32_t *elem, const int *rank,
                             int *elem_cnt, const int *elem_off, int *sorted, int *list,
                             int *count, int phase, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (phase == 0) {
        hipLaunchKernelGGL(k_eval_dense, dim3((unsigned)((m->nel + 255) / 256)), dim3(256), 0, s,
                           (int)m->nel, elem_cnt);
    } else {
        hipLaunchKernelGGL(k_eval_split, dim3((unsigned)((n + kSplitChunk - 1) / kSplitChunk)),
                           dim3(256), 0, s, (int)n, elem, rank, elem_cnt, elem_off, sorted, list,
                           count);
    }
    return hipGetLastError();
}

hipError_t launch_eval_sparse(const fpts_mesh *m, int64_t n, const double *r, int n_fields,
                              int field_n, const double *field, double *out,
                              const int32_t *elem, const int *list, const int *count,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // line meshes only: the other meshes interpolate every point on the
    // matrix cores (the same bits in both calls need the same arithmetic)
    SparseFn fn = m->R == 1 ? pick_sparse<1>(field_n) : nullptr;
    if (!fn) return hipErrorInvalidValue;
    EvalArgs a{};
    a.r = r;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.n_fields = n_fields;
    a.field = field;
    a.out = out;
    if (field_n == m->N) a.basis = m->basis;
    else gll::fill(field_n, a.basis.z, a.basis.w);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, m->cus * 8));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, a, elem, list, count);
    return hipGetLastError();
}

hipError_t launch_near_rows(const fpts_mesh *m, hipStream_t s)
{
    const int64_t total = m->nel * m->near_npad;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_near_rows, dim3(grid), dim3(256), 0, s, m->d_nodes, m->d_xc, m->d_near,
                       (int64_t)m->nel, m->D, m->NP, m->near_npad);
    return hipGetLastError();
}

hipError_t launch_nodes32(const fpts_mesh *m, hipStream_t s)
{
    hipLaunchKernelGGL(k_nodes32, dim3(4096), dim3(256), 0, s, m->d_nodes, m->d_xc,
                       m->d_nodes32, (int64_t)m->nel, m->D, m->NP);
    return hipGetLastError();
}

}  // namespace fpts
