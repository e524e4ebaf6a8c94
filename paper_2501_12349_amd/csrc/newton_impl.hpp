// Trust-region Newton inversion of the element map (Section 3.2.1) for
// (point, candidate element) pairs grouped by element.  Shared by the
// per-element-kind translation units kernels_newton_*.hip.
//
// Work decomposition: pairs are bucketed by element; a task is a chunk of up
// to 64 pairs of ONE element, run by one wavefront with one pair per lane.
// The wave copies the element's nodal coordinates into LDS once per task
// (coalesced 16-byte loads); all lanes then read the same LDS words
// (broadcast) while each evaluates the map at its own reference point by sum
// factorisation
//     A_jk = sum_i x_ijk phi_i(r),  B_k = sum_j A_jk phi_j(s),
//     x = sum_k B_k phi_k(t)   (and the derivative variants),
// without re-reading the element per point.  Waves take tasks from an
// atomic counter until none are left.
//
// Map evaluation comes in two sweeps over the element:
//   sweep 1: x(r) and G = dx/dr            2N^3 + 3N^2 + 4N FMAs per coordinate
//   sweep 2: S_ab = sum_c dx_c d2x_c/dr_a dr_b, the second-derivative term
//            of the Hessian (eq. eq_newton_hessian), contracted with the
//            lane's residual dx before the sum over nodes, so one set of
//            accumulators serves all coordinates.
// Sweep 2 runs only when a lane has accepted a point on a face or edge of
// the reference box (the only places the paper uses beta = 1), and for the
// rare case of a rejected first step from a start node on the boundary.
//
// Mixed precision: an FP32 phase runs the same iteration on FP32 nodes
// stored as offsets from the element centre (the point shifted the same way
// in FP64 before rounding) to ||dr|| < 1e-5 or 10 passes; the FP64 phase
// then restarts the iteration from that r with alpha = 1.  Codes, distances
// and the final residual come from the FP64 phase.
#pragma once
#include <cfloat>

#include "fpts_internal.hpp"
#include "gll_table.hpp"

namespace fpts {
namespace newton {

// Element nodal data is staged in LDS once per task and read by every lane
// at the same address (broadcast reads).
template <typename T> struct CPtr { typedef const T *type; };

template <typename T> __device__ inline T eps_of();
template <> __device__ inline double eps_of<double>() { return DBL_EPSILON; }
template <> __device__ inline float eps_of<float>() { return FLT_EPSILON; }

struct NewtonArgs {
    const double *nodes;     // [nel][D][NP]
    const float *nodes32;    // [nel][D][NP] (mixed mode)
    const double *xc;        // [nel][D]     (mixed mode)
    const double *pts;       // [D][n]
    int n;
    int nel;
    NewtonIO io;
    int max_iter;
    double tol;
    double eps_d;
    int max_iter32;
    float tol32;
};

// Packed symmetric R x R matrices: diagonal first, then the upper triangle.
template <int R> constexpr int kSym = R * (R + 1) / 2;
template <int R>
__device__ constexpr int sym(int a, int b)
{
    if (a == b) return a;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return R == 2 ? 2 : (lo == 0 ? (hi == 1 ? 3 : 4) : 5);
}

// phi_i, phi_i' (and phi_i'') at r for all i, in product form
// w_i prod_{m!=i}(r - z_m), by prefix and suffix products carried with
// their first two derivatives.
template <typename T, int N, bool H2>
struct Bas {
    T v[N], d[N], dd[H2 ? N : 1];
};

template <typename T, int N, bool H2>
__device__ __forceinline__ void make_basis(T r, Bas<T, N, H2> &b)
{
    constexpr gll::Table<N> G = gll::Nodes<N>::t;
    T pv[N], pd[N], pdd[N];
    pv[0] = T(1);
    pd[0] = T(0);
    pdd[0] = T(0);
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const T t = r - T(G.z[i - 1]);
        if (H2) pdd[i] = pdd[i - 1] * t + T(2) * pd[i - 1];
        pd[i] = pd[i - 1] * t + pv[i - 1];
        pv[i] = pv[i - 1] * t;
    }
    T sv = T(1), sd = T(0), sdd = T(0);
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        b.v[i] = T(G.w[i]) * (pv[i] * sv);
        b.d[i] = T(G.w[i]) * (pd[i] * sv + pv[i] * sd);
        if (H2) b.dd[H2 ? i : 0] = T(G.w[i]) * (pdd[i] * sv + T(2) * pd[i] * sd + pv[i] * sdd);
        const T t = r - T(G.z[i]);
        if (H2) sdd = sdd * t + T(2) * sd;
        sd = sd * t + sv;
        sv = sv * t;
    }
}

// Shift a basis table down by one entry, so that a loop over a runtime index
// k always finds entry k at position 0 (register arrays cannot be indexed at
// run time without leaving registers).
template <typename T, int N, bool H2>
__device__ __forceinline__ void rotate(Bas<T, N, H2> &b)
{
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) {
        b.v[i] = b.v[i + 1];
        b.d[i] = b.d[i + 1];
        if (H2) b.dd[H2 ? i : 0] = b.dd[H2 ? i + 1 : 0];
    }
}

// Sweep 1: x(q) and G = dx/dr.
template <typename T, int D, int R, int N>
__device__ __forceinline__ void sweep1(typename CPtr<T>::type xe, const T (&q)[R], T (&X)[D],
                                       T (&G)[D][R])
{
    Bas<T, N, false> b0, b1;
    make_basis<T, N, false>(q[0], b0);
    make_basis<T, N, false>(q[1], b1);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        X[c] = T(0);
#pragma unroll
        for (int a = 0; a < R; ++a) G[c][a] = T(0);
    }
    if constexpr (R == 3) {
        constexpr int NP = N * N * N;
        Bas<T, N, false> b2;
        make_basis<T, N, false>(q[2], b2);
#pragma unroll 1
        for (int k = 0; k < N; ++k) {
            const T tv = b2.v[0], td = b2.d[0];
            rotate(b2);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T B0 = 0, Br = 0, Bs = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    T A0 = 0, A1 = 0;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        const T xv = xe[c * NP + i + N * (j + N * k)];
                        A0 = fma(xv, b0.v[i], A0);
                        A1 = fma(xv, b0.d[i], A1);
                    }
                    B0 = fma(A0, b1.v[j], B0);
                    Br = fma(A1, b1.v[j], Br);
                    Bs = fma(A0, b1.d[j], Bs);
                }
                X[c] = fma(B0, tv, X[c]);
                G[c][0] = fma(Br, tv, G[c][0]);
                G[c][1] = fma(Bs, tv, G[c][1]);
                G[c][2] = fma(B0, td, G[c][2]);
            }
        }
    } else {
        constexpr int NP = N * N;
#pragma unroll 1
        for (int j = 0; j < N; ++j) {
            const T sv = b1.v[0], sd = b1.d[0];
            rotate(b1);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T A0 = 0, A1 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const T xv = xe[c * NP + i + N * j];
                    A0 = fma(xv, b0.v[i], A0);
                    A1 = fma(xv, b0.d[i], A1);
                }
                X[c] = fma(A0, sv, X[c]);
                G[c][0] = fma(A1, sv, G[c][0]);
                G[c][1] = fma(A0, sd, G[c][1]);
            }
        }
    }
}

// Sweep 2: S_ab = sum_c dx_c d2x_c/dr_a dr_b at q (symmetric, packed).
template <typename T, int D, int R, int N>
__device__ __forceinline__ void sweep2(typename CPtr<T>::type xe, const T (&q)[R],
                                       const T (&dx)[D], T (&S)[kSym<R>])
{
    Bas<T, N, true> b0, b1;
    make_basis<T, N, true>(q[0], b0);
    make_basis<T, N, true>(q[1], b1);
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) S[a] = T(0);
    if constexpr (R == 3) {
        constexpr int NP = N * N * N;
        Bas<T, N, true> b2;
        make_basis<T, N, true>(q[2], b2);
#pragma unroll 1
        for (int k = 0; k < N; ++k) {
            const T tv = b2.v[0], td = b2.d[0], tdd = b2.dd[0];
            rotate(b2);
            T B0 = 0, Br = 0, Bs = 0, Brr = 0, Brs = 0, Bss = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                T A0 = 0, A1 = 0, A2 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    T wv = T(0);
#pragma unroll
                    for (int c = 0; c < D; ++c) wv = fma(dx[c], xe[c * NP + i + N * (j + N * k)], wv);
                    A0 = fma(wv, b0.v[i], A0);
                    A1 = fma(wv, b0.d[i], A1);
                    A2 = fma(wv, b0.dd[i], A2);
                }
                B0 = fma(A0, b1.v[j], B0);
                Br = fma(A1, b1.v[j], Br);
                Bs = fma(A0, b1.d[j], Bs);
                Brr = fma(A2, b1.v[j], Brr);
                Brs = fma(A1, b1.d[j], Brs);
                Bss = fma(A0, b1.dd[j], Bss);
            }
            S[0] = fma(Brr, tv, S[0]);
            S[1] = fma(Bss, tv, S[1]);
            S[2] = fma(B0, tdd, S[2]);
            S[3] = fma(Brs, tv, S[3]);
            S[4] = fma(Br, td, S[4]);
            S[5] = fma(Bs, td, S[5]);
        }
    } else {
        constexpr int NP = N * N;
#pragma unroll 1
        for (int j = 0; j < N; ++j) {
            const T sv = b1.v[0], sd = b1.d[0], sdd = b1.dd[0];
            rotate(b1);
            T A0 = 0, A1 = 0, A2 = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T wv = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) wv = fma(dx[c], xe[c * NP + i + N * j], wv);
                A0 = fma(wv, b0.v[i], A0);
                A1 = fma(wv, b0.d[i], A1);
                A2 = fma(wv, b0.dd[i], A2);
            }
            S[0] = fma(A2, sv, S[0]);
            S[1] = fma(A0, sdd, S[1]);
            S[2] = fma(A1, sd, S[2]);
        }
    }
}

// Objective at a point: f = |x* - x|^2, g = G^T dx, Hgn = G^T G (packed).
template <typename T, int D, int R>
struct Obj {
    T f;
    T g[R];
    T Hgn[kSym<R>];
};

template <typename T, int D, int R>
__device__ __forceinline__ void objective(const T (&xs)[D], const T (&X)[D], const T (&G)[D][R],
                                          Obj<T, D, R> &o, T (&dx)[D])
{
    o.f = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) o.g[a] = T(0);
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) o.Hgn[a] = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        dx[c] = xs[c] - X[c];
        o.f = fma(dx[c], dx[c], o.f);
#pragma unroll
        for (int a = 0; a < R; ++a) {
            o.g[a] = fma(G[c][a], dx[c], o.g[a]);
#pragma unroll
            for (int b = a; b < R; ++b) o.Hgn[sym<R>(a, b)] = fma(G[c][a], G[c][b], o.Hgn[sym<R>(a, b)]);
        }
    }
}

// Solve H dr = g on the free coordinates (rows/columns of held coordinates
// replaced by the identity, right-hand side 0) by LDL^T; false when a pivot
// is not positive.
template <typename T, int R>
__device__ __forceinline__ bool solve_free(const T (&H)[kSym<R>], const T (&g)[R],
                                           const bool (&held)[R], T (&x)[R])
{
    T A[R][R], b[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        b[a] = held[a] ? T(0) : g[a];
#pragma unroll
        for (int c = 0; c < R; ++c)
            A[a][c] = (held[a] || held[c]) ? (a == c ? T(1) : T(0)) : H[sym<R>(a, c)];
    }
    T L[R][R], d[R];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < R; ++a) {
        T s = A[a][a];
#pragma unroll
        for (int k = 0; k < a; ++k) s -= L[a][k] * L[a][k] * d[k];
        d[a] = s;
        ok = ok && (s > T(0));
        const T inv = T(1) / s;
#pragma unroll
        for (int c = a + 1; c < R; ++c) {
            T t = A[c][a];
#pragma unroll
            for (int k = 0; k < a; ++k) t -= L[c][k] * L[a][k] * d[k];
            L[c][a] = t * inv;
        }
    }
    T y[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        T s = b[a];
#pragma unroll
        for (int k = 0; k < a; ++k) s -= L[a][k] * y[k];
        y[a] = s;
    }
#pragma unroll
    for (int a = R - 1; a >= 0; --a) {
        T s = y[a] / d[a];
#pragma unroll
        for (int k = a + 1; k < R; ++k) s -= L[k][a] * x[k];
        x[a] = s;
    }
    return ok;
}

enum { M_INIT = 0, M_STEP = 1, M_REFRESH = 2 };

struct LaneStats {
    unsigned long long passes = 0, evals = 0, evals_h2 = 0, passes32 = 0, evals32 = 0,
                       evals_h2_exec = 0;
};

template <typename T, int R>
__device__ __forceinline__ bool on_face(const T (&r)[R])
{
    bool b = false;
#pragma unroll
    for (int a = 0; a < R; ++a) b = b || (fabs(r[a]) == T(1));
    return b;
}

// The iteration of Section 3.2.1 for one lane; all lanes of the wave step
// together and `active` masks finished ones.  r holds the start on entry and
// the result on exit, f the squared distance.  Each trip evaluates the map
// once (sweep 1) at the start point (INIT), the trial point (STEP) or the
// current point (REFRESH: a face pass needs second derivatives that were not
// computed there yet); sweep 2 follows when some lane needs S at the point.
template <typename T, int D, int R, int N, bool IS32>
__device__ __forceinline__ void newton_loop(typename CPtr<T>::type xe, const T (&xs)[D],
                                            T (&r)[R], T &f, bool active, int max_iter, T tol,
                                            LaneStats &st)
{
    T xnorm = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) xnorm = fma(xs[c], xs[c], xnorm);
    xnorm = sqrt(xnorm);
    Obj<T, D, R> cur;
    T Hs[kSym<R>];
    cur.f = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) cur.g[a] = T(0);
#pragma unroll
    for (int a = 0; a < kSym<R>; ++a) {
        cur.Hgn[a] = T(0);
        Hs[a] = T(0);
    }
    bool hb_ok = false;
    T alpha = T(1);
    int mode = M_INIT, pass = 0;
    T q[R], pred = T(0), dmax = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) q[a] = r[a];
    for (int trip = 0; trip < 2 * max_iter + 2; ++trip) {
        if (!__any(active)) break;
        if (active && mode == M_STEP) {
            const bool beta = (pass > 0) && on_face(r);
            if (beta && !hb_ok) {
                mode = M_REFRESH;
#pragma unroll
                for (int a = 0; a < R; ++a) q[a] = r[a];
            } else {
                T H[kSym<R>];
#pragma unroll
                for (int a = 0; a < kSym<R>; ++a) H[a] = beta ? cur.Hgn[a] - Hs[a] : cur.Hgn[a];
                bool held[R];
#pragma unroll
                for (int a = 0; a < R; ++a)
                    held[a] = (r[a] == T(1) && cur.g[a] > T(0)) ||
                              (r[a] == T(-1) && cur.g[a] < T(0));
                T x[R];
                bool ok = solve_free<T, R>(H, cur.g, held, x);
                if (!ok && beta) {
#pragma unroll
                    for (int a = 0; a < kSym<R>; ++a) H[a] = cur.Hgn[a];
                    ok = solve_free<T, R>(H, cur.g, held, x);
                }
                T dr[R];
                dmax = T(0);
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    T d = ok ? x[a] : T(0);
                    d = fmin(fmax(d, -alpha), alpha);
                    const T t = fmin(fmax(r[a] + d, T(-1)), T(1));
                    q[a] = t;
                    dr[a] = t - r[a];
                    dmax = fmax(dmax, fabs(dr[a]));
                }
                T gd = T(0), dHd = T(0);
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    gd = fma(cur.g[a], dr[a], gd);
#pragma unroll
                    for (int b = 0; b < R; ++b) dHd = fma(dr[a] * H[sym<R>(a, b)], dr[b], dHd);
                }
                pred = T(2) * gd - dHd;
            }
        }
        T X[D], G[D][R], dxn[D];
        sweep1<T, D, R, N>(xe, q, X, G);
        Obj<T, D, R> nw;
        objective<T, D, R>(xs, X, G, nw, dxn);
        bool need_s2 = false;
        if (active) {
            if (IS32) st.evals32++;
            else st.evals++;
            if (mode == M_INIT) {
                cur = nw;
                hb_ok = false;
                mode = M_STEP;
            } else if (mode == M_REFRESH) {
                need_s2 = true;
            } else {
                ++pass;
                if (IS32) st.passes32++;
                else st.passes++;
                bool accept, stop = false;
                if (dmax < tol) {
                    accept = true;
                    stop = true;
                } else {
                    const T decr = cur.f - nw.f;
                    const T sf = sqrt(cur.f);
                    const T noise = T(64) * eps_of<T>() * sf * (xnorm + sf);
                    if (pred > T(0) && pred <= noise) {
                        accept = true;
                    } else if (pred > T(0) && decr >= T(0.9) * pred) {
                        accept = true;
                        alpha *= T(2);
                    } else if (pred > T(0) && decr >= T(0.01) * pred) {
                        accept = true;
                    } else {
                        accept = false;
                        alpha *= T(0.25);
                    }
                }
                if (accept) {
#pragma unroll
                    for (int a = 0; a < R; ++a) r[a] = q[a];
                    cur = nw;
                    hb_ok = false;
                }
                if (stop || pass >= max_iter) active = false;
                // the next pass uses beta = 1 here only if r sits on a face
                need_s2 = accept && active && on_face(r);
            }
        }
        if (__any(need_s2)) {
            T S[kSym<R>];
            sweep2<T, D, R, N>(xe, q, dxn, S);
            if (need_s2) {
#pragma unroll
                for (int a = 0; a < kSym<R>; ++a) Hs[a] = S[a];
                hb_ok = true;
                mode = M_STEP;
                if (!IS32) st.evals_h2++;
            }
            if (active && !IS32) st.evals_h2_exec++;
        }
    }
    f = cur.f;
}

// Nearest element node (Euclidean; lowest index on ties) -> its reference
// coordinates (Section 3.2.1 initial guess).
template <typename T, int D, int R, int N>
__device__ __forceinline__ void nearest_node(typename CPtr<T>::type xe, const T (&xs)[D],
                                             T (&r)[R])
{
    constexpr gll::Table<N> G = gll::Nodes<N>::t;
    constexpr int NP = (R == 3) ? N * N * N : N * N;
    T best = T(__builtin_huge_valf());
    int bi = 0;
#pragma unroll 1
    for (int row = 0; row < NP / N; ++row) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int idx = row * N + i;
            T d2 = T(0);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T t = xs[c] - xe[c * NP + idx];
                d2 = fma(t, t, d2);
            }
            if (d2 < best) {
                best = d2;
                bi = idx;
            }
        }
    }
    const int ii[3] = {bi % N, (bi / N) % N, bi / (N * N)};
#pragma unroll
    for (int a = 0; a < R; ++a) {
        T v = T(G.z[0]);
#pragma unroll
        for (int m = 1; m < N; ++m)
            if (ii[a] == m) v = T(G.z[m]);
        r[a] = v;
    }
}

// Copy `count` values (a multiple of 2) of one element into LDS with 16-byte
// loads spread over the wave, then wait for the whole wave.
template <typename T>
__device__ __forceinline__ void stage(T *lds, const T *src, int count, int lane)
{
    typedef __attribute__((ext_vector_type(4))) unsigned int u4;
    const int words = count * (int)sizeof(T) / 16;
    const u4 *s = reinterpret_cast<const u4 *>(src);
    u4 *d = reinterpret_cast<u4 *>(lds);
    for (int k = lane; k < words; k += kWave) d[k] = s[k];
    const int tail = count * (int)sizeof(T) - words * 16;   // 0 or 8 bytes
    if (tail && lane == 0) {
        const unsigned long long *s8 = reinterpret_cast<const unsigned long long *>(src);
        reinterpret_cast<unsigned long long *>(lds)[words * 2] = s8[words * 2];
    }
    __syncthreads();
}

template <int D, int R, int N, bool MIXED>
__global__ __launch_bounds__(64) void k_newton(NewtonArgs a)
{
    constexpr int NP = (R == 3) ? N * N * N : N * N;
    extern __shared__ double lds_nodes[];
    const int lane = threadIdx.x;
    const NewtonIO &io = a.io;
    const int total = io.chunk_off[a.nel];
    LaneStats st;
    unsigned long long pairs = 0;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(io.counter, 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
        if (t >= total) break;
        // element of task t: last e with chunk_off[e] <= t
        int lo = 0, hi = a.nel;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (io.chunk_off[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int e = __builtin_amdgcn_readfirstlane(lo);
        const int beg = io.elem_off[e] + (t - io.chunk_off[e]) * kChunk;
        const int end = min(io.elem_off[e + 1], beg + kChunk);
        const int idx = beg + lane;
        const bool has = idx < end;
        const int item = has ? io.list[idx] : 0;
        const int p = has ? (io.slot_pt ? io.slot_pt[item] : item) : 0;
        pairs += has ? 1 : 0;
        double xs[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xs[c] = has ? a.pts[(size_t)c * a.n + p] : 0.0;
        double r[R], f = 0.0;
        __syncthreads();   // the previous task is done with the LDS copy
        if constexpr (MIXED) {
            float *xl32 = reinterpret_cast<float *>(lds_nodes);
            stage<float>(xl32, a.nodes32 + (size_t)e * D * NP, D * NP, lane);
            float xs32[D], r32[R], f32;
#pragma unroll
            for (int c = 0; c < D; ++c) xs32[c] = (float)(xs[c] - a.xc[(size_t)e * D + c]);
            nearest_node<float, D, R, N>(xl32, xs32, r32);
            newton_loop<float, D, R, N, true>(xl32, xs32, r32, f32, has, a.max_iter32, a.tol32,
                                              st);
#pragma unroll
            for (int k = 0; k < R; ++k) r[k] = (double)r32[k];
            __syncthreads();
            stage<double>(lds_nodes, a.nodes + (size_t)e * D * NP, D * NP, lane);
        } else {
            stage<double>(lds_nodes, a.nodes + (size_t)e * D * NP, D * NP, lane);
            nearest_node<double, D, R, N>(lds_nodes, xs, r);
        }
        newton_loop<double, D, R, N, false>(lds_nodes, xs, r, f, has, a.max_iter, a.tol, st);
        if (has) {
            bool inside = true;
#pragma unroll
            for (int k = 0; k < R; ++k) inside = inside && (fabs(r[k]) < 1.0);
            if (R < D) inside = inside && (f < a.eps_d);
            io.code[item] = inside ? FPTS_INTERIOR : FPTS_BORDER;
            if (io.elem) io.elem[item] = e;
            io.dist[item] = sqrt(f);
#pragma unroll
            for (int k = 0; k < R; ++k) io.r[(size_t)k * io.ostride + item] = r[k];
        }
    }
    // wave-reduce the counters, one atomic per wave and counter
    unsigned long long v[7] = {pairs, st.passes, st.evals, st.evals_h2, st.passes32, st.evals32,
                               st.evals_h2_exec};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        unsigned long long x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0 && x) atomicAdd(&io.stats[k], x);
    }
}

typedef void (*KernelFn)(NewtonArgs);

template <int D, int R, bool MIXED>
KernelFn pick_kernel(int N)
{
    switch (N) {
    case 2: return k_newton<D, R, 2, MIXED>;
    case 3: return k_newton<D, R, 3, MIXED>;
    case 4: return k_newton<D, R, 4, MIXED>;
    case 5: return k_newton<D, R, 5, MIXED>;
    case 6: return k_newton<D, R, 6, MIXED>;
    case 7: return k_newton<D, R, 7, MIXED>;
    case 8: return k_newton<D, R, 8, MIXED>;
    case 9: return k_newton<D, R, 9, MIXED>;
    case 10: return k_newton<D, R, 10, MIXED>;
    default: return nullptr;
    }
}

template <int D, int R>
hipError_t launch_newton_kind(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, hipStream_t s)
{
    KernelFn fn = mixed ? pick_kernel<D, R, true>(m->N) : pick_kernel<D, R, false>(m->N);
    if (!fn) return hipErrorInvalidValue;
    NewtonArgs a;
    a.nodes = m->d_nodes;
    a.nodes32 = m->d_nodes32;
    a.xc = m->d_xc;
    a.pts = pts;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.io = io;
    a.max_iter = m->p.max_iter;
    a.tol = m->p.newton_tol;
    a.eps_d = m->p.surf_eps_d;
    a.max_iter32 = 10;
    a.tol32 = 1e-5f;
    const size_t lds = sizeof(double) * (size_t)m->D * m->NP;
    hipLaunchKernelGGL(fn, dim3(m->cus * 16), dim3(64), lds, s, a);
    return hipGetLastError();
}

}  // namespace newton
}  // namespace fpts
