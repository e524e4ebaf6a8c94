// Trust-region Newton inversion of the element map (Section 3.2.1) for all
// (point, candidate element) pairs, grouped by element.
//
// Work decomposition: pairs are bucketed by element; a task is a chunk of
// up to 64 pairs of ONE element and is run by one wavefront, one pair per
// lane.  Because the element is wave-uniform its nodal coordinates are read
// with scalar loads (through the scalar cache) and enter the FMAs as SGPR
// operands, so each lane evaluates x(r), G = dx/dr and, on faces/edges, the
// second derivatives by sum factorisation
//     A_jk = sum_i x_ijk phi_i(r),  B_k = sum_j A_jk phi_j(s),
//     x = sum_k B_k phi_k(t)   (and the derivative variants)
// at 2N^3 + 3N^2 + 4N FMAs per coordinate, without re-reading the element
// per point.  Waves take tasks from an atomic counter until none are left.
//
// Mixed precision: an FP32 phase runs the same iteration on FP32 nodes
// stored as offsets from the element centre (and the point shifted the same
// way in FP64 before rounding), to ||dr|| < 1e-5 or 10 passes; the FP64
// phase then restarts the iteration from that r with alpha = 1.  Codes,
// distances and the final residual come from the FP64 phase.
#include <cfloat>

#include "fpts_internal.hpp"

namespace fpts {
namespace {

typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) float cfloat;

template <typename T> struct CPtr;
template <> struct CPtr<double> { typedef cdouble *type; };
template <> struct CPtr<float> { typedef cfloat *type; };

template <typename T> __device__ inline T eps_of();
template <> __device__ inline double eps_of<double>() { return DBL_EPSILON; }
template <> __device__ inline float eps_of<float>() { return FLT_EPSILON; }

struct BasisF {
    float z[16];
    float w[16];
};

struct NewtonArgs {
    const double *nodes;     // [nel][D][NP]
    const float *nodes32;    // [nel][D][NP] (mixed mode)
    const double *xc;        // [nel][D]     (mixed mode)
    const double *pts;       // [D][n]
    int n;
    int nel;
    const int *slot_pt;
    const int *sorted;
    const int *elem_off;
    const int *chunk_off;
    int64_t cap;
    double *res_r;           // [R][cap]
    double *res_dist;        // [cap]
    int *res_code;           // [cap]
    int *counter;
    unsigned long long *stats;
    Basis basis;
    BasisF basis32;
    int max_iter;
    double tol;
    double eps_d;
    int mixed;
    int max_iter32;
    float tol32;
};

// phi_i, phi_i', phi_i'' at r in product form w_i prod_{m!=i}(r - z_m), by
// prefix and suffix products carried with their first two derivatives.
template <typename T, int N, bool H2>
struct Bas {
    T v[N], d[N], dd[H2 ? N : 1];
};

template <typename T, int N, bool H2>
__device__ __forceinline__ void make_basis(T r, const T *z, const T *w, Bas<T, N, H2> &b)
{
    T pv[N], pd[N], pdd[N];
    pv[0] = T(1);
    pd[0] = T(0);
    pdd[0] = T(0);
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const T t = r - z[i - 1];
        if (H2) pdd[i] = pdd[i - 1] * t + T(2) * pd[i - 1];
        pd[i] = pd[i - 1] * t + pv[i - 1];
        pv[i] = pv[i - 1] * t;
    }
    T sv = T(1), sd = T(0), sdd = T(0);
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        b.v[i] = w[i] * (pv[i] * sv);
        b.d[i] = w[i] * (pd[i] * sv + pv[i] * sd);
        if (H2) b.dd[H2 ? i : 0] = w[i] * (pdd[i] * sv + T(2) * pd[i] * sd + pv[i] * sdd);
        const T t = r - z[i];
        if (H2) sdd = sdd * t + T(2) * sd;
        sd = sd * t + sv;
        sv = sv * t;
    }
}

// Objective data at one reference point: f = |x* - x|^2, g = G^T dx,
// Hgn = G^T G, Hs = -sum_c dx_c d2x_c/dr dr (only with H2).
template <typename T, int R>
struct Obj {
    T f;
    T g[R];
    T Hgn[R][R];
    T Hs[R][R];
};

template <typename T, int R>
__device__ __forceinline__ void obj_zero(Obj<T, R> &o)
{
    o.f = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) {
        o.g[a] = T(0);
#pragma unroll
        for (int b = 0; b < R; ++b) {
            o.Hgn[a][b] = T(0);
            o.Hs[a][b] = T(0);
        }
    }
}

template <typename T, int R, bool H2>
__device__ __forceinline__ void obj_add(Obj<T, R> &o, T dx, const T (&G)[R], const T (&S)[R][R])
{
    o.f += dx * dx;
#pragma unroll
    for (int a = 0; a < R; ++a) {
        o.g[a] += G[a] * dx;
#pragma unroll
        for (int b = 0; b < R; ++b) {
            o.Hgn[a][b] += G[a] * G[b];
            if (H2) o.Hs[a][b] -= dx * S[a][b];
        }
    }
}

// Hex element: D = R = 3.
template <typename T, int D, int N, bool H2>
__device__ __forceinline__ void eval_hex(typename CPtr<T>::type xe, const T (&xs)[D],
                                         const Bas<T, N, H2> &br, const Bas<T, N, H2> &bs,
                                         const Bas<T, N, H2> &bt, Obj<T, 3> &o)
{
    constexpr int NP = N * N * N;
    obj_zero(o);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T X = 0, Xr = 0, Xs = 0, Xt = 0, Xrr = 0, Xss = 0, Xtt = 0, Xrs = 0, Xrt = 0, Xst = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T B0 = 0, Br = 0, Bs = 0, Brr = 0, Brs = 0, Bss = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                T A0 = 0, A1 = 0, A2 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const T xv = xe[c * NP + i + N * (j + N * k)];
                    A0 = fma(xv, br.v[i], A0);
                    A1 = fma(xv, br.d[i], A1);
                    if (H2) A2 = fma(xv, br.dd[H2 ? i : 0], A2);
                }
                B0 = fma(A0, bs.v[j], B0);
                Br = fma(A1, bs.v[j], Br);
                Bs = fma(A0, bs.d[j], Bs);
                if (H2) {
                    Brr = fma(A2, bs.v[j], Brr);
                    Brs = fma(A1, bs.d[j], Brs);
                    Bss = fma(A0, bs.dd[H2 ? j : 0], Bss);
                }
            }
            X = fma(B0, bt.v[k], X);
            Xr = fma(Br, bt.v[k], Xr);
            Xs = fma(Bs, bt.v[k], Xs);
            Xt = fma(B0, bt.d[k], Xt);
            if (H2) {
                Xrr = fma(Brr, bt.v[k], Xrr);
                Xrs = fma(Brs, bt.v[k], Xrs);
                Xss = fma(Bss, bt.v[k], Xss);
                Xrt = fma(Br, bt.d[k], Xrt);
                Xst = fma(Bs, bt.d[k], Xst);
                Xtt = fma(B0, bt.dd[H2 ? k : 0], Xtt);
            }
        }
        const T G[3] = {Xr, Xs, Xt};
        const T S[3][3] = {{Xrr, Xrs, Xrt}, {Xrs, Xss, Xst}, {Xrt, Xst, Xtt}};
        obj_add<T, 3, H2>(o, xs[c] - X, G, S);
    }
}

// Quad element (D = 2) or surface quad (D = 3): R = 2.
template <typename T, int D, int N, bool H2>
__device__ __forceinline__ void eval_quad(typename CPtr<T>::type xe, const T (&xs)[D],
                                          const Bas<T, N, H2> &br, const Bas<T, N, H2> &bs,
                                          Obj<T, 2> &o)
{
    constexpr int NP = N * N;
    obj_zero(o);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T X = 0, Xr = 0, Xs = 0, Xrr = 0, Xrs = 0, Xss = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T A0 = 0, A1 = 0, A2 = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T xv = xe[c * NP + i + N * j];
                A0 = fma(xv, br.v[i], A0);
                A1 = fma(xv, br.d[i], A1);
                if (H2) A2 = fma(xv, br.dd[H2 ? i : 0], A2);
            }
            X = fma(A0, bs.v[j], X);
            Xr = fma(A1, bs.v[j], Xr);
            Xs = fma(A0, bs.d[j], Xs);
            if (H2) {
                Xrr = fma(A2, bs.v[j], Xrr);
                Xrs = fma(A1, bs.d[j], Xrs);
                Xss = fma(A0, bs.dd[H2 ? j : 0], Xss);
            }
        }
        const T G[2] = {Xr, Xs};
        const T S[2][2] = {{Xrr, Xrs}, {Xrs, Xss}};
        obj_add<T, 2, H2>(o, xs[c] - X, G, S);
    }
}

template <typename T, int D, int R, int N, bool H2>
__device__ __forceinline__ void eval_obj(typename CPtr<T>::type xe, const T (&xs)[D],
                                         const T (&q)[R], const T *z, const T *w, Obj<T, R> &o)
{
    Bas<T, N, H2> b0, b1;
    make_basis<T, N, H2>(q[0], z, w, b0);
    make_basis<T, N, H2>(q[1], z, w, b1);
    if constexpr (R == 3) {
        Bas<T, N, H2> b2;
        make_basis<T, N, H2>(q[2], z, w, b2);
        eval_hex<T, D, N, H2>(xe, xs, b0, b1, b2, o);
    } else {
        eval_quad<T, D, N, H2>(xe, xs, b0, b1, o);
    }
}

// Solve H dr = g on the free coordinates (rows/columns of held coordinates
// replaced by the identity, right-hand side 0) by LDL^T; false when a pivot
// is not positive.
template <typename T, int R>
__device__ __forceinline__ bool solve_free(const T (&H)[R][R], const T (&g)[R],
                                           const bool (&held)[R], T (&x)[R])
{
    T A[R][R], b[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
        b[a] = held[a] ? T(0) : g[a];
#pragma unroll
        for (int c = 0; c < R; ++c)
            A[a][c] = (held[a] || held[c]) ? (a == c ? T(1) : T(0)) : H[a][c];
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
    unsigned long long passes = 0, evals = 0, evals_h2 = 0, passes32 = 0, evals32 = 0;
};

// The iteration of Section 3.2.1 for one lane (all lanes of the wave step
// together; `active` masks finished lanes).  r holds the start on entry and
// the result on exit; f the squared distance.  Each loop trip makes one map
// evaluation: at the start point (INIT), at the trial point (STEP), or at the
// current point with second derivatives when a face pass needs them and they
// were not computed there yet (REFRESH).
template <typename T, int D, int R, int N, bool IS32>
__device__ __forceinline__ void newton_loop(typename CPtr<T>::type xe, const T (&xs)[D],
                                            T (&r)[R], T &f, bool active, const T *z,
                                            const T *w, int max_iter, T tol, LaneStats &st)
{
    T xnorm = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) xnorm += xs[c] * xs[c];
    xnorm = sqrt(xnorm);
    Obj<T, R> cur;
    obj_zero(cur);
    bool hb_ok = false;
    T alpha = T(1);
    int mode = M_INIT, pass = 0;
    T q[R], dr[R], pred = T(0), dmax = T(0);
#pragma unroll
    for (int a = 0; a < R; ++a) {
        q[a] = r[a];
        dr[a] = T(0);
    }
    for (int trip = 0; trip < 2 * max_iter + 2; ++trip) {
        if (!__any(active)) break;
        bool want_h2 = false;
        if (active && mode == M_STEP) {
            bool onb = false;
#pragma unroll
            for (int a = 0; a < R; ++a) onb = onb || (fabs(r[a]) == T(1));
            const bool beta = (pass > 0) && onb;
            if (beta && !hb_ok) {
                mode = M_REFRESH;
                want_h2 = true;
#pragma unroll
                for (int a = 0; a < R; ++a) q[a] = r[a];
            } else {
                T H[R][R];
#pragma unroll
                for (int a = 0; a < R; ++a)
#pragma unroll
                    for (int b = 0; b < R; ++b)
                        H[a][b] = beta ? cur.Hgn[a][b] + cur.Hs[a][b] : cur.Hgn[a][b];
                bool held[R];
#pragma unroll
                for (int a = 0; a < R; ++a)
                    held[a] = (r[a] == T(1) && cur.g[a] > T(0)) ||
                              (r[a] == T(-1) && cur.g[a] < T(0));
                T x[R];
                bool ok = solve_free<T, R>(H, cur.g, held, x);
                if (!ok && beta) {
#pragma unroll
                    for (int a = 0; a < R; ++a)
#pragma unroll
                        for (int b = 0; b < R; ++b) H[a][b] = cur.Hgn[a][b];
                    ok = solve_free<T, R>(H, cur.g, held, x);
                }
                dmax = T(0);
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    T d = ok ? x[a] : T(0);
                    d = fmin(fmax(d, -alpha), alpha);
                    T t = fmin(fmax(r[a] + d, T(-1)), T(1));
                    q[a] = t;
                    dr[a] = t - r[a];
                    dmax = fmax(dmax, fabs(dr[a]));
                    want_h2 = want_h2 || (fabs(t) == T(1));
                }
                T gd = T(0), dHd = T(0);
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    gd += cur.g[a] * dr[a];
#pragma unroll
                    for (int b = 0; b < R; ++b) dHd += dr[a] * H[a][b] * dr[b];
                }
                pred = T(2) * gd - dHd;
            }
        }
        Obj<T, R> nw;
        const bool h2 = __any(active && want_h2);
        if (h2)
            eval_obj<T, D, R, N, true>(xe, xs, q, z, w, nw);
        else
            eval_obj<T, D, R, N, false>(xe, xs, q, z, w, nw);
        if (active) {
            if (IS32) st.evals32++;
            else {
                st.evals++;
                if (h2) st.evals_h2++;
            }
            if (mode == M_INIT) {
                cur = nw;
                hb_ok = h2;
                mode = M_STEP;
            } else if (mode == M_REFRESH) {
#pragma unroll
                for (int a = 0; a < R; ++a)
#pragma unroll
                    for (int b = 0; b < R; ++b) cur.Hs[a][b] = nw.Hs[a][b];
                hb_ok = true;
                mode = M_STEP;
            } else {
                ++pass;
                if (IS32) st.passes32++;
                else st.passes++;
                bool accept;
                bool stop = false;
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
                    hb_ok = h2;
                }
                if (stop || pass >= max_iter) active = false;
            }
        }
    }
    f = cur.f;
}

template <typename T>
__device__ __forceinline__ T pick(const T *z, int idx, int N)
{
    T v = z[0];
#pragma unroll
    for (int m = 1; m < 16; ++m)
        if (m < N && m == idx) v = z[m];
    return v;
}

// Nearest element node (Euclidean; lowest index on ties) -> its reference
// coordinates (Section 3.2.1 initial guess).
template <typename T, int D, int R, int N>
__device__ __forceinline__ void nearest_node(typename CPtr<T>::type xe, const T (&xs)[D],
                                             const T *z, T (&r)[R])
{
    constexpr int NP = (R == 3) ? N * N * N : N * N;
    T best = T(__builtin_huge_valf());
    int bi = 0;
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
    r[0] = pick(z, bi % N, N);
    r[1] = pick(z, (bi / N) % N, N);
    if constexpr (R == 3) r[2] = pick(z, bi / (N * N), N);
}

template <int D, int R, int N>
__global__ __launch_bounds__(64) void k_newton(NewtonArgs a)
{
    constexpr int NP = (R == 3) ? N * N * N : N * N;
    const int lane = threadIdx.x;
    const int total = a.chunk_off[a.nel];
    LaneStats st;
    unsigned long long pairs = 0;
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(a.counter, 1);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
        if (t >= total) break;
        // element of task t: last e with chunk_off[e] <= t
        int lo = 0, hi = a.nel;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.chunk_off[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int e = __builtin_amdgcn_readfirstlane(lo);
        const int beg = a.elem_off[e] + (t - a.chunk_off[e]) * kChunk;
        const int end = min(a.elem_off[e + 1], beg + kChunk);
        const int idx = beg + lane;
        const bool has = idx < end;
        const int s = has ? a.sorted[idx] : 0;
        const int p = has ? a.slot_pt[s] : 0;
        pairs += has ? 1 : 0;
        double xs[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xs[c] = has ? a.pts[(size_t)c * a.n + p] : 0.0;
        cdouble *xe = (cdouble *)(a.nodes + (size_t)e * D * NP);
        double r[R], f = 0.0;
        if (a.mixed) {
            cfloat *xe32 = (cfloat *)(a.nodes32 + (size_t)e * D * NP);
            float xs32[D], r32[R], f32;
#pragma unroll
            for (int c = 0; c < D; ++c) xs32[c] = (float)(xs[c] - a.xc[(size_t)e * D + c]);
            nearest_node<float, D, R, N>(xe32, xs32, a.basis32.z, r32);
            newton_loop<float, D, R, N, true>(xe32, xs32, r32, f32, has, a.basis32.z,
                                              a.basis32.w, a.max_iter32, a.tol32, st);
#pragma unroll
            for (int k = 0; k < R; ++k) r[k] = (double)r32[k];
        } else {
            nearest_node<double, D, R, N>(xe, xs, a.basis.z, r);
        }
        newton_loop<double, D, R, N, false>(xe, xs, r, f, has, a.basis.z, a.basis.w, a.max_iter,
                                            a.tol, st);
        if (has) {
            bool inside = true;
#pragma unroll
            for (int k = 0; k < R; ++k) inside = inside && (fabs(r[k]) < 1.0);
            if (R < D) inside = inside && (f < a.eps_d);
            a.res_code[s] = inside ? FPTS_INTERIOR : FPTS_BORDER;
            a.res_dist[s] = sqrt(f);
#pragma unroll
            for (int k = 0; k < R; ++k) a.res_r[(size_t)k * a.cap + s] = r[k];
        }
    }
    // wave-reduce the counters, one atomic per wave
    unsigned long long v[6] = {pairs, st.passes, st.evals, st.evals_h2, st.passes32, st.evals32};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        unsigned long long x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0 && x) atomicAdd(&a.stats[k], x);
    }
}

typedef void (*KernelFn)(NewtonArgs);

template <int D, int R>
KernelFn pick_kernel(int N)
{
    switch (N) {
    case 2: return k_newton<D, R, 2>;
    case 3: return k_newton<D, R, 3>;
    case 4: return k_newton<D, R, 4>;
    case 5: return k_newton<D, R, 5>;
    case 6: return k_newton<D, R, 6>;
    case 7: return k_newton<D, R, 7>;
    case 8: return k_newton<D, R, 8>;
    case 9: return k_newton<D, R, 9>;
    case 10: return k_newton<D, R, 10>;
    default: return nullptr;
    }
}

}  // namespace

hipError_t launch_newton(const fpts_mesh *m, int precision, int64_t n, const double *pts,
                         const int *slot_pt, const int *sorted, const int *elem_off,
                         const int *chunk_off, int64_t cap, double *res_r, double *res_dist,
                         int *res_code, int *counter, unsigned long long *stats, hipStream_t s)
{
    KernelFn fn = nullptr;
    if (m->D == 3 && m->R == 3) fn = pick_kernel<3, 3>(m->N);
    else if (m->D == 2 && m->R == 2) fn = pick_kernel<2, 2>(m->N);
    else if (m->D == 3 && m->R == 2) fn = pick_kernel<3, 2>(m->N);
    if (!fn) return hipErrorInvalidValue;
    NewtonArgs a;
    a.nodes = m->d_nodes;
    a.nodes32 = m->d_nodes32;
    a.xc = m->d_xc;
    a.pts = pts;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.slot_pt = slot_pt;
    a.sorted = sorted;
    a.elem_off = elem_off;
    a.chunk_off = chunk_off;
    a.cap = cap;
    a.res_r = res_r;
    a.res_dist = res_dist;
    a.res_code = res_code;
    a.counter = counter;
    a.stats = stats;
    a.basis = m->basis;
    for (int i = 0; i < 16; ++i) {
        a.basis32.z[i] = (float)m->basis.z[i];
        a.basis32.w[i] = (float)m->basis.w[i];
    }
    a.max_iter = m->p.max_iter;
    a.tol = m->p.newton_tol;
    a.eps_d = m->p.surf_eps_d;
    a.mixed = precision == FPTS_MIXED;
    a.max_iter32 = 10;
    a.tol32 = 1e-5f;
    const int grid = m->cus * 16;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace fpts
