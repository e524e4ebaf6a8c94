// Nearest-node start and trust-region Newton for line elements (D_r = 1) in
// 2D and 3D: Section 3.2.1 with one reference coordinate and the manifold
// codes of Section 4.4.
//
// Pairs arrive bucketed by element in tasks of at most 64 (the task grid of
// the other kernels); a wave takes one task and each lane one pair.  The
// element's D x N node coordinates are wave-uniform, read with scalar loads,
// so a lane's map evaluation is N-term sums on the VALU: x(r), x'(r) and,
// where the Hessian needs them, x''(r), with the Lagrange bases and their
// derivatives in product form.  With a single reference coordinate there is
// no contraction for the matrix cores to take.  Every pass follows the
// oracle's order of operations; a 1 x 1 Cholesky factor is used for the
// solve, as there.
#include <cfloat>

#include "fpts_internal.hpp"
#include "gll_table.hpp"

namespace fpts {
namespace {

typedef const __attribute__((address_space(4))) double cdouble;

struct LineArgs {
    const double *nodes;    // [nel][D][N]
    const double *pts;      // [D][n]
    int n;
    int nel;
    NewtonIO io;
    int max_iter;
    double tol;
    double eps_d;
    int which;              // 1: nearest-node start, 2: Newton from io.r, 3: both
};

// phi_i(r) = w_i prod_{m != i} (r - z_m) and its first two derivatives from
// prefix and suffix product jets (value, first, second derivative).
template <int N>
__device__ inline void line_basis(double r, double (&v)[N], double (&d1)[N], double (&d2)[N])
{
    constexpr gll::Table<N> T = gll::Nodes<N>::t;
    double pv[N], pd[N], pe[N];
    pv[0] = 1.0;
    pd[0] = 0.0;
    pe[0] = 0.0;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const double a = r - T.z[i - 1];
        pe[i] = pe[i - 1] * a + 2.0 * pd[i - 1];
        pd[i] = pd[i - 1] * a + pv[i - 1];
        pv[i] = pv[i - 1] * a;
    }
    double sv = 1.0, sd = 0.0, se = 0.0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        v[i] = T.w[i] * (pv[i] * sv);
        d1[i] = T.w[i] * (pd[i] * sv + pv[i] * sd);
        d2[i] = T.w[i] * (pe[i] * sv + 2.0 * pd[i] * sd + pv[i] * se);
        const double a = r - T.z[i];
        se = se * a + 2.0 * sd;
        sd = sd * a + sv;
        sv = sv * a;
    }
}

template <int D, int N>
__device__ inline void line_map(const double (&X)[D][N], double r, double (&x)[D], double (&g)[D],
                                double (&h)[D])
{
    double v[N], d1[N], d2[N];
    line_basis<N>(r, v, d1, d2);
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double a = 0.0, b = 0.0, e = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            a = fma(X[c][i], v[i], a);
            b = fma(X[c][i], d1[i], b);
            e = fma(X[c][i], d2[i], e);
        }
        x[c] = a;
        g[c] = b;
        h[c] = e;
    }
}

__device__ inline unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int D, int N>
__global__ __launch_bounds__(64) void k_newton_line(LineArgs a)
{
    constexpr gll::Table<N> T = gll::Nodes<N>::t;
    const NewtonIO &io = a.io;
    const int lane = threadIdx.x;
    const int total = io.chunk_off[a.nel];
    unsigned long long n_pairs = 0, n_passes = 0, n_evals = 0, n_h2 = 0;
    for (int t = task_of_block(); t < total; t += gridDim.x) {
        const int e = __builtin_amdgcn_readfirstlane(io.task_elem[t]);
        const int beg = io.elem_off[e] + (t - io.chunk_off[e]) * kChunk;
        const int end = min(io.elem_off[e + 1], beg + kChunk);
        const int idx = beg + lane;
        cdouble *xe = (cdouble *)(a.nodes + (size_t)e * D * N);
        double X[D][N];
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
            for (int i = 0; i < N; ++i) X[c][i] = xe[c * N + i];
        if (idx >= end) continue;
        const int item = io.list[idx];
        const int p = io.slot_pt ? io.slot_pt[item] : item;
        double xs[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xs[c] = a.pts[(size_t)c * a.n + p];
        double r;
        if (a.which & 1) {
            // start: the nearest node, ties to the lowest index
            double best = INFINITY;
            int bi = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double d2 = 0.0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const double q = xs[c] - X[c][i];
                    d2 += q * q;
                }
                if (d2 < best) {
                    best = d2;
                    bi = i;
                }
            }
            r = T.z[0];
#pragma unroll
            for (int i = 1; i < N; ++i)
                if (bi == i) r = T.z[i];
            if (!(a.which & 2)) {
                io.r[item] = r;
                continue;
            }
        } else {
            r = io.r[item];
        }
        double x[D], G[D], Hx[D], dx[D], f = 0.0, xn2 = 0.0;
        line_map<D, N>(X, r, x, G, Hx);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            dx[c] = xs[c] - x[c];
            f += dx[c] * dx[c];
            xn2 += xs[c] * xs[c];
        }
        const double xnorm = sqrt(xn2);
        ++n_pairs;
        ++n_evals;
        double alpha = 1.0;
        bool converged = false;
        for (int l = 0; l < a.max_iter; ++l) {
            ++n_passes;
            double g = 0.0, H = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                g += G[c] * dx[c];
                H += G[c] * G[c];
            }
            const bool onb = fabs(r) == 1.0;
            if (l > 0 && onb) {
                // beta = 1: the residual-weighted second derivative
                ++n_h2;
#pragma unroll
                for (int c = 0; c < D; ++c) H -= dx[c] * Hx[c];
            }
            const bool active = (r == 1.0 && g > 0.0) || (r == -1.0 && g < 0.0);
            double dr = 0.0;
            if (!active) {
                if (!(H > 0.0) || !__builtin_isfinite(H)) {
                    H = 0.0;   // not SPD: G^T G
#pragma unroll
                    for (int c = 0; c < D; ++c) H += G[c] * G[c];
                }
                if (H > 0.0 && __builtin_isfinite(H)) {
                    const double L = sqrt(H);
                    dr = (g / L) / L;
                }
            }
            double d = fmin(fmax(dr, -alpha), alpha);
            const double rn = fmin(fmax(r + d, -1.0), 1.0);
            dr = rn - r;
            const double dmax = fabs(dr);
            double xn[D], Gn[D], Hn[D], dxn[D], fn = 0.0;
            line_map<D, N>(X, rn, xn, Gn, Hn);
            ++n_evals;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                dxn[c] = xs[c] - xn[c];
                fn += dxn[c] * dxn[c];
            }
            bool accept, conv = false;
            if (dmax < a.tol) {
                accept = true;
                conv = true;
            } else {
                const double pred = 2.0 * (g * dr) - dr * H * dr, decr = f - fn;
                const double sf = sqrt(f);
                const double noise = 64.0 * DBL_EPSILON * sf * (xnorm + sf);
                if (pred > 0.0 && pred <= noise) {
                    accept = true;
                } else if (pred > 0.0 && decr >= 0.9 * pred) {
                    accept = true;
                    alpha *= 2.0;
                } else if (pred > 0.0 && decr >= 0.01 * pred) {
                    accept = true;
                } else {
                    accept = false;
                    alpha *= 0.25;
                }
            }
            if (accept) {
                r = rn;
                f = fn;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    x[c] = xn[c];
                    G[c] = Gn[c];
                    Hx[c] = Hn[c];
                    dx[c] = dxn[c];
                }
            }
            if (conv) {
                converged = true;
                break;
            }
        }
        if (io.conv) io.conv[item] = converged ? 1 : 0;
        const bool inside = fabs(r) < 1.0 && f < a.eps_d;
        io.code[item] = inside ? FPTS_INTERIOR : FPTS_BORDER;
        if (io.elem) io.elem[item] = e;
        io.r[item] = r;
        io.dist[item] = sqrt(f);
        if (io.rs) io.rs[idx] = inside && 1.0 - fabs(r) > kSettleGuard ? r : __builtin_nan("");
    }
    // counters: pairs, passes, evaluations, evaluations with x''
    n_pairs = wave_sum(n_pairs);
    n_passes = wave_sum(n_passes);
    n_evals = wave_sum(n_evals);
    n_h2 = wave_sum(n_h2);
    if (lane == 0 && n_pairs) {
        atomicAdd(&io.stats[0], n_pairs);
        atomicAdd(&io.stats[1], n_passes);
        atomicAdd(&io.stats[2], n_evals);
        atomicAdd(&io.stats[3], n_h2);
    }
}

typedef void (*LineFn)(LineArgs);

template <int D>
LineFn pick_line(int N)
{
    switch (N) {
    case 2: return k_newton_line<D, 2>;
    case 3: return k_newton_line<D, 3>;
    case 4: return k_newton_line<D, 4>;
    case 5: return k_newton_line<D, 5>;
    case 6: return k_newton_line<D, 6>;
    case 7: return k_newton_line<D, 7>;
    case 8: return k_newton_line<D, 8>;
    case 9: return k_newton_line<D, 9>;
    case 10: return k_newton_line<D, 10>;
    default: return nullptr;
    }
}

}  // namespace

hipError_t launch_newton_line(const fpts_mesh *m, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s)
{
    if (m->R != 1 || n <= 0) return m->R != 1 ? hipErrorInvalidValue : hipSuccess;
    LineFn fn = m->D == 2 ? pick_line<2>(m->N) : pick_line<3>(m->N);
    if (!fn) return hipErrorInvalidValue;
    LineArgs a;
    a.nodes = m->d_nodes;
    a.pts = pts;
    a.n = (int)n;
    a.nel = (int)m->nel;
    a.io = io;
    a.max_iter = io.max_iter > 0 ? io.max_iter : m->p.max_iter;
    a.tol = m->p.newton_tol;
    a.eps_d = m->p.surf_eps_d;
    // phase C calls the start (which 1) and the iteration (which 2) apart;
    // the second call recomputes nothing but reads the start back
    a.which = which & 3;
    hipLaunchKernelGGL(fn, dim3(task_grid(io.task_bound, m->cus)), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace fpts
