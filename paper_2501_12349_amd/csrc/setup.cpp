// Host side of Setup (Section 3.1 and 4.1-4.3): GLL basis, piecewise-linear
// basis bounds, per-element AABB and OBB, and the local Cartesian map.  The
// paper runs Setup on the CPU (Section 5); elements are processed in
// parallel with std::thread.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "fpts_internal.hpp"
#include "gll_table.hpp"

namespace fpts {
namespace {

// Legendre P_n and P_n' by recurrence.
void leg(int n, double x, double &p, double &dp)
{
    double a = 1.0, b = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    p = b;
    // P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), valid for |x| < 1
    dp = n * (x * b - a) / (x * x - 1.0);
}

// Gauss-Legendre rule with Q points.
void gauss_rule(int Q, double *x, double *w)
{
    for (int j = 0; j < Q; ++j) {
        double t = std::cos(M_PI * (Q - j - 0.25) / (Q + 0.5));
        for (int it = 0; it < 60; ++it) {
            double a = 1.0, b = t;
            for (int k = 2; k <= Q; ++k) {
                double c = ((2 * k - 1) * t * b - (k - 1) * a) / k;
                a = b;
                b = c;
            }
            double dp = Q * (t * b - a) / (t * t - 1.0);
            double step = b / dp;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double p, dp;
        leg(Q, t, p, dp);
        x[j] = t;
        w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// phi_i(r) and phi_i'(r) in product form via prefix/suffix jets.
void basis_eval(const Basis &B, int N, double r, double *v, double *d)
{
    double pv[16], pd[16];
    pv[0] = 1.0;
    pd[0] = 0.0;
    for (int i = 1; i < N; ++i) {
        double t = r - B.z[i - 1];
        pd[i] = pd[i - 1] * t + pv[i - 1];
        pv[i] = pv[i - 1] * t;
    }
    double sv = 1.0, sd = 0.0;
    for (int i = N - 1; i >= 0; --i) {
        v[i] = B.w[i] * (pv[i] * sv);
        if (d) d[i] = B.w[i] * (pd[i] * sv + pv[i] * sd);
        double t = r - B.z[i];
        sd = sd * t + sv;
        sv = sv * t;
    }
}

// Tables shared by all elements of one mesh.
struct Tables {
    int N, M;
    std::vector<double> eta;        // [M]
    std::vector<double> vlo, vhi;   // [N][M] basis bound values
    std::vector<double> mom0, mom1; // [N] int phi_i P_0, int phi_i P_1
    std::vector<double> pmin, pmax; // [N*M][N*M]: min/max of the four
                                    // products of basis-bound values
};

void make_tables(const Basis &B, int N, Tables &T)
{
    const int M = 2 * N;           // Section 3.1.1 default
    T.N = N;
    T.M = M;
    T.eta.resize(M);
    for (int j = 0; j < M; ++j) T.eta[j] = -std::cos(M_PI * j / (M - 1.0));
    T.eta[0] = -1.0;
    T.eta[M - 1] = 1.0;
    T.vlo.assign(N * M, 0.0);
    T.vhi.assign(N * M, 0.0);
    double v[16], d[16], vm[16], dm[16], vp[16], dp[16];
    for (int j = 0; j < M; ++j) {
        basis_eval(B, N, T.eta[j], v, nullptr);
        if (j == 0 || j == M - 1) {
            for (int i = 0; i < N; ++i) T.vlo[i * M + j] = T.vhi[i * M + j] = v[i];
            continue;
        }
        // tangents at the adjacent interval mid-points, evaluated at eta_j
        double em = 0.5 * (T.eta[j - 1] + T.eta[j]);
        double ep = 0.5 * (T.eta[j] + T.eta[j + 1]);
        basis_eval(B, N, em, vm, dm);
        basis_eval(B, N, ep, vp, dp);
        for (int i = 0; i < N; ++i) {
            double a = v[i];
            double b = vm[i] + (T.eta[j] - em) * dm[i];
            double c = vp[i] - (ep - T.eta[j]) * dp[i];
            T.vlo[i * M + j] = std::min(a, std::min(b, c));
            T.vhi[i * M + j] = std::max(a, std::max(b, c));
        }
    }
    (void)d;
    // Legendre moments of the bases, exact with N Gauss points
    double xq[16], wq[16];
    gauss_rule(N, xq, wq);
    T.mom0.assign(N, 0.0);
    T.mom1.assign(N, 0.0);
    for (int q = 0; q < N; ++q) {
        basis_eval(B, N, xq[q], v, nullptr);
        for (int i = 0; i < N; ++i) {
            T.mom0[i] += wq[q] * v[i];
            T.mom1[i] += wq[q] * v[i] * xq[q];
        }
    }
    // min / max of {lo lo, lo hi, hi lo, hi hi} per (i,k) x (j,l)
    const int NM = N * M;
    T.pmin.assign((size_t)NM * NM, 0.0);
    T.pmax.assign((size_t)NM * NM, 0.0);
    for (int a = 0; a < NM; ++a)
        for (int b = 0; b < NM; ++b) {
            double p1 = T.vlo[a] * T.vlo[b], p2 = T.vlo[a] * T.vhi[b];
            double p3 = T.vhi[a] * T.vlo[b], p4 = T.vhi[a] * T.vhi[b];
            T.pmin[(size_t)a * NM + b] = std::min(std::min(p1, p2), std::min(p3, p4));
            T.pmax[(size_t)a * NM + b] = std::max(std::max(p1, p2), std::max(p3, p4));
        }
}

// Bound of u(r) = sum_i u_i phi_i(r) with the linear Legendre part removed
// (eqs. eq_1D_bound_final_1/2).
void bound1(const Tables &T, const Basis &B, const double *u, double &lo, double &hi)
{
    const int N = T.N, M = T.M;
    double a0 = 0.0, a1 = 0.0;
    for (int i = 0; i < N; ++i) {
        a0 += u[i] * T.mom0[i];
        a1 += u[i] * T.mom1[i];
    }
    a0 *= 0.5;
    a1 *= 1.5;
    double w[16];
    for (int i = 0; i < N; ++i) w[i] = u[i] - (a0 + a1 * B.z[i]);
    lo = INFINITY;
    hi = -INFINITY;
    for (int j = 0; j < M; ++j) {
        double l = a0 + a1 * T.eta[j], h = l;
        for (int i = 0; i < N; ++i) {
            double x = w[i] * T.vlo[i * M + j], y = w[i] * T.vhi[i * M + j];
            l += std::min(x, y);
            h += std::max(x, y);
        }
        lo = std::min(lo, l);
        hi = std::max(hi, h);
    }
}

// Bound of u(r,s) = sum_ij u_ij phi_i(r) phi_j(s), u indexed i + N j, with
// the bilinear Legendre part removed; the min over the four products of
// w_ij with basis-bound values equals w_ij times the smallest (w >= 0) or
// the largest (w < 0) product (eqs. eq_2D_function_bound_1/2).
void bound2(const Tables &T, const Basis &B, const double *u, double &lo, double &hi)
{
    const int N = T.N, M = T.M, NM = N * M;
    double a00 = 0, a10 = 0, a01 = 0, a11 = 0;
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            double x = u[i + N * j];
            a00 += x * T.mom0[i] * T.mom0[j];
            a10 += x * T.mom1[i] * T.mom0[j];
            a01 += x * T.mom0[i] * T.mom1[j];
            a11 += x * T.mom1[i] * T.mom1[j];
        }
    a00 *= 0.25;
    a10 *= 0.75;
    a01 *= 0.75;
    a11 *= 2.25;
    double w[256];
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i)
            w[i + N * j] = u[i + N * j] - (a00 + a10 * B.z[i] + a01 * B.z[j] +
                                           a11 * B.z[i] * B.z[j]);
    lo = INFINITY;
    hi = -INFINITY;
    for (int l = 0; l < M; ++l)
        for (int k = 0; k < M; ++k) {
            double b = a00 + a10 * T.eta[k] + a01 * T.eta[l] + a11 * T.eta[k] * T.eta[l];
            double sl = b, sh = b;
            for (int i = 0; i < N; ++i) {
                const size_t row = (size_t)(i * M + k) * NM;
                for (int j = 0; j < N; ++j) {
                    double x = w[i + N * j];
                    double pn = T.pmin[row + j * M + l], px = T.pmax[row + j * M + l];
                    sl += x >= 0.0 ? x * pn : x * px;
                    sh += x >= 0.0 ? x * px : x * pn;
                }
            }
            lo = std::min(lo, sl);
            hi = std::max(hi, sh);
        }
}

// Bound of one coordinate function f[NP] of an element: edges of a quad,
// faces of a hex, the whole patch of a surface quad, the whole curve of a
// line element.
void bound_fun(const fpts_mesh *m, const Tables &T, const double *f, double &lo, double &hi)
{
    const int N = m->N;
    double buf[256], a, b;
    lo = INFINITY;
    hi = -INFINITY;
    auto take = [&](double x, double y) { lo = std::min(lo, x); hi = std::max(hi, y); };
    if (m->R == 2 && m->D == 2) {
        for (int e = 0; e < 2; ++e) {
            const int q = e ? N - 1 : 0;
            for (int i = 0; i < N; ++i) buf[i] = f[i + N * q];
            bound1(T, m->basis, buf, a, b);
            take(a, b);
            for (int j = 0; j < N; ++j) buf[j] = f[q + N * j];
            bound1(T, m->basis, buf, a, b);
            take(a, b);
        }
    } else if (m->R == 3) {
        for (int e = 0; e < 2; ++e) {
            const int q = e ? N - 1 : 0;
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) buf[i + N * j] = f[i + N * (j + N * q)];
            bound2(T, m->basis, buf, a, b);
            take(a, b);
            for (int k = 0; k < N; ++k)
                for (int i = 0; i < N; ++i) buf[i + N * k] = f[i + N * (q + N * k)];
            bound2(T, m->basis, buf, a, b);
            take(a, b);
            for (int k = 0; k < N; ++k)
                for (int j = 0; j < N; ++j) buf[j + N * k] = f[q + N * (j + N * k)];
            bound2(T, m->basis, buf, a, b);
            take(a, b);
        }
    } else if (m->R == 2) {
        bound2(T, m->basis, f, a, b);
        take(a, b);
    } else {
        bound1(T, m->basis, f, a, b);
        take(a, b);
    }
}

// Thin-extent rule (manifolds only, Section 4.1) and expansion by tol of the
// extent in total (Section 3.1.1).  `len` scales extents to physical length.
// The rule's reference is the smallest other extent for surface quads and
// the largest for lines (a straight line in 3D has two zero extents).
void finish(const fpts_mesh *m, double *lo, double *hi, const double *len)
{
    const int D = m->D;
    const double tol = m->p.bbox_tol;
    double L[3];
    for (int d = 0; d < D; ++d) L[d] = hi[d] - lo[d];
    if (m->R < m->D) {
        double P[3];
        for (int d = 0; d < D; ++d) P[d] = L[d] * len[d];
        for (int d = 0; d < D; ++d) {
            double ref = m->R == 1 ? 0.0 : INFINITY;
            for (int q = 0; q < D; ++q)
                if (q != d) ref = m->R == 1 ? std::max(ref, P[q]) : std::min(ref, P[q]);
            double need = tol * ref / len[d];
            if (L[d] < need) {
                double c = 0.5 * (lo[d] + hi[d]);
                lo[d] = c - 0.5 * need;
                hi[d] = c + 0.5 * need;
                L[d] = need;
            }
        }
    }
    for (int d = 0; d < D; ++d) {
        lo[d] -= 0.5 * tol * L[d];
        hi[d] += 0.5 * tol * L[d];
    }
}

bool invert(int D, const double *A, double *I)
{
    if (D == 2) {
        double det = A[0] * A[3] - A[1] * A[2];
        if (!(det != 0.0) || !std::isfinite(det)) return false;
        I[0] = A[3] / det;
        I[1] = -A[1] / det;
        I[2] = -A[2] / det;
        I[3] = A[0] / det;
        return true;
    }
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8],
           c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(det != 0.0) || !std::isfinite(det)) return false;
    double id = 1.0 / det;
    I[0] = c00 * id;
    I[3] = c01 * id;
    I[6] = c02 * id;
    I[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    I[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    I[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    I[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    I[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    I[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return true;
}

// AABB and OBB of element e (Section 3.1.1, 3.1.2, 4.1, 4.2).
void element_setup(fpts_mesh *m, const Tables &T, const double *x, int64_t e)
{
    const int D = m->D, R = m->R, N = m->N, NP = m->NP, W = box_words(D);
    const double *xe = x + (size_t)e * D * NP;
    double *rec = &m->box[(size_t)e * W];
    double lo[3], hi[3], one[3] = {1, 1, 1};
    for (int c = 0; c < D; ++c) bound_fun(m, T, xe + c * NP, lo[c], hi[c]);
    finish(m, lo, hi, one);
    for (int c = 0; c < D; ++c) {
        rec[c] = lo[c];
        rec[D + c] = hi[c];
    }
    // centre and centre Jacobian
    double v[16], d[16];
    basis_eval(m->basis, N, 0.0, v, d);
    double xc[3] = {0, 0, 0}, G[3][3] = {{0}};
    for (int idx = 0; idx < NP; ++idx) {
        int ii = idx % N, jj = (idx / N) % N, kk = idx / (N * N);
        double b0 = v[ii] * v[jj], br = d[ii] * v[jj], bs = v[ii] * d[jj], bt = 0.0;
        if (R == 1) {
            b0 = v[ii];
            br = d[ii];
            bs = 0.0;
        }
        if (R == 3) {
            bt = b0 * d[kk];
            b0 *= v[kk];
            br *= v[kk];
            bs *= v[kk];
        }
        for (int c = 0; c < D; ++c) {
            double xv = xe[c * NP + idx];
            xc[c] += xv * b0;
            G[c][0] += xv * br;
            G[c][1] += xv * bs;
            if (R == 3) G[c][2] += xv * bt;
        }
    }
    for (int c = 0; c < D; ++c) m->xc[(size_t)e * D + c] = xc[c];
    double Jc[9] = {0}, Ji[9] = {0}, len[3] = {1, 1, 1};
    if (R == D) {
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) Jc[a * D + b] = G[a][b];
    } else if (R == 1) {
        // Section 4.2, line elements: the rotation Q that takes the unit
        // tangent u at the centre to e1, by Rodrigues' formula about
        // k = u x e1 with cos = u.e1, sin = |u x e1|; x~ = Q (x - x_c) keeps
        // physical length, so J_c = Q^T.  u = -e1 takes the half turn about
        // e3; a zero tangent leaves J_c singular (OBB off).
        rodrigues_frame(D, G[0][0], G[1][0], D == 3 ? G[2][0] : 0.0, Jc);
    } else {
        double t1[3] = {G[0][0], G[1][0], G[2][0]}, t2[3] = {G[0][1], G[1][1], G[2][1]};
        double n[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                       t1[0] * t2[1] - t1[1] * t2[0]};
        double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int c = 0; c < 3; ++c) {
            Jc[c * 3 + 0] = t1[c];
            Jc[c * 3 + 1] = t2[c];
            Jc[c * 3 + 2] = nn > 0.0 ? n[c] / nn : 0.0;
        }
        len[0] = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        len[1] = std::sqrt(t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2]);
    }
    double *oc = rec + 2 * D, *oA = rec + 3 * D;
    if (!invert(D, Jc, Ji)) {
        for (int c = 0; c < D; ++c) oc[c] = xc[c];
        for (int a = 0; a < D * D; ++a) oA[a] = 0.0;
        return;
    }
    std::vector<double> f(NP);
    double tl[3], th[3];
    for (int c = 0; c < D; ++c) {
        for (int idx = 0; idx < NP; ++idx) {
            double s = 0.0;
            for (int q = 0; q < D; ++q) s += Ji[c * D + q] * (xe[q * NP + idx] - xc[q]);
            f[idx] = s;
        }
        bound_fun(m, T, f.data(), tl[c], th[c]);
    }
    finish(m, tl, th, len);
    for (int a = 0; a < D; ++a) {
        double half = 0.5 * (th[a] - tl[a]);
        for (int b = 0; b < D; ++b) oA[a * D + b] = Ji[a * D + b] / half;
    }
    for (int c = 0; c < D; ++c) {
        double s = xc[c];
        for (int q = 0; q < D; ++q) s += Jc[c * D + q] * 0.5 * (th[q] + tl[q]);
        oc[c] = s;
    }
}

template <class F>
void parallel_for(int64_t n, F f)
{
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (n < 64) nt = 1;
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            int64_t b = next.fetch_add(32);
            if (b >= n) break;
            int64_t e = std::min(n, b + 32);
            for (int64_t i = b; i < e; ++i) f(i);
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

int cell_coord(const fpts_mesh *m, int d, double x)
{
    double t = std::floor((x - m->hlo[d]) / m->hdel[d]);
    if (t < 0.0) t = 0.0;
    if (t > m->NL - 1) t = m->NL - 1;
    return (int)t;
}

}  // namespace

void bound_tables(const fpts_mesh *m, BoundTables *t)
{
    const int N = m->N;
    Tables T;
    make_tables(m->basis, N, T);
    std::memset(t, 0, sizeof(*t));
    t->N = N;
    t->M = T.M;
    for (int j = 0; j < T.M; ++j) t->eta[j] = T.eta[j];
    for (int a = 0; a < N * T.M; ++a) {
        t->vlo[a] = T.vlo[a];
        t->vhi[a] = T.vhi[a];
    }
    for (int i = 0; i < N; ++i) {
        t->mom0[i] = T.mom0[i];
        t->mom1[i] = T.mom1[i];
        t->z[i] = m->basis.z[i];
    }
    basis_eval(m->basis, N, 0.0, t->v0, t->d0);
}

int host_setup(fpts_mesh *m, const double *h_nodes)
{
    const int D = m->D, N = m->N, W = box_words(D);
    // the same compile-time GLL table the kernels use
    gll::fill(N, m->basis.z, m->basis.w);
    Tables T;
    make_tables(m->basis, N, T);
    m->box.assign((size_t)m->nel * W, 0.0);
    m->xc.assign((size_t)m->nel * D, 0.0);
    parallel_for(m->nel, [&](int64_t e) { element_setup(m, T, h_nodes, e); });
    // local map (Section 3.1.3)
    for (int d = 0; d < D; ++d) {
        m->hlo[d] = INFINITY;
        m->hhi[d] = -INFINITY;
    }
    for (int64_t e = 0; e < m->nel; ++e)
        for (int d = 0; d < D; ++d) {
            m->hlo[d] = std::min(m->hlo[d], m->box[(size_t)e * W + d]);
            m->hhi[d] = std::max(m->hhi[d], m->box[(size_t)e * W + D + d]);
        }
    for (int d = 0; d < D; ++d)
        if (!std::isfinite(m->hlo[d]) || !std::isfinite(m->hhi[d]) || !(m->hhi[d] > m->hlo[d]))
            return FPTS_EINVAL;
    int NL = m->p.hash_n;
    if (NL <= 0) {
        NL = 1;
        while (std::pow((double)NL, D) < (double)m->nel) ++NL;
    }
    if ((int64_t)std::pow((double)NL, D) > (int64_t)1 << 30) return FPTS_EINVAL;
    m->NL = NL;
    for (int d = 0; d < D; ++d) m->hdel[d] = (m->hhi[d] - m->hlo[d]) / NL;
    int64_t ncell = 1;
    for (int d = 0; d < D; ++d) ncell *= NL;
    std::vector<int64_t> cnt(ncell + 1, 0);
    auto span = [&](int64_t e, int c0[3], int c1[3]) {
        for (int d = 0; d < 3; ++d) c0[d] = c1[d] = 0;
        for (int d = 0; d < D; ++d) {
            c0[d] = cell_coord(m, d, m->box[(size_t)e * W + d]);
            c1[d] = cell_coord(m, d, m->box[(size_t)e * W + D + d]);
        }
    };
    for (int64_t e = 0; e < m->nel; ++e) {
        int c0[3], c1[3];
        span(e, c0, c1);
        for (int k = c0[2]; k <= c1[2]; ++k)
            for (int j = c0[1]; j <= c1[1]; ++j)
                for (int i = c0[0]; i <= c1[0]; ++i)
                    cnt[1 + i + (int64_t)NL * (j + (int64_t)NL * k)]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cnt[c + 1] += cnt[c];
    if (cnt[ncell] >= ((int64_t)1 << 31)) return FPTS_EINVAL;
    m->cell_off.resize(ncell + 1);
    m->max_cell = 0;
    for (int64_t c = 0; c <= ncell; ++c) m->cell_off[c] = (int)cnt[c];
    for (int64_t c = 0; c < ncell; ++c)
        m->max_cell = std::max(m->max_cell, (int)(cnt[c + 1] - cnt[c]));
    m->cell_el.assign(std::max<int64_t>(cnt[ncell], 1), 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < m->nel; ++e) {
        int c0[3], c1[3];
        span(e, c0, c1);
        for (int k = c0[2]; k <= c1[2]; ++k)
            for (int j = c0[1]; j <= c1[1]; ++j)
                for (int i = c0[0]; i <= c1[0]; ++i)
                    m->cell_el[fill[i + (int64_t)NL * (j + (int64_t)NL * k)]++] = (int)e;
    }
    return FPTS_OK;
}

}  // namespace fpts
