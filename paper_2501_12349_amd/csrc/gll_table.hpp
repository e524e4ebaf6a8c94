// Gauss-Lobatto-Legendre nodes and product-form Lagrange weights as
// compile-time tables (Section 2: the bases are Lagrange interpolants at the
// GLL points), shared by the host setup and the kernels of this library so
// that both use bit-identical nodes.  Interior nodes are the roots of
// P'_{N-1}, found by Newton's method from Chebyshev-Gauss-Lobatto guesses,
// with P'' from Legendre's differential equation; the weights are
// w_i = 1 / prod_{m != i}(z_i - z_m), so phi_i(r) = w_i prod_{m != i}(r - z_m).
#pragma once

namespace fpts {
namespace gll {

constexpr double kPi = 3.14159265358979323846264338327950288;

// cos on [0, pi] by Taylor series about 0 (|x| <= pi/2 after reflection).
constexpr double ce_cos(double x)
{
    double sign = 1.0;
    if (x > kPi / 2) {
        x = kPi - x;
        sign = -1.0;
    }
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sign * sum;
}

constexpr double ce_abs(double x) { return x < 0 ? -x : x; }

// P_n(x), P_n'(x) by the three-term recurrence.
constexpr void legendre(int n, double x, double &p, double &dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        const double d2 = d0 + (2.0 * k - 1.0) * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    p = p1;
    dp = d1;
}

template <int N>
struct Table {
    double z[N];
    double w[N];
};

template <int N>
constexpr Table<N> make()
{
    Table<N> t{};
    const int n = N - 1;
    t.z[0] = -1.0;
    t.z[N - 1] = 1.0;
    for (int j = 1; j < N - 1; ++j) {
        double x = -ce_cos(kPi * j / n);
        for (int it = 0; it < 100; ++it) {
            double p = 0, dp = 0;
            legendre(n, x, p, dp);
            const double ddp = (2.0 * x * dp - n * (n + 1.0) * p) / (1.0 - x * x);
            const double step = dp / ddp;
            x -= step;
            if (ce_abs(step) < 1e-17) break;
        }
        t.z[j] = x;
    }
    for (int j = 0; j < N / 2; ++j) {
        const double h = 0.5 * (t.z[N - 1 - j] - t.z[j]);
        t.z[j] = -h;
        t.z[N - 1 - j] = h;
    }
    if (N % 2) t.z[N / 2] = 0.0;
    for (int i = 0; i < N; ++i) {
        double den = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != i) den *= t.z[i] - t.z[m];
        t.w[i] = 1.0 / den;
    }
    return t;
}

template <int N> struct Nodes {
    static constexpr Table<N> t = make<N>();
};

// Host access by runtime N (2..16).
inline void fill(int N, double *z, double *w)
{
    auto put = [&](const auto &t, int n) {
        for (int i = 0; i < n; ++i) {
            z[i] = t.z[i];
            w[i] = t.w[i];
        }
    };
    switch (N) {
    case 2: put(Nodes<2>::t, 2); break;
    case 3: put(Nodes<3>::t, 3); break;
    case 4: put(Nodes<4>::t, 4); break;
    case 5: put(Nodes<5>::t, 5); break;
    case 6: put(Nodes<6>::t, 6); break;
    case 7: put(Nodes<7>::t, 7); break;
    case 8: put(Nodes<8>::t, 8); break;
    case 9: put(Nodes<9>::t, 9); break;
    case 10: put(Nodes<10>::t, 10); break;
    case 11: put(Nodes<11>::t, 11); break;
    case 12: put(Nodes<12>::t, 12); break;
    case 13: put(Nodes<13>::t, 13); break;
    case 14: put(Nodes<14>::t, 14); break;
    case 15: put(Nodes<15>::t, 15); break;
    case 16: put(Nodes<16>::t, 16); break;
    default: break;
    }
}

}  // namespace gll
}  // namespace fpts
