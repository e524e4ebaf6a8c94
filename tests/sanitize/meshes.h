/* Small curved meshes for the sanitizer drivers: a structured mesh of
 * [0,1]^D with n elements per direction and N equispaced-in-GLL-order nodes
 * (Chebyshev-Gauss-Lobatto points stand in for the GLL points: node
 * placement only has to be inside each element), curved by
 * x_c += a sin(pi x) sin(pi y) [sin(pi z)], nodes laid out [nel][D][N^D]
 * with the first reference index fastest; and a closed curve of line
 * elements in 2D. */
#ifndef SAN_MESHES_H
#define SAN_MESHES_H
#include <math.h>
#include <stdlib.h>

static double san_node1d(int N, int i)
{
    return 0.5 * (1.0 - cos(M_PI * i / (N - 1)));
}

/* volume mesh: returns malloc'd [n^D][D][N^D] */
static double *san_volume(int D, int n, int N, double amp)
{
    const int NP = D == 3 ? N * N * N : N * N, nel = D == 3 ? n * n * n : n * n;
    double *x = (double *)malloc(sizeof(double) * (size_t)nel * D * NP);
    for (int e = 0; e < nel; ++e) {
        const int a = e % n, b = (e / n) % n, c = e / (n * n);
        for (int q = 0; q < NP; ++q) {
            const int i = q % N, j = (q / N) % N, k = q / (N * N);
            double p[3] = {(a + san_node1d(N, i)) / n, (b + san_node1d(N, j)) / n,
                           D == 3 ? (c + san_node1d(N, k)) / n : 0.0};
            double d = amp * sin(M_PI * p[0]) * sin(M_PI * p[1]);
            if (D == 3) d *= sin(M_PI * p[2]);
            for (int cc = 0; cc < D; ++cc) x[((size_t)e * D + cc) * NP + q] = p[cc] + d;
        }
    }
    return x;
}

/* surface: the graph z = 0.1 sin(2 pi x) sin(2 pi y) over [0,1]^2 as n x n
 * quads in 3D: [n^2][3][N^2] */
static double *san_surface(int n, int N)
{
    const int NP = N * N, nel = n * n;
    double *x = (double *)malloc(sizeof(double) * (size_t)nel * 3 * NP);
    for (int e = 0; e < nel; ++e) {
        const int a = e % n, b = e / n;
        for (int q = 0; q < NP; ++q) {
            const int i = q % N, j = q / N;
            const double u = (a + san_node1d(N, i)) / n, v = (b + san_node1d(N, j)) / n;
            x[((size_t)e * 3 + 0) * NP + q] = u;
            x[((size_t)e * 3 + 1) * NP + q] = v;
            x[((size_t)e * 3 + 2) * NP + q] = 0.1 * sin(2 * M_PI * u) * sin(2 * M_PI * v);
        }
    }
    return x;
}

/* lines: a circle of radius 1 + 0.1 cos(3t) as nel elements in 2D:
 * [nel][2][N] */
static double *san_lines(int nel, int N)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)nel * 2 * N);
    for (int e = 0; e < nel; ++e)
        for (int i = 0; i < N; ++i) {
            const double t = 2 * M_PI * (e + san_node1d(N, i)) / nel;
            const double rr = 1.0 + 0.1 * cos(3 * t);
            x[((size_t)e * 2 + 0) * N + i] = rr * cos(t);
            x[((size_t)e * 2 + 1) * N + i] = rr * sin(t);
        }
    return x;
}
#endif
