/*
 * findpts oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, FP64 CPU implementation of the processor-local part of
 * general field evaluation ("findpts") on high-order quad, hex and surface
 * meshes, written from Mittal, Parik, Dutta, Fischer, Kolev, Lottes,
 * "General Field Evaluation in High-Order Meshes on GPUs" (arXiv 2501.12349).
 *
 * Only the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the HIP library:
 * every formula is written out here directly from the paper, one point at a
 * time, with direct (not sum-factorised) tensor sums and no binning.
 *
 * Where the paper is silent, garbled or ambiguous, the reading taken is stated
 * at the function that implements it.  Parity status: every function below is
 * pinned by a CPU test (closed forms, the paper's (N, M_min) footnote table,
 * containment, recovery of known coordinates, brute force, polynomial
 * reproduction) except the per-iteration path of Newton for points whose
 * closest point is not unique ("parity unpinned" for that path only).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 16
#define ORC_INTERIOR 0
#define ORC_BORDER 1
#define ORC_NOT_FOUND 2

/* ------------------------------------------------------------------------ */
/* Section 2: Legendre polynomials, Gauss-Lobatto-Legendre (GLL) nodes.      */
/* ------------------------------------------------------------------------ */

/* P_n(x) and P_n'(x) by the three-term recurrence, with
 * P_k' = P_{k-2}' + (2k-1) P_{k-1}. */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        double d2 = d0 + (2.0 * k - 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1; *dp = d1;
}

/* GLL nodes zeta_1..zeta_N on [-1,1] (Section 2: the Lagrange bases are
 * interpolants at these nodes) and their quadrature weights.  The end nodes
 * are -1 and 1; the interior nodes are the roots of P'_{N-1}, found by Newton
 * from Chebyshev-Gauss-Lobatto guesses using P'' from Legendre's equation. */
int orc_gll(int N, double *z, double *w)
{
    if (N < 2 || N > ORC_MAXN) return -1;
    const int n = N - 1;
    z[0] = -1.0; z[N - 1] = 1.0;
    for (int j = 1; j < N - 1; ++j) {
        double x = -cos(M_PI * j / n);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, x, &p, &dp);
            double d2p = (2.0 * x * dp - n * (n + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        z[j] = x;
    }
    for (int j = 0; j < N / 2; ++j) {        /* exact symmetry about 0 */
        double a = 0.5 * (z[N - 1 - j] - z[j]);
        z[j] = -a; z[N - 1 - j] = a;
    }
    if (N % 2) z[N / 2] = 0.0;
    if (w) {
        for (int j = 0; j < N; ++j) {
            double p, dp;
            legendre(n, z[j], &p, &dp);
            w[j] = 2.0 / (n * (n + 1.0) * p * p);
        }
    }
    return 0;
}

/* Gauss-Legendre nodes/weights with Q points; used only for the exact
 * Legendre moments of the bound compaction (Section 3.1.1). */
static void gauss_legendre(int Q, double *x, double *w)
{
    for (int j = 0; j < Q; ++j) {
        double t = -cos(M_PI * (j + 0.75) / (Q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(Q, t, &p, &dp);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double p, dp;
        legendre(Q, t, &p, &dp);
        x[j] = t;
        w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

/* Lagrange interpolants at the nodes z (eq. eq_x: phi_i(zeta_j) = delta_ij),
 * in product form phi_i(r) = prod_{m!=i} (r - z_m)/(z_i - z_m), with the
 * first and second derivatives by the product rule.  Any of dphi/d2phi may
 * be NULL. */
void orc_lagrange(int N, const double *z, double r, double *phi, double *dphi,
                  double *d2phi)
{
    for (int i = 0; i < N; ++i) {
        double den = 1.0, p = 1.0;
        for (int m = 0; m < N; ++m)
            if (m != i) { den *= (z[i] - z[m]); p *= (r - z[m]); }
        phi[i] = p / den;
        if (dphi) {
            double s = 0.0;
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                double t = 1.0;
                for (int m = 0; m < N; ++m)
                    if (m != i && m != k) t *= (r - z[m]);
                s += t;
            }
            dphi[i] = s / den;
        }
        if (d2phi) {
            double s = 0.0;
            for (int k = 0; k < N; ++k) {
                if (k == i) continue;
                for (int l = 0; l < N; ++l) {
                    if (l == i || l == k) continue;
                    double t = 1.0;
                    for (int m = 0; m < N; ++m)
                        if (m != i && m != k && m != l) t *= (r - z[m]);
                    s += t;
                }
            }
            d2phi[i] = s / den;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Section 3.1.1: piecewise-linear bounds of the bases and of functions.     */
/* ------------------------------------------------------------------------ */

/* Chebyshev interval points eta_j = -cos((j-1) pi / (M-1)), j = 1..M
 * (eq. eq_chebyshev). */
void orc_cheb_points(int M, double *eta)
{
    for (int j = 0; j < M; ++j) eta[j] = -cos(M_PI * j / (M - 1.0));
    eta[0] = -1.0; eta[M - 1] = 1.0;
}

/* Lower/upper values lo[i*M+j], hi[i*M+j] of the piecewise-linear bounds of
 * phi_i at eta_j (eqs. eq_1D_bases_bounds .. eq_1D_bases_bounds_3).
 * Reading of the garbled case split: at the two end points the set V_ij holds
 * only phi_i(eta_j); at interior points it holds phi_i(eta_j) and the values
 * at eta_j of the tangents taken at the two adjacent interval mid-points
 * eta_{j-} and eta_{j+}, i.e. offsets (eta_j - eta_{j-}) and
 * (eta_{j+} - eta_j).  This reading reproduces the paper's footnote table of
 * minimal M for N = 2..12. */
int orc_basis_bounds(int N, int M, double *lo, double *hi)
{
    if (N < 2 || N > ORC_MAXN || M < 2) return -1;
    double z[ORC_MAXN], eta[4 * ORC_MAXN * 4];
    if (M > (int)(sizeof(eta) / sizeof(eta[0]))) return -1;
    orc_gll(N, z, NULL);
    orc_cheb_points(M, eta);
    double ph[ORC_MAXN], phm[ORC_MAXN], dphm[ORC_MAXN],
        php[ORC_MAXN], dphp[ORC_MAXN];
    for (int j = 0; j < M; ++j) {
        orc_lagrange(N, z, eta[j], ph, NULL, NULL);
        if (j == 0 || j == M - 1) {
            for (int i = 0; i < N; ++i) lo[i * M + j] = hi[i * M + j] = ph[i];
            continue;
        }
        double em = 0.5 * (eta[j] + eta[j - 1]);
        double ep = 0.5 * (eta[j] + eta[j + 1]);
        orc_lagrange(N, z, em, phm, dphm, NULL);
        orc_lagrange(N, z, ep, php, dphp, NULL);
        for (int i = 0; i < N; ++i) {
            double v0 = ph[i];
            double v1 = phm[i] + (eta[j] - em) * dphm[i];
            double v2 = php[i] - (ep - eta[j]) * dphp[i];
            double mn = v0, mx = v0;
            if (v1 < mn) mn = v1;
            if (v1 > mx) mx = v1;
            if (v2 < mn) mn = v2;
            if (v2 > mx) mx = v2;
            lo[i * M + j] = mn;
            hi[i * M + j] = mx;
        }
    }
    return 0;
}

/* Bound of a 1D function u(r) = sum_i u_i phi_i(r) over [-1,1] with the
 * Legendre compaction u = a0 + a1 r + sum_i w_i phi_i (eqs.
 * eq_1D_bound_final_1/2):  a_l = (2l+1)/2 * int u P_l, w_i = u_i - a0 - a1
 * zeta_i, and the overall bound is the min / max over j of the bounding
 * functions at eta_j.  The moments are integrated exactly with N-point
 * Gauss-Legendre quadrature (the paper leaves the quadrature open). */
void orc_bound_1d(int N, int M, const double *u, double *umin, double *umax)
{
    double z[ORC_MAXN], eta[4 * ORC_MAXN * 4];
    double lo[ORC_MAXN * 4 * ORC_MAXN * 4], hi[ORC_MAXN * 4 * ORC_MAXN * 4];
    double xq[ORC_MAXN], wq[ORC_MAXN], ph[ORC_MAXN];
    orc_gll(N, z, NULL);
    orc_cheb_points(M, eta);
    orc_basis_bounds(N, M, lo, hi);
    gauss_legendre(N, xq, wq);
    double a0 = 0.0, a1 = 0.0;
    for (int q = 0; q < N; ++q) {
        orc_lagrange(N, z, xq[q], ph, NULL, NULL);
        double uq = 0.0;
        for (int i = 0; i < N; ++i) uq += u[i] * ph[i];
        a0 += wq[q] * uq;
        a1 += wq[q] * uq * xq[q];
    }
    a0 *= 0.5;
    a1 *= 1.5;
    double w[ORC_MAXN];
    for (int i = 0; i < N; ++i) w[i] = u[i] - a0 - a1 * z[i];
    double mn = INFINITY, mx = -INFINITY;
    for (int j = 0; j < M; ++j) {
        double l = a0 + a1 * eta[j], h = a0 + a1 * eta[j];
        for (int i = 0; i < N; ++i) {
            double p = w[i] * lo[i * M + j], q = w[i] * hi[i * M + j];
            l += (p < q) ? p : q;
            h += (p > q) ? p : q;
        }
        if (l < mn) mn = l;
        if (h > mx) mx = h;
    }
    *umin = mn;
    *umax = mx;
}

/* Bound of a 2D tensor function u(r,s) = sum_ij u_ij phi_i(r) phi_j(s)
 * (eqs. eq_2D_function_bound_1/2): at each grid point (eta_k, eta_l) the
 * bound is the sum over ij of the min / max of u_ij times the four products
 * of basis-bound values; the overall bound is the min / max over the M x M
 * grid.  Reading (the paper is silent on compaction in 2D): the tensor
 * extension of the 1D Legendre compaction is applied, i.e. the bilinear part
 * b(r,s) = sum_{l,m<=1} a_lm P_l(r) P_m(s), a_lm = (2l+1)(2m+1)/4 * iint u P_l
 * P_m, is subtracted from the nodal values and added back exactly at the grid
 * points.  u is indexed u[i + N*j]. */
void orc_bound_2d(int N, int M, const double *u, double *umin, double *umax)
{
    double z[ORC_MAXN], eta[4 * ORC_MAXN * 4];
    double lo[ORC_MAXN * 4 * ORC_MAXN * 4], hi[ORC_MAXN * 4 * ORC_MAXN * 4];
    double xq[ORC_MAXN], wq[ORC_MAXN], phq[ORC_MAXN][ORC_MAXN];
    orc_gll(N, z, NULL);
    orc_cheb_points(M, eta);
    orc_basis_bounds(N, M, lo, hi);
    gauss_legendre(N, xq, wq);
    for (int q = 0; q < N; ++q) orc_lagrange(N, z, xq[q], phq[q], NULL, NULL);
    double a00 = 0, a10 = 0, a01 = 0, a11 = 0;
    for (int q1 = 0; q1 < N; ++q1)
        for (int q2 = 0; q2 < N; ++q2) {
            double uq = 0.0;
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i)
                    uq += u[i + N * j] * phq[q1][i] * phq[q2][j];
            double wt = wq[q1] * wq[q2] * uq;
            a00 += wt;
            a10 += wt * xq[q1];
            a01 += wt * xq[q2];
            a11 += wt * xq[q1] * xq[q2];
        }
    a00 *= 0.25;
    a10 *= 0.75;
    a01 *= 0.75;
    a11 *= 2.25;
    double w[ORC_MAXN * ORC_MAXN];
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i)
            w[i + N * j] = u[i + N * j] -
                (a00 + a10 * z[i] + a01 * z[j] + a11 * z[i] * z[j]);
    double mn = INFINITY, mx = -INFINITY;
    for (int l = 0; l < M; ++l)
        for (int k = 0; k < M; ++k) {
            double b = a00 + a10 * eta[k] + a01 * eta[l] + a11 * eta[k] * eta[l];
            double sl = b, sh = b;
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    double wij = w[i + N * j];
                    double c[4] = {wij * lo[i * M + k] * lo[j * M + l],
                                   wij * lo[i * M + k] * hi[j * M + l],
                                   wij * hi[i * M + k] * lo[j * M + l],
                                   wij * hi[i * M + k] * hi[j * M + l]};
                    double cmn = c[0], cmx = c[0];
                    for (int t = 1; t < 4; ++t) {
                        if (c[t] < cmn) cmn = c[t];
                        if (c[t] > cmx) cmx = c[t];
                    }
                    sl += cmn;
                    sh += cmx;
                }
            if (sl < mn) mn = sl;
            if (sh > mx) mx = sh;
        }
    *umin = mn;
    *umax = mx;
}

/* ------------------------------------------------------------------------ */
/* Mesh: element map (eqs. eq_x_tensor, eq_x_tensor_surf), boxes, hash.      */
/* ------------------------------------------------------------------------ */

typedef struct orc_mesh {
    int D, R, N, NP;          /* space dim, reference dim, nodes/dir, nodes/elem */
    long long nel;
    const double *x;          /* caller-owned [nel][D][NP], i fastest */
    double tol, eps_d, newton_tol;
    int max_iter, M;
    double z[ORC_MAXN];
    double *aabb;             /* [nel][D][2] expanded */
    double *obbA;             /* [nel][D][D] : Acute{J}^{-1} */
    double *obbc;             /* [nel][D]    : Acute{x}_c */
    int *obb_ok;              /* [nel] 0 when J_c is singular: OBB test skipped */
    double hlo[3], hhi[3], hdel[3];
    int NL;
    long long ncell;
    long long *cell_off;      /* [ncell+1] */
    int *cell_el;             /* [nnz] ascending element ids per cell */
} orc_mesh;

static inline double node(const orc_mesh *m, long long e, int c, int idx)
{
    return m->x[((size_t)e * m->D + c) * m->NP + idx];
}

/* x(r), G = dx/dr (G[c*R + a]) and, if H2 != NULL, the second derivatives
 * H2[(c*R + a)*R + b] of element e at reference point r, as direct tensor
 * sums over all nodes (eq. eq_x_tensor and its derivatives). */
static void map_eval(const orc_mesh *m, long long e, const double *r, double *x,
                     double *G, double *H2)
{
    const int D = m->D, R = m->R, N = m->N;
    double ph[3][ORC_MAXN], dph[3][ORC_MAXN], d2ph[3][ORC_MAXN];
    for (int a = 0; a < R; ++a)
        orc_lagrange(N, m->z, r[a], ph[a], dph[a], H2 ? d2ph[a] : NULL);
    for (int c = 0; c < D; ++c) {
        x[c] = 0.0;
        if (G) for (int a = 0; a < R; ++a) G[c * R + a] = 0.0;
        if (H2) for (int a = 0; a < R * R; ++a) H2[c * R * R + a] = 0.0;
    }
    for (int idx = 0; idx < m->NP; ++idx) {
        int ii[3] = {idx % N, (idx / N) % N, idx / (N * N)};
        double v[3], dv[3], d2v[3];
        for (int a = 0; a < R; ++a) {
            v[a] = ph[a][ii[a]];
            dv[a] = dph[a][ii[a]];
            d2v[a] = H2 ? d2ph[a][ii[a]] : 0.0;
        }
        double prod = 1.0;
        for (int a = 0; a < R; ++a) prod *= v[a];
        /* derivative products: d/dr_a replaces factor a by its derivative */
        double dprod[3], d2prod[3][3];
        for (int a = 0; a < R; ++a) {
            double t = 1.0;
            for (int b = 0; b < R; ++b) t *= (b == a) ? dv[b] : v[b];
            dprod[a] = t;
        }
        if (H2) {
            for (int a = 0; a < R; ++a)
                for (int b = 0; b < R; ++b) {
                    double t = 1.0;
                    for (int q = 0; q < R; ++q) {
                        if (a == b) t *= (q == a) ? d2v[q] : v[q];
                        else t *= (q == a || q == b) ? dv[q] : v[q];
                    }
                    d2prod[a][b] = t;
                }
        }
        for (int c = 0; c < D; ++c) {
            double xv = node(m, e, c, idx);
            x[c] += xv * prod;
            if (G) for (int a = 0; a < R; ++a) G[c * R + a] += xv * dprod[a];
            if (H2)
                for (int a = 0; a < R; ++a)
                    for (int b = 0; b < R; ++b)
                        H2[(c * R + a) * R + b] += xv * d2prod[a][b];
        }
    }
}

void orc_map(const orc_mesh *m, long long e, const double *r, double *x,
             double *G, double *H2)
{
    map_eval(m, e, r, x, G, H2);
}

/* Bound [lo,hi] of one coordinate function given by nodal values f[NP] of
 * element-shaped data.  Volume quad: union of the 1D bounds of its 4 edges.
 * Hex: union of the 2D bounds of its 6 faces (Section 3.1.1).  Surface quad
 * in 3D: the 2D bound of the whole element function (Section 4.1 bounds the
 * nodal position function itself; a curved patch can bulge past its edges). */
static void bound_coord(const orc_mesh *m, const double *f, double *lo, double *hi)
{
    const int N = m->N, M = m->M;
    double mn = INFINITY, mx = -INFINITY, a, b;
    double buf[ORC_MAXN * ORC_MAXN];
    if (m->R == 2 && m->D == 2) {
        /* edges s=-1, s=1 (vary i), r=-1, r=1 (vary j) */
        for (int side = 0; side < 2; ++side) {
            int j = side ? N - 1 : 0;
            for (int i = 0; i < N; ++i) buf[i] = f[i + N * j];
            orc_bound_1d(N, M, buf, &a, &b);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
            int i0 = side ? N - 1 : 0;
            for (int jj = 0; jj < N; ++jj) buf[jj] = f[i0 + N * jj];
            orc_bound_1d(N, M, buf, &a, &b);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
        }
    } else if (m->R == 3) {
        for (int side = 0; side < 2; ++side) {
            int q = side ? N - 1 : 0;
            /* face t = +-1: vary (i,j) */
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) buf[i + N * j] = f[i + N * (j + N * q)];
            orc_bound_2d(N, M, buf, &a, &b);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
            /* face s = +-1: vary (i,k) */
            for (int k = 0; k < N; ++k)
                for (int i = 0; i < N; ++i) buf[i + N * k] = f[i + N * (q + N * k)];
            orc_bound_2d(N, M, buf, &a, &b);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
            /* face r = +-1: vary (j,k) */
            for (int k = 0; k < N; ++k)
                for (int j = 0; j < N; ++j) buf[j + N * k] = f[q + N * (j + N * k)];
            orc_bound_2d(N, M, buf, &a, &b);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
        }
    } else if (m->R == 2) { /* surface quad in 3D */
        orc_bound_2d(N, M, f, &mn, &mx);
    } else { /* line element: the whole curve's coordinate function */
        orc_bound_1d(N, M, f, &mn, &mx);
    }
    *lo = mn;
    *hi = mx;
}

/* Thin-extent rule for manifold elements (Section 4.1): a (near) zero extent
 * is raised to tol times the smallest other extent, about its centre.
 * Reading: applied to every direction of surface elements (a no-op unless the
 * extent is below that value); not applied to volume elements.  For line
 * elements the reference is the largest other extent: in 2D that is the one
 * other extent, as printed; in 3D a straight line has two zero extents and
 * the smallest other one would be zero.  Then the
 * box is expanded by tol of its extent in total, half on each side (Section
 * 3.1.1, "expanded by a nominal percentage"). */
static void finish_box(const orc_mesh *m, double *lo, double *hi, const double *scale)
{
    const int D = m->D;
    double L[3];
    for (int d = 0; d < D; ++d) L[d] = hi[d] - lo[d];
    if (m->R < m->D) {
        double Lp[3];
        for (int d = 0; d < D; ++d) Lp[d] = L[d] * (scale ? scale[d] : 1.0);
        for (int d = 0; d < D; ++d) {
            double mo = m->R == 1 ? 0.0 : INFINITY;
            for (int q = 0; q < D; ++q)
                if (q != d && (m->R == 1 ? Lp[q] > mo : Lp[q] < mo)) mo = Lp[q];
            double need = m->tol * mo / (scale ? scale[d] : 1.0);
            if (L[d] < need) {
                double c = 0.5 * (lo[d] + hi[d]);
                lo[d] = c - 0.5 * need;
                hi[d] = c + 0.5 * need;
                L[d] = need;
            }
        }
    }
    for (int d = 0; d < D; ++d) {
        lo[d] -= 0.5 * m->tol * L[d];
        hi[d] += 0.5 * m->tol * L[d];
    }
}

static int inv3(int n, const double *A, double *Ai)
{
    if (n == 2) {
        double det = A[0] * A[3] - A[1] * A[2];
        if (!(fabs(det) > 0) || !isfinite(det)) return -1;
        Ai[0] = A[3] / det; Ai[1] = -A[1] / det;
        Ai[2] = -A[2] / det; Ai[3] = A[0] / det;
        return 0;
    }
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(fabs(det) > 0) || !isfinite(det)) return -1;
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return 0;
}

/* AABB (Section 3.1.1 and 4.1) and OBB (Section 3.1.2 and 4.2) of element e.
 * OBB: x_c = x(0), J_c = G(0) (surface: the columns t1, t2, n/|n|, which is
 * the inverse of the rotation R = R2 R1 of Section 4.2); the nodes are mapped
 * to x~ = J_c^{-1}(x - x_c), bounded like the AABB, and the box of x~ with
 * half-widths L~/2 and centre x~_c gives Acute{J} = J_c diag(L~/2) and
 * Acute{x}_c = x_c + J_c x~_c (eq. eq_OBB_test uses Acute{J}^{-1}).  For the
 * surface normal direction the thin-extent rule compares physical lengths,
 * L~_d |t_d| (reading: x~_3 is a physical distance, x~_1,2 reference ones). */
static void element_boxes(orc_mesh *m, long long e)
{
    const int D = m->D, R = m->R, NP = m->NP;
    double f[ORC_MAXN * ORC_MAXN * ORC_MAXN];
    double lo[3], hi[3];
    for (int c = 0; c < D; ++c) {
        for (int i = 0; i < NP; ++i) f[i] = node(m, e, c, i);
        bound_coord(m, f, &lo[c], &hi[c]);
    }
    finish_box(m, lo, hi, NULL);
    for (int c = 0; c < D; ++c) {
        m->aabb[((size_t)e * D + c) * 2 + 0] = lo[c];
        m->aabb[((size_t)e * D + c) * 2 + 1] = hi[c];
    }
    /* OBB */
    double r0[3] = {0, 0, 0}, xc[3], G[9], Jc[9] = {0}, Ji[9] = {0};
    map_eval(m, e, r0, xc, G, NULL);
    double scale[3] = {1, 1, 1};
    if (R == D) {
        for (int i = 0; i < D * D; ++i) Jc[i] = G[i];
    } else if (R == 1) {
        /* line (Section 4.2): Rodrigues' rotation Q about k = u x e1 by the
         * angle between the unit tangent u = t/|t| and e1 takes u to e1,
         * Q = I + sin(th) K + (1 - cos(th)) K^2 with K v = k x v.  x~ =
         * Q (x - x_c) is in physical length, so J_c = Q^T.  u = -e1: the
         * half turn about e3.  A zero tangent leaves the OBB off. */
        double t[3] = {G[0], G[1], D == 3 ? G[2] : 0.0};
        double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        double Q[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (tn > 0) {
            double u[3] = {t[0] / tn, t[1] / tn, t[2] / tn};
            double k[3] = {0.0, u[2], -u[1]};          /* u x e1 */
            double sn = sqrt(k[1] * k[1] + k[2] * k[2]), cs = u[0];
            if (sn > 0) {
                for (int i = 0; i < 3; ++i) k[i] /= sn;
                double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double k2 = 0.0;
                        for (int q = 0; q < 3; ++q) k2 += K[i * 3 + q] * K[q * 3 + j];
                        Q[i * 3 + j] = (i == j ? 1.0 : 0.0) + sn * K[i * 3 + j] + (1.0 - cs) * k2;
                    }
            } else if (cs < 0) {
                Q[0] = -1.0;
                Q[4] = -1.0;
            }
            for (int c = 0; c < D; ++c)
                for (int q = 0; q < D; ++q) Jc[c * D + q] = Q[q * 3 + c];
        }
    } else { /* surface: columns t1, t2, n/|n| ; G[c*2 + a] */
        double t1[3] = {G[0], G[2], G[4]}, t2[3] = {G[1], G[3], G[5]};
        double n[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                       t1[0] * t2[1] - t1[1] * t2[0]};
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int c = 0; c < 3; ++c) {
            Jc[c * 3 + 0] = t1[c];
            Jc[c * 3 + 1] = t2[c];
            Jc[c * 3 + 2] = nn > 0 ? n[c] / nn : 0.0;
        }
        scale[0] = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        scale[1] = sqrt(t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2]);
        scale[2] = 1.0;
    }
    int ok = inv3(D, Jc, Ji) == 0;
    m->obb_ok[e] = ok;
    if (!ok) {
        for (int i = 0; i < D * D; ++i) m->obbA[(size_t)e * D * D + i] = 0.0;
        for (int c = 0; c < D; ++c) m->obbc[(size_t)e * D + c] = xc[c];
        return;
    }
    double tl[3], th[3];
    for (int c = 0; c < D; ++c) {
        for (int i = 0; i < NP; ++i) {
            double s = 0.0;
            for (int q = 0; q < D; ++q) s += Ji[c * D + q] * (node(m, e, q, i) - xc[q]);
            f[i] = s;
        }
        bound_coord(m, f, &tl[c], &th[c]);
    }
    finish_box(m, tl, th, scale);
    double half[3], tc[3];
    for (int c = 0; c < D; ++c) {
        half[c] = 0.5 * (th[c] - tl[c]);
        tc[c] = 0.5 * (th[c] + tl[c]);
    }
    /* Acute{J}^{-1} = diag(1/half) J_c^{-1} ; Acute{x}_c = x_c + J_c tc */
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
            m->obbA[(size_t)e * D * D + a * D + b] = Ji[a * D + b] / half[a];
    for (int c = 0; c < D; ++c) {
        double s = xc[c];
        for (int q = 0; q < D; ++q) s += Jc[c * D + q] * tc[q];
        m->obbc[(size_t)e * D + c] = s;
    }
}

/* Cell index of coordinate x along dim d of the local Cartesian mesh
 * (Section 3.1.3), clamped to [0, NL-1]. */
static int cell_of(const orc_mesh *m, int d, double x)
{
    double t = floor((x - m->hlo[d]) / m->hdel[d]);
    if (t < 0) t = 0;
    if (t > m->NL - 1) t = m->NL - 1;
    return (int)t;
}

/* Section 3.1.3: N_L cells per direction spanning the union of the element
 * boxes; element e is registered in every cell between the cells of its
 * AABB's opposite corners.  Default N_L: the smallest n with n^D >= N_E
 * ("resolution similar to that of the mesh"). */
static int build_hash(orc_mesh *m, int hash_n)
{
    const int D = m->D;
    for (int d = 0; d < D; ++d) { m->hlo[d] = INFINITY; m->hhi[d] = -INFINITY; }
    for (long long e = 0; e < m->nel; ++e)
        for (int d = 0; d < D; ++d) {
            double lo = m->aabb[((size_t)e * D + d) * 2], hi = m->aabb[((size_t)e * D + d) * 2 + 1];
            if (lo < m->hlo[d]) m->hlo[d] = lo;
            if (hi > m->hhi[d]) m->hhi[d] = hi;
        }
    int NL = hash_n;
    if (NL <= 0) {
        NL = 1;
        for (;;) {
            double p = 1.0;
            for (int d = 0; d < D; ++d) p *= NL;
            if (p >= (double)m->nel) break;
            ++NL;
        }
    }
    m->NL = NL;
    for (int d = 0; d < D; ++d) m->hdel[d] = (m->hhi[d] - m->hlo[d]) / NL;
    long long nc = 1;
    for (int d = 0; d < D; ++d) nc *= NL;
    m->ncell = nc;
    long long *cnt = calloc((size_t)nc + 1, sizeof(long long));
    if (!cnt) return -1;
    for (int pass = 0; pass < 2; ++pass) {
        for (long long e = 0; e < m->nel; ++e) {
            int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
            for (int d = 0; d < D; ++d) {
                c0[d] = cell_of(m, d, m->aabb[((size_t)e * D + d) * 2]);
                c1[d] = cell_of(m, d, m->aabb[((size_t)e * D + d) * 2 + 1]);
            }
            for (int k = c0[2]; k <= c1[2]; ++k)
                for (int j = c0[1]; j <= c1[1]; ++j)
                    for (int i = c0[0]; i <= c1[0]; ++i) {
                        long long cell = i + (long long)NL * (j + (long long)NL * k);
                        if (pass == 0) cnt[cell + 1]++;
                        else m->cell_el[cnt[cell]++] = (int)e;
                    }
        }
        if (pass == 0) {
            for (long long c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
            m->cell_off = malloc(sizeof(long long) * ((size_t)nc + 1));
            m->cell_el = malloc(sizeof(int) * ((size_t)cnt[nc] + 1));
            if (!m->cell_off || !m->cell_el) { free(cnt); return -1; }
            memcpy(m->cell_off, cnt, sizeof(long long) * ((size_t)nc + 1));
        }
    }
    free(cnt);
    return 0;
}

void orc_free(orc_mesh *m)
{
    if (!m) return;
    free(m->aabb); free(m->obbA); free(m->obbc); free(m->obb_ok);
    free(m->cell_off); free(m->cell_el);
    free(m);
}

/* Setup (Section 3.1): boxes per element and the local map.  `x` must stay
 * alive for the life of the mesh.  M = 2N Chebyshev interval points. */
orc_mesh *orc_setup(int D, int R, int N, long long nel, const double *x, double tol,
                    int hash_n, double eps_d, int max_iter, double newton_tol)
{
    if (!(D == 2 || D == 3) || !(R == D || R == 1 || (R == 2 && D == 3))) return NULL;
    if (N < 2 || N > ORC_MAXN || nel < 1 || !x) return NULL;
    orc_mesh *m = calloc(1, sizeof(orc_mesh));
    if (!m) return NULL;
    m->D = D; m->R = R; m->N = N; m->nel = nel; m->x = x;
    m->NP = (R == 3) ? N * N * N : (R == 2) ? N * N : N;
    m->tol = tol; m->eps_d = eps_d; m->max_iter = max_iter; m->newton_tol = newton_tol;
    m->M = 2 * N;
    orc_gll(N, m->z, NULL);
    m->aabb = malloc(sizeof(double) * (size_t)nel * D * 2);
    m->obbA = malloc(sizeof(double) * (size_t)nel * D * D);
    m->obbc = malloc(sizeof(double) * (size_t)nel * D);
    m->obb_ok = malloc(sizeof(int) * (size_t)nel);
    if (!m->aabb || !m->obbA || !m->obbc || !m->obb_ok) { orc_free(m); return NULL; }
#pragma omp parallel for schedule(dynamic, 16)
    for (long long e = 0; e < nel; ++e) element_boxes(m, e);
    if (build_hash(m, hash_n)) { orc_free(m); return NULL; }
    return m;
}

void orc_get_boxes(const orc_mesh *m, double *aabb, double *obbA, double *obbc, int *obb_ok)
{
    if (aabb) memcpy(aabb, m->aabb, sizeof(double) * (size_t)m->nel * m->D * 2);
    if (obbA) memcpy(obbA, m->obbA, sizeof(double) * (size_t)m->nel * m->D * m->D);
    if (obbc) memcpy(obbc, m->obbc, sizeof(double) * (size_t)m->nel * m->D);
    if (obb_ok) memcpy(obb_ok, m->obb_ok, sizeof(int) * (size_t)m->nel);
}

/* hash description: out[0..2] lo, out[3..5] hi, out[6..8] cell size; returns N_L */
int orc_get_hash(const orc_mesh *m, double *out, long long *nnz)
{
    for (int d = 0; d < 3; ++d) {
        out[d] = d < m->D ? m->hlo[d] : 0;
        out[3 + d] = d < m->D ? m->hhi[d] : 0;
        out[6 + d] = d < m->D ? m->hdel[d] : 0;
    }
    if (nnz) *nnz = m->cell_off[m->ncell];
    return m->NL;
}

/* cell lists: off[ncell+1], el[nnz] (ascending ids per cell) */
void orc_get_cells(const orc_mesh *m, long long *off, int *el)
{
    if (off) memcpy(off, m->cell_off, sizeof(long long) * ((size_t)m->ncell + 1));
    if (el) memcpy(el, m->cell_el, sizeof(int) * (size_t)m->cell_off[m->ncell]);
}

/* Box slacks of x against element e: AABB (eq. eq_AABB_test, inclusive) as
 * the smallest normalised distance to a face (negative outside) and OBB
 * (eq. eq_OBB_test) as 1 - ||Acute{J}^{-1}(x - Acute{x}_c)||_inf. */
static void box_slack(const orc_mesh *m, long long e, const double *x, double *sa, double *so)
{
    const int D = m->D;
    double s = INFINITY;
    for (int d = 0; d < D; ++d) {
        double lo = m->aabb[((size_t)e * D + d) * 2], hi = m->aabb[((size_t)e * D + d) * 2 + 1];
        double t1 = (x[d] - lo) / (hi - lo), t2 = (hi - x[d]) / (hi - lo);
        if (t1 < s) s = t1;
        if (t2 < s) s = t2;
    }
    *sa = s;
    if (!m->obb_ok[e]) { *so = INFINITY; return; }
    double mx = 0.0;
    for (int a = 0; a < D; ++a) {
        double t = 0.0;
        for (int b = 0; b < D; ++b)
            t += m->obbA[(size_t)e * D * D + a * D + b] * (x[b] - m->obbc[(size_t)e * D + b]);
        if (fabs(t) > mx) mx = fabs(t);
    }
    *so = 1.0 - mx;
}

static int box_pass(const orc_mesh *m, long long e, const double *x)
{
    const int D = m->D;
    for (int d = 0; d < D; ++d) {
        double lo = m->aabb[((size_t)e * D + d) * 2], hi = m->aabb[((size_t)e * D + d) * 2 + 1];
        if (!((x[d] - lo) * (hi - x[d]) >= 0.0)) return 0;
    }
    if (!m->obb_ok[e]) return 1;
    for (int a = 0; a < D; ++a) {
        double t = 0.0;
        for (int b = 0; b < D; ++b)
            t += m->obbA[(size_t)e * D * D + a * D + b] * (x[b] - m->obbc[(size_t)e * D + b]);
        if (!(fabs(t) <= 1.0)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2.1: trust-region Newton.                                       */
/* ------------------------------------------------------------------------ */

/* Cholesky solve of the n x n system A x = b restricted to the index list
 * idx; returns -1 when a pivot is not positive (A not SPD there). */
static int chol_solve(int R, const double *A, int n, const int *idx, const double *b, double *x)
{
    double L[3][3] = {{0}};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[idx[i] * R + idx[j]];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return -1;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    double y[3];
    for (int i = 0; i < n; ++i) {
        double s = b[idx[i]];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * x[idx[k]];
        x[idx[i]] = s / L[i][i];
    }
    return 0;
}

/* Minimise f(r) = 1/2 ||x* - x(r)||^2 over r in [-1,1]^R for element e
 * (Section 3.2.1).  Start: the reference coordinates of the element node
 * nearest to x* (ties: lowest lexicographic node index).  Each pass:
 *   g = G^T dx (= -J, eq. eq_newton_jacobian);
 *   coordinates at a bound whose descent direction leaves the box are held
 *   (reading: active set), the rest are free;
 *   beta = 1 only for passes l > 0 with the iterate on a face / edge;
 *   H = G^T G - beta sum_i dx_i d2x_i/dr dr (eq. eq_newton_hessian); if H is
 *   not SPD on the free set, G^T G is used (reading);
 *   dr = H^{-1} g on the free set (eq. eq_newton), clipped componentwise to
 *   [-alpha, alpha], and r + dr clipped to [-1,1];
 *   x is evaluated at the trial point; ||dr||_inf < tol accepts it and stops;
 *   otherwise pred = 2 g.dr - dr.H.dr (the model decrease of ||dx||^2,
 *   reading of the garbled quadratic formula), decr = ||dx||^2 - ||dx'||^2,
 *   and alpha <- 2 alpha (decr >= 0.9 pred, accept), alpha (>= 0.01 pred,
 *   accept), alpha / 4 (otherwise, reject).  Reading (the paper is silent on
 *   rounding): when 0 < pred <= 64 eps sqrt(f) (|x*| + sqrt(f)), the rounding
 *   noise of f itself, decr cannot judge the step; it is accepted and alpha
 *   kept.  Without this, non-zero-residual problems (BORDER points, surface
 *   closest points) stall about 1e-8 short of the fixed point.
 * At most max_iter passes, accepted or not.  Returns r, ||x* - x(r)||_2, the
 * number of passes and whether the step test was met. */
void orc_newton(const orc_mesh *m, long long e, const double *xs, double *r_out,
                double *dist_out, int *iters_out, int *conv_out)
{
    const int D = m->D, R = m->R, N = m->N, NP = m->NP;
    double best = INFINITY;
    int bi = 0;
    for (int idx = 0; idx < NP; ++idx) {
        double d2 = 0.0;
        for (int c = 0; c < D; ++c) {
            double t = xs[c] - node(m, e, c, idx);
            d2 += t * t;
        }
        if (d2 < best) { best = d2; bi = idx; }
    }
    double r[3] = {0, 0, 0};
    r[0] = m->z[bi % N];
    r[1] = m->z[(bi / N) % N];
    if (R == 3) r[2] = m->z[bi / (N * N)];
    double x[3], G[9], dx[3], f = 0.0;
    map_eval(m, e, r, x, G, NULL);
    for (int c = 0; c < D; ++c) { dx[c] = xs[c] - x[c]; f += dx[c] * dx[c]; }
    double alpha = 1.0;
    int it = 0, conv = 0;
    for (int l = 0; l < m->max_iter; ++l) {
        ++it;
        double g[3] = {0, 0, 0};
        for (int a = 0; a < R; ++a)
            for (int c = 0; c < D; ++c) g[a] += G[c * R + a] * dx[c];
        int onb = 0;
        for (int a = 0; a < R; ++a)
            if (fabs(r[a]) == 1.0) onb = 1;
        int beta = (l > 0) && onb;
        double H[9];
        for (int a = 0; a < R; ++a)
            for (int b = 0; b < R; ++b) {
                double s = 0.0;
                for (int c = 0; c < D; ++c) s += G[c * R + a] * G[c * R + b];
                H[a * R + b] = s;
            }
        if (beta) {
            double xx[3], GG[9], H2[27];
            map_eval(m, e, r, xx, GG, H2);
            for (int a = 0; a < R; ++a)
                for (int b = 0; b < R; ++b)
                    for (int c = 0; c < D; ++c)
                        H[a * R + b] -= dx[c] * H2[(c * R + a) * R + b];
        }
        int fidx[3], nf = 0;
        for (int a = 0; a < R; ++a) {
            int act = (r[a] == 1.0 && g[a] > 0.0) || (r[a] == -1.0 && g[a] < 0.0);
            if (!act) fidx[nf++] = a;
        }
        double dr[3] = {0, 0, 0};
        if (nf > 0 && chol_solve(R, H, nf, fidx, g, dr) != 0) {
            for (int a = 0; a < R; ++a)
                for (int b = 0; b < R; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < D; ++c) s += G[c * R + a] * G[c * R + b];
                    H[a * R + b] = s;
                }
            dr[0] = dr[1] = dr[2] = 0.0;
            if (chol_solve(R, H, nf, fidx, g, dr) != 0) dr[0] = dr[1] = dr[2] = 0.0;
        }
        double rn[3] = {0, 0, 0}, dmax = 0.0;
        for (int a = 0; a < R; ++a) {
            double d = dr[a];
            if (d > alpha) d = alpha;
            if (d < -alpha) d = -alpha;
            double t = r[a] + d;
            if (t > 1.0) t = 1.0;
            if (t < -1.0) t = -1.0;
            rn[a] = t;
            dr[a] = t - r[a];
            if (fabs(dr[a]) > dmax) dmax = fabs(dr[a]);
        }
        double xn[3], Gn[9], dxn[3], fn = 0.0;
        map_eval(m, e, rn, xn, Gn, NULL);
        for (int c = 0; c < D; ++c) { dxn[c] = xs[c] - xn[c]; fn += dxn[c] * dxn[c]; }
        int accept;
        if (dmax < m->newton_tol) {
            accept = 1;
            conv = 1;
        } else {
            double gd = 0.0, dHd = 0.0;
            for (int a = 0; a < R; ++a) {
                gd += g[a] * dr[a];
                for (int b = 0; b < R; ++b) dHd += dr[a] * H[a * R + b] * dr[b];
            }
            double pred = 2.0 * gd - dHd, decr = f - fn;
            double sf = sqrt(f), xn2 = 0.0;
            for (int c = 0; c < D; ++c) xn2 += xs[c] * xs[c];
            double noise = 64.0 * DBL_EPSILON * sf * (sqrt(xn2) + sf);
            if (pred > 0.0 && pred <= noise) { accept = 1; }
            else if (pred > 0.0 && decr >= 0.9 * pred) { accept = 1; alpha *= 2.0; }
            else if (pred > 0.0 && decr >= 0.01 * pred) { accept = 1; }
            else { accept = 0; alpha *= 0.25; }
        }
        if (accept) {
            for (int a = 0; a < R; ++a) r[a] = rn[a];
            for (int c = 0; c < D; ++c) { x[c] = xn[c]; dx[c] = dxn[c]; }
            for (int i = 0; i < D * R; ++i) G[i] = Gn[i];
            f = fn;
        }
        if (conv) break;
    }
    for (int a = 0; a < R; ++a) r_out[a] = r[a];
    *dist_out = sqrt(f);
    if (iters_out) *iters_out = it;
    if (conv_out) *conv_out = conv;
}

/* Code of a Newton result: INTERIOR when r is inside the open reference box
 * (Section 3.2) and, for manifolds, the squared distance is below eps_d
 * (Section 4.4); BORDER otherwise. */
static int code_of(const orc_mesh *m, const double *r, double dist)
{
    for (int a = 0; a < m->R; ++a)
        if (!(fabs(r[a]) < 1.0)) return ORC_BORDER;
    if (m->R < m->D && !(dist * dist < m->eps_d)) return ORC_BORDER;
    return ORC_INTERIOR;
}

/* Section 3.2: find one point.  mode 0: candidates from the local map;
 * mode 1: every element whose boxes contain the point (no map); mode 2:
 * every element (no map, no boxes).  Candidates are visited in ascending
 * element id; the first INTERIOR result ends the search, otherwise the
 * smallest distance wins (ties: the lower id).  margin[0..4]: see orc_find. */
static void find_one(const orc_mesh *m, const double *xs, int mode, int *code, int *elem,
                     double *r, double *dist, double *margin, int *iters, int *ncand)
{
    const int D = m->D, R = m->R;
    *code = ORC_NOT_FOUND; *elem = -1; *dist = INFINITY; *iters = 0; *ncand = 0;
    for (int a = 0; a < R; ++a) r[a] = 0.0;
    for (int k = 0; k < 5; ++k) margin[k] = INFINITY;
    int finite = 1, inside = 1;
    for (int d = 0; d < D; ++d) {
        if (!isfinite(xs[d])) finite = 0;
        else if (!(xs[d] >= m->hlo[d] && xs[d] <= m->hhi[d])) inside = 0;
    }
    if (!finite) return;
    /* box margin over the neighbourhood of the point's cell */
    {
        int c[3] = {0, 0, 0};
        for (int d = 0; d < D; ++d) c[d] = cell_of(m, d, xs[d]);
        double bm = INFINITY;
        for (int d = 0; d < D; ++d) {
            double t = fmin(fabs(xs[d] - m->hlo[d]), fabs(m->hhi[d] - xs[d])) /
                       (m->hhi[d] - m->hlo[d]);
            if (t < bm) bm = t;
        }
        int k0 = D == 3 ? c[2] - 1 : 0, k1 = D == 3 ? c[2] + 1 : 0;
        for (int k = k0; k <= k1; ++k)
            for (int j = c[1] - 1; j <= c[1] + 1; ++j)
                for (int i = c[0] - 1; i <= c[0] + 1; ++i) {
                    if (i < 0 || j < 0 || k < 0 || i >= m->NL || j >= m->NL || k >= m->NL) continue;
                    long long cell = i + (long long)m->NL * (j + (long long)m->NL * k);
                    for (long long q = m->cell_off[cell]; q < m->cell_off[cell + 1]; ++q) {
                        double sa, so;
                        box_slack(m, m->cell_el[q], xs, &sa, &so);
                        double t = fabs(fmin(sa, so));
                        if (t < bm) bm = t;
                    }
                }
        margin[1] = bm;
    }
    if (!inside && mode == 0) return;
    long long q0, q1;
    if (mode == 0) {
        long long cell = 0, mul = 1;
        for (int d = 0; d < D; ++d) { cell += mul * cell_of(m, d, xs[d]); mul *= m->NL; }
        q0 = m->cell_off[cell];
        q1 = m->cell_off[cell + 1];
    } else {
        q0 = 0;
        q1 = m->nel;
    }
    double second = INFINITY;
    for (long long q = q0; q < q1; ++q) {
        long long e = (mode == 0) ? m->cell_el[q] : q;
        if (mode != 2 && !box_pass(m, e, xs)) continue;
        (*ncand)++;
        double rr[3], dd;
        int it, cv;
        orc_newton(m, e, xs, rr, &dd, &it, &cv);
        *iters += it;
        int cd = code_of(m, rr, dd);
        if (cd == ORC_INTERIOR) {
            *code = cd; *elem = (int)e; *dist = dd;
            for (int a = 0; a < R; ++a) r[a] = rr[a];
            double mr = INFINITY;
            for (int a = 0; a < R; ++a)
                if (1.0 - fabs(rr[a]) < mr) mr = 1.0 - fabs(rr[a]);
            margin[0] = mr;
            break;
        }
        if (*elem < 0 || dd < *dist) {
            if (*elem >= 0) second = *dist;
            *code = cd; *elem = (int)e; *dist = dd;
            for (int a = 0; a < R; ++a) r[a] = rr[a];
        } else if (dd < second) {
            second = dd;
        }
    }
    if (*elem >= 0) {
        const double *bx = &m->aabb[(size_t)(*elem) * D * 2];
        double h = 0.0;
        for (int d = 0; d < D; ++d)
            if (bx[2 * d + 1] - bx[2 * d] > h) h = bx[2 * d + 1] - bx[2 * d];
        h /= (1.0 + m->tol);
        if (*code == ORC_BORDER) {
            margin[2] = (second - *dist) / h;
            margin[3] = *dist / h;
            /* distance of r from the reference box edges along the free
               coordinates: small values mean the closest point sits near an
               edge/corner shared with a neighbour */
            double mr = INFINITY;
            for (int a = 0; a < R; ++a)
                if (fabs(r[a]) < 1.0 && 1.0 - fabs(r[a]) < mr) mr = 1.0 - fabs(r[a]);
            margin[0] = mr;
        }
        if (R < D) margin[4] = fabs(*dist * *dist - m->eps_d) / m->eps_d;
    }
}

/* Find n points (SoA pts[D][n]).  Outputs: code, elem (-1 if NOT_FOUND),
 * r (SoA [R][n], 0 if NOT_FOUND), dist (+inf if NOT_FOUND), and optional
 * margin[5][n] (0: 1-max|r| of the result, 1: smallest |box slack| near the
 * point, 2: BORDER gap to the second-best distance / h, 3: BORDER
 * distance / h, 4: surface |dist^2 - eps_d| / eps_d), iters[n] (Newton
 * passes over all candidates), ncand[n]. */
void orc_find(const orc_mesh *m, long long n, const double *pts, int mode, int32_t *code,
              int32_t *elem, double *r, double *dist, double *margin, int32_t *iters,
              int32_t *ncand, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
    (void)nthreads;
#pragma omp parallel for schedule(dynamic, 32) num_threads(nthreads)
    for (long long p = 0; p < n; ++p) {
        double xs[3], rr[3], mg[5], dd;
        int cd, el, it, nc;
        for (int d = 0; d < m->D; ++d) xs[d] = pts[(size_t)d * n + p];
        find_one(m, xs, mode, &cd, &el, rr, &dd, mg, &it, &nc);
        code[p] = cd;
        elem[p] = el;
        dist[p] = dd;
        for (int a = 0; a < m->R; ++a) r[(size_t)a * n + p] = rr[a];
        if (margin)
            for (int k = 0; k < 5; ++k) margin[(size_t)k * n + p] = mg[k];
        if (iters) iters[p] = it;
        if (ncand) ncand[p] = nc;
    }
}

/* Section 3.3: u_f(r*) = sum over the field's nodes of u_f,e(node) times
 * the product of Lagrange bases at r* (eq. eq_u_tensor).  The field has its
 * own order: Nf GLL nodes per direction (Nf = N-tilde, which need not equal
 * the geometry's N), laid out [nf][nel][Nf^R] with the first reference index
 * fastest.  NaN for NOT_FOUND points.  Returns -1 for Nf out of range. */
int orc_eval_order(const orc_mesh *m, long long n, const int32_t *code, const int32_t *elem,
                   const double *r, int nf, int Nf, const double *field, double *out,
                   int nthreads)
{
    const int R = m->R;
    if (Nf < 2 || Nf > ORC_MAXN) return -1;
    int NPf = Nf;
    for (int a = 1; a < R; ++a) NPf *= Nf;
    double zf[ORC_MAXN], wf[ORC_MAXN];
    if (Nf == m->N) {
        for (int i = 0; i < Nf; ++i) zf[i] = m->z[i];
    } else if (orc_gll(Nf, zf, wf) != 0) {
        return -1;
    }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (long long p = 0; p < n; ++p) {
        if (code[p] == ORC_NOT_FOUND || elem[p] < 0) {
            for (int f = 0; f < nf; ++f) out[(size_t)f * n + p] = NAN;
            continue;
        }
        double ph[3][ORC_MAXN];
        for (int a = 0; a < R; ++a) orc_lagrange(Nf, zf, r[(size_t)a * n + p], ph[a], NULL, NULL);
        for (int f = 0; f < nf; ++f) {
            const double *u = field + ((size_t)f * m->nel + elem[p]) * NPf;
            double s = 0.0;
            for (int idx = 0; idx < NPf; ++idx) {
                double b = ph[0][idx % Nf];
                if (R >= 2) b *= ph[1][(idx / Nf) % Nf];
                if (R == 3) b *= ph[2][idx / (Nf * Nf)];
                s += u[idx] * b;
            }
            out[(size_t)f * n + p] = s;
        }
    }
    return 0;
}

/* Interpolation of fields with the geometry's order (Nf = N). */
void orc_eval(const orc_mesh *m, long long n, const int32_t *code, const int32_t *elem,
              const double *r, int nf, const double *field, double *out, int nthreads)
{
    (void)orc_eval_order(m, n, code, elem, r, nf, m->N, field, out, nthreads);
}

/* Threads an OpenMP region of this library uses by default. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
