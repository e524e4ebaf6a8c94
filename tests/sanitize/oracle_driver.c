/* Runs the oracle (setup, find, eval) on small meshes of every kind; built
 * with -fsanitize=address,undefined by tests/test_sanitizers.py.  Prints one
 * line per mesh; any sanitizer report makes the process fail. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "meshes.h"

typedef struct orc_mesh orc_mesh;
orc_mesh *orc_setup(int D, int R, int N, long long nel, const double *x, double tol,
                    int hash_n, double eps_d, int max_iter, double newton_tol);
void orc_free(orc_mesh *m);
void orc_find(const orc_mesh *m, long long n, const double *pts, int mode, int32_t *code,
              int32_t *elem, double *r, double *dist, double *margin, int32_t *iters,
              int32_t *ncand, int nthreads);
void orc_eval(const orc_mesh *m, long long n, const int32_t *code, const int32_t *elem,
              const double *r, int nf, const double *field, double *out, int nthreads);

static int run(const char *name, int D, int R, int N, long long nel, const double *x,
               double lo, double hi)
{
    orc_mesh *m = orc_setup(D, R, N, nel, x, 0.1, 0, 1e-10, 50, 1e-10);
    if (!m) return 1;
    const long long n = 3000;
    double *pts = malloc(sizeof(double) * D * n), *r = malloc(sizeof(double) * R * n);
    double *dist = malloc(sizeof(double) * n), *margin = malloc(sizeof(double) * 5 * n);
    int32_t *code = malloc(4 * n), *elem = malloc(4 * n), *it = malloc(4 * n), *nc = malloc(4 * n);
    srand(7);
    for (long long i = 0; i < D * n; ++i) pts[i] = lo + (hi - lo) * (rand() / (double)RAND_MAX);
    int NP = 1;
    for (int a = 0; a < R; ++a) NP *= N;
    double *field = malloc(sizeof(double) * nel * NP), *out = malloc(sizeof(double) * n);
    for (long long i = 0; i < nel * NP; ++i) field[i] = x[(i / NP) * D * NP + i % NP];
    for (int mode = 0; mode < 3; ++mode) {
        orc_find(m, n, pts, mode, code, elem, r, dist, margin, it, nc, 2);
        orc_eval(m, n, code, elem, r, 1, field, out, 2);
    }
    long long cnt[3] = {0, 0, 0};
    for (long long i = 0; i < n; ++i) cnt[code[i]]++;
    printf("%s: %lld %lld %lld\n", name, cnt[0], cnt[1], cnt[2]);
    orc_free(m);
    free(pts); free(r); free(dist); free(margin); free(code); free(elem); free(it); free(nc);
    free(field); free(out);
    return 0;
}

int main(void)
{
    int bad = 0;
    double *h = san_volume(3, 3, 5, 0.1);
    bad |= run("hex", 3, 3, 5, 27, h, -0.05, 1.05);
    double *q = san_volume(2, 4, 6, 0.05);
    bad |= run("quad", 2, 2, 6, 16, q, -0.05, 1.05);
    double *s = san_surface(3, 4);
    bad |= run("surface", 3, 2, 4, 9, s, -0.05, 1.05);
    double *l = san_lines(12, 4);
    bad |= run("line", 2, 1, 4, 12, l, -1.3, 1.3);
    free(h); free(q); free(s); free(l);
    return bad;
}
