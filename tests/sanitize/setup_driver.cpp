// Runs the library's host setup (boxes, OBBs, local map; the part of
// fpts_setup that runs on the CPU) on small meshes of every kind; built with
// host-side -fsanitize=address,undefined by tests/test_sanitizers.py.  No
// device is touched.
#include <cstdio>
#include <cstdlib>

#include "fpts_internal.hpp"

extern "C" {
#include "meshes.h"
}

static int run(const char *name, int D, int R, int N, int64_t nel, const double *x)
{
    fpts_mesh m{};
    m.p.dim = D;
    m.p.ref_dim = R;
    m.p.nodes_1d = N;
    m.p.n_elem = nel;
    m.p.bbox_tol = 0.1;
    m.p.surf_eps_d = 1e-10;
    m.p.max_iter = 50;
    m.p.newton_tol = 1e-10;
    m.p.mixed_max_iter = 10;
    m.p.mixed_tol = 1e-3;
    m.D = D;
    m.R = R;
    m.N = N;
    m.NP = R == 3 ? N * N * N : R == 2 ? N * N : N;
    m.nel = nel;
    const int st = fpts::host_setup(&m, x);
    std::printf("%s: status %d, N_L %d, cell entries %d, largest cell %d\n", name, st, m.NL,
                m.cell_off.empty() ? 0 : m.cell_off.back(), m.max_cell);
    return st != 0;
}

int main()
{
    int bad = 0;
    double *h = san_volume(3, 3, 5, 0.1);
    bad |= run("hex", 3, 3, 5, 27, h);
    double *q = san_volume(2, 4, 6, 0.05);
    bad |= run("quad", 2, 2, 6, 16, q);
    double *s = san_surface(3, 4);
    bad |= run("surface", 3, 2, 4, 9, s);
    double *l = san_lines(12, 4);
    bad |= run("line", 2, 1, 4, 12, l);
    std::free(h);
    std::free(q);
    std::free(s);
    std::free(l);
    return bad;
}
