// Particle transport step of the particle-tracking application (Section 6.7):
// Stokes drag a = (u - v) / tau, second-order Adams-Bashforth for x' = v and
// v' = a (forward Euler on the first step) and the box boundary condition,
// one particle per lane and direction by direction on SoA arrays.
//
// The kernel is HBM-bound and tiny next to Find and Interpolate: per particle
// and direction it reads x, v, v_prev, a_prev and u and writes x, v, v_prev,
// a_prev (72 bytes), plus one 4-byte code.  Loads are unit-stride across the
// wavefront.  This file is built without FP contraction so that every
// operation rounds as written (no fused multiply-adds).
#include "fpts_internal.hpp"

namespace fpts {
namespace {

template <int D>
__global__ __launch_bounds__(256) void k_lpt_advance(LptArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += stride) {
        if (a.code[p] == FPTS_NOT_FOUND) continue;     // lost: keeps its state
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const size_t o = (size_t)d * a.n + p;
            const double x = a.x[o], v = a.v[o], u = a.u[o];
            const double acc = (u - v) / a.tau;
            double xn, vn;
            if (a.first) {
                xn = x + a.dt * v;
                vn = v + a.dt * acc;
            } else {
                const double hv = a.hist_v[o], ha = a.hist_a[o];
                xn = x + a.dt * (1.5 * v - 0.5 * hv);
                vn = v + a.dt * (1.5 * acc - 0.5 * ha);
            }
            double nhv = v, nha = acc;
            const double lo = a.lo[d], hi = a.hi[d];
            if (a.periodic[d]) {
                if (xn < lo || xn >= hi) {
                    const double L = hi - lo;
                    xn = xn - L * floor((xn - lo) / L);
                }
            } else {
                const bool up = xn > hi, dn = xn < lo;
                if (up) xn = 2.0 * hi - xn;
                else if (dn) xn = 2.0 * lo - xn;
                if (up || dn) {
                    vn = -vn;
                    nhv = -nhv;
                    nha = -nha;
                }
                xn = fmin(fmax(xn, lo), hi);
            }
            a.x[o] = xn;
            a.v[o] = vn;
            a.hist_v[o] = nhv;
            a.hist_a[o] = nha;
        }
    }
}

}  // namespace

hipError_t launch_lpt_advance(const fpts_mesh *m, const LptArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((a.n + 255) / 256, (int64_t)m->cus * 16);
    if (m->D == 2)
        hipLaunchKernelGGL(k_lpt_advance<2>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_lpt_advance<3>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fpts
