// Trust-region Newton kernels (Section 3.2.1) of the volume and surface
// element kinds: hexahedra (D = 3, R = 3), quadrilaterals (D = 2, R = 2) and
// surface quadrilaterals (D = 3, R = 2), every order N, both precisions; the
// kernels themselves are the templates of newton_mfma.hpp.
#include "newton_mfma.hpp"

namespace fpts {

hipError_t launch_newton_hex(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                             const NewtonIO &io, int which, hipStream_t s)
{
    return newton::launch_newton_kind<3, 3>(m, mixed, n, pts, io, which, s);
}

hipError_t launch_newton_quad(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s)
{
    return newton::launch_newton_kind<2, 2>(m, mixed, n, pts, io, which, s);
}

hipError_t launch_newton_surf(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                              const NewtonIO &io, int which, hipStream_t s)
{
    return newton::launch_newton_kind<3, 2>(m, mixed, n, pts, io, which, s);
}

}  // namespace fpts
