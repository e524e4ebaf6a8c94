// Trust-region Newton kernels for surface quadrilateral elements (D = 3, R = 2).
#include "newton_mfma.hpp"

namespace fpts {

hipError_t launch_newton_surf(const fpts_mesh *m, bool mixed, int64_t n, const double *pts,
                            const NewtonIO &io, int which, hipStream_t s)
{
    return newton::launch_newton_kind<3, 2>(m, mixed, n, pts, io, which, s);
}

}  // namespace fpts
