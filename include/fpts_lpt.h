/*
 * fpts_lpt -- one-way coupled inertial point particles carried by a fluid
 * velocity field that lives on the same high-order mesh (fpts.h), on one GPU.
 *
 * This is the Lagrangian particle tracking application of the paper (Section
 * 6.7, its algorithm "Lagrangian Particle Tracking" and the table of its time
 * breakdown), where Find and Interpolate take almost all of the particle
 * time.  One call advances every particle by one time step, in the paper's
 * order of operations:
 *
 *   Interpolate  u = fluid velocity at each particle, from the Find result
 *                of its current position (fpts_eval, D fields)
 *   ParticleRHS  a = (u - v) / tau                       (Stokes drag)
 *   Integrate    x' = v, v' = a by second-order Adams-Bashforth,
 *                  x <- x + dt (3/2 v - 1/2 v_prev)
 *                  v <- v + dt (3/2 a - 1/2 a_prev)
 *                or by forward Euler (x <- x + dt v, v <- v + dt a) on the
 *                first step, which has no history
 *   ParticleBC   per direction of the domain box [lo, hi]: periodic
 *                directions wrap x into [lo, hi) as
 *                x - (hi - lo) floor((x - lo) / (hi - lo)); wall directions
 *                mirror a particle that left (x <- 2 hi - x or 2 lo - x) and
 *                negate that component of v, v_prev and a_prev, then clamp x
 *                to [lo, hi]
 *   Find         element and reference coordinates of the new positions
 *                (fpts_find)
 *
 * The boundary condition is applied before Find (the paper lists it after
 * Find and leaves its form open) so that Find sees positions inside the
 * domain.  A particle whose current Find result is NOT_FOUND keeps its
 * position, velocity and history.  The fluid solve and the migration of
 * particles between ranks are not part of this library: the field is given
 * and the mesh is on one GPU.  The integration arithmetic is evaluated
 * operation by operation in the order written above, without fused
 * multiply-adds.
 *
 * Pointers named d_* are caller-owned device memory; the call only enqueues
 * work on `stream`.  Status codes are those of fpts.h.
 */
#ifndef FPTS_LPT_H
#define FPTS_LPT_H

#include <stddef.h>
#include <stdint.h>

#include "fpts.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpts_lpt_params {
    double tau;          /* particle response (Stokes) time, > 0 */
    double dt;           /* time step, > 0 */
    double lo[3];        /* domain box, lo[d] < hi[d] for d < dim */
    double hi[3];
    int periodic[3];     /* per direction: 1 wrap, 0 walls that mirror */
    int hint;            /* nonzero: hinted Find.  A particle whose last code
                            was INTERIOR is first searched in its previous
                            element from its previous r, for at most 8
                            Newton passes; when that converges INTERIOR at
                            least 1e-9 inside the reference box no other
                            element can hold the particle in its interior,
                            so the full Find would give the same element and
                            r, and the particle keeps it.  All other
                            particles take the full Find.  Not part of the
                            paper's method, which runs the full Find every
                            step; 0 runs exactly that */
} fpts_lpt_params;

/* Bytes of device workspace fpts_lpt_step needs for n particles (the
 * interpolated velocity, the hinted-search flags and the larger of the Find
 * and Interpolate workspaces), or 0 when n is out of range. */
size_t fpts_lpt_workspace_size(const fpts_mesh *m, int64_t n);

/* One time step of n particles on a volume mesh (ref_dim == dim).
 *   d_x      [dim][n]     positions, updated in place
 *   d_v      [dim][n]     velocities, updated in place
 *   d_hist   [2][dim][n]  v_prev then a_prev: read unless `first`, and
 *                         overwritten with this step's v and a
 *   d_field  [dim][n_elem][nodes_1d^dim]  fluid velocity at the mesh nodes
 *   d_code, d_elem, d_r, d_dist           the fpts_find result of d_x on
 *                         entry (from fpts_find or the previous step); on
 *                         return that of the new positions
 *   first    nonzero: forward Euler, d_hist is not read
 *   precision, d_ws, ws_bytes             as for fpts_find; the workspace
 *                         holds at least fpts_lpt_workspace_size(m, n) bytes
 *                         and is 256-byte aligned
 * n == 0 is a no-op.  FPTS_EINVAL for null pointers, n out of range, a
 * surface mesh, tau or dt not positive and finite, lo >= hi, or a too small
 * workspace; FPTS_EDEVICE for HIP errors. */
int fpts_lpt_step(fpts_mesh *m, const fpts_lpt_params *p, int64_t n, int first, double *d_x,
                  double *d_v, double *d_hist, const double *d_field, int32_t *d_code,
                  int32_t *d_elem, double *d_r, double *d_dist, int precision, void *d_ws,
                  size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif
