"""Particle-transport oracle -- TEST INFRASTRUCTURE ONLY.

One time step of one-way coupled inertial point particles carried by a
frozen fluid velocity field, the Lagrangian particle tracking application
of arXiv 2501.12349 (Section 6.7, the algorithm "Lagrangian Particle
Tracking" and the table of its time breakdown), written with numpy in FP64
over the oracle's Find and Interpolate.  Per step, in the paper's order:

  Interpolate  u = fluid velocity at each particle, from the last Find
  ParticleRHS  a = (u - v) / tau                      (Stokes drag)
  Integrate    x' = v and v' = a by second-order Adams-Bashforth, the
               order the paper pairs with its second-order flow solver;
               the first step has no history and takes forward Euler
  ParticleBC   the box: wrap in periodic directions, mirror at walls
  Find         element and reference coordinates of the new positions

Readings where the paper is silent (also listed with the design notes):
the boundary condition is applied to the integrated positions before Find
so that Find sees positions inside the domain; at a wall the particle is
mirrored (position reflected, the normal component of its velocity and of
its Adams-Bashforth history negated); a particle whose last Find said
NOT_FOUND keeps its state (it is not moved).  FluidSolve and Migrate are
outside the one-GPU path: the fluid field is frozen and nothing migrates.

Only ``tests/``, the package smoke check and the CPU-baseline leg of the
benchmark may import this module; it imports nothing from the product.
"""
import numpy as np

from . import NOT_FOUND

# Adams-Bashforth 2: y_{n+1} = y_n + dt (3/2 f_n - 1/2 f_{n-1})
AB2_NEW, AB2_OLD = 1.5, 0.5


def advance(x, v, hist_v, hist_a, u, code, tau, dt, first, lo, hi, periodic):
    """ParticleRHS + Integrate + ParticleBC for all particles at once.

    x, v, hist_v, hist_a, u: [D][n] float64 (hist_*: v and a of the previous
    step, ignored when ``first``); code: [n] from the last Find.  Returns new
    (x, v, hist_v, hist_a); the inputs are not modified."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    hv = np.array(hist_v, dtype=np.float64)
    ha = np.array(hist_a, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    live = np.asarray(code) != NOT_FOUND
    D = x.shape[0]
    for d in range(D):
        a = (u[d] - v[d]) / tau                          # Stokes drag
        if first:
            xn = x[d] + dt * v[d]                        # forward Euler
            vn = v[d] + dt * a
        else:
            xn = x[d] + dt * (AB2_NEW * v[d] - AB2_OLD * hv[d])
            vn = v[d] + dt * (AB2_NEW * a - AB2_OLD * ha[d])
        nhv, nha = v[d].copy(), a
        L = hi[d] - lo[d]
        if periodic[d]:
            out = (xn < lo[d]) | (xn >= hi[d])
            xn = np.where(out, xn - L * np.floor((xn - lo[d]) / L), xn)
        else:
            up = xn > hi[d]
            dn = xn < lo[d]
            xn = np.where(up, 2.0 * hi[d] - xn, np.where(dn, 2.0 * lo[d] - xn, xn))
            flip = up | dn
            vn = np.where(flip, -vn, vn)
            nhv = np.where(flip, -nhv, nhv)
            nha = np.where(flip, -nha, nha)
            xn = np.minimum(np.maximum(xn, lo[d]), hi[d])   # a move longer than the box
        x[d] = np.where(live, xn, x[d])
        v[d] = np.where(live, vn, v[d])
        hv[d] = np.where(live, nhv, hv[d])
        ha[d] = np.where(live, nha, ha[d])
    return x, v, hv, ha


def step(mesh, field, state, tau, dt, lo, hi, periodic, first):
    """One time step.  ``state`` = dict(x, v, hist_v, hist_a, find) where
    ``find`` is the oracle Find result for x; returns the new state with the
    Find result of the new positions and the interpolated velocity ``u``."""
    u = mesh.eval(state["find"], field)
    x, v, hv, ha = advance(state["x"], state["v"], state["hist_v"], state["hist_a"], u,
                           state["find"]["code"], tau, dt, first, lo, hi, periodic)
    return dict(x=x, v=v, hist_v=hv, hist_a=ha, find=mesh.find(x), u=u)


def run(mesh, field, x0, v0, steps, tau, dt, lo, hi, periodic):
    """Find x0, then ``steps`` time steps (the first one Euler)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    st = dict(x=x0, v=np.array(v0, dtype=np.float64), hist_v=np.zeros_like(x0),
              hist_a=np.zeros_like(x0), find=mesh.find(x0))
    for k in range(steps):
        st = step(mesh, field, st, tau, dt, lo, hi, periodic, first=(k == 0))
    return st
