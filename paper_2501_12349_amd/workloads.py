"""Seeded synthetic workloads (meshes, query points, nodal fields).

This module only produces inputs: node coordinates of structured, curved
quad/hex meshes and of a bumpy cubed-sphere surface, query points and nodal
field values.  It holds none of the field-evaluation method's arithmetic (no
element map, no bounds, no Newton): node positions are placed at
Gauss-Lobatto-Legendre points computed here with ``numpy.polynomial`` and the
curving maps are analytic functions of the node positions.  Both the oracle
tests and the HIP library consume these arrays.

Layouts: nodes ``[n_elem][D][N^R]`` (i fastest, then j, then k), points
``[D][n]``, fields ``[n_fields][n_elem][N^R]``; all float64.

The paper's meshes (spiral, triple point, turbine blade, channel) are not
available; these stand in for them with the shapes and sizes of the five
workloads:

* ``quad2d``  : 8x8 quads on [0,1]^2, p=4, X += 0.05 h sin(2 pi X) sin(2 pi Y)
* ``hex16``   : 16^3 hexes, p=5, x += 0.1 sin(pi x) sin(pi y) sin(pi z)
* ``hex48``   : 48^3 hexes, p=7, amplitude 0.15, 16M points, 3 fields
* ``serving`` : four resident hex meshes p=3,5,7,9
* ``sphere``  : cubed sphere 6x32x32, p=6, radius 1 + 0.05 B(x)
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(N):
    """GLL points on [-1,1] for node placement (numpy's Legendre roots)."""
    if N == 2:
        return np.array([-1.0, 1.0])
    inner = npleg.Legendre.basis(N - 1).deriv().roots()
    z = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    z = 0.5 * (z - z[::-1])
    return z


def box_mesh(D, n, N):
    """Uncurved structured mesh of [0,1]^D with n elements per direction and
    N GLL nodes per direction.  Element id = a + n*(b + n*c)."""
    t = 0.5 * (gll_points(N) + 1.0) / n           # local offsets in [0, 1/n]
    a = np.arange(n) / n
    if D == 2:
        X = (a[None, :, None, None] + t[None, None, None, :])  # [b][a][j][i]
        Y = (a[:, None, None, None] + t[None, None, :, None])
        X = np.broadcast_to(X, (n, n, N, N))
        Y = np.broadcast_to(Y, (n, n, N, N))
        nodes = np.stack([X, Y], axis=2)          # [b][a][D][j][i]
        return np.ascontiguousarray(nodes.reshape(n * n, 2, N * N))
    X = a[None, None, :, None, None, None] + t[None, None, None, None, None, :]
    Y = a[None, :, None, None, None, None] + t[None, None, None, None, :, None]
    Z = a[:, None, None, None, None, None] + t[None, None, None, :, None, None]
    shp = (n, n, n, N, N, N)
    nodes = np.stack([np.broadcast_to(X, shp), np.broadcast_to(Y, shp),
                      np.broadcast_to(Z, shp)], axis=3)   # [c][b][a][D][k][j][i]
    return np.ascontiguousarray(nodes.reshape(n ** 3, 3, N ** 3))


def curve_quad2d(nodes, n):
    """X += 0.05 h sin(2 pi X) sin(2 pi Y) applied to both components."""
    h = 1.0 / n
    X, Y = nodes[:, 0].copy(), nodes[:, 1].copy()
    d = 0.05 * h * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    out = nodes.copy()
    out[:, 0] = X + d
    out[:, 1] = Y + d
    return out


def curve_hex(nodes, amp, chunk=4096):
    """x_c += amp sin(pi x) sin(pi y) sin(pi z) for every component c."""
    out = np.empty_like(nodes)
    for s in range(0, nodes.shape[0], chunk):
        blk = nodes[s:s + chunk]
        d = amp * (np.sin(np.pi * blk[:, 0]) * np.sin(np.pi * blk[:, 1]) *
                   np.sin(np.pi * blk[:, 2]))
        out[s:s + chunk] = blk + d[:, None, :]
    return out


def poly_coeffs(D, deg, rng):
    """Random total-degree-``deg`` polynomial: list of (exponents, coeff)."""
    terms = []
    if D == 2:
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                terms.append(((a, b), rng.uniform(-1, 1)))
    else:
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                for c in range(deg + 1 - a - b):
                    terms.append(((a, b, c), rng.uniform(-1, 1)))
    return terms


def _poly_chunk(terms, blk, deg):
    D = blk.shape[0]
    pw = [[np.ones(blk.shape[1])] for _ in range(D)]
    for d in range(D):
        for _ in range(deg):
            pw[d].append(pw[d][-1] * blk[d])
    acc = np.zeros(blk.shape[1])
    for e, c in terms:
        t = c * pw[0][e[0]]
        for d in range(1, D):
            t = t * pw[d][e[d]]
        acc += t
    return acc


def poly_eval(terms, X, chunk=1 << 20):
    """Evaluate a polynomial given by ``poly_coeffs`` at points X [D][...]
    (chunks in a thread pool; numpy releases the GIL on array arithmetic)."""
    import concurrent.futures as cf
    import os
    X = np.asarray(X)
    D = X.shape[0]
    flat = X.reshape(D, -1)
    out = np.empty(flat.shape[1])
    deg = max(sum(e) for e, _ in terms)
    starts = list(range(0, flat.shape[1], chunk))
    nthreads = max(1, min(16, os.cpu_count() or 1, len(starts)))

    def work(s0):
        out[s0:s0 + chunk] = _poly_chunk(terms, flat[:, s0:s0 + chunk], deg)

    if nthreads == 1:
        for s0 in starts:
            work(s0)
    else:
        with cf.ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, starts))
    return out.reshape(X.shape[1:])


def nodal_field(nodes, terms):
    """Field values u(x_node) of a physical polynomial: [nel][NP]."""
    X = np.moveaxis(nodes, 1, 0)          # [D][nel][NP]
    return poly_eval(terms, X)


def uniform_points(rng, n, D, lo, hi):
    return rng.uniform(lo, hi, size=(D, n))


def shell_points(rng, n, D, inner=(0.0, 1.0), outer=(-0.05, 1.05)):
    """n points uniform in the outer box minus the inner box (rejection)."""
    out = np.empty((D, 0))
    while out.shape[1] < n:
        p = rng.uniform(outer[0], outer[1], size=(D, 2 * n + 16))
        ins = np.all((p >= inner[0]) & (p <= inner[1]), axis=0)
        out = np.concatenate([out, p[:, ~ins]], axis=1)
    return np.ascontiguousarray(out[:, :n])


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------

def quad2d(n_pts=10000, seed=1000):
    """8x8 curved quads, p=4; points uniform in [-0.05,1.05]^2; a total-degree
    4 field plus the linear field x (rows 0 and 1 of ``fields``)."""
    rng = np.random.default_rng(seed)
    n, N = 8, 5
    nodes = curve_quad2d(box_mesh(2, n, N), n)
    pts = uniform_points(rng, n_pts, 2, -0.05, 1.05)
    terms = poly_coeffs(2, 4, rng)
    fields = np.stack([nodal_field(nodes, terms), nodes[:, 0].copy()])
    return dict(name="quad2d_8x8_p4", dim=2, ref_dim=2, N=N, nodes=nodes, pts=pts,
                fields=fields, terms=[terms, [((1, 0), 1.0)]], h=1.0 / n)


def hex16(n_in=1000000, n_out=20000, seed=1001):
    """16^3 curved hexes, p=5; 1M points in the cube plus 2% in the shell
    [-0.05,1.05]^3 minus [0,1]^3; a total-degree 5 scalar field."""
    rng = np.random.default_rng(seed)
    n, N = 16, 6
    nodes = curve_hex(box_mesh(3, n, N), 0.1)
    pts = np.concatenate([uniform_points(rng, n_in, 3, 0.0, 1.0),
                          shell_points(rng, n_out, 3)], axis=1)
    terms = poly_coeffs(3, 5, rng)
    fields = nodal_field(nodes, terms)[None]
    return dict(name="hex16_p5", dim=3, ref_dim=3, N=N, nodes=nodes, pts=pts,
                fields=fields, terms=[terms], h=1.0 / n)


def hex48(n_pts=1 << 24, seed=1002, with_fields=True, n_elem_side=48):
    """48^3 curved hexes (amplitude 0.15), p=7; 2^24 points uniform in the
    cube; three total-degree 7 fields."""
    rng = np.random.default_rng(seed)
    n, N = n_elem_side, 8
    nodes = curve_hex(box_mesh(3, n, N), 0.15)
    pts = uniform_points(rng, n_pts, 3, 0.0, 1.0)
    terms = [poly_coeffs(3, 7, rng) for _ in range(3)]
    fields = None
    if with_fields:
        fields = np.stack([nodal_field(nodes, t) for t in terms])
    return dict(name="hex48_p7", dim=3, ref_dim=3, N=N, nodes=nodes, pts=pts,
                fields=fields, terms=terms, h=1.0 / n)


SERVING_MESHES = ((4, 46), (6, 36), (8, 27), (10, 22))   # (N = p+1, elems/dir)


def serving_mesh(k, seed=1003, scale=1.0):
    """Resident mesh k of the serving workload: p = 3,5,7,9 with 46^3, 36^3,
    27^3, 22^3 hexes (amplitude 0.1) and a degree-p scalar field.  ``scale``
    < 1 shrinks the element count per direction (for small tests)."""
    N, n = SERVING_MESHES[k]
    n = max(2, int(round(n * scale)))
    rng = np.random.default_rng(seed + 17 * k)
    nodes = curve_hex(box_mesh(3, n, N), 0.1)
    terms = poly_coeffs(3, N - 1, rng)
    fields = nodal_field(nodes, terms)[None]
    return dict(name="serve_p%d_%d3" % (N - 1, n), dim=3, ref_dim=3, N=N,
                nodes=nodes, fields=fields, terms=[terms], h=1.0 / n)


def serving_requests(n_req, seed=1004, lo=3.0, hi=6.0, n_mesh=4):
    """Request sizes round(10^U(lo,hi)), uniform mesh choice."""
    rng = np.random.default_rng(seed)
    sizes = np.round(10.0 ** rng.uniform(lo, hi, size=n_req)).astype(np.int64)
    meshes = rng.integers(0, n_mesh, size=n_req)
    return sizes, meshes, rng


# --------------------------------------------------------------------------
# Cubed sphere with random spherical-harmonic bumps.
# --------------------------------------------------------------------------

def _face_dirs(f, X, Y):
    """Unnormalised direction of gnomonic coordinates (X, Y) on face f."""
    one = np.ones_like(X)
    if f == 0:
        return np.stack([one, X, Y])
    if f == 1:
        return np.stack([-one, -X, Y])
    if f == 2:
        return np.stack([-X, one, Y])
    if f == 3:
        return np.stack([X, -one, Y])
    if f == 4:
        return np.stack([-Y, X, one])
    return np.stack([Y, X, -one])


def _real_sph(l, m, theta, phi):
    from scipy.special import sph_harm_y
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    if m > 0:
        return math.sqrt(2.0) * sph_harm_y(l, m, theta, phi).real
    return math.sqrt(2.0) * sph_harm_y(l, -m, theta, phi).imag


class Bumps:
    """B(x_hat) = sum_{l=2..6} sum_m c_lm Y_lm(x_hat), c_lm ~ N(0,1),
    normalised to max |B| = 1 over a fine sample of the sphere."""

    def __init__(self, rng):
        self.terms = [(l, m, rng.standard_normal()) for l in range(2, 7)
                      for m in range(-l, l + 1)]
        th = np.linspace(0, np.pi, 181)
        ph = np.linspace(0, 2 * np.pi, 361)
        T, P = np.meshgrid(th, ph, indexing="ij")
        self.scale = 1.0
        self.scale = 1.0 / np.abs(self._raw(T.ravel(), P.ravel())).max()

    def _raw(self, theta, phi):
        acc = np.zeros_like(theta)
        for l, m, c in self.terms:
            acc += c * _real_sph(l, m, theta, phi)
        return acc * self.scale

    def __call__(self, u):
        """u: unit vectors [3][n]."""
        theta = np.arccos(np.clip(u[2], -1.0, 1.0))
        phi = np.arctan2(u[1], u[0])
        return self._raw(theta, phi)


def _sphere_surface(bumps, f, xi, eta, amp):
    d = _face_dirs(f, np.tan(xi), np.tan(eta))
    u = d / np.linalg.norm(d, axis=0)
    return (1.0 + amp * bumps(u)) * u


def sphere(n_pts=1 << 22, seed=1005, ne=32, N=7, amp=0.05, far_frac=0.01,
           offset=1e-3):
    """Cubed sphere 6 x ne x ne quads, N nodes per direction, equiangular
    gnomonic faces, radius 1 + amp B.  Points: (1-far_frac) at signed normal
    offsets U[-offset, offset] from the analytic surface at uniformly drawn
    (element, local coordinates); far_frac uniform in 1.5 <= |x| <= 2."""
    rng = np.random.default_rng(seed)
    bumps = Bumps(rng)
    z = gll_points(N)
    edges = np.linspace(-np.pi / 4, np.pi / 4, ne + 1)
    nel = 6 * ne * ne
    nodes = np.empty((nel, 3, N * N))
    e = 0
    for f in range(6):
        for b in range(ne):
            for a in range(ne):
                xa = edges[a] + 0.5 * (z + 1.0) * (edges[a + 1] - edges[a])
                yb = edges[b] + 0.5 * (z + 1.0) * (edges[b + 1] - edges[b])
                XI, ETA = np.meshgrid(xa, yb, indexing="xy")   # [j][i]
                nodes[e] = _sphere_surface(bumps, f, XI.ravel(), ETA.ravel(), amp)
                e += 1
    n_far = int(round(n_pts * far_frac))
    n_near = n_pts - n_far
    ef = rng.integers(0, nel, size=n_near)
    rr = rng.uniform(-1.0, 1.0, size=(2, n_near))
    dl = rng.uniform(-offset, offset, size=n_near)
    f = ef // (ne * ne)
    a = ef % ne
    b = (ef // ne) % ne
    xi = edges[a] + 0.5 * (rr[0] + 1.0) * (edges[a + 1] - edges[a])
    eta = edges[b] + 0.5 * (rr[1] + 1.0) * (edges[b + 1] - edges[b])
    near = np.empty((3, n_near))
    hs = 1e-6
    for face in range(6):
        sel = np.nonzero(f == face)[0]
        if sel.size == 0:
            continue
        x0 = _sphere_surface(bumps, face, xi[sel], eta[sel], amp)
        x1 = _sphere_surface(bumps, face, xi[sel] + hs, eta[sel], amp)
        x2 = _sphere_surface(bumps, face, xi[sel], eta[sel] + hs, amp)
        nrm = np.cross((x1 - x0).T, (x2 - x0).T).T
        nrm /= np.linalg.norm(nrm, axis=0)
        near[:, sel] = x0 + dl[sel] * nrm
    u = rng.standard_normal((3, n_far))
    u /= np.linalg.norm(u, axis=0)
    rad = np.cbrt(rng.uniform(1.5 ** 3, 2.0 ** 3, size=n_far))
    far = u * rad
    pts = np.ascontiguousarray(np.concatenate([near, far], axis=1))
    terms = poly_coeffs(3, N - 1, rng)
    fields = np.stack([nodal_field(nodes, terms), nodes[:, 0].copy()])
    return dict(name="sphere_6x%dx%d_p%d" % (ne, ne, N - 1), dim=3, ref_dim=2, N=N,
                nodes=nodes, pts=pts, fields=fields,
                terms=[terms, [((1, 0, 0), 1.0)]], h=(np.pi / 2) / ne)


# --------------------------------------------------------------------------
# Channel flow for particle tracking.
# --------------------------------------------------------------------------

CHANNEL_L = (2.0 * math.pi, 2.0, math.pi)     # Lx, height (y in [-1, 1]), Lz


def channel_mesh(n_el, N, beta=1.5, L=CHANNEL_L):
    """Channel [0,Lx] x [-1,1] (x [0,Lz]) with n_el = (nx, ny[, nz]) elements,
    N GLL nodes per direction, uniform in x and z and graded towards the
    walls in y by y = tanh(beta eta) / tanh(beta) applied node by node (so
    the element maps are curved in y).  Element id = a + nx*(b + ny*c);
    nodes shared by two elements are bit-identical."""
    D = len(n_el)
    t = 0.5 * (gll_points(N) + 1.0)
    s = [(np.arange(n)[:, None] + t[None, :]) / n for n in n_el]     # [n][N] in [0, 1]
    cx = L[0] * s[0]
    eta = 2.0 * s[1] - 1.0
    cy = np.sign(eta) * np.tanh(beta * np.abs(eta)) / np.tanh(beta)
    if D == 2:
        nx, ny = n_el
        X = np.broadcast_to(cx[None, :, None, :], (ny, nx, N, N))    # [b][a][j][i]
        Y = np.broadcast_to(cy[:, None, :, None], (ny, nx, N, N))
        nodes = np.stack([X, Y], axis=2)
        return np.ascontiguousarray(nodes.reshape(nx * ny, 2, N * N))
    nx, ny, nz = n_el
    cz = L[2] * s[2]
    shp = (nz, ny, nx, N, N, N)                                       # [c][b][a][k][j][i]
    X = np.broadcast_to(cx[None, None, :, None, None, :], shp)
    Y = np.broadcast_to(cy[None, :, None, None, :, None], shp)
    Z = np.broadcast_to(cz[:, None, None, :, None, None], shp)
    nodes = np.stack([X, Y, Z], axis=3)
    return np.ascontiguousarray(nodes.reshape(nx * ny * nz, 3, N ** 3))


def channel_modes(rng, n_modes=4, L=CHANNEL_L):
    """Random perturbation modes (kx, kz, A, B, phase_x, phase_z, phase_w),
    periodic in x and z."""
    modes = []
    for _ in range(n_modes):
        kx = 2.0 * math.pi * rng.integers(1, 4) / L[0]
        kz = 2.0 * math.pi * rng.integers(0, 3) / L[2]
        modes.append((kx, kz, rng.uniform(0.02, 0.08), rng.uniform(0.02, 0.08),
                      rng.uniform(0, 2 * math.pi), rng.uniform(0, 2 * math.pi),
                      rng.uniform(0, 2 * math.pi)))
    return modes


def channel_velocity(X, modes):
    """Analytic fluid velocity at X [D][...]: the laminar profile
    1.5 (1 - y^2) (bulk velocity 1 along x) plus, per mode, the curl of the
    stream function A (1-y^2)^2 sin(kx x + px) cos(kz z + pz) in the x-y
    plane and (3D) a spanwise B (1-y^2) sin(kx x + pw).  Divergence-free,
    zero at the walls y = +-1, periodic in x and z."""
    X = np.asarray(X, dtype=np.float64)
    D = X.shape[0]
    y = X[1]
    w = 1.0 - y * y
    out = np.zeros_like(X)
    out[0] = 1.5 * w
    for kx, kz, A, B, px, pz, pw in modes:
        cz = np.cos(kz * X[2] + pz) if D == 3 else 1.0
        out[0] += A * 2.0 * w * (-2.0 * y) * np.sin(kx * X[0] + px) * cz
        out[1] -= A * w * w * kx * np.cos(kx * X[0] + px) * cz
        if D == 3:
            out[2] += B * w * np.sin(kx * X[0] + pw)
    return out


def particle_lattice(n_y, D=3, L=CHANNEL_L):
    """n_x : n_y (: n_z) = 2 : 1 (: 1) particles at the centres of a uniform
    lattice of the channel; particle id = i + n_x*(j + n_y*k)."""
    n_x = 2 * n_y
    gx = (np.arange(n_x) + 0.5) / n_x * L[0]
    gy = -1.0 + (np.arange(n_y) + 0.5) / n_y * 2.0
    if D == 2:
        Y, X = np.meshgrid(gy, gx, indexing="ij")
        return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()]))
    gz = (np.arange(n_y) + 0.5) / n_y * L[2]
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


def lattice_n_y(ratio, n_comp):
    """n_y = n_z = ceil((ratio n_comp / 2)^(1/3)) for ratio = particles per
    computational point (Section 6.7)."""
    n = int(math.ceil((0.5 * ratio * n_comp) ** (1.0 / 3.0) - 1e-9))
    return max(n, 1)


def channel(n_el=(36, 24, 36), N=8, ratio=1.02, seed=1007, n_y=None, tau=5.0, dt=1e-3):
    """Particle-tracking workload: the channel mesh (31104 hexes, p=7 by
    default: 15.9M computational points), the fluid velocity at its nodes
    ([D][nel][NP], three fields), the particle lattice for ``ratio``
    particles per computational point, their initial velocity (the fluid's,
    analytic), Stokes time tau = 5 and dt = 1e-3 as in the paper."""
    rng = np.random.default_rng(seed)
    D = len(n_el)
    nodes = channel_mesh(n_el, N)
    modes = channel_modes(rng)
    fields = np.ascontiguousarray(channel_velocity(np.moveaxis(nodes, 1, 0), modes))
    n_comp = nodes.shape[0] * N ** D
    if n_y is None:
        n_y = lattice_n_y(ratio, n_comp)
    pts = particle_lattice(n_y, D)
    v0 = np.ascontiguousarray(channel_velocity(pts, modes))
    L = CHANNEL_L
    lo = (0.0, -1.0, 0.0)[:D]
    hi = (L[0], 1.0, L[2])[:D]
    periodic = (1, 0, 1)[:D]
    name = "channel_%s_p%d" % ("x".join(str(n) for n in n_el), N - 1)
    return dict(name=name, dim=D, ref_dim=D, N=N, nodes=nodes, fields=fields, pts=pts, v0=v0,
                modes=modes, lo=lo, hi=hi, periodic=periodic, tau=tau, dt=dt, n_y=n_y,
                n_comp=n_comp, h=min(L[0] / n_el[0], 2.0 / n_el[1]))


# --------------------------------------------------------------------------
# Line meshes (D_r = 1) in 2D and 3D.
# --------------------------------------------------------------------------

def _line_pieces_2d():
    """Curve pieces of the 2D line workload: the boundary of [0,7] x [0,3]
    (straight) and two curved interfaces meeting it and each other at
    element ends, 84 elements at level 0.  Each piece: (function of the
    parameter s in [0, 1] -> (x, y), elements at level 0)."""
    def seg(p, q):
        return lambda s: (p[0] + s * (q[0] - p[0]), p[1] + s * (q[1] - p[1]))
    iface1 = lambda s: (1.0 + 0.08 * np.sin(2.0 * np.pi * s), 3.0 * s)
    iface2 = lambda s: (1.0 + 6.0 * s, 1.5 + 0.3 * np.sin(np.pi * s))
    return [(seg((0, 0), (7, 0)), 21), (seg((7, 0), (7, 3)), 6), (seg((7, 3), (0, 3)), 21),
            (seg((0, 3), (0, 0)), 6), (iface1, 6), (iface2, 24)]


def _trefoil(s):
    t = 2.0 * np.pi * s
    return (np.sin(t) + 2.0 * np.sin(2.0 * t), np.cos(t) - 2.0 * np.cos(2.0 * t),
            -np.sin(3.0 * t))


def line_mesh(pieces, N, level):
    """Nodes [nel][D][N] of curve pieces split into 2^level times their
    level-0 element count, uniform in the curve parameter; nodes at the GLL
    points of each element's parameter interval.  Also the parameter
    interval of every element, for sampling points on the curves."""
    t = 0.5 * (gll_points(N) + 1.0)
    nodes, spans = [], []
    for f, m0 in pieces:
        m = m0 * 2 ** level
        a = np.arange(m) / m
        S = (a[:, None] + t[None, :] / m)             # [m][N]
        S[:, -1] = (np.arange(m) + 1) / m              # shared ends bit-identical
        X = np.stack([np.asarray(c, dtype=np.float64) for c in f(S)], axis=1)   # [m][D][N]
        nodes.append(X)
        spans.append((f, a, 1.0 / m))
    return np.ascontiguousarray(np.concatenate(nodes)), spans


def line_points_on_curves(spans, per_elem, rng, offset=0.0):
    """per_elem points per element at uniform random curve parameters of its
    interval, on the analytic curve (not on the element's polynomial), plus,
    with offset > 0, a random displacement of length U(0, offset) in a random
    direction."""
    out = []
    for f, a, h in spans:
        s = (a[:, None] + h * rng.uniform(0, 1, (a.size, per_elem))).ravel()
        out.append(np.stack([np.asarray(c, dtype=np.float64) for c in f(s)]))
    P = np.concatenate(out, axis=1)
    if offset > 0:
        u = rng.standard_normal(P.shape)
        u /= np.linalg.norm(u, axis=0)
        P = P + u * rng.uniform(0, offset, P.shape[1])
    return np.ascontiguousarray(P)


def line2d(level=8, per_elem=1000, N=4, seed=1008):
    """Cubic line mesh in 2D standing in for the paper's cubic surface mesh
    of the 2D triple-point problem (Section 6.3): 84 elements at level 0, 84
    x 2^level after uniform refinement (21 504 at level 8), per_elem points
    per element on the curves, a cubic field of (x, y)."""
    rng = np.random.default_rng(seed)
    nodes, spans = line_mesh(_line_pieces_2d(), N, level)
    pts = line_points_on_curves(spans, per_elem, rng)
    terms = poly_coeffs(2, 3, rng)
    fields = nodal_field(nodes, terms)[None]
    return dict(name="line2d_%del_p%d" % (nodes.shape[0], N - 1), dim=2, ref_dim=1, N=N,
                nodes=nodes, pts=pts, fields=fields, terms=[terms], h=3.0 / 6 / 2 ** level)


def line3d(n_elem=64, per_elem=200, N=5, seed=1009, offset=1e-3):
    """A trefoil knot in 3D with n_elem curved elements of N nodes; points
    near the curve (random offsets up to `offset`) and a degree N-1 field."""
    rng = np.random.default_rng(seed)
    nodes, spans = line_mesh([(_trefoil, n_elem)], N, 0)
    pts = line_points_on_curves(spans, per_elem, rng, offset)
    terms = poly_coeffs(3, N - 1, rng)
    fields = nodal_field(nodes, terms)[None]
    return dict(name="line3d_trefoil_%del_p%d" % (n_elem, N - 1), dim=3, ref_dim=1, N=N,
                nodes=nodes, pts=pts, fields=fields, terms=[terms], h=10.0 / n_elem)
