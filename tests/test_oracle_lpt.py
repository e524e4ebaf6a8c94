"""Pins of the particle-transport oracle (oracle.lpt) against closed forms,
order of accuracy, symmetry and the channel workload's own properties."""
import math

import numpy as np
import pytest

import oracle
from oracle import lpt
from paper_2501_12349_amd import workloads as W

BIG = (-1e9, -1e9, -1e9), (1e9, 1e9, 1e9), (0, 0, 0)      # no boundary in reach


def _integrate(x0, v0, U, tau, dt, steps, lo=BIG[0], hi=BIG[1], periodic=BIG[2]):
    """advance() alone with a given fluid velocity U (constant per particle)."""
    D, n = x0.shape
    x, v = x0.copy(), v0.copy()
    hv, ha = np.zeros_like(x), np.zeros_like(x)
    code = np.zeros(n, np.int32)
    for k in range(steps):
        x, v, hv, ha = lpt.advance(x, v, hv, ha, U, code, tau, dt, k == 0, lo[:D], hi[:D],
                                   periodic[:D])
    return x, v, hv, ha


def test_first_step_is_forward_euler():
    rng = np.random.default_rng(0)
    x0, v0, U = rng.uniform(-1, 1, (3, 50)), rng.uniform(-1, 1, (3, 50)), rng.uniform(-1, 1, (3, 50))
    x, v, hv, ha = _integrate(x0, v0, U, 0.7, 0.01, 1)
    assert np.array_equal(x, x0 + 0.01 * v0)
    assert np.array_equal(v, v0 + 0.01 * ((U - v0) / 0.7))
    assert np.array_equal(hv, v0) and np.array_equal(ha, (U - v0) / 0.7)


def test_tracer_in_uniform_flow_moves_at_the_flow_velocity():
    """v0 = U: the drag is zero and x = x0 + t U exactly up to rounding."""
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-1, 1, (3, 40))
    U = np.broadcast_to(np.array([[0.7], [-0.2], [0.3]]), x0.shape).copy()
    x, v, _, _ = _integrate(x0, U.copy(), U, 5.0, 1e-3, 200)
    assert np.array_equal(v, U)
    assert np.abs(x - (x0 + 0.2 * U)).max() < 1e-13


def _relax_errors(dt, T=1.0, tau=0.5):
    """Particles at rest released in a uniform flow: error at time T against
    v = U (1 - e^{-t/tau}), x = x0 + U (t - tau (1 - e^{-t/tau}))."""
    U = np.array([[1.0], [-0.5], [0.25]])
    x0 = np.zeros((3, 1))
    steps = int(round(T / dt))
    x, v, _, _ = _integrate(x0, np.zeros((3, 1)), U, tau, dt, steps)
    g = 1.0 - math.exp(-T / tau)
    return np.abs(v - U * g).max(), np.abs(x - U * (T - tau * g)).max()


def test_integrator_is_second_order():
    """Halving dt divides the error by about 4 (Adams-Bashforth 2 with one
    Euler start step); forward Euler throughout would give 2."""
    e = [_relax_errors(0.02 / 2 ** k) for k in range(4)]
    for k in range(3):
        for c in range(2):
            ratio = e[k][c] / e[k + 1][c]
            assert 3.6 < ratio < 4.4, (k, c, ratio)
    assert e[-1][0] < 1e-5


def test_wall_reflection_mirrors_the_free_trajectory():
    """Zero fluid velocity, particles thrown at the wall y = 1: with the wall
    the trajectory is the mirror image 2 - y of the free one once it crosses,
    velocity and history negated (linear drag keeps mirror symmetry)."""
    y0 = np.linspace(0.5, 0.95, 10)
    x0 = np.stack([np.zeros(10), y0, np.zeros(10)])
    v0 = np.stack([np.full(10, 0.3), np.full(10, 1.0), np.zeros(10)])
    U = np.zeros((3, 10))
    lo, hi, per = (0.0, -1.0, 0.0), (10.0, 1.0, 10.0), (0, 0, 0)
    crossed = np.zeros(10, bool)
    xf, vf, hvf, haf = x0.copy(), v0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    xw, vw, hvw, haw = x0.copy(), v0.copy(), np.zeros_like(x0), np.zeros_like(x0)
    code = np.zeros(10, np.int32)
    for k in range(40):
        xf, vf, hvf, haf = lpt.advance(xf, vf, hvf, haf, U, code, 2.0, 0.02, k == 0,
                                       BIG[0], BIG[1], BIG[2])
        xw, vw, hvw, haw = lpt.advance(xw, vw, hvw, haw, U, code, 2.0, 0.02, k == 0, lo, hi, per)
        crossed |= xf[1] > 1.0
        assert np.all(np.abs(xw[1]) <= 1.0)
        my = np.where(crossed, 2.0 - xf[1], xf[1])
        sv = np.where(crossed, -1.0, 1.0)
        assert np.abs(xw[1] - my).max() < 1e-14, k
        assert np.abs(vw[1] - sv * vf[1]).max() < 1e-15, k
        assert np.abs(hvw[1] - sv * hvf[1]).max() < 1e-15, k
        assert np.abs(haw[1] - sv * haf[1]).max() < 1e-15, k
        assert np.array_equal(xw[0], xf[0]) and np.array_equal(vw[0], vf[0])
    assert crossed.all()


def test_periodic_wrap():
    L = 2.0 * math.pi
    x0 = np.array([[L - 0.01, 0.005], [0.0, 0.0], [0.0, 0.0]])
    U = np.array([[1.0, -1.0], [0.0, 0.0], [0.0, 0.0]])
    x, v, _, _ = _integrate(x0, U.copy(), U, 5.0, 0.004, 5, lo=(0.0, -1.0, 0.0),
                            hi=(L, 1.0, math.pi), periodic=(1, 0, 1))
    assert abs(x[0, 0] - 0.01) < 1e-14
    assert abs(x[0, 1] - (L - 0.015)) < 1e-14
    assert np.all((x[0] >= 0) & (x[0] < L))


def test_lost_particles_keep_their_state():
    rng = np.random.default_rng(3)
    x0, v0 = rng.uniform(-1, 1, (3, 8)), rng.uniform(-1, 1, (3, 8))
    hv, ha, U = rng.uniform(-1, 1, (3, 8)), rng.uniform(-1, 1, (3, 8)), np.full((3, 8), np.nan)
    code = np.full(8, oracle.NOT_FOUND, np.int32)
    out = lpt.advance(x0, v0, hv, ha, U, code, 1.0, 0.1, False, BIG[0], BIG[1], BIG[2])
    for a, b in zip(out, (x0, v0, hv, ha)):
        assert np.array_equal(a, b)


def test_channel_velocity_properties():
    """Divergence-free (central differences), no-slip at the walls, bulk
    velocity 1 (Gauss-Legendre in y), periodic in x and z."""
    rng = np.random.default_rng(5)
    modes = W.channel_modes(rng)
    P = np.stack([rng.uniform(0, 6.28, 200), rng.uniform(-0.99, 0.99, 200),
                  rng.uniform(0, 3.14, 200)])
    h = 1e-5
    div = np.zeros(200)
    for d in range(3):
        e = np.zeros((3, 1))
        e[d] = h
        div += (W.channel_velocity(P + e, modes)[d] - W.channel_velocity(P - e, modes)[d]) / (2 * h)
    assert np.abs(div).max() < 1e-8
    for yw in (-1.0, 1.0):
        Q = P.copy()
        Q[1] = yw
        assert np.array_equal(W.channel_velocity(Q, modes), np.zeros_like(Q))
    yq, wq = np.polynomial.legendre.leggauss(20)
    for k in range(5):
        Q = np.stack([np.full(20, P[0, k]), yq, np.full(20, P[2, k])])
        assert abs(0.5 * np.dot(wq, W.channel_velocity(Q, modes)[0]) - 1.0) < 1e-12
    L = W.CHANNEL_L
    Q = P + np.array([[L[0]], [0.0], [L[2]]])
    assert np.abs(W.channel_velocity(Q, modes) - W.channel_velocity(P, modes)).max() < 1e-12


def test_lattice_sizes_follow_the_particle_ratio():
    n_comp = 31104 * 8 ** 3
    for ratio in (0.01, 0.10, 0.23, 0.50, 1.02, 5.03):
        n = W.lattice_n_y(ratio, n_comp)
        assert n - 1 < (0.5 * ratio * n_comp) ** (1 / 3) <= n
        assert 2 * n ** 3 >= ratio * n_comp
    pts = W.particle_lattice(3)
    assert pts.shape == (3, 2 * 27)
    assert np.all((pts[0] > 0) & (pts[0] < W.CHANNEL_L[0]) & (np.abs(pts[1]) < 1))


@pytest.fixture(scope="module")
def small_channel():
    wl = W.channel(n_el=(6, 4, 6), N=6, n_y=6)
    om = oracle.Mesh(wl["nodes"], 3, 3, 6)
    return wl, om


def test_oracle_loop_on_the_channel(small_channel):
    """Twenty steps through the oracle's Find and Interpolate: every particle
    stays in the box and is found, the interpolated fluid velocity matches
    the analytic field to the interpolation error of p = 5 elements, and the
    tracer limit (tau -> small) follows the fluid."""
    wl, om = small_channel
    st = lpt.run(om, wl["fields"], wl["pts"], wl["v0"], 20, 0.05, 0.01, wl["lo"], wl["hi"],
                 wl["periodic"])
    x = st["x"]
    assert np.all(st["find"]["code"] != oracle.NOT_FOUND)
    assert np.all((x[0] >= 0) & (x[0] <= W.CHANNEL_L[0]) & (np.abs(x[1]) <= 1.0))
    u_exact = W.channel_velocity(x, wl["modes"])
    u_int = om.eval(st["find"], wl["fields"])
    assert np.abs(u_int - u_exact).max() < 2e-3
    # with tau = 0.05 the particle velocity lags the fluid by about tau * Du/Dt
    assert np.abs(st["v"] - u_int).max() < 0.05


def test_oracle_loop_lost_particle(small_channel):
    """A particle outside the channel is NOT_FOUND and stays put."""
    wl, om = small_channel
    x0 = np.array([[1.0, 1.0], [0.2, 1.5], [1.0, 1.0]])
    v0 = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    st = lpt.run(om, wl["fields"], x0, v0, 3, 5.0, 0.01, wl["lo"], wl["hi"], wl["periodic"])
    assert st["find"]["code"][1] == oracle.NOT_FOUND
    assert np.array_equal(st["x"][:, 1], x0[:, 1]) and np.array_equal(st["v"][:, 1], v0[:, 1])
    assert st["find"]["code"][0] != oracle.NOT_FOUND
