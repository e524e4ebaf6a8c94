"""Pins of the oracle's basis, basis bounds and function bounds
(Section 2 and Section 3.1.1 of arXiv 2501.12349)."""
import os

import numpy as np
import pytest

import oracle
from tests import indep

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_gll_closed_forms():
    z, w = oracle.gll(2)
    assert np.allclose(z, [-1, 1], atol=0) and np.allclose(w, [1, 1], atol=1e-15)
    z, w = oracle.gll(3)
    assert np.allclose(z, [-1, 0, 1], atol=0)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    z, w = oracle.gll(4)
    a = 1 / np.sqrt(5)
    assert np.allclose(z, [-1, -a, a, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    z, w = oracle.gll(5)
    a = np.sqrt(3 / 7)
    assert np.allclose(z, [-1, -a, 0, a, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("N", range(2, 17))
def test_gll_against_numpy_roots(N):
    z, w = oracle.gll(N)
    zr = indep.gll_points(N)
    assert np.max(np.abs(z - zr)) < 1e-14
    assert abs(w.sum() - 2.0) < 1e-13
    # GLL quadrature is exact to degree 2N-3
    for k in range(0, 2 * N - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, z ** k) - exact) < 1e-13


@pytest.mark.parametrize("N", [2, 3, 5, 8, 10, 12])
def test_lagrange_identities_and_derivatives(N):
    z, _ = oracle.gll(N)
    for j in range(N):
        ph, _, _ = oracle.lagrange(N, z[j], 0)
        assert np.allclose(ph, np.eye(N)[j], atol=1e-14)
    rng = np.random.default_rng(0)
    for r in rng.uniform(-1, 1, 7):
        ph, d1, d2 = oracle.lagrange(N, r, 2)
        assert abs(ph.sum() - 1) < 1e-13                 # partition of unity
        assert abs(np.dot(z, ph) - r) < 1e-13            # reproduces r
        assert abs(d1.sum()) < 1e-11 and abs(np.dot(z, d1) - 1) < 1e-11
        assert abs(d2.sum()) < 1e-9
        assert np.allclose(ph, indep.lag(N, r, 0)[0], atol=1e-12)
        assert np.allclose(d1, indep.lag(N, r, 1)[0], atol=1e-10)
        assert np.allclose(d2, indep.lag(N, r, 2)[0], rtol=1e-9, atol=1e-8)


def _basis_violation(N, M, ph_dense, r_dense):
    lo, hi = oracle.basis_bounds(N, M)
    eta = oracle.cheb_points(M)
    worst = 0.0
    for i in range(N):
        L = np.interp(r_dense, eta, lo[i])
        H = np.interp(r_dense, eta, hi[i])
        worst = min(worst, (ph_dense[:, i] - L).min(), (H - ph_dense[:, i]).min())
    return worst


def _load_mmin():
    rows = []
    with open(os.path.join(GOLD, "basis_bound_mmin.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, b = line.split()
                rows.append((int(a), int(b)))
    return rows


@pytest.mark.parametrize("N,Mmin", _load_mmin())
def test_basis_bound_minimal_M_matches_footnote(N, Mmin):
    """The smallest M whose piecewise-linear bounds contain every basis on a
    dense grid is the paper's M_min (footnote in Section 3.1.1).  This pins
    the reading of the garbled basis-bound formula."""
    r = np.linspace(-1, 1, 20001)
    ph = indep.lag(N, r, 0)
    assert _basis_violation(N, Mmin, ph, r) > -1e-12
    for M in range(2, Mmin):
        assert _basis_violation(N, M, ph, r) < -1e-12, (N, M)


@pytest.mark.parametrize("N", range(2, 17))
def test_basis_bounds_hold_at_M_2N(N):
    r = np.linspace(-1, 1, 8001)
    ph = indep.lag(N, r, 0)
    assert _basis_violation(N, 2 * N, ph, r) > -1e-12


def test_chebyshev_points():
    for M in (2, 5, 8, 16):
        eta = oracle.cheb_points(M)
        j = np.arange(1, M + 1)
        assert np.allclose(eta, -np.cos((j - 1) * np.pi / (M - 1)), atol=1e-15)


def _cubic_from_nodes(u):
    z = indep.gll_points(4)
    c = np.polyfit(z, u, 3)
    crit = [x.real for x in np.roots(np.polyder(c)) if abs(x.imag) < 1e-14 and -1 <= x.real <= 1]
    cand = np.array([-1.0, 1.0] + crit)
    v = np.polyval(c, cand)
    return v.min(), v.max()


def test_worked_example_1d_bounds_contain_and_tighten():
    with open(os.path.join(GOLD, "bound_example_1d.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    u = np.array([float(x) for x in rows[0]])
    Ms = [int(x) for x in rows[1]]
    umin, umax = _cubic_from_nodes(u)
    widths = []
    for M in Ms:
        lo, hi = oracle.bound_1d(u, M)
        assert lo <= umin + 1e-14 and hi >= umax - 1e-14
        widths.append(hi - lo)
    assert widths[0] > widths[1] > widths[2]


@pytest.mark.parametrize("N", [2, 3, 4, 6, 8, 10])
def test_bound_1d_containment_and_linear_exactness(N):
    rng = np.random.default_rng(N)
    z = indep.gll_points(N)
    r = np.linspace(-1, 1, 4001)
    ph = indep.lag(N, r, 0)
    for _ in range(20):
        u = rng.normal(size=N) * rng.uniform(0.1, 10) + rng.uniform(-50, 50)
        lo, hi = oracle.bound_1d(u, 2 * N)
        vals = ph @ u
        assert lo <= vals.min() + 1e-12 * max(1, abs(vals).max())
        assert hi >= vals.max() - 1e-12 * max(1, abs(vals).max())
    a, b = 3.7, -1.3                               # linear: exact after compaction
    lo, hi = oracle.bound_1d(a + b * z, 2 * N)
    assert abs(lo - (a - abs(b))) < 1e-13 and abs(hi - (a + abs(b))) < 1e-13


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_bound_2d_containment_and_bilinear_exactness(N):
    rng = np.random.default_rng(10 + N)
    z = indep.gll_points(N)
    r = np.linspace(-1, 1, 301)
    ph = indep.lag(N, r, 0)
    for _ in range(10):
        u = rng.normal(size=(N, N)) + rng.uniform(-20, 20)      # u[j][i]
        lo, hi = oracle.bound_2d(u, 2 * N)
        vals = ph @ u @ ph.T        # [s][r]: sum_ij u[j][i] phi_j(s) phi_i(r)
        vals = np.einsum("ai,ji,bj->ab", ph, u, ph)
        assert lo <= vals.min() + 1e-11 and hi >= vals.max() - 1e-11
    ZI, ZJ = np.meshgrid(z, z, indexing="xy")                   # [j][i]
    u = 1.5 + 2.0 * ZI - 0.5 * ZJ + 0.25 * ZI * ZJ
    lo, hi = oracle.bound_2d(u, 2 * N)
    corners = [1.5 + 2 * a - 0.5 * b + 0.25 * a * b for a in (-1, 1) for b in (-1, 1)]
    assert abs(lo - min(corners)) < 1e-13 and abs(hi - max(corners)) < 1e-13
