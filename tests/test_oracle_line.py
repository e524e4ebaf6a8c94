"""Pins of the oracle for line elements (D_r = 1) in 2D and 3D: boxes of
straight segments in closed form (Rodrigues' rotation included), containment
for curved elements, closest points of explicit polynomial curves, brute
force over all elements and dense sampling, interpolation of polynomials."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W

TOL = 0.1     # box expansion


def _segment_nodes(p, q, N):
    t = 0.5 * (W.gll_points(N) + 1.0)
    p, q = np.asarray(p, float), np.asarray(q, float)
    return (p[:, None] + t[None, :] * (q - p)[:, None])[None]     # [1][D][N]


@pytest.mark.parametrize("D", [2, 3])
def test_straight_segment_boxes_closed_form(D):
    """AABB: the end points' box, zero (or tiny) extents raised to tol times
    the largest other extent, then expanded by tol in total.  OBB: x~ = Q(x -
    x_c) with Q taking the unit tangent u to e1; along u the box is the
    segment, across it tol L; so A (Acute{J}^{-1}) has first row u / h_t and
    the others orthogonal to u with norm 1 / h_n."""
    rng = np.random.default_rng(D)
    dirs = [np.eye(D)[0], -np.eye(D)[0], np.eye(D)[1]] + \
        [v / np.linalg.norm(v) for v in rng.standard_normal((6, D))]
    for u in dirs:
        L = 0.7
        p = rng.uniform(-1, 1, D)
        q = p + L * u
        om = oracle.Mesh(_segment_nodes(p, q, 4), D, 1, 4, bbox_tol=TOL)
        aabb, A, c, ok = om.boxes()
        lo, hi = np.minimum(p, q), np.maximum(p, q)
        ext = hi - lo
        for d in range(D):
            ref = max(ext[k] for k in range(D) if k != d)
            e = max(ext[d], TOL * ref)
            mid = 0.5 * (lo[d] + hi[d]) if ext[d] < TOL * ref else None
            if mid is not None:
                lo_d, hi_d = mid - 0.5 * e, mid + 0.5 * e
            else:
                lo_d, hi_d = lo[d], hi[d]
            assert abs(aabb[0, d, 0] - (lo_d - 0.5 * TOL * e)) < 1e-14
            assert abs(aabb[0, d, 1] - (hi_d + 0.5 * TOL * e)) < 1e-14
        assert ok[0] == 1
        h_t = 0.5 * L * (1 + TOL)
        h_n = 0.5 * TOL * L * (1 + TOL)
        assert np.allclose(A[0, 0], u / h_t, atol=1e-12)
        for k in range(1, D):
            assert abs(np.dot(A[0, k], u)) < 1e-12
            assert abs(np.linalg.norm(A[0, k]) - 1 / h_n) < 1e-9 / h_n
        for a in range(1, D):
            for b in range(a + 1, D):
                assert abs(np.dot(A[0, a], A[0, b])) < 1e-9 / h_n ** 2
        assert np.allclose(c[0], 0.5 * (p + q), atol=1e-14)


def _curve_poly(D, N, rng, scale=0.3):
    """Random polynomial curve x(r) = sum_k a_k r^k of degree N-1 (mild
    curvature) and its nodes at numpy's GLL points."""
    a = rng.uniform(-scale, scale, (D, N))
    a[:, 1] = rng.uniform(0.5, 1.0, D) * np.sign(rng.uniform(-1, 1, D))
    z = W.gll_points(N)
    x = np.stack([np.polynomial.polynomial.polyval(z, a[d]) for d in range(D)])
    return a, x


@pytest.mark.parametrize("D", [2, 3])
def test_curved_boxes_contain_the_curve(D):
    rng = np.random.default_rng(10 + D)
    nodes = np.stack([_curve_poly(D, 6, rng)[1] for _ in range(20)])
    om = oracle.Mesh(nodes, D, 1, 6)
    aabb, A, c, ok = om.boxes()
    rs = np.linspace(-1, 1, 801)
    for e in range(20):
        X = np.stack([om.map(e, [r])[0] for r in rs])        # [801][D]
        assert np.all(X >= aabb[e, :, 0] - 1e-14) and np.all(X <= aabb[e, :, 1] + 1e-14)
        if ok[e]:
            y = (X - c[e]) @ A[e].T
            assert np.abs(y).max() <= 1.0 + 1e-12


@pytest.mark.parametrize("D", [2, 3])
def test_closest_point_of_polynomial_curve(D):
    """Points at x(r0) + delta n with n normal to x'(r0): the closest point
    is r0 at distance |delta| while delta is below the radius of curvature;
    codes follow the manifold rule (INTERIOR iff delta^2 < 1e-10)."""
    rng = np.random.default_rng(20 + D)
    N = 5
    for trial in range(12):
        a, x = _curve_poly(D, N, rng, scale=0.1)
        om = oracle.Mesh(x[None], D, 1, N)
        r0 = rng.uniform(-0.9, 0.9)
        t = np.array([np.polynomial.polynomial.polyval(r0, np.polynomial.polynomial.polyder(a[d]))
                      for d in range(D)])
        v = rng.standard_normal(D)
        nrm = v - np.dot(v, t) / np.dot(t, t) * t
        nrm /= np.linalg.norm(nrm)
        x0 = np.array([np.polynomial.polynomial.polyval(r0, a[d]) for d in range(D)])
        for delta, code in ((0.0, oracle.INTERIOR), (3e-6, oracle.INTERIOR),
                            (2e-3, oracle.BORDER)):
            p = (x0 + delta * nrm)[:, None]
            res = om.find(p)
            assert res["code"][0] == code, (trial, delta, res["code"][0])
            assert abs(res["r"][0, 0] - r0) < 1e-10, (trial, delta, res["r"][0, 0], r0)
            assert abs(res["dist"][0] - delta) < 1e-12


@pytest.mark.parametrize("D", [2, 3])
def test_find_matches_brute_force_and_dense_sampling(D):
    """Points on the curves: the local map gives what a search of every
    element gives.  Points up to 0.05 off the curves: the same as a search
    of every element whose boxes hold the point (off-curve points are only
    judged against such elements), and the distance is the smallest over a
    dense sampling of those elements."""
    wl = W.line2d(level=1, per_elem=20) if D == 2 else W.line3d(n_elem=24, per_elem=20)
    om = oracle.Mesh(wl["nodes"], D, 1, wl["N"])
    rng = np.random.default_rng(30 + D)
    pts = np.ascontiguousarray(wl["pts"][:, ::7])
    a = om.find(pts, mode=0)
    b = om.find(pts, mode=2)
    assert np.all(a["code"] != oracle.NOT_FOUND)
    assert np.array_equal(a["code"], b["code"])
    assert np.allclose(a["dist"], b["dist"], atol=1e-12)
    near = np.ascontiguousarray(pts + rng.uniform(-0.005, 0.005, pts.shape))
    a = om.find(near, mode=0)
    b = om.find(near, mode=1)
    assert np.array_equal(a["code"], b["code"]) and np.array_equal(a["elem"], b["elem"])
    assert np.allclose(a["dist"], b["dist"], atol=1e-12, equal_nan=True)
    aabb, A, c, ok = om.boxes()
    rs = np.linspace(-1, 1, 2001)
    found = np.nonzero(a["code"] != oracle.NOT_FOUND)[0]
    assert found.size > 0.3 * near.shape[1]
    for p in found[::5]:
        x = near[:, p]
        best = np.inf
        for e in range(om.nel):
            if not (np.all(x >= aabb[e, :, 0]) and np.all(x <= aabb[e, :, 1])):
                continue
            if ok[e] and np.abs(A[e] @ (x - c[e])).max() > 1.0:
                continue
            X = np.stack([om.map(e, [r])[0] for r in rs])
            k = int(np.argmin(np.linalg.norm(X - x, axis=1)))
            fine = np.clip(np.linspace(rs[k] - 1e-3, rs[k] + 1e-3, 2001), -1, 1)
            X = np.stack([om.map(e, [r])[0] for r in fine])
            best = min(best, np.min(np.linalg.norm(X - x, axis=1)))
        assert a["dist"][p] <= best + 1e-12
        assert best - a["dist"][p] < 1e-9


def test_far_points_are_not_found():
    wl = W.line3d(n_elem=16, per_elem=5)
    om = oracle.Mesh(wl["nodes"], 3, 1, wl["N"])
    res = om.find(np.array([[50.0, -40.0], [0.0, 3.0], [0.0, 100.0]]))
    assert np.all(res["code"] == oracle.NOT_FOUND) and np.all(res["elem"] == -1)


@pytest.mark.parametrize("Nf", [3, 5, 7])
def test_line_interpolation_reproduces_polynomials(Nf):
    rng = np.random.default_rng(Nf)
    wl = W.line3d(n_elem=10, per_elem=5)
    om = oracle.Mesh(wl["nodes"], 3, 1, wl["N"])
    c = rng.uniform(-1, 1, (om.nel, Nf))
    z = W.gll_points(Nf)
    field = np.stack([np.polynomial.polynomial.polyval(z, c[e]) for e in range(om.nel)])
    n = 300
    res = dict(code=np.zeros(n, np.int32), elem=rng.integers(0, om.nel, n).astype(np.int32),
               r=rng.uniform(-1, 1, (1, n)))
    u = om.eval(res, field[None], field_nodes_1d=Nf)[0]
    ref = np.array([np.polynomial.polynomial.polyval(res["r"][0, p], c[res["elem"][p]])
                    for p in range(n)])
    assert np.abs(u - ref).max() < 1e-12
