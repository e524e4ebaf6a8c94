"""Pins of the oracle's trust-region Newton iteration (Section 3.2.1: the
Newton step of eqs. eq_newton / eq_newton_jacobian / eq_newton_hessian, the
trust-region radius update, the rule that second derivatives enter only after
the first pass and only on a face or edge, the closest-node start) and of the
selection tie-break (Section 3.2), one pass at a time.

Each case is a constructed element whose map is reproduced exactly by its
nodes (a quadratic map with N = 3 nodes -1, 0, 1), so every quantity of a
pass -- residual, gradient, Hessian, the step before and after clipping, the
predicted and the actual decrease -- is a rational number.  The expected
iterates below are derived by hand, pass by pass; the Fraction arithmetic
only checks each stated number and which branch of the radius update the
ratio decr / pred selects.  The oracle is run with max_iter = 1, 2, 3, ...
and its iterate after each pass is compared with the derivation.

Notation (the oracle's objective): f(r) = ||x* - x(r)||^2, g = G^T dx,
H = G^T G (pass 0, or off the boundary) or G^T G - sum_i dx_i d2x_i
(passes l > 0 on a face), pred = 2 g.dr - dr.H.dr, decr = f(r) - f(r + dr);
decr >= 0.9 pred doubles the radius alpha, decr >= 0.01 pred keeps it,
anything else rejects the step and divides alpha by 4.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

Z3 = (-1.0, 0.0, 1.0)          # GLL nodes for N = 3


def quad_nodes(fx, fy):
    """One quad, N = 3, node (i, j) at index i + 3 j with x = fx(z_i, z_j),
    y = fy(z_i, z_j)."""
    nodes = np.zeros((1, 2, 9))
    for j in range(3):
        for i in range(3):
            nodes[0, 0, i + 3 * j] = fx(Z3[i], Z3[j])
            nodes[0, 1, i + 3 * j] = fy(Z3[i], Z3[j])
    return nodes


def line_nodes(fx, fy):
    """One line element in 2D, N = 3."""
    nodes = np.zeros((1, 2, 3))
    for i in range(3):
        nodes[0, 0, i] = fx(Z3[i])
        nodes[0, 1, i] = fy(Z3[i])
    return nodes


def run(nodes, R, x, k):
    """Oracle Newton on element 0 with at most k passes."""
    m = oracle.Mesh(nodes, 2, R, 3, max_iter=k)
    return m.newton(0, np.asarray(x, dtype=np.float64))


def ratio(f_old, f_new, g, dr, H):
    """decr / pred of a one-coordinate step."""
    pred = 2 * g * dr - H * dr * dr
    return (f_old - f_new) / pred, pred


# --------------------------------------------------------------------------
# Case A: a rejected step, alpha / 4, a non-SPD Hessian on the face, growth.
#
# x(r, s) = (r - 9/20 r^2, s): x_r = 1 - 9/10 r in [1/10, 19/10], so the
# element is valid but strongly stretched near r = 1.  x* = (13/40, 0).  The
# s-coordinate starts at its exact value (s = 0 is a node) and never moves,
# so every pass reduces to the scalar p(r) = r - 9/20 r^2 and e = 13/40 - p(r).

def test_case_a_reject_quarter_growth():
    X = Fr(13, 40)
    p = lambda r: r - Fr(9, 20) * r * r
    dp = lambda r: 1 - Fr(9, 10) * r
    d2p = Fr(-9, 10)
    # start: the nodes' x are p(-1) = -29/20, p(0) = 0, p(1) = 11/20; x* is
    # nearest to p(1) (distance 9/40 < 13/40), so r0 = 1.
    assert abs(X - p(1)) < abs(X - p(0)) < abs(X - p(-1))
    r0 = Fr(1)
    e0 = X - p(r0)
    assert e0 == Fr(-9, 40)
    # pass 0 (beta = 0): the Gauss-Newton step e / p' = -9/4 is clipped to
    # -alpha = -1, trial r = 0.  f rises from 81/1600 to 169/1600: rejected,
    # alpha = 1/4, r stays 1.
    assert e0 / dp(r0) == Fr(-9, 4)
    assert (X - p(0)) ** 2 > e0 ** 2
    # pass 1: l > 0 on the face r = 1, so beta = 1: H = p'^2 - e p'' =
    # 1/100 - 81/400 < 0 is not SPD, the oracle falls back to G^T G = 1/100;
    # the step -9/4 is clipped to -1/4, r = 3/4.
    H1 = dp(r0) ** 2 - e0 * d2p
    assert H1 < 0
    r1 = r0 - Fr(1, 4)
    rho1, pred1 = ratio(e0 ** 2, (X - p(r1)) ** 2, dp(r0) * e0, -Fr(1, 4), dp(r0) ** 2)
    assert pred1 > 0 and rho1 >= Fr(9, 10)        # accepted, alpha = 1/2
    # pass 2 (beta = 0: off the face): Newton step from 3/4 is -55/104,
    # beyond alpha = 1/2, clipped to -1/2: r = 1/4.
    e1 = X - p(r1)
    step2 = e1 / dp(r1)
    assert step2 == Fr(-55, 104) and step2 < -Fr(1, 2)
    r2 = r1 - Fr(1, 2)
    rho2, pred2 = ratio(e1 ** 2, (X - p(r2)) ** 2, dp(r1) * e1, -Fr(1, 2), dp(r1) ** 2)
    assert Fr(1, 100) <= rho2 < Fr(9, 10)          # accepted, alpha stays 1/2
    # pass 3 on: plain Newton steps for p(r) = X (below alpha), converging to
    # the root of 9/20 r^2 - r + 13/40 = 0 in [-1, 1].
    e2 = X - p(r2)
    r3 = r2 + e2 / dp(r2)
    assert abs(e2 / dp(r2)) < Fr(1, 2)
    rstar = (1 - np.sqrt(1 - 4 * 0.45 * 0.325)) / 0.9
    expect = [r0, r1, r2, r3]
    for k, re in enumerate(expect, start=1):
        r, _, it, conv = run(quad_nodes(lambda r, s: r - 0.45 * r * r, lambda r, s: s), 2,
                             [0.325, 0.0], k)
        assert it == k and not conv
        assert abs(r[0] - float(re)) <= 1e-15, (k, r, float(re))
        assert r[1] == 0.0
    r, d, it, conv = run(quad_nodes(lambda r, s: r - 0.45 * r * r, lambda r, s: s), 2,
                         [0.325, 0.0], 50)
    assert conv and abs(r[0] - rstar) <= 1e-14 and d <= 1e-15
    # steps after pass 3 shrink quadratically: 1.2e-2, 1.0e-4, 7.5e-9, then
    # one below 1e-10 stops the iteration: 8 passes in all
    steps, rr = [], r3
    while True:
        s_ = (X - p(rr)) / dp(rr)
        steps.append(s_)
        rr += s_
        if abs(s_) < Fr(1, 10 ** 10):
            break
    assert it == 4 + len(steps), (it, [float(s) for s in steps])


# --------------------------------------------------------------------------
# Case B: an accepted step with decr / pred between 0.01 and 0.3.
#
# x(r, s) = (r - 7/20 r^2, s), x* = (2/5, 0).

def test_case_b_poor_but_accepted_step():
    X = Fr(2, 5)
    p = lambda r: r - Fr(7, 20) * r * r
    dp = lambda r: 1 - Fr(7, 10) * r
    assert abs(X - p(1)) < abs(X - p(0))            # r0 = 1 (13/20 vs 0)
    e0 = X - p(1)
    step = e0 / dp(1)
    assert step == Fr(-5, 6)                        # inside alpha = 1: not clipped
    r1 = 1 + step
    rho, pred = ratio(e0 ** 2, (X - p(r1)) ** 2, dp(1) * e0, step, dp(1) ** 2)
    assert pred == e0 ** 2                          # full Gauss-Newton step
    assert Fr(1, 100) <= rho < Fr(3, 10)            # accepted (rho ~ 0.055)
    nodes = quad_nodes(lambda r, s: r - 0.35 * r * r, lambda r, s: s)
    r, _, it, _ = run(nodes, 2, [0.4, 0.0], 1)
    assert abs(r[0] - 1 / 6) <= 1e-15 and it == 1
    # the next pass starts from r1 with alpha = 1 and takes the full Newton
    # step (1/6 -> 1/6 + e1 / p'(1/6))
    e1 = X - p(r1)
    r2 = r1 + e1 / dp(r1)
    assert abs(e1 / dp(r1)) < 1
    r, _, it, _ = run(nodes, 2, [0.4, 0.0], 2)
    assert abs(r[0] - float(r2)) <= 1e-15


# --------------------------------------------------------------------------
# Case C: decr / pred between 0.5 and 0.9 keeps alpha, and the next step is
# clipped by it.  A parabolic line element x(r) = (r, -r^2) in 2D and the
# point x* = (-7/4, 1) off the curve: the closest point is r* = -1/2, the
# only real root of d/dr ||x* - x(r)||^2 / 2 = 2 r^3 + 3 r + 7/4, with
# distance 5 sqrt(2) / 4.

def test_case_c_keep_radius_then_clip():
    X, Y = Fr(-7, 4), Fr(1)
    x = lambda r: (r, -r * r)
    G = lambda r: (Fr(1), -2 * r)
    f = lambda r: (X - x(r)[0]) ** 2 + (Y - x(r)[1]) ** 2
    g = lambda r: G(r)[0] * (X - x(r)[0]) + G(r)[1] * (Y - x(r)[1])
    GG = lambda r: G(r)[0] ** 2 + G(r)[1] ** 2
    # start: node distances^2 are 73/16 (r = -1), 65/16 (r = 0), 137/16 (r = 1)
    assert f(0) < f(-1) < f(1)
    # pass 0 at r = 0: step g / G^T G = -7/4, clipped to -1; f(-1) > f(0):
    # rejected, alpha = 1/4
    assert g(0) / GG(0) == Fr(-7, 4)
    assert f(-1) > f(0)
    # pass 1: the same step clipped to -1/4; ratio in [0.5, 0.9): accepted,
    # alpha stays 1/4
    rho1, _ = ratio(f(0), f(Fr(-1, 4)), g(0), Fr(-1, 4), GG(0))
    assert Fr(1, 2) <= rho1 < Fr(9, 10)
    # pass 2 at r = -1/4: the step g / G^T G = -31/40 is clipped to -1/4 (a
    # radius of 1/2 would give r = -3/4); ratio >= 0.01: r = -1/2
    r1 = Fr(-1, 4)
    assert g(r1) / GG(r1) == Fr(-31, 40)
    rho2, _ = ratio(f(r1), f(Fr(-1, 2)), g(r1), Fr(-1, 4), GG(r1))
    assert Fr(1, 100) <= rho2
    # pass 3 at r = -1/2: g = 0 exactly, step 0 < 1e-10: converged
    assert g(Fr(-1, 2)) == 0
    nodes = line_nodes(lambda r: r, lambda r: -r * r)
    for k, re in enumerate([0.0, -0.25, -0.5], start=1):
        r, _, it, conv = run(nodes, 1, [-1.75, 1.0], k)
        assert r[0] == re and it == k and not conv, (k, r)
    r, d, it, conv = run(nodes, 1, [-1.75, 1.0], 50)
    assert r[0] == -0.5 and conv and it == 4
    assert abs(d - 1.25 * np.sqrt(2.0)) <= 1e-15


# --------------------------------------------------------------------------
# Case D: second derivatives on a face.  x(r, s) = (r + 3/10 s^2, s): the
# face r = 1 is the parabola x = 1 + 3/10 s^2.  x* = (6/5, 3/10) lies outside
# it; the closest point of the element is on that face at s* = 1/3 (the root
# of 9/50 s^3 + 22/25 s - 3/10), with distance sqrt(26) / 30.

def test_case_d_face_second_derivatives():
    X, Y = Fr(6, 5), Fr(3, 10)
    c = Fr(3, 10)
    ex = lambda s: X - (1 + c * s * s)              # on the face r = 1
    ey = lambda s: Y - s
    # start: node (1, 0) (distance^2 13/100) is the nearest; on it g_r =
    # e_x = 1/5 > 0 points out of the element, so r is held at 1.
    # pass 0 (l = 0: beta = 0 although r is on a face): H_ss = (G^T G)_ss = 1,
    # g_s = e_y = 3/10, step 3/10 -> s = 3/10, ratio >= 0.9 (alpha = 2)
    s1 = Fr(3, 10)
    rho, _ = ratio(ex(0) ** 2 + ey(0) ** 2, ex(s1) ** 2 + ey(s1) ** 2, ey(0), s1, 1)
    assert rho >= Fr(9, 10)
    # with beta = 1 already at l = 0, H_ss would be 1 - e_x * 2c = 22/25 and
    # the step 15/44 instead
    # pass 1 (l = 1, on the face: beta = 1): x_s = 2 c s, g_s = x_s e_x +
    # e_y, H_ss = x_s^2 + 1 - e_x * 2c (the G^T G value alone would be
    # x_s^2 + 1)
    xs = 2 * c * s1
    g1 = xs * ex(s1) + ey(s1)
    H1 = xs * xs + 1 - ex(s1) * 2 * c
    s2 = s1 + g1 / H1
    assert H1 != xs * xs + 1
    # pass 2: the same Newton step from s2
    xs2 = 2 * c * s2
    s3 = s2 + (xs2 * ex(s2) + ey(s2)) / (xs2 * xs2 + 1 - ex(s2) * 2 * c)
    nodes = quad_nodes(lambda r, s: r + 0.3 * s * s, lambda r, s: s)
    for k, se in enumerate([s1, s2, s3], start=1):
        r, _, it, _ = run(nodes, 2, [1.2, 0.3], k)
        assert r[0] == 1.0 and abs(r[1] - float(se)) <= 1e-15, (k, r, float(se))
    # passes 2 on are Newton's method for the scalar stationarity equation
    # (exact Hessian: quadratic convergence to s* = 1/3)
    r, d, it, conv = run(nodes, 2, [1.2, 0.3], 50)
    assert conv and r[0] == 1.0 and abs(r[1] - 1 / 3) <= 1e-15
    assert abs(d - np.sqrt(26.0) / 30) <= 1e-15
    assert it == 5


# --------------------------------------------------------------------------
# Case E: the start node decides a BORDER result.  Line element x(r) =
# (r, r^2 / 2), x* = (0, 2): the two end nodes (-1, 1/2) and (1, 1/2) are
# equally near (distance^2 13/4 < 4 to the middle node), and each end is a
# local minimum of the distance over [-1, 1] (the free minimisers r = +-sqrt 2
# lie outside).  The lowest node index wins the tie, so the result is r = -1;
# the middle node, a stationary point of the distance, would stay put.

def test_case_e_closest_node_start_and_its_tie_break():
    nodes = line_nodes(lambda r: r, lambda r: 0.5 * r * r)
    r, d, it, conv = run(nodes, 1, [0.0, 2.0], 50)
    assert r[0] == -1.0 and conv and it == 1
    assert d == np.sqrt(3.25)
    # shifted a little to the right, the end node r = 1 is nearest
    r, d, it, conv = run(nodes, 1, [0.1, 2.0], 50)
    assert r[0] == 1.0 and abs(d - np.sqrt(0.81 + 2.25)) <= 1e-15


# --------------------------------------------------------------------------
# Case F: selection among BORDER candidates with equal distance (Section
# 3.2: the lowest element id).  Two affine unit squares share the edge
# x = 1; the point (1, -1/25) lies below their common corner, inside both
# expanded boxes, and is at distance 1/25 from both (the corner itself,
# r = (1, -1) in element 0 and (-1, -1) in element 1).

def test_case_f_equal_distance_tie_goes_to_lowest_id():
    z = np.array([-1.0, 1.0])
    nodes = np.zeros((2, 2, 4))
    for e in range(2):
        for j in range(2):
            for i in range(2):
                nodes[e, 0, i + 2 * j] = e + 0.5 * (z[i] + 1)
                nodes[e, 1, i + 2 * j] = 0.5 * (z[j] + 1)
    pts = np.array([[1.0], [-0.04]])
    for order in (nodes, nodes[::-1].copy()):
        m = oracle.Mesh(order, 2, 2, 2)
        res = m.find(pts)
        assert res["code"][0] == oracle.BORDER
        assert res["elem"][0] == 0
        assert res["dist"][0] == 0.04
        assert res["ncand"][0] == 2
    # element 0 of the first ordering is the left square
    m = oracle.Mesh(nodes, 2, 2, 2)
    res = m.find(pts)
    assert res["r"][0, 0] == 1.0 and res["r"][1, 0] == -1.0
    m = oracle.Mesh(nodes[::-1].copy(), 2, 2, 2)
    res = m.find(pts)
    assert res["r"][0, 0] == -1.0 and res["r"][1, 0] == -1.0
