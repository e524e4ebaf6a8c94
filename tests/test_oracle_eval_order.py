"""Pins of the oracle's interpolation with a field order N-tilde different
from the geometry's N (eq. eq_u_tensor with its own N-tilde): polynomial
reproduction in reference space, the degree limit, equality with the plain
interpolation when N-tilde = N, and a physical linear field on an affine
mesh through Find."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W


def _ref_poly_field(nel, R, Nf, rng):
    """Nodal values at the Nf GLL nodes (numpy's Legendre roots) of a random
    tensor polynomial of degree Nf-1 per reference variable, plus its
    coefficients [nel][Nf]*R."""
    z = W.gll_points(Nf)
    C = rng.uniform(-1, 1, (nel,) + (Nf,) * R)
    grids = np.meshgrid(*([z] * R), indexing="ij")     # grids[a][i0, i1, ...] = z[i_a]
    field = np.zeros((nel, Nf ** R))
    for e in range(nel):
        val = np.polynomial.polynomial.polyval(grids[0], C[e]) if R == 1 else \
            _tensor_polyval([g.ravel() for g in grids], C[e])
        # node (i, j, k) sits at i + Nf j + Nf^2 k: first reference index fastest
        field[e] = val.reshape((Nf,) * R).transpose(tuple(range(R))[::-1]).ravel()
    return field, C


def _tensor_polyval(X, C):
    R = len(X)
    out = np.zeros_like(X[0])
    for idx in np.ndindex(C.shape):
        t = np.full_like(X[0], C[idx])
        for a in range(R):
            t = t * X[a] ** idx[a]
        out += t
    return out


@pytest.mark.parametrize("R,N,Nf", [(3, 6, 3), (3, 4, 9), (3, 5, 2), (2, 5, 7), (2, 6, 4)])
def test_reference_polynomials_of_the_field_order_are_reproduced(R, N, Nf):
    rng = np.random.default_rng(10 * N + Nf)
    nodes = W.curve_hex(W.box_mesh(3, 3, N), 0.05) if R == 3 else \
        W.curve_quad2d(W.box_mesh(2, 4, N), 4)
    om = oracle.Mesh(nodes, R, R, N)
    field, C = _ref_poly_field(om.nel, R, Nf, rng)
    n = 400
    res = dict(code=np.zeros(n, np.int32), elem=rng.integers(0, om.nel, n).astype(np.int32),
               r=rng.uniform(-1, 1, (R, n)))
    u = om.eval(res, field[None], field_nodes_1d=Nf)[0]
    ref = np.array([_tensor_polyval([res["r"][a, p:p + 1] for a in range(R)],
                                    C[res["elem"][p]])[0] for p in range(n)])
    assert np.abs(u - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_degree_above_the_field_order_is_not_reproduced():
    """The field's own order is used: r^Nf in one variable is not in the
    space of Nf nodes per direction and must miss at random points."""
    N, Nf = 6, 3
    om = oracle.Mesh(W.box_mesh(3, 2, N), 3, 3, N)
    z = W.gll_points(Nf)
    Z = np.meshgrid(z, z, z, indexing="ij")[0]          # r at node (i, j, k)
    vals = (Z ** Nf).transpose(2, 1, 0).ravel()
    field = np.tile(vals, (om.nel, 1))
    rng = np.random.default_rng(2)
    n = 100
    res = dict(code=np.zeros(n, np.int32), elem=np.zeros(n, np.int32),
               r=rng.uniform(-1, 1, (3, n)))
    u = om.eval(res, field[None], field_nodes_1d=Nf)[0]
    assert np.abs(u - res["r"][0] ** Nf).max() > 1e-2


def test_field_order_equal_to_geometry_is_the_plain_interpolation():
    wl = W.hex16(n_in=3000, n_out=100)
    om = oracle.Mesh(wl["nodes"], 3, 3, wl["N"])
    res = om.find(wl["pts"])
    a = om.eval(res, wl["fields"])
    b = om.eval(res, wl["fields"], field_nodes_1d=wl["N"])
    assert np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("Nf", [2, 4, 8])
def test_linear_physical_field_on_affine_mesh(Nf):
    """On an affine mesh a linear physical field, sampled at the Nf GLL nodes
    of each element, interpolates exactly at found points."""
    n_el, N = 3, 5
    om = oracle.Mesh(W.box_mesh(3, n_el, N), 3, 3, N)
    t = 0.5 * (W.gll_points(Nf) + 1.0) / n_el
    a = np.arange(n_el) / n_el
    e = np.arange(om.nel)
    ea, eb, ec = e % n_el, (e // n_el) % n_el, e // (n_el * n_el)
    K, J, I = np.meshgrid(t, t, t, indexing="ij")       # node (i, j, k), i fastest
    X = a[ea][:, None] + I.ravel()[None]
    Y = a[eb][:, None] + J.ravel()[None]
    Z = a[ec][:, None] + K.ravel()[None]
    field = 0.3 + 1.5 * X - 0.7 * Y + 2.0 * Z
    rng = np.random.default_rng(4)
    pts = rng.uniform(0, 1, (3, 500))
    res = om.find(pts)
    assert np.all(res["code"] == oracle.INTERIOR)
    u = om.eval(res, field[None], field_nodes_1d=Nf)[0]
    ref = 0.3 + 1.5 * pts[0] - 0.7 * pts[1] + 2.0 * pts[2]
    assert np.abs(u - ref).max() < 1e-13


def test_field_order_out_of_range_is_refused():
    om = oracle.Mesh(W.box_mesh(2, 2, 3), 2, 2, 3)
    res = dict(code=np.zeros(1, np.int32), elem=np.zeros(1, np.int32), r=np.zeros((2, 1)))
    with pytest.raises(ValueError):
        om.eval(res, np.zeros((1, om.nel, 1)), field_nodes_1d=1)
