"""Interpolation of fields whose order differs from the geometry's
(fpts_eval_order) against the oracle: each side finds the points on its
own, the interpolants are compared where both chose the same element, to
the interpolation bar (relative 1e-10)."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_eval, compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(nodes, D, N, pts, Nf, seed, nf=2):
    from paper_2501_12349_amd import fpts
    rng = np.random.default_rng(seed)
    nel = nodes.shape[0]
    field = rng.uniform(-1, 1, (nf, nel, Nf ** D))
    gm = fpts.Mesh(nodes, N)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    res = gm.find(tp)
    u = gm.eval(res, torch.from_numpy(field).cuda(), field_nodes_1d=Nf)
    torch.cuda.synchronize()
    g = to_np(res)
    ug = u.cpu().numpy()
    om = oracle.Mesh(nodes, D, D, N)
    orc = om.find(pts)
    compare_find(om, pts, orc, g, 1.0)
    uo = om.eval(orc, field, field_nodes_1d=Nf)
    same = g["elem"] == orc["elem"]
    err = compare_eval(uo[:, same], ug[:, same], orc["code"][same])
    print("D=%d N=%d Nf=%d: %d points, %d same element, max rel %.2e" % (
        D, N, Nf, pts.shape[1], int(same.sum()), err), flush=True)
    return gm, res, field


@pytest.mark.parametrize("Nf", [2, 3, 8, 10])
def test_hex_field_orders(Nf):
    N = 6
    nodes = W.curve_hex(W.box_mesh(3, 5, N), 0.08)
    pts = W.uniform_points(np.random.default_rng(40 + Nf), 20000, 3, -0.02, 1.02)
    _case(nodes, 3, N, pts, Nf, 50 + Nf)


@pytest.mark.parametrize("Nf", [3, 7])
def test_quad_field_orders(Nf):
    wl = W.quad2d(n_pts=8000)
    _case(wl["nodes"], 2, wl["N"], wl["pts"], Nf, 60 + Nf)


def test_same_order_is_fpts_eval_and_bad_order_is_refused():
    from paper_2501_12349_amd import fpts
    N = 5
    nodes = W.curve_hex(W.box_mesh(3, 4, N), 0.05)
    pts = W.uniform_points(np.random.default_rng(7), 5000, 3, 0.0, 1.0)
    gm, res, field = _case(nodes, 3, N, pts, N, 70)
    f = torch.from_numpy(field).cuda()
    a = gm.eval(res, f)
    b = gm.eval(res, f, field_nodes_1d=N)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(fpts.FptsError):
        gm.eval(res, torch.zeros((1, gm.n_elem, 11 ** 3), dtype=torch.float64, device="cuda"),
                field_nodes_1d=11)
