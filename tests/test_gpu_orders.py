"""Every supported order on the GPU against the oracle: curved hex and quad
meshes with N = 2 .. 10 nodes per direction (p = 1 .. 9), and the four
resident meshes of the serving workload (p = 3, 5, 7, 9 with 46^3, 36^3,
27^3, 22^3 hexes) at full size on sampled points, in both precisions."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_eval, compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(nodes, D, N, pts, fields, precision, idx=None, h=1.0):
    from paper_2501_12349_amd import fpts
    gm = fpts.Mesh(nodes, N)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    res = gm.find(tp, precision=precision)
    u = gm.eval(res, torch.from_numpy(fields).cuda())
    torch.cuda.synchronize()
    g, ug = to_np(res), u.cpu().numpy()
    if idx is not None:
        g = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in g.items()}
        ug = ug[:, idx]
        pts = np.ascontiguousarray(pts[:, idx])
    om = oracle.Mesh(nodes, D, D, N)
    orc = om.find(pts)
    rep = compare_find(om, pts, orc, g, h, max_ambiguous=1e-3)
    uo = om.eval(orc, fields)
    same = g["elem"] == orc["elem"]
    rep["eval_rel"] = compare_eval(uo[:, same], ug[:, same], orc["code"][same])
    rep["codes"] = np.bincount(g["code"], minlength=3).tolist()
    return rep


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", list(range(2, 11)))
def test_hex_every_order(N, precision):
    n = 4
    nodes = W.curve_hex(W.box_mesh(3, n, N), 0.1)
    rng = np.random.default_rng(300 + N)
    pts = np.concatenate([W.uniform_points(rng, 20000, 3, 0.0, 1.0),
                          W.shell_points(rng, 2000, 3)], axis=1)
    fields = W.nodal_field(nodes, W.poly_coeffs(3, N - 1, rng))[None]
    rep = _run(nodes, 3, N, pts, fields, precision, h=1.0 / n)
    print("hex N=%d %s" % (N, precision), rep, flush=True)
    assert rep["codes"][0] > 15000 and rep["codes"][1] > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", list(range(2, 11)))
def test_quad_every_order(N, precision):
    n = 6
    nodes = W.curve_quad2d(W.box_mesh(2, n, N), n)
    rng = np.random.default_rng(400 + N)
    pts = W.uniform_points(rng, 10000, 2, -0.05, 1.05)
    fields = W.nodal_field(nodes, W.poly_coeffs(2, N - 1, rng))[None]
    rep = _run(nodes, 2, N, pts, fields, precision, h=1.0 / n)
    print("quad N=%d %s" % (N, precision), rep, flush=True)


@pytest.fixture(scope="module", params=[0, 1, 2, 3])
def serving_mesh(request):
    return W.serving_mesh(request.param, scale=1.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_serving_meshes_full_size(serving_mesh, precision):
    wl = serving_mesh
    N, nodes = wl["N"], wl["nodes"]
    rng = np.random.default_rng(500 + N)
    n = 1 << 20
    pts = W.uniform_points(rng, n, 3, 0.0, 1.0)
    idx = np.sort(rng.choice(n, 8000, replace=False))
    print("serving mesh %s: %d elements, %d points, %d checked" % (
        wl["name"], nodes.shape[0], n, idx.size), flush=True)
    rep = _run(nodes, 3, N, pts, wl["fields"], precision, idx=idx, h=wl["h"])
    print(wl["name"], precision, rep, flush=True)
