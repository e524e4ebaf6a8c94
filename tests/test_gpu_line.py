"""Line elements (D_r = 1) in 2D and 3D on the GPU against the oracle: the
find bars of the volume and surface cases (manifold codes, ambiguous
points checked for validity) and the interpolation bar."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_eval, compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fpts():
    from paper_2501_12349_amd import fpts
    return fpts


def _run(wl, pts, precision="fp64", idx=None):
    fpts = _fpts()
    gm = fpts.Mesh(wl["nodes"], wl["N"], dim=wl["dim"], ref_dim=1)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    res = gm.find(tp, precision=precision)
    u = gm.eval(res, torch.from_numpy(wl["fields"]).cuda())
    torch.cuda.synchronize()
    g = to_np(res)
    ug = u.cpu().numpy()
    if idx is not None:
        g = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in g.items()}
        ug = ug[:, idx]
        pts = np.ascontiguousarray(pts[:, idx])
    om = oracle.Mesh(wl["nodes"], wl["dim"], 1, wl["N"])
    orc = om.find(pts)
    rep = compare_find(om, pts, orc, g, wl["h"], surface=True)
    uo = om.eval(orc, wl["fields"])
    same = g["elem"] == orc["elem"]
    rep["eval_rel"] = compare_eval(uo[:, same], ug[:, same], orc["code"][same])
    rep["codes"] = np.bincount(g["code"], minlength=3).tolist()
    print(wl["name"], precision, rep, flush=True)
    return gm, g, rep


def _with_offsets(pts, rng, scale):
    off = pts + rng.uniform(-scale, scale, pts.shape)
    far = rng.uniform(-10, 10, (pts.shape[0], 200))
    return np.ascontiguousarray(np.concatenate([pts, off, far], axis=1))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_line2d(precision):
    wl = W.line2d(level=2, per_elem=100)
    pts = _with_offsets(wl["pts"], np.random.default_rng(81), 0.02)
    _, g, rep = _run(wl, pts, precision)
    assert rep["codes"][0] > 0 and rep["codes"][1] > 0 and rep["codes"][2] > 0


@pytest.mark.parametrize("N", [3, 5, 8])
def test_line3d_trefoil(N):
    wl = W.line3d(n_elem=48, per_elem=150, N=N)
    pts = _with_offsets(wl["pts"], np.random.default_rng(82 + N), 0.05)
    _run(wl, pts)


def test_line_ragged_and_empty():
    fpts = _fpts()
    wl = W.line3d(n_elem=20, per_elem=3)
    for n in (1, 63, 64, 65, 0):
        pts = np.ascontiguousarray(wl["pts"][:, :n])
        if n == 0:
            gm = fpts.Mesh(wl["nodes"], wl["N"], dim=3, ref_dim=1)
            gm.find(torch.zeros((3, 0), dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            continue
        _run(wl, pts)


@pytest.mark.parametrize("D", [2, 3])
def test_line_update_nodes_matches_fresh_setup(D):
    """Device setup of a moved line mesh equals a fresh host setup bit for
    bit, and both find the same results."""
    fpts = _fpts()
    wl = W.line2d(level=1, per_elem=50) if D == 2 else W.line3d(n_elem=40, per_elem=50)
    a = wl["nodes"]
    X = np.moveaxis(a, 1, 0)
    b = np.ascontiguousarray(a * 1.05 + 0.02 * np.sin(2.0 * X.sum(axis=0))[:, None, :])
    moved = fpts.Mesh(a, wl["N"], dim=D, ref_dim=1)
    moved.update_nodes(torch.from_numpy(b).cuda())
    fresh = fpts.Mesh(b, wl["N"], dim=D, ref_dim=1)
    for u, v in zip(moved.boxes(), fresh.boxes()):
        assert np.array_equal(u, v), np.abs(u - v).max()
    hu, hv = moved.hash_info(), fresh.hash_info()
    for k in hu:
        assert np.array_equal(np.asarray(hu[k]), np.asarray(hv[k])), k
    pts = torch.from_numpy(np.ascontiguousarray(wl["pts"] * 1.05)).cuda()
    ra, rb = to_np(moved.find(pts)), to_np(fresh.find(pts))
    torch.cuda.synchronize()
    for k in ra:
        assert np.array_equal(ra[k], rb[k], equal_nan=True), k


def test_line2d_full_size_sampled():
    """84 x 2^8 = 21 504 cubic line elements with 1000 points each (the size
    of the paper's largest surface-mesh case), 20 000 points checked."""
    wl = W.line2d()
    n = wl["pts"].shape[1]
    print("line2d full size: %d elements, %d points" % (wl["nodes"].shape[0], n), flush=True)
    idx = np.sort(np.random.default_rng(83).choice(n, 20000, replace=False))
    _run(wl, wl["pts"], idx=idx)
