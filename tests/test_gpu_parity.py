"""GPU parity of find and eval against the oracle, through the C-ABI."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests import indep
from tests.parity import compare_eval, compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fpts():
    from paper_2501_12349_amd import fpts
    return fpts


def _run(wl, pts, precision="fp64", fields=True):
    fpts = _fpts()
    gm = fpts.Mesh(wl["nodes"], wl["N"], dim=wl["dim"], ref_dim=wl["ref_dim"])
    tp = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    res = gm.find(tp, precision=precision)
    out = None
    if fields and wl.get("fields") is not None:
        out = gm.eval(res, torch.from_numpy(wl["fields"]).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    return gm, to_np(res), out


def _check(wl, pts, precision="fp64", surface=False, max_ambiguous=0.01):
    om = oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])
    orc = om.find(pts)
    gm, gpu, u = _run(wl, pts, precision)
    rep = compare_find(om, pts, orc, gpu, wl["h"], surface=surface,
                       max_ambiguous=max_ambiguous)
    if u is not None:
        uo = om.eval(orc, wl["fields"])
        # compare eval on the GPU's own coordinates where they agree with the
        # oracle's element
        same = gpu["elem"] == orc["elem"]
        rep["eval_rel"] = compare_eval(uo[:, same], u[:, same], orc["code"][same])
    print(wl["name"], precision, rep)
    return rep, gm


def test_quad2d_full_fp64():
    wl = W.quad2d()
    _check(wl, wl["pts"])


def test_quad2d_full_mixed():
    wl = W.quad2d()
    _check(wl, wl["pts"], "mixed")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex16_subset(precision):
    wl = W.hex16(n_in=200000, n_out=4000)
    _check(wl, wl["pts"], precision)


def test_sphere_subset_fp64():
    wl = W.sphere(n_pts=100000, ne=32, N=7)
    _check(wl, wl["pts"], "fp64", surface=True)


def test_sphere_subset_mixed():
    wl = W.sphere(n_pts=100000, ne=32, N=7)
    _check(wl, wl["pts"], "mixed", surface=True)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4097])
def test_ragged_sizes(n):
    wl = W.quad2d(n_pts=n, seed=2000 + n)
    _check(wl, wl["pts"])


def test_empty_call():
    fpts = _fpts()
    wl = W.quad2d(n_pts=10)
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    res = gm.find(torch.zeros((2, 0), dtype=torch.float64, device="cuda"))
    assert res["code"].numel() == 0


def test_invalid_and_far_points():
    wl = W.quad2d(n_pts=10)
    pts = np.array([[np.nan, np.inf, -np.inf, 5.0, -3.0, 0.5, 1e300, 0.0, 1.0, 0.5],
                    [0.5, 0.5, 0.5, 0.5, 0.5, np.nan, 0.5, 0.0, 1.0, 0.5]])
    om = oracle.Mesh(wl["nodes"], 2, 2, wl["N"])
    orc = om.find(pts)
    gm, gpu, _ = _run(wl, pts, fields=False)
    assert np.all(gpu["code"][:7] == oracle.NOT_FOUND)
    assert np.all(gpu["elem"][:7] == -1)
    compare_find(om, pts, orc, gpu, wl["h"], max_ambiguous=1.0)


def test_all_points_in_one_element_many_chunks():
    """Thousands of pairs of one element: many 64-pair tasks of the same
    element, plus a ragged last task."""
    wl = W.quad2d(n_pts=10)
    rng = np.random.default_rng(5)
    e = np.full(5000 + 17, 27)
    rt = rng.uniform(-0.999, 0.999, (2, e.size))
    pts = indep.map_points(wl["nodes"], wl["N"], 2, e, rt)
    gm, gpu, _ = _run(wl, pts, fields=False)
    assert np.all(gpu["elem"] == 27) and np.all(gpu["code"] == oracle.INTERIOR)
    assert np.abs(gpu["r"] - rt).max() < 1e-10


def test_points_at_nodes_and_corners():
    wl = W.hex16(n_in=10, n_out=0)
    nodes = wl["nodes"]
    sel = nodes[::97]                          # every 97th element
    pts = np.ascontiguousarray(np.moveaxis(sel, 1, 0).reshape(3, -1))
    # every point sits on a node: corners and faces are ambiguous by design
    _check(dict(wl, fields=None), pts, max_ambiguous=1.0)


def test_recovery_hex_gpu():
    wl = W.hex16(n_in=10, n_out=0)
    rng = np.random.default_rng(9)
    n = 20000
    e = rng.integers(0, wl["nodes"].shape[0], n)
    rt = rng.uniform(-0.999, 0.999, (3, n))
    pts = indep.map_points(wl["nodes"], wl["N"], 3, e, rt)
    for prec in ("fp64", "mixed"):
        gm, gpu, _ = _run(dict(wl, fields=None), pts, prec, fields=False)
        assert np.array_equal(gpu["elem"], e.astype(np.int32))
        assert np.all(gpu["code"] == oracle.INTERIOR)
        assert np.abs(gpu["r"] - rt).max() < 1e-10, prec


def test_deterministic_bitwise():
    wl = W.hex16(n_in=50000, n_out=1000)
    a = _run(wl, wl["pts"])
    b = _run(wl, wl["pts"])
    for k in ("code", "elem", "r", "dist"):
        assert np.array_equal(a[1][k], b[1][k], equal_nan=True), k
    assert np.array_equal(a[2], b[2], equal_nan=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_second_search_overflow(precision):
    """Boxes expanded fivefold overlap so much that the points outside the
    domain have far more candidates than the second search's slots hold
    (one per point): the overflowing points go through the one-point-per-
    wavefront path, and every result still meets the parity bars."""
    wl = W.quad2d(n_pts=6000, seed=2077)
    rng = np.random.default_rng(2078)
    pts = rng.uniform(-0.15, 1.15, (2, 6000))
    fpts = _fpts()
    gm = fpts.Mesh(wl["nodes"], wl["N"], bbox_tol=4.0)
    om = oracle.Mesh(wl["nodes"], 2, 2, wl["N"], bbox_tol=4.0)
    orc = om.find(pts)
    res = gm.find(torch.from_numpy(pts).cuda(), precision=precision)
    st = gm.find_stats()
    torch.cuda.synchronize()
    gpu = to_np(res)
    rep = compare_find(om, pts, orc, gpu, wl["h"])
    print(precision, rep, "overflow points", st["overflow_points"])
    assert st["overflow_points"] > 100
    assert (orc["code"] == oracle.BORDER).sum() > 1000


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_face_pairs_beyond_the_saved_states(precision):
    """Points just outside the cube (offsets up to 2e-3, inside the boxes of
    the boundary elements, whose map is the identity on the cube's faces):
    the primary pair of nearly every point iterates to the boundary face,
    needs second derivatives there and leaves the primary kernel's slots.
    The park records keep the iteration state of the first n/8 + 1024 such
    pairs only, so the face kernel resumes some pairs from their state and
    re-evaluates the others, within the same waves.  Results as the
    oracle's (BORDER at the offset's distance)."""
    wl = W.hex16(n_in=0, n_out=0)
    rng = np.random.default_rng(2024)
    n = 60000
    pts = rng.uniform(0.0, 1.0, size=(3, n))
    axis = rng.integers(0, 3, size=n)
    side = rng.integers(0, 2, size=n)
    off = rng.uniform(1e-5, 2e-3, size=n)
    pts[axis, np.arange(n)] = np.where(side == 1, 1.0 + off, -off)
    rep, gm = _check(wl, pts, precision)
    st = gm.find_stats()
    cap = min(n, n // 8 + 1024)
    print("parked", st["parked_pairs"], "saved states", cap)
    assert st["parked_pairs"] > cap
