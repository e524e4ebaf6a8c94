"""fpts_find_eval (Find and Interpolate in one call) gives exactly what
fpts_find followed by fpts_eval gives, on workloads that exercise every
branch: interior points settled by their primary candidate, points the
second search settles, BORDER points, NOT_FOUND points, surfaces, lines,
both precisions and fields of another order."""
import numpy as np
import pytest

from paper_2501_12349_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _same(wl, precision, ref_dim=None, field_nodes_1d=None, field=None):
    from paper_2501_12349_amd import fpts
    gm = fpts.Mesh(wl["nodes"], wl["N"], dim=wl["dim"], ref_dim=ref_dim or wl["ref_dim"])
    pts = torch.from_numpy(np.ascontiguousarray(wl["pts"])).cuda()
    f = torch.from_numpy(wl["fields"] if field is None else field).cuda()
    a = gm.find(pts, precision=precision)
    ua = gm.eval(a, f, field_nodes_1d=field_nodes_1d)
    b, ub = gm.find_eval(pts, f, precision=precision, field_nodes_1d=field_nodes_1d)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(torch.isnan(ua), torch.isnan(ub))
    assert torch.equal(torch.nan_to_num(ua), torch.nan_to_num(ub))
    codes = torch.bincount(b["code"].long(), minlength=3).tolist()
    print(wl["name"], precision, codes, flush=True)
    return codes


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex16(precision):
    codes = _same(W.hex16(n_in=200000, n_out=20000), precision)
    assert codes[0] > 0 and codes[2] > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_quad2d(precision):
    _same(W.quad2d(n_pts=50000), precision)


def test_sphere_surface():
    codes = _same(W.sphere(n_pts=100000, ne=8), "fp64")
    assert codes[1] > 0


def test_line2d():
    wl = W.line2d(level=2, per_elem=200)
    rng = np.random.default_rng(5)
    wl["pts"] = np.ascontiguousarray(np.concatenate(
        [wl["pts"], wl["pts"] + rng.uniform(-0.02, 0.02, wl["pts"].shape)], axis=1))
    _same(wl, "fp64", ref_dim=1)


def test_field_of_another_order():
    wl = W.hex16(n_in=50000, n_out=1000)
    rng = np.random.default_rng(6)
    field = rng.uniform(-1, 1, (2, wl["nodes"].shape[0], 4 ** 3))
    _same(wl, "fp64", field_nodes_1d=4, field=field)


@pytest.fixture(scope="module")
def hex48():
    return W.hex48()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex48_full_size(hex48, precision):
    _same(hex48, precision)


def test_ragged_sizes_and_arguments():
    """Sizes around the task size, n = 0, and argument errors."""
    from paper_2501_12349_amd import fpts
    wl = W.hex16(n_in=3000, n_out=100)
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    f = torch.from_numpy(wl["fields"]).cuda()
    allp = torch.from_numpy(np.ascontiguousarray(wl["pts"])).cuda()
    for n in (1, 63, 64, 65, 257):
        pts = allp[:, :n].contiguous()
        a = gm.find(pts)
        ua = gm.eval(a, f)
        b, ub = gm.find_eval(pts, f)
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), (n, k)
        assert torch.equal(torch.nan_to_num(ua), torch.nan_to_num(ub)), n
    empty = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    b, ub = gm.find_eval(empty, f)
    torch.cuda.synchronize()
    assert ub.shape == (1, 0)
    L = fpts.load_library()
    assert L.fpts_find_eval_workspace_size(None, 10) == 0
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    out = {k: v for k, v in gm.find(allp[:, :10].contiguous()).items()}
    u = torch.empty((1, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(fpts.FptsError):      # workspace too small
        gm.find_eval(allp[:, :10].contiguous(), f, out=out, u=u, ws=ws)
    with pytest.raises(fpts.FptsError):      # field order out of range
        gm.find_eval(allp[:, :10].contiguous(),
                     torch.zeros((1, gm.n_elem, 11 ** 3), dtype=torch.float64, device="cuda"),
                     field_nodes_1d=11)
    st = L.fpts_find_eval(gm._h, 10, None, None, None, None, None, 0, 1, wl["N"], None, None,
                          None, 0, None)
    assert st == -1       # null pointers
    torch.cuda.synchronize()
