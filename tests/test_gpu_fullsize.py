"""Full-size workloads in the launch configuration bench.py times.

The GPU finds and interpolates every point of the workload with the same
Mesh.find / Mesh.eval calls as bench.py; the oracle checks all of them where
it finishes in seconds (16^3 hexes, 1.02M points; the cubed sphere, 2^22
points) and a seeded random sample of 10^6 points otherwise (48^3 hexes with
2^24 points), point by point, to the same bars as the small parity tests.
The oracle's results are computed once per workload and shared by both
precisions."""
import sys

import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_eval, compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_all(wl, precision):
    from paper_2501_12349_amd import fpts
    gm = fpts.Mesh(wl["nodes"], wl["N"], dim=wl["dim"], ref_dim=wl["ref_dim"])
    tp = torch.from_numpy(np.ascontiguousarray(wl["pts"])).cuda()
    res = gm.find(tp, precision=precision)
    u = None
    if wl.get("fields") is not None:
        u = gm.eval(res, torch.from_numpy(wl["fields"]).cuda())
    torch.cuda.synchronize()
    out = to_np(res)
    return out, (u.cpu().numpy() if u is not None else None)


def _subset(gpu, u, idx):
    g = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in gpu.items()}
    return g, (u[:, idx] if u is not None else None)


_ORACLE = {}


def _oracle_results(wl, om, idx):
    """Oracle find (and eval) of the sampled points, once per workload."""
    key = (wl["name"], len(idx), int(idx[0]), int(idx[-1]))
    if key not in _ORACLE:
        pts = np.ascontiguousarray(wl["pts"][:, idx])
        orc = om.find(pts)
        uo = om.eval(orc, wl["fields"]) if wl.get("fields") is not None else None
        _ORACLE[key] = (pts, orc, uo)
    return _ORACLE[key]


def _check_sample(wl, om, precision, idx, surface=False):
    print("full-size %s %s: %d points on the GPU, %d checked" % (
        wl["name"], precision, wl["pts"].shape[1], len(idx)), flush=True)
    sys.stdout.flush()
    gpu, u = _gpu_all(wl, precision)
    g, us = _subset(gpu, u, idx)
    pts, orc, uo = _oracle_results(wl, om, idx)
    rep = compare_find(om, pts, orc, g, wl["h"], surface=surface, max_ambiguous=1e-3)
    if us is not None:
        same = g["elem"] == orc["elem"]
        rep["eval_rel"] = compare_eval(uo[:, same], us[:, same], orc["code"][same])
    # every point of the full run is accounted for
    assert np.all(np.isin(gpu["code"], [oracle.INTERIOR, oracle.BORDER, oracle.NOT_FOUND]))
    print(wl["name"], precision, rep, flush=True)
    return rep


@pytest.fixture(scope="module")
def hex16():
    wl = W.hex16()
    return wl, oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])


@pytest.fixture(scope="module")
def hex48():
    wl = W.hex48()
    return wl, oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])


@pytest.fixture(scope="module")
def sphere():
    wl = W.sphere()
    return wl, oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex16_every_point(hex16, precision):
    wl, om = hex16
    rep = _check_sample(wl, om, precision, np.arange(wl["pts"].shape[1]))
    assert rep["n"] == 1020000


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex48_sampled(hex48, precision):
    wl, om = hex48
    n = wl["pts"].shape[1]
    idx = np.sort(np.random.default_rng(77).choice(n, size=1000000, replace=False))
    # plus the first and last points of the batch
    idx = np.unique(np.concatenate([idx, [0, 1, n - 2, n - 1]]))
    _check_sample(wl, om, precision, idx)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sphere_every_point(sphere, precision):
    wl, om = sphere
    n = wl["pts"].shape[1]
    rep = _check_sample(wl, om, precision, np.arange(n), surface=True)
    assert rep["n"] == 1 << 22


def test_hex48_1e8_points_one_call(hex48):
    """10^8 points (the largest point count of the paper's Find runs) found
    and interpolated on the 48^3 mesh in one fpts_find_eval call; a seeded
    sample of 20 000 points checked against the oracle."""
    from paper_2501_12349_amd import fpts
    wl, om = hex48
    n = 100_000_000
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    g = torch.Generator(device="cuda")
    g.manual_seed(1_000_003)
    pts = torch.rand((3, n), generator=g, dtype=torch.float64, device="cuda")
    fields = torch.from_numpy(wl["fields"]).cuda()
    wsb = gm.find_eval_workspace_bytes(n)
    print("1e8 points: workspace %.2f GB (%.0f B per point)" % (wsb / 1e9, wsb / n), flush=True)
    res, u = gm.find_eval(pts, fields)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(79).choice(n, 20000, replace=False))
    ti = torch.from_numpy(idx).cuda()
    sp = np.ascontiguousarray(pts[:, ti].cpu().numpy())
    gsub = {k: (v[:, ti] if v.dim() == 2 else v[ti]).cpu().numpy() for k, v in res.items()}
    us = u[:, ti].cpu().numpy()
    orc = om.find(sp)
    rep = compare_find(om, sp, orc, gsub, wl["h"], max_ambiguous=1e-3)
    uo = om.eval(orc, wl["fields"])
    same = gsub["elem"] == orc["elem"]
    rep["eval_rel"] = compare_eval(uo[:, same], us[:, same], orc["code"][same])
    codes = torch.bincount(res["code"].long(), minlength=3).cpu().tolist()
    print("1e8 points:", rep, "codes", codes, flush=True)
    assert codes[0] == n
    assert wsb / n < 400
