"""Setup products of the library (fpts_setup: element AABB and OBB, local
map; Sections 3.1.1-3.1.3 and 4.1-4.2) against the oracle's, element by
element, through the C-ABI read-only views.

The two sides compute the boxes with different arithmetic (the library from
Gauss moments of the bases and tabulated basis bounds, the oracle with
Gauss-Legendre quadrature and direct sums), so box values agree to rounding:
1e-13 of the element's box extent.  The local map is discrete: N_L, the
element count of every cell and the element lists are identical."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _meshes():
    out = [("quad2d", W.quad2d(n_pts=10)),
           ("hex_p5", dict(W.hex16(n_in=10, n_out=0), nodes=W.curve_hex(W.box_mesh(3, 6, 6), 0.1),
                           N=6)),
           ("sphere", W.sphere(n_pts=100, ne=8, N=7)),
           ("line2d", W.line2d(level=1, per_elem=10)),
           ("line3d", W.line3d(n_elem=40, per_elem=10))]
    for k in range(4):
        out.append(("serving%d" % k, W.serving_mesh(k, scale=0.25)))
    return out


MESHES = _meshes()


@pytest.mark.parametrize("name,wl", MESHES, ids=[m[0] for m in MESHES])
def test_boxes_and_map_match_the_oracle(name, wl):
    from paper_2501_12349_amd import fpts
    nodes, N = wl["nodes"], wl["N"]
    D = nodes.shape[1]
    R = wl.get("ref_dim", D)
    if name.startswith("line"):
        R = 1
    gm = fpts.Mesh(nodes, N, dim=D, ref_dim=R)
    om = oracle.Mesh(nodes, D, R, N)
    la, lA, lc = gm.boxes()
    oa, oA, oc, ok = om.boxes()
    assert np.all(ok == 1)
    ext = (oa[:, :, 1] - oa[:, :, 0])                        # [nel][D]
    scale = np.maximum(ext, 1e-300)
    assert np.all(np.abs(la - oa) <= 1e-13 * scale[:, :, None]), \
        np.max(np.abs(la - oa) / scale[:, :, None])
    assert np.all(np.abs(lc - oc) <= 1e-13 * scale), np.max(np.abs(lc - oc) / scale)
    an = np.abs(oA).max(axis=(1, 2))
    assert np.all(np.abs(lA - oA) <= 1e-13 * an[:, None, None]), \
        np.max(np.abs(lA - oA) / an[:, None, None])
    lh, oh = gm.hash_info(), om.hash_info()
    assert lh["NL"] == oh["NL"] and lh["nnz"] == oh["nnz"]
    span = oh["hi"] - oh["lo"]
    for k in ("lo", "hi", "delta"):
        assert np.all(np.abs(lh[k] - oh[k]) <= 1e-13 * span), k
    loff, lel = gm.cells()
    ooff, oel = om.cells()
    assert np.array_equal(loff.astype(np.int64), ooff)
    assert np.array_equal(lel, oel)
    assert lh["max_cell"] == int(np.diff(ooff).max())
    print(name, "elements", nodes.shape[0], "NL", lh["NL"], "nnz", lh["nnz"],
          "max box diff %.2e" % np.max(np.abs(la - oa) / scale[:, :, None]))
