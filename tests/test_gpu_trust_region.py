"""The trust-region Newton iteration on the GPU, pass by pass (Section
3.2.1), against the oracle, through the C-ABI.

The constructed elements of the oracle's trust-region pins (a rejected step,
a non-SPD face Hessian, radius growth and clipping, second derivatives on a
face, the closest-node start and its tie-break, the equal-distance selection
tie) are searched on the GPU: the result must equal the oracle's and, in
FP64, the number of Newton passes (accepted or not, the converging one
included) must equal the oracle's exactly.  On single curved elements the
pass counts of many interior points are compared the same way: a different
radius rule, start or Hessian would change them even where the converged
result agrees."""
import numpy as np
import pytest

import oracle
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_find, to_np
from tests.test_oracle_trust_region import line_nodes, quad_nodes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fpts():
    from paper_2501_12349_amd import fpts
    return fpts


CASES = [
    # (name, nodes, ref_dim, point, bbox_tol): the cases of the oracle pins;
    # the points off the line elements lie far outside the default boxes, so
    # those cases widen the boxes on both sides
    ("reject_quarter_growth", quad_nodes(lambda r, s: r - 0.45 * r * r, lambda r, s: s), 2,
     (0.325, 0.0), 0.1),
    ("poor_but_accepted", quad_nodes(lambda r, s: r - 0.35 * r * r, lambda r, s: s), 2,
     (0.4, 0.0), 0.1),
    ("keep_radius_then_clip", line_nodes(lambda r: r, lambda r: -r * r), 1, (-1.75, 1.0), 8.0),
    ("face_second_derivatives", quad_nodes(lambda r, s: r + 0.3 * s * s, lambda r, s: s), 2,
     (1.2, 0.3), 0.1),
    ("closest_node_tie", line_nodes(lambda r: r, lambda r: 0.5 * r * r), 1, (0.0, 2.0), 8.0),
    ("closest_node_right", line_nodes(lambda r: r, lambda r: 0.5 * r * r), 1, (0.1, 2.0), 8.0),
]


def _gpu_find(nodes, R, pts, precision, bbox_tol=0.1):
    fpts = _fpts()
    D = nodes.shape[1]
    N = int(round(nodes.shape[2] ** (1.0 / R)))
    gm = fpts.Mesh(nodes, N, dim=D, ref_dim=R, bbox_tol=bbox_tol)
    tp = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
    res = gm.find(tp, precision=precision)
    st = gm.find_stats()
    torch.cuda.synchronize()
    return to_np(res), st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_constructed_case(case, precision):
    name, nodes, R, x, tol = case
    D = nodes.shape[1]
    N = int(round(nodes.shape[2] ** (1.0 / R)))
    pts = np.array(x, dtype=np.float64).reshape(D, 1)
    om = oracle.Mesh(nodes, D, R, N, bbox_tol=tol)
    orc = om.find(pts)
    assert orc["code"][0] != oracle.NOT_FOUND and orc["iters"][0] > 0
    gpu, st = _gpu_find(nodes, R, pts, precision, tol)
    print(name, precision, gpu, orc["iters"], st["passes"])
    assert gpu["code"][0] == orc["code"][0] and gpu["elem"][0] == orc["elem"][0]
    assert np.abs(gpu["r"][:, 0] - orc["r"][:, 0]).max() <= 1e-13
    assert abs(gpu["dist"][0] - orc["dist"][0]) <= 1e-13
    if precision == "fp64":
        assert st["passes"] == int(orc["iters"][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_equal_distance_tie_goes_to_lowest_id(precision):
    z = np.array([-1.0, 1.0])
    nodes = np.zeros((2, 2, 4))
    for e in range(2):
        for j in range(2):
            for i in range(2):
                nodes[e, 0, i + 2 * j] = e + 0.5 * (z[i] + 1)
                nodes[e, 1, i + 2 * j] = 0.5 * (z[j] + 1)
    pts = np.array([[1.0], [-0.04]])
    for order, r0 in ((nodes, 1.0), (nodes[::-1].copy(), -1.0)):
        gpu, _ = _gpu_find(order, 2, pts, precision)
        assert gpu["code"][0] == oracle.BORDER
        assert gpu["elem"][0] == 0
        assert abs(gpu["dist"][0] - 0.04) <= 1e-16
        assert gpu["r"][0, 0] == r0 and gpu["r"][1, 0] == -1.0


def _curved_element(D, N, seed):
    """One element on [0,1]^D with curved faces: x_c += 0.08 sin(a.x + b)."""
    rng = np.random.default_rng(seed)
    nodes = W.box_mesh(D, 1, N)
    X = nodes.copy()
    for c in range(D):
        a = rng.uniform(-2.0, 2.0, D)
        b = rng.uniform(0, 2 * np.pi)
        X[:, c] += 0.08 * np.sin(np.einsum("d,edn->en", a, nodes) + b)
    return X


@pytest.mark.parametrize("D,N", [(2, 5), (3, 4), (3, 6), (3, 8)])
def test_pass_counts_single_curved_element(D, N):
    nodes = _curved_element(D, N, 77 + D * 10 + N)
    rng = np.random.default_rng(5 + N)
    pts = rng.uniform(-0.1, 1.1, (D, 4000))
    om = oracle.Mesh(nodes, D, D, N)
    orc = om.find(pts)
    # interior points away from the faces: zero-residual problems whose
    # trust-region decisions are far from rounding
    keep = (orc["code"] == oracle.INTERIOR) & (orc["margin"][0] > 1e-3)
    assert keep.sum() > 1000
    sub = np.ascontiguousarray(pts[:, keep])
    osub = {k: (v[..., keep] if v.ndim > 1 else v[keep]) for k, v in orc.items()}
    gpu, st = _gpu_find(nodes, D, sub, "fp64")
    compare_find(om, sub, osub, gpu, 1.0)
    print(D, N, st["passes"], int(osub["iters"].sum()), st["pairs"])
    assert st["pairs"] == sub.shape[1]
    assert st["passes"] == int(osub["iters"].sum())
    # all points, both precisions: results only
    for precision in ("fp64", "mixed"):
        gpu, _ = _gpu_find(nodes, D, pts, precision)
        compare_find(om, pts, orc, gpu, 1.0)


@pytest.mark.parametrize("D,N", [(2, 5), (3, 8)])
def test_fp32_phase_evaluates_starts_at_their_nodes(D, N):
    """Mixed mode: every FP32 pair starts at its nearest node, and that first
    evaluation is taken from the element's nodes and differentiation matrix
    rows instead of a sweep; the results still match the oracle."""
    nodes = _curved_element(D, N, 91 + D * 10 + N)
    rng = np.random.default_rng(17 + N)
    pts = rng.uniform(-0.1, 1.1, (D, 3000))
    om = oracle.Mesh(nodes, D, D, N)
    orc = om.find(pts)
    gpu, st = _gpu_find(nodes, D, pts, "mixed")
    compare_find(om, pts, orc, gpu, 1.0)
    fpts = _fpts()
    gm = fpts.Mesh(nodes, N, dim=D, ref_dim=D)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    gm.find(tp, precision="mixed")
    primary = gm.find_stats(newton_pass=1)
    print(D, N, primary)
    assert primary["evals_fp32_node"] == primary["pairs"] > 0
    # the swept evaluations fit the sweeps' slots
    swept = primary["evals_fp32"] - primary["evals_fp32_node"]
    assert 0 < swept <= 16 * primary["sweeps_fp32"]
