"""The request loop: results are bit-identical alone and in the mix, every
served result meets the oracle parity bars, admission respects the memory
budget, oversize requests are refused."""
import numpy as np
import pytest

import oracle
from tests.parity import compare_eval, compare_find

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def meshes():
    from paper_2501_12349_amd import serve
    return serve.build_meshes(scale=0.25)


def _server(meshes, budget, streams):
    from paper_2501_12349_amd import fpts
    s = fpts.Server(budget, n_streams=streams, max_batch_points=1 << 21)
    ids = [s.add_mesh(m, f) for _, m, f in meshes]
    return s, ids


def _reqs(n, seed):
    from paper_2501_12349_amd import serve
    return serve.make_requests(n, seed=seed, lo=2.5, hi=5.0)


def _snap(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_identical_alone_and_in_the_mix(meshes, precision):
    sizes, mids, pts = _reqs(40, seed=11)
    # alone: one stream, one request at a time
    s1, ids1 = _server(meshes, 4 << 30, 1)
    alone = []
    for i in range(len(sizes)):
        rid, out = s1.submit(ids1[mids[i]], pts[i], precision)
        s1.wait(rid)
        alone.append(_snap(out))
    s1.close()
    # in the mix: everything at once, four streams, batching allowed
    s4, ids4 = _server(meshes, 4 << 30, 4)
    outs = []
    for i in range(len(sizes)):
        rid, out = s4.submit(ids4[mids[i]], pts[i], precision)
        outs.append(out)
    s4.drain()
    st = s4.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0
    assert st["max_batch_requests"] > 1          # requests were concatenated
    for i in range(len(sizes)):
        mix = _snap(outs[i])
        for k in ("code", "elem", "r", "dist", "u"):
            assert np.array_equal(mix[k], alone[i][k], equal_nan=True), (i, k)
    s4.close()
    # and equal to a direct find + eval of the same points
    wl, m, f = meshes[mids[0]]
    res = m.find(pts[0], precision=precision)
    u = m.eval(res, f)
    torch.cuda.synchronize()
    assert np.array_equal(res["elem"].cpu().numpy(), alone[0]["elem"])
    assert np.array_equal(u.cpu().numpy(), alone[0]["u"][:u.shape[0]], equal_nan=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_results_match_the_oracle(meshes, precision):
    """Requests of every mesh served in the mix (four streams, batching),
    each request's outputs checked against the oracle point by point."""
    sizes, mids, pts = _reqs(24, seed=21)
    s, ids = _server(meshes, 4 << 30, 4)
    outs = []
    for i in range(len(sizes)):
        rid, out = s.submit(ids[mids[i]], pts[i], precision)
        outs.append(out)
    s.drain()
    assert s.stats()["completed"] == len(sizes)
    s.close()
    oms = {}
    for i in range(len(sizes)):
        wl, _, _ = meshes[mids[i]]
        if mids[i] not in oms:
            oms[mids[i]] = oracle.Mesh(wl["nodes"], 3, 3, wl["N"])
        om = oms[mids[i]]
        p = pts[i].cpu().numpy()
        g = _snap(outs[i])
        orc = om.find(p)
        rep = compare_find(om, p, orc, g, wl["h"])
        uo = om.eval(orc, wl["fields"])
        same = g["elem"] == orc["elem"]
        rep["eval_rel"] = compare_eval(uo[:, same], g["u"][:uo.shape[0], same],
                                       orc["code"][same])
        print("request", i, "mesh", int(mids[i]), precision, rep, flush=True)
    assert len(set(int(m) for m in mids)) == 4


def test_points_written_on_the_callers_stream():
    """A non-contiguous input (transposed [n][3] tensor) is copied on the
    caller's stream inside submit, and the points of a second request are
    produced by a kernel queued just before it: both requests wait for that
    work and match direct calls."""
    from paper_2501_12349_amd import serve
    meshes = serve.build_meshes(scale=0.25)
    s, ids = _server(meshes, 1 << 30, 2)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    raw = torch.rand((200000, 3), generator=g, dtype=torch.float64, device="cuda")
    pts_t = raw.t()                                  # non-contiguous view
    assert not pts_t.is_contiguous()
    rid1, out1 = s.submit(ids[1], pts_t, "fp64")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        torch.cuda._sleep(2000000)                   # keep the producer busy
        pts2 = raw.t().contiguous() * 0.5 + 0.25
        rid2, out2 = s.submit(ids[2], pts2, "fp64", stream=side)
    s.drain()
    torch.cuda.synchronize()
    for (wl, m, f), p, out in ((meshes[1], pts_t.contiguous(), out1),
                               (meshes[2], raw.t().contiguous() * 0.5 + 0.25, out2)):
        res = m.find(p)
        u = m.eval(res, f)
        torch.cuda.synchronize()
        for k in ("code", "elem", "r", "dist"):
            assert torch.equal(res[k], out[k]), k
        assert torch.equal(torch.nan_to_num(u), torch.nan_to_num(out["u"][:u.shape[0]]))
    s.close()


def test_admission_is_memory_gated(meshes):
    from paper_2501_12349_amd import fpts
    sizes, mids, pts = _reqs(24, seed=12)
    wl, m, f = meshes[0]
    need = max(m.find_workspace_bytes(int(n)) for n in sizes)
    budget = int(need * 2.5)
    s, ids = _server(meshes, budget, 4)
    for i in range(len(sizes)):
        s.submit(ids[mids[i]], pts[i], "fp64")
    s.drain()
    st = s.stats()
    assert st["completed"] == len(sizes)
    assert st["peak_bytes"] <= budget
    # a request that can never fit is refused at submission
    big = torch.rand((3, 2_000_000), dtype=torch.float64, device="cuda")
    with pytest.raises(fpts.FptsError):
        s.submit(ids[0], big, "fp64")
    s.close()


def test_load_generator_reports_latency(meshes):
    from paper_2501_12349_amd import serve
    sizes, mids, pts = _reqs(30, seed=13)
    s, ids = _server(meshes, 4 << 30, 4)
    rep = serve.run(s, ids, sizes, mids, pts, rate=2000.0, precision="mixed")
    assert rep["requests"] == 30 and rep["p50_ms"] <= rep["p99_ms"] and rep["mpts_s"] > 0
    print(rep)
    s.close()
