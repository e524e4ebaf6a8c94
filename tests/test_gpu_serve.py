"""The request loop: results are bit-identical alone and in the mix,
admission respects the memory budget, oversize requests are refused."""
import numpy as np
import pytest

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
