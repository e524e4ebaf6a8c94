"""Load generator for the request loop (fpts_serve.h).

Four resident hex meshes (p = 3, 5, 7, 9), a Poisson stream of find + eval
requests with log-uniform point counts, submitted at their arrival times;
latency = device completion - submission, reported as p50 / p99 beside the
throughput.  Points are generated on the device (uniform in the unit cube)
before the clock starts.
"""
import time

import numpy as np

from . import fpts
from . import workloads as W

REQ_DONE = 2      # FPTS_REQ_DONE of fpts_serve.h


def build_meshes(scale=1.0, seed=1003):
    """Set up the four resident meshes with their fields on the device."""
    import torch
    out = []
    for k in range(len(W.SERVING_MESHES)):
        wl = W.serving_mesh(k, seed=seed, scale=scale)
        m = fpts.Mesh(wl["nodes"], wl["N"])
        f = torch.from_numpy(wl["fields"]).cuda()
        out.append((wl, m, f))
    return out


def make_requests(n_req, seed=1004, lo=3.0, hi=6.0, n_mesh=4, dim=3):
    """Request sizes round(10^U(lo,hi)), mesh ids uniform, points uniform in
    [0,1]^3 on the device (torch generator seeded per request)."""
    import torch
    sizes, meshes, _ = W.serving_requests(n_req, seed=seed, lo=lo, hi=hi, n_mesh=n_mesh)
    g = torch.Generator(device="cuda")
    pts = []
    for i, n in enumerate(sizes):
        g.manual_seed(seed * 100003 + i)
        pts.append(torch.rand((dim, int(n)), generator=g, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return sizes, meshes, pts


def run(server, mesh_ids, sizes, meshes, pts, rate, precision="mixed", seed=7):
    """Submit the requests with exponential inter-arrival times of mean
    1/rate seconds (rate = inf: all at once), wait for all, and return the
    latency and throughput summary.  Output buffers are allocated before
    the first arrival."""
    import torch
    rng = np.random.default_rng(seed)
    n = len(sizes)
    gaps = np.zeros(n) if not np.isfinite(rate) else rng.exponential(1.0 / rate, size=n)
    arrive = np.cumsum(gaps)
    outs = [server.outputs(mesh_ids[meshes[i]], int(sizes[i])) for i in range(n)]
    torch.cuda.synchronize()
    rids = []
    t0 = time.perf_counter()
    for i in range(n):
        while time.perf_counter() - t0 < arrive[i]:
            pass
        rid, _ = server.submit(mesh_ids[meshes[i]], pts[i], precision=precision, out=outs[i])
        rids.append(rid)
    server.drain()
    lat, t_sub, t_done = [], [], []
    for rid in rids:
        st, ts, tst, td = server.poll(rid)
        assert st == REQ_DONE, (rid, st)
        lat.append(td - ts)
        t_sub.append(ts)
        t_done.append(td)
        server.release(rid)
    lat = np.array(lat) * 1e-3            # ms
    span = (max(t_done) - min(t_sub)) * 1e-6
    pts_total = float(np.sum(sizes))
    return dict(requests=n, points=int(pts_total), rate_req_s=float(rate),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), makespan_s=float(span),
                mpts_s=float(pts_total / span / 1e6))


def sweep(server, mesh_ids, sizes, meshes, pts, loads=(0.5, 0.8, 1.0, 1.2), precision="mixed"):
    """Saturation run (all requests at once) and Poisson runs at the given
    fractions of the saturated request rate."""
    run(server, mesh_ids, sizes[:8], meshes[:8], pts[:8], float("inf"), precision)   # warm-up
    sat = run(server, mesh_ids, sizes, meshes, pts, float("inf"), precision)
    rate_sat = sat["requests"] / sat["makespan_s"]
    out = []
    for k, ld in enumerate(loads):
        rep = run(server, mesh_ids, sizes, meshes, pts, ld * rate_sat, precision, seed=100 + k)
        rep["load"] = ld
        out.append(rep)
    st = server.stats()
    return dict(saturation=sat, saturated_rate_req_s=rate_sat, loads=out,
                batches=st["batches"], max_batch_requests=st["max_batch_requests"],
                max_in_flight=st["max_in_flight"], peak_bytes=st["peak_bytes"],
                budget_bytes=st["budget_bytes"])
