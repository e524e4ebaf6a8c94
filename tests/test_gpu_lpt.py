"""Particle transport through fpts_lpt_step against the oracle's loop
(oracle.lpt) on the same seeded channel, particles and fluid velocity.

Both sides start from the same positions and velocities and take the same
number of steps; the integration arithmetic is the same operation by
operation, so the two trajectories differ only through the interpolated
velocity.  Bar: the Find results of the final positions meet the find
parity bar, and x, v and the history agree to 1e-9, the bound that the
interpolation bar (relative 1e-10 of |u| <= 2) gives over these runs:
|dv| <= K dt / tau * 2e-10 and |dx| <= K dt |dv| with K dt / tau <= 4."""
import numpy as np
import pytest

import oracle
from oracle import lpt as olpt
from paper_2501_12349_amd import workloads as W
from tests.parity import compare_find, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-9


def _fpts():
    from paper_2501_12349_amd import fpts
    return fpts


def _extra_particles(wl):
    """Particles thrown at the walls, across the periodic ends, and one
    outside the channel (NOT_FOUND, frozen)."""
    L = W.CHANNEL_L
    D = wl["dim"]
    x = [[0.3, 1.0, 2.0, L[0] - 0.02, 0.01, 1.0],
         [0.97, -0.985, 0.5, 0.0, -0.3, 1.5],
         [1.0, 2.0, L[2] - 0.03, 1.0, 0.02, 1.0]][:D]
    v = [[0.2, 0.0, 0.5, 1.5, -1.2, 0.0],
         [1.5, -1.0, 0.0, 0.1, 0.0, 0.0],
         [0.0, 0.3, 1.4, 0.0, -1.0, 0.0]][:D]
    return np.array(x), np.array(v)


def _run_both(wl, steps, tau, dt, precision="fp64", hint=False):
    fpts = _fpts()
    xe, ve = _extra_particles(wl)
    x0 = np.ascontiguousarray(np.concatenate([wl["pts"], xe], axis=1))
    v0 = np.ascontiguousarray(np.concatenate([wl["v0"], ve], axis=1))
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    field = torch.from_numpy(wl["fields"]).cuda()
    P = fpts.Particles(torch.from_numpy(x0).cuda(), torch.from_numpy(v0).cuda(), tau, dt,
                       wl["lo"], wl["hi"], wl["periodic"], hint=hint).start(gm, precision)
    for k in range(steps):
        gm.lpt_step(P, field, first=(k == 0), precision=precision)
    torch.cuda.synchronize()
    g = dict(x=P.x.cpu().numpy(), v=P.v.cpu().numpy(), hist=P.hist.cpu().numpy(),
             find=to_np(P.find))
    om = oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])
    o = olpt.run(om, wl["fields"], x0, v0, steps, tau, dt, wl["lo"], wl["hi"], wl["periodic"])
    return om, g, o


def _compare(wl, om, g, o):
    rep = dict(dx=float(np.abs(g["x"] - o["x"]).max()), dv=float(np.abs(g["v"] - o["v"]).max()),
               dhv=float(np.abs(g["hist"][0] - o["hist_v"]).max()),
               dha=float(np.abs(g["hist"][1] - o["hist_a"]).max()))
    print(wl["name"], rep, flush=True)
    for k, val in rep.items():
        assert val <= TOL, (k, val)
    # Find of the final positions: the GPU's positions through the oracle
    orc = om.find(g["x"])
    rep["find"] = compare_find(om, g["x"], orc, g["find"], wl["h"])
    # the wall-bound particles stayed inside, the outside one is frozen
    assert np.all(np.abs(g["x"][1, :-1]) <= 1.0)
    assert g["find"]["code"][-1] == oracle.NOT_FOUND
    assert np.all(g["find"]["code"][:-1] != oracle.NOT_FOUND)
    return rep


@pytest.mark.parametrize("hint", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tau", [0.05, 5.0])
def test_channel3d_matches_oracle_loop(precision, tau, hint):
    """The hinted Find (previous element first) is held to the same bars as
    the full Find the oracle runs every step."""
    wl = W.channel(n_el=(6, 4, 6), N=6, n_y=6)
    om, g, o = _run_both(wl, 20, tau, 0.01, precision, hint)
    _compare(wl, om, g, o)


@pytest.mark.parametrize("hint", [False, True])
def test_channel2d_matches_oracle_loop(hint):
    wl = W.channel(n_el=(8, 4), N=5, n_y=10)
    om, g, o = _run_both(wl, 25, 0.1, 0.01, hint=hint)
    _compare(wl, om, g, o)


def test_deterministic_and_empty():
    fpts = _fpts()
    wl = W.channel(n_el=(4, 3, 4), N=5, n_y=5)
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    field = torch.from_numpy(wl["fields"]).cuda()
    outs = []
    for _ in range(2):
        P = fpts.Particles(torch.from_numpy(wl["pts"]).cuda(), torch.from_numpy(wl["v0"]).cuda(),
                           0.2, 0.01, wl["lo"], wl["hi"], wl["periodic"]).start(gm)
        for k in range(5):
            gm.lpt_step(P, field, first=(k == 0))
        torch.cuda.synchronize()
        outs.append((P.x.cpu().numpy(), P.v.cpu().numpy(), to_np(P.find)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    for k in outs[0][2]:
        assert np.array_equal(outs[0][2][k], outs[1][2][k], equal_nan=True), k
    E = fpts.Particles(torch.zeros((3, 0), dtype=torch.float64, device="cuda"),
                       torch.zeros((3, 0), dtype=torch.float64, device="cuda"),
                       0.2, 0.01, wl["lo"], wl["hi"], wl["periodic"]).start(gm)
    gm.lpt_step(E, field, first=True)
    torch.cuda.synchronize()


def test_rejects_bad_arguments():
    fpts = _fpts()
    wl = W.channel(n_el=(4, 3, 4), N=5, n_y=3)
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    field = torch.from_numpy(wl["fields"]).cuda()
    x = torch.from_numpy(wl["pts"]).cuda()
    v = torch.from_numpy(wl["v0"]).cuda()
    for tau, dt, lo in ((0.0, 0.01, 0.0), (1.0, -0.01, 0.0), (1.0, float("nan"), 0.0),
                        (1.0, 0.01, 10.0)):
        P = fpts.Particles(x, v, tau, dt, (lo, -1.0, 0.0), wl["hi"], wl["periodic"]).start(gm)
        with pytest.raises(fpts.FptsError):
            gm.lpt_step(P, field, first=True)
    P = fpts.Particles(x, v, 1.0, 0.01, wl["lo"], wl["hi"], wl["periodic"]).start(gm)
    with pytest.raises(fpts.FptsError):
        gm.lpt_step(P, field[:2].contiguous(), first=True)
    torch.cuda.synchronize()


@pytest.mark.parametrize("hint", [False, True])
def test_channel_full_size_sampled(hint):
    """The channel of the particle-tracking table (36 x 24 x 36 hexes, p = 7,
    15.9M computational points) with 1.02 particles per point: 16.5M
    particles, three steps on the GPU; 3000 sampled particles run through
    the oracle loop (one-way coupling: particles are independent)."""
    fpts = _fpts()
    wl = W.channel()
    n = wl["pts"].shape[1]
    print("channel full size: %d particles, %d elements" % (n, wl["nodes"].shape[0]), flush=True)
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    field = torch.from_numpy(wl["fields"]).cuda()
    P = fpts.Particles(torch.from_numpy(wl["pts"]).cuda(), torch.from_numpy(wl["v0"]).cuda(),
                       wl["tau"], wl["dt"], wl["lo"], wl["hi"], wl["periodic"],
                       hint=hint).start(gm)
    steps = 3
    for k in range(steps):
        gm.lpt_step(P, field, first=(k == 0))
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.random.default_rng(79).choice(n, 3000, replace=False),
                                    [0, n - 1]]))
    g = dict(x=P.x[:, idx].cpu().numpy(), v=P.v[:, idx].cpu().numpy(),
             hist=P.hist[:, :, idx].cpu().numpy(),
             find={k: (t[:, idx] if t.dim() == 2 else t[idx]).cpu().numpy()
                   for k, t in P.find.items()})
    codes = P.find["code"].cpu().numpy()
    assert np.all(codes != oracle.NOT_FOUND)
    del P, field, gm
    om = oracle.Mesh(wl["nodes"], 3, 3, wl["N"])
    o = olpt.run(om, wl["fields"], wl["pts"][:, idx], wl["v0"][:, idx], steps, wl["tau"],
                 wl["dt"], wl["lo"], wl["hi"], wl["periodic"])
    rep = dict(dx=float(np.abs(g["x"] - o["x"]).max()), dv=float(np.abs(g["v"] - o["v"]).max()))
    print(wl["name"], rep, flush=True)
    assert rep["dx"] <= TOL and rep["dv"] <= TOL
    assert np.abs(g["hist"][0] - o["hist_v"]).max() <= TOL
    assert np.abs(g["hist"][1] - o["hist_a"]).max() <= TOL
    compare_find(om, g["x"], om.find(g["x"]), g["find"], wl["h"])
