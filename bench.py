"""Benchmark: located + interpolated points per second on one MI355X.

One step = Find (hash lookup, box filter, trust-region Newton, selection)
and Interpolate of all fields over one batch of device-resident points, as
one fpts_find_eval call (bit for bit the outputs of fpts_find followed by
fpts_eval; the two separate calls are timed beside it).  Default workload: 48^3 curved hexes, p = 7 (N = 8 GLL nodes per
direction), 2^24 points uniform in the cube, 3 fields.  Both Newton
precisions are timed (FP64, and FP32 passes + FP64 polish); `value` is the
FP64 path, the mixed result sits beside it.  Beside them: the particle
tracking loop of the paper's channel case (fpts_lpt_step), a 2D line mesh
of the paper's surface-mesh size, device-side setup, host-to-host
throughput, the serving loop and the oracle on the CPU.

Prints one JSON line (see the driver contract) with a roofline object for
the dominant kernel (trust-region Newton, measured with HIP events on the
stream it runs on) and the oracle timed on the host cores over a bounded
sample of the same points.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6    # 256 CUs x 2.4 GHz x 128 FP64 flop/clk
FP32_VALU_PEAK_TFLOPS = 157.3
TRAFFIC_SUMMARY = "k_newton_hex48_p7_fp64_traffic.md"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eval_flops(D, R, N, h2):
    """Algorithmic FLOPs of one map evaluation (x, G = dx/dr and, with h2,
    the second derivatives) at one reference point, as the kernel computes
    it: sum-factorised contraction + product-form basis jets + objective
    terms (FMA = 2 FLOPs)."""
    if R == 3:
        con = 2 * D * ((3 * N ** 3 + 6 * N ** 2 + 10 * N) if h2 else
                       (2 * N ** 3 + 3 * N ** 2 + 4 * N))
    else:
        con = 2 * D * ((3 * N ** 2 + 6 * N) if h2 else (2 * N ** 2 + 3 * N))
    basis = R * (27 * N if h2 else 14 * N)
    obj = 2 * D * (1 + R + (2 * R * R if h2 else R * R))
    return con + basis + obj


def newton_flops(stats, D, R, N):
    """FLOPs of one k_newton launch from its exact counters: every map
    evaluation the iteration needs (first derivatives at each query point,
    second derivatives where a face pass needs them), FP32 and FP64."""
    f = stats["evals"] * eval_flops(D, R, N, False)
    f += stats["evals_h2"] * (eval_flops(D, R, N, True) - eval_flops(D, R, N, False))
    f += stats["evals_fp32"] * eval_flops(D, R, N, False)
    return float(f)


def nearest_flops(stats, D, R, N):
    """FLOPs of one k_nearest launch: a squared distance (D subtractions and
    D FMAs = 3 D FLOPs) per element node and pair."""
    return float(stats["pairs"] * N ** R * 3 * D)


def slot_use(stats):
    """Fraction of busy pair slots per sweep (16 slots per wavefront)."""
    out = {}
    if stats["sweeps"]:
        out["sweep1"] = round(stats["evals"] / (16.0 * stats["sweeps"]), 4)
    if stats["sweeps_h2"]:
        out["sweep2"] = round(stats["evals_h2"] / (16.0 * stats["sweeps_h2"]), 4)
    if stats["sweeps_fp32"]:
        swept = stats["evals_fp32"] - stats.get("evals_fp32_node", 0)
        out["fp32"] = round(swept / (16.0 * stats["sweeps_fp32"]), 4)
    return out


def make_workload(name):
    from paper_2501_12349_amd import workloads as W
    if name == "hex48":
        return W.hex48()
    if name == "hex16":
        return W.hex16()
    if name == "sphere":
        return W.sphere()
    if name == "quad2d":
        return W.quad2d()
    raise SystemExit("unknown workload %s" % name)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(wl, sample, log_, sample_1core=100000):
    """The oracle (FP64, OpenMP over points) on the first `sample` points:
    find + eval timed, setup excluded; then the first `sample_1core` points
    on one thread.  Returns the report and the oracle's results on the
    sample (for the error of the GPU results)."""
    import oracle
    t0 = time.perf_counter()
    om = oracle.Mesh(wl["nodes"], wl["dim"], wl["ref_dim"], wl["N"])
    t_setup = time.perf_counter() - t0
    pts = np.ascontiguousarray(wl["pts"][:, :sample])
    log_("cpu baseline: oracle setup %.1f s, timing find+eval on %d points" % (t_setup, sample))
    t0 = time.perf_counter()
    res = om.find(pts)
    u = om.eval(res, wl["fields"]) if wl.get("fields") is not None else None
    t = time.perf_counter() - t0
    n1 = min(sample_1core, sample)
    p1 = np.ascontiguousarray(wl["pts"][:, :n1])
    t0 = time.perf_counter()
    r1 = om.find(p1, nthreads=1)
    if wl.get("fields") is not None:
        om.eval(r1, wl["fields"], nthreads=1)
    t1 = time.perf_counter() - t0
    model, ncpu = cpu_model()
    log_("cpu baseline: %.3f Mpts/s on %d threads, %.3f Mpts/s on one (%s)" % (
        sample / t / 1e6, oracle.max_threads(), n1 / t1 / 1e6, model))
    rep = dict(value=sample / t / 1e6, unit="Mpts/s", cores=oracle.max_threads(),
               kind="oracle", cpu_model=model, logical_cpus=ncpu,
               value_1core=round(n1 / t1 / 1e6, 5),
               sample="first %d of the %d points, same mesh and %d fields; find+eval %.1f s, "
                      "oracle setup %.1f s excluded; one-thread figure on the first %d points "
                      "(%.1f s)" % (
                          sample, wl["pts"].shape[1],
                          0 if wl.get("fields") is None else wl["fields"].shape[0], t, t_setup,
                          n1, t1))
    return rep, om, res, u


# oracle margins below which a point is ambiguous (its answer may change under
# rounding-level changes of the inputs): reference units from a face, box
# slack, BORDER gap and distance over h, surface threshold
_AMB_R, _AMB_BOX, _AMB_GAP, _AMB_EPS = 2e-6, 1e-9, 1e-8, 1e-6


def error_vs_oracle(orc, uo, gpu, ug, h, surface):
    """Error of GPU results against the oracle's on the same points: element
    / code mismatches on the unambiguous points, max |dr|, max |ddist| / h
    and the max field error relative to max(|u_oracle|, max |u|)."""
    m, code = orc["margin"], orc["code"]
    amb = (code == 0) & (m[0] < _AMB_R)
    amb |= (code != 0) & (m[1] < _AMB_BOX)
    amb |= (code == 1) & ((m[2] < _AMB_GAP) | (m[3] < _AMB_GAP))
    if surface:
        amb |= (code != 2) & (m[4] < _AMB_EPS)
    una = ~amb
    found = una & (code != 2)
    out = dict(points=int(code.size), ambiguous=int(amb.sum()),
               elem_mismatch=int((una & (gpu["elem"] != orc["elem"])).sum()),
               code_mismatch=int((una & (gpu["code"] != code)).sum()))
    same = found & (gpu["elem"] == orc["elem"])
    out["max_dr"] = float(np.abs(gpu["r"][:, same] - orc["r"][:, same]).max()) if same.any() \
        else 0.0
    out["max_ddist_over_h"] = float(np.abs(gpu["dist"][same] - orc["dist"][same]).max() / h) \
        if same.any() else 0.0
    if uo is not None and ug is not None and same.any():
        scale = np.maximum(np.abs(uo[:, same]), np.abs(uo[:, same]).max(axis=1, keepdims=True))
        out["max_du_rel"] = float((np.abs(ug[:, same] - uo[:, same]) / scale).max())
    return out


def pcie_inclusive(gm, wl, fields, ws_f, ws_e, mode, steps):
    """Points from pinned host memory to results in pinned host memory:
    H2D of the points, find + eval, D2H of code/elem/r/dist/u, on one
    stream."""
    import torch
    n = wl["pts"].shape[1]
    R = wl["ref_dim"]
    nf = fields.shape[0]
    dev = fields.device
    h_pts = torch.from_numpy(wl["pts"]).pin_memory()
    h_out = dict(code=torch.empty(n, dtype=torch.int32).pin_memory(),
                 elem=torch.empty(n, dtype=torch.int32).pin_memory(),
                 r=torch.empty((R, n), dtype=torch.float64).pin_memory(),
                 dist=torch.empty(n, dtype=torch.float64).pin_memory(),
                 u=torch.empty((nf, n), dtype=torch.float64).pin_memory())
    d_pts = torch.empty_like(h_pts, device=dev)
    d_out = {k: torch.empty_like(v, device=dev) for k, v in h_out.items()}

    def once():
        d_pts.copy_(h_pts, non_blocking=True)
        res = {k: d_out[k] for k in ("code", "elem", "r", "dist")}
        gm.find(d_pts, precision=mode, out=res, ws=ws_f)
        gm.eval(res, fields, out=d_out["u"], ws=ws_e)
        for k in h_out:
            h_out[k].copy_(d_out[k], non_blocking=True)

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    moved = h_pts.numel() * 8 + sum(v.numel() * v.element_size() for v in h_out.values())
    return dict(value=round(n / dt / 1e6, 3), unit="Mpts/s", ms_per_step=round(dt * 1e3, 3),
                steps=steps, precision=mode, bytes_over_pcie=int(moved))


def serving(n_req, budget, n_streams=4, max_batch=1 << 22):
    """The request loop over four resident curved hex meshes (p = 3, 5, 7,
    9; 46^3, 36^3, 27^3, 22^3 elements), Poisson arrivals of find + eval
    requests with 10^U(3,6) points, mixed precision; p50/p99 latency at
    0.5 / 0.8 / 1.0 / 1.2 x the saturated request rate."""
    from paper_2501_12349_amd import fpts
    from paper_2501_12349_amd import serve as SV
    t0 = time.perf_counter()
    meshes = SV.build_meshes(scale=1.0)
    sizes, mids, pts = SV.make_requests(n_req)
    log("serving: 4 meshes + %d requests (%d points) ready in %.1f s" % (
        n_req, int(sizes.sum()), time.perf_counter() - t0))
    srv = fpts.Server(budget, n_streams=n_streams, max_batch_points=max_batch)
    ids = [srv.add_mesh(m, f) for _, m, f in meshes]
    rep = SV.sweep(srv, ids, sizes, mids, pts)
    srv.close()
    for r in rep["loads"]:
        log("serving load %.1f: %.0f req/s  p50 %.2f ms  p99 %.2f ms  %.1f Mpts/s" % (
            r["load"], r["rate_req_s"], r["p50_ms"], r["p99_ms"], r["mpts_s"]))
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    return dict(meshes=[wl["name"] for wl, _, _ in meshes], requests=n_req,
                points=int(sizes.sum()), precision="mixed", budget_bytes=budget,
                n_streams=n_streams, max_batch_points=max_batch,
                saturation=rnd(rep["saturation"]),
                saturated_rate_req_s=round(rep["saturated_rate_req_s"], 2),
                loads=[rnd(r) for r in rep["loads"]], batches=rep["batches"],
                max_batch_requests=rep["max_batch_requests"],
                max_in_flight=rep["max_in_flight"], peak_bytes=rep["peak_bytes"])


def particle_tracking(ratios, steps, warmup, precision):
    """The particle-tracking loop of the paper's channel case: 36 x 24 x 36
    hexes with p = 7 (15.9M computational points), a frozen synthetic
    fluid velocity, tau = 5, dt = 1e-3, particles on a 2:1:1 lattice with
    `ratio` particles per computational point.  One step = Interpolate +
    particle update + Find of every particle (fpts_lpt_step); the time of
    each part comes from HIP events on the stream."""
    import torch
    from paper_2501_12349_amd import fpts
    from paper_2501_12349_amd import workloads as W
    t0 = time.perf_counter()
    wl = W.channel(ratio=ratios[0])
    gm = fpts.Mesh(wl["nodes"], wl["N"])
    field = torch.from_numpy(wl["fields"]).cuda()
    log("particle tracking: %s (%d elements) ready in %.1f s" % (
        wl["name"], wl["nodes"].shape[0], time.perf_counter() - t0))
    out = []
    # every ratio with the paper's full Find; the first one also hinted
    # (previous element first, fpts_lpt.h)
    for ratio, hint in [(r, False) for r in ratios] + [(ratios[0], True)]:
        n_y = W.lattice_n_y(ratio, wl["n_comp"])
        pts = W.particle_lattice(n_y)
        v0 = W.channel_velocity(pts, wl["modes"])
        n = pts.shape[1]
        P = fpts.Particles(torch.from_numpy(pts).cuda(), torch.from_numpy(v0).cuda(), wl["tau"],
                           wl["dt"], wl["lo"], wl["hi"], wl["periodic"],
                           hint=hint).start(gm, precision)
        del pts, v0
        ws = torch.empty(gm.lpt_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        for k in range(warmup):
            gm.lpt_step(P, field, first=(k == 0), precision=precision, ws=ws)
        torch.cuda.synchronize()
        gm.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            gm.lpt_step(P, field, first=(warmup == 0 and k == 0), precision=precision, ws=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        kt = gm.profile_read()
        gm.profile(False)
        lost = int((P.find["code"] == fpts.NOT_FOUND).sum().item())
        c = max(kt["lpt_calls"], 1)
        find_ms = (kt["locate_ms"] + kt["nearest_ms"] + kt["newton_ms"] + kt["face_ms"] +
                   kt["select_ms"]) / c
        interp_ms = (kt["eval_bin_ms"] + kt["eval_ms"]) / c
        adv_ms = kt["advance_ms"] / c
        tot = find_ms + interp_ms + adv_ms
        rep = dict(ratio=ratio, hinted_find=hint, particles=n, ms_per_step=round(dt * 1e3, 4),
                   mparticle_steps_per_s=round(n / dt / 1e6, 3),
                   find_ms=round(find_ms, 4), interpolate_ms=round(interp_ms, 4),
                   advance_ms=round(adv_ms, 4),
                   fractions=dict(find=round(find_ms / tot, 4),
                                  interpolate=round(interp_ms / tot, 4),
                                  advance=round(adv_ms / tot, 4)),
                   not_found=lost)
        log("particle tracking %.2f particles/point (%d)%s: %.3f ms/step  %.1f M particle-steps/s  "
            "find %.3f interpolate %.3f advance %.3f ms  lost %d" % (
                ratio, n, " hinted" if hint else "", dt * 1e3, n / dt / 1e6, find_ms, interp_ms,
                adv_ms, lost))
        out.append(rep)
        del P, ws
        torch.cuda.empty_cache()
    return dict(workload="%s_%dhex_tau%g_dt%g" % (wl["name"], wl["nodes"].shape[0], wl["tau"],
                                                   wl["dt"]),
                n_comp=wl["n_comp"], precision=precision, steps=steps, warmup=warmup,
                step="interpolate (3 fields) + drag/AB2/boundary + find, fpts_lpt_step",
                runs=out)


def line_surface(level, steps, warmup):
    """Find + Interpolate on the cubic 2D line mesh that stands in for the
    paper's surface-mesh case (84 x 2^level elements, 1000 points per
    element on the curves, one cubic field), FP64."""
    import torch
    from paper_2501_12349_amd import fpts
    from paper_2501_12349_amd import workloads as W
    t0 = time.perf_counter()
    wl = W.line2d(level=level)
    gm = fpts.Mesh(wl["nodes"], wl["N"], dim=2, ref_dim=1)
    t_setup = time.perf_counter() - t0
    n = wl["pts"].shape[1]
    pts = torch.from_numpy(wl["pts"]).cuda()
    field = torch.from_numpy(wl["fields"]).cuda()
    out = dict(code=torch.empty(n, dtype=torch.int32, device="cuda"),
               elem=torch.empty(n, dtype=torch.int32, device="cuda"),
               r=torch.empty((1, n), dtype=torch.float64, device="cuda"),
               dist=torch.empty(n, dtype=torch.float64, device="cuda"))
    u = torch.empty((1, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(gm.find_workspace_bytes(n), gm.eval_workspace_bytes(n)),
                     dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        gm.find(pts, out=out, ws=ws)
        gm.eval(out, field, out=u, ws=ws)
    torch.cuda.synchronize()
    gm.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gm.find(pts, out=out, ws=ws)
        gm.eval(out, field, out=u, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kt = gm.profile_read()
    gm.profile(False)
    stats = gm.find_stats()
    c = max(kt["find_calls"], 1)
    find_ms = (kt["locate_ms"] + kt["nearest_ms"] + kt["newton_ms"] + kt["face_ms"] +
                   kt["select_ms"]) / c
    eval_ms = (kt["eval_bin_ms"] + kt["eval_ms"]) / max(kt["eval_calls"], 1)
    codes = torch.bincount(out["code"].long(), minlength=3).cpu().tolist()
    log("line2d %d elements, %d points: %.3f ms/step  %.1f Mpts/s  find %.3f eval %.3f ms  "
        "newton %.3f ms  codes %s  evals/pair %.2f" % (
            wl["nodes"].shape[0], n, dt * 1e3, n / dt / 1e6, find_ms, eval_ms,
            kt["newton_ms"] / c, codes, stats["evals"] / max(stats["pairs"], 1)))
    return dict(workload="%s_%dpts_1field" % (wl["name"], n), n_elem=int(wl["nodes"].shape[0]),
                n_points=n, precision="fp64", steps=steps, ms_per_step=round(dt * 1e3, 4),
                mpts_s=round(n / dt / 1e6, 3), find_ms=round(find_ms, 4),
                eval_ms=round(eval_ms, 4), newton_ms=round(kt["newton_ms"] / c, 4),
                setup_s=round(t_setup, 3),
                codes=dict(zip(("interior", "border", "not_found"), codes)),
                evals_per_pair=round(stats["evals"] / max(stats["pairs"], 1), 3),
                paper_context="same element and point counts: Find 8.6 s, Interpolate 2.4 s "
                              "on one node with 4 V100 GPUs")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hex48")
    ap.add_argument("--cpu-sample", type=int, default=4000000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--mixed-tol", type=float, default=None,
                    help="step size that ends the FP32 phase of mixed mode (default: the "
                         "library's, fpts_params_default)")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests per serving run (0: no serving measurement)")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=1 << 22)
    ap.add_argument("--pcie-steps", type=int, default=3,
                    help="steps of the host-to-host measurement (0: skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 1 GiB device copy first (HBM counter calibration); "
                         "implies --no-setup-device, whose node copy is larger")
    ap.add_argument("--no-setup-device", action="store_true",
                    help="skip timing the device-side setup (fpts_update_nodes)")
    ap.add_argument("--lpt-ratios", default="1.02",
                    help="particles per computational point of the particle-tracking runs "
                         "(comma list; empty: skip)")
    ap.add_argument("--lpt-steps", type=int, default=10,
                    help="timed steps per particle-tracking run (0: skip)")
    ap.add_argument("--line-level", type=int, default=8,
                    help="refinement level of the 2D line-mesh run (84 x 2^level elements; "
                         "-1: skip)")
    ap.add_argument("--only", choices=("lpt", "line", "serve"),
                    help="run only the particle-tracking or the line-mesh leg and print its "
                         "object (for profiling those kernels; not the benchmark line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on exactly one GPU: the find/eval path has no "
              "multi-GPU mode (points would shard across GPUs with the mesh replicated)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_12349_amd import fpts

    if args.only == "lpt":
        print(json.dumps(particle_tracking([float(r) for r in args.lpt_ratios.split(",")],
                                           args.lpt_steps, args.warmup, "fp64")), flush=True)
        return
    if args.only == "serve":
        print(json.dumps(serving(args.serve_requests, int(args.serve_budget_gb * (1 << 30)),
                                 args.serve_streams, args.serve_max_batch)), flush=True)
        return
    if args.only == "line":
        print(json.dumps(line_surface(max(args.line_level, 0), args.steps, args.warmup)),
              flush=True)
        return

    t0 = time.perf_counter()
    wl = make_workload(args.workload)
    log("workload %s generated in %.1f s" % (wl["name"], time.perf_counter() - t0))
    D, R, N = wl["dim"], wl["ref_dim"], wl["N"]
    n = wl["pts"].shape[1]
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    gm = fpts.Mesh(wl["nodes"], N, dim=D, ref_dim=R, mixed_tol=args.mixed_tol)
    t_setup = time.perf_counter() - t0
    log("setup %.2f s (host boxes + map, upload)" % t_setup)
    # setup on the device from nodes already there (fpts_update_nodes, the
    # moving-mesh path), timed after a first call
    t_setup_dev = None
    if not (args.no_setup_device or args.calib_copy):
        d_nodes = torch.from_numpy(wl["nodes"]).to(dev)
        gm.update_nodes(d_nodes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gm.update_nodes(d_nodes)
        t_setup_dev = time.perf_counter() - t0
        del d_nodes
        log("device setup %.1f ms (boxes, centres, local map from device nodes)"
            % (t_setup_dev * 1e3))
    pts = torch.from_numpy(wl["pts"]).to(dev)
    fields = torch.from_numpy(wl["fields"]).to(dev)
    nf = fields.shape[0]
    out = dict(code=torch.empty(n, dtype=torch.int32, device=dev),
               elem=torch.empty(n, dtype=torch.int32, device=dev),
               r=torch.empty((R, n), dtype=torch.float64, device=dev),
               dist=torch.empty(n, dtype=torch.float64, device=dev))
    u = torch.empty((nf, n), dtype=torch.float64, device=dev)
    # one workspace serves fpts_find_eval and, for the comparison with the two
    # separate calls, fpts_find (its layout starts the same way)
    ws_f = torch.empty(gm.find_eval_workspace_bytes(n), dtype=torch.uint8, device=dev)
    ws_e = torch.empty(gm.eval_workspace_bytes(n), dtype=torch.uint8, device=dev)
    log("workspace find+eval %.2f GB (%.0f B per point), eval %.2f GB" % (
        ws_f.numel() / 1e9, ws_f.numel() / n, ws_e.numel() / 1e9))

    def step(prec):
        # one pass of the path: Find and Interpolate of every point
        gm.find_eval(pts, fields, precision=prec, out=out, u=u, ws=ws_f)

    def step_separate(prec):
        gm.find(pts, precision=prec, out=out, ws=ws_f)
        gm.eval(out, fields, out=u, ws=ws_e)

    if args.calib_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per byte
        # scales the counters of the other kernels
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    results = {}
    for mode in args.modes.split(","):
        for _ in range(args.warmup):
            step(mode)
        torch.cuda.synchronize()
        gm.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = gm.profile_read()
        gm.profile(False)
        # counters of the last find (the iteration counts are deterministic)
        stats = gm.find_stats(newton_pass=1)
        stats_all = gm.find_stats()
        stats_other = gm.find_stats(newton_pass=2)
        stats_face = gm.find_stats(newton_pass=3)
        codes = torch.bincount(out["code"].long(), minlength=3).cpu().tolist()
        # the sample the oracle checks: the first points of the batch
        ns = min(args.cpu_sample, n)
        snap = {k: (v[..., :ns].cpu().numpy()) for k, v in out.items()}
        snap_u = u[:, :ns].cpu().numpy()
        ms = dt / args.steps * 1e3
        newton_ms = kt["newton_ms"] / max(kt["find_calls"], 1)
        fl = newton_flops(stats, D, R, N)
        results[mode] = dict(ms_per_step=ms, mpts=n / (dt / args.steps) / 1e6, kt=kt,
                             newton_ms=newton_ms, stats=stats, stats_all=stats_all,
                             stats_other=stats_other, stats_face=stats_face, flops=fl,
                             codes=codes, snap=snap, snap_u=snap_u)
        log("%s: other candidates %s  face %s" % (mode, stats_other, stats_face))
        log("%s: %.3f ms/step  %.1f Mpts/s  k_newton %.3f ms (%.1f TFLOP/s)  face %.3f  "
            "nearest %.3f locate %.3f select %.3f eval_bin %.3f eval %.3f ms/call  codes %s  "
            "slots %s  stats %s" % (
                mode, ms, n / (dt / args.steps) / 1e6, newton_ms, fl / newton_ms / 1e9,
                kt["face_ms"] / kt["find_calls"], kt["nearest_ms"] / kt["find_calls"],
                kt["locate_ms"] / kt["find_calls"], kt["select_ms"] / kt["find_calls"],
                kt["eval_bin_ms"] / kt["eval_calls"], kt["eval_ms"] / kt["eval_calls"],
                codes, slot_use(stats), stats_all))

    main_mode = "fp64" if "fp64" in results else list(results)[0]
    r0 = results[main_mode]
    # the same work as fpts_find + fpts_eval called one after the other
    for _ in range(args.warmup):
        step_separate(main_mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_separate(main_mode)
    torch.cuda.synchronize()
    dt_sep = (time.perf_counter() - t0) / args.steps
    log("%s, fpts_find + fpts_eval as two calls: %.3f ms/step  %.1f Mpts/s" % (
        main_mode, dt_sep * 1e3, n / dt_sep / 1e6))
    achieved = r0["flops"] / (r0["newton_ms"] * 1e-3) / 1e12
    kt0 = r0["kt"]
    # HBM bytes per k_newton launch from the committed counter summary of this
    # workload (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated); None when
    # the Newton sources changed since the counters were taken
    traffic = None
    if args.workload == "hex48" and main_mode == "fp64":
        from paper_2501_12349_amd import prof
        traffic = prof.read_newton_traffic(os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY))
    line = {
        "metric": "located+interpolated points/s (Mpts/s) FP64 vs mixed; p50/p99 request latency",
        "value": round(r0["mpts"], 3),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r0["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s_%dpts_%dfields" % (wl["name"], n, nf),
                   "n_elem": int(wl["nodes"].shape[0]), "nodes_1d": N, "dim": D,
                   "ref_dim": R, "n_points": n, "n_fields": nf, "precision": main_mode,
                   "step": "find + eval of all fields (fpts_find_eval), inputs resident "
                           "in HBM"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4), "traffic": traffic,
                     "kernel": "k_newton (FP64 trust-region Newton, primary candidates)",
                     "kernel_ms": round(r0["newton_ms"], 4),
                     "flops_per_launch": r0["flops"],
                     "slot_use": slot_use(r0["stats"])},
        "workspace_bytes_per_point": round(gm.find_eval_workspace_bytes(n) / n, 1),
        "newton_total_ms": round((kt0["newton_ms"] + kt0["face_ms"]) / max(kt0["find_calls"], 1), 4),
        "setup_s": round(t_setup, 3),
        "setup_device_s": round(t_setup_dev, 4) if t_setup_dev is not None else None,
        "codes": dict(zip(("interior", "border", "not_found"), r0["codes"])),
    }
    if "mixed" in results and main_mode != "mixed":
        rm = results["mixed"]
        line["mixed"] = {"value": round(rm["mpts"], 3), "unit": "Mpts/s",
                         "ms_per_step": round(rm["ms_per_step"], 4),
                         "speedup_vs_fp64": round(rm["mpts"] / r0["mpts"], 4),
                         "newton_kernel_ms": round(rm["newton_ms"], 4)}
    kt = r0["kt"]
    line["kernel_ms"] = {k: round(kt[k + "_ms"] / max(kt["find_calls" if k in
                         ("locate", "nearest", "newton", "face", "select") else "eval_calls"], 1), 4)
                         for k in ("locate", "nearest", "newton", "face", "select", "eval_bin",
                                   "eval")}
    line["newton_stats"] = {"primary": r0["stats"], "other_candidates": r0["stats_other"],
                            "face": r0["stats_face"], "all": r0["stats_all"]}
    line["separate_calls"] = {"value": round(n / dt_sep / 1e6, 3), "unit": "Mpts/s",
                              "ms_per_step": round(dt_sep * 1e3, 4),
                              "calls": "fpts_find then fpts_eval"}
    if args.pcie_steps > 0:
        line["pcie_inclusive"] = pcie_inclusive(gm, wl, fields, ws_f, ws_e, main_mode,
                                                args.pcie_steps)
        log("host-to-host (PCIe copies included): %.1f Mpts/s" %
            line["pcie_inclusive"]["value"])
    del ws_f, ws_e, out, u, pts
    torch.cuda.empty_cache()
    if args.lpt_ratios and args.lpt_steps > 0:
        line["particle_tracking"] = particle_tracking(
            [float(r) for r in args.lpt_ratios.split(",")], args.lpt_steps, 2, main_mode)
    if args.line_level >= 0:
        line["line_mesh_2d"] = line_surface(args.line_level, 5, 1)
    if args.serve_requests > 0:
        line["serving"] = serving(args.serve_requests, int(args.serve_budget_gb * (1 << 30)),
                                  args.serve_streams, args.serve_max_batch)
    if not args.no_cpu:
        rep, om, orc, uo = cpu_baseline(wl, min(args.cpu_sample, n), log)
        line["cpu_baseline"] = rep
        # error of every GPU result against the FP64 oracle on that sample
        line["error_vs_oracle"] = {
            mode: error_vs_oracle(orc, uo, results[mode]["snap"], results[mode]["snap_u"],
                                  wl["h"], R < D)
            for mode in results}
        for mode, e in line["error_vs_oracle"].items():
            log("error vs oracle, %s: %s" % (mode, e))
        del om, orc, uo
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
