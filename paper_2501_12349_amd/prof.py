"""Summaries of rocprofv3 CSV output for the profiles/ folder.

    python -m paper_2501_12349_amd.prof stats  <dir>/run_kernel_stats.csv  "<command>" "<title>"
    python -m paper_2501_12349_amd.prof traffic <fetch_dir> <write_dir> "<commands>" "<title>"
    python -m paper_2501_12349_amd.prof sq <dir1> <dir2> "<commands>" "<title>"

`stats` turns a --kernel-trace --stats run into a table of kernels (calls,
average and total time).  `sq` summarises two --pmc runs of SQ counters
(instruction counts, MFMA busy cycles, waits, LDS bank conflicts) per
dispatch of the Newton and nearest-node kernels.  `traffic` combines a --pmc FETCH_SIZE run and a
--pmc WRITE_SIZE run (same program, one pass each) into HBM bytes per
dispatch.  Each counter is scaled by what it reads for a plain device copy of
known size in the same run (bench.py --calib-copy: 1 GiB), because the raw
counters need not count bytes one to one.  The traffic summary ends with a
line that bench.py reads back for its roofline object, together with a hash
of the Newton kernel sources, so that a stale figure is never reported.
"""
import csv
import hashlib
import os
import sys
from collections import OrderedDict

PKG = os.path.dirname(os.path.abspath(__file__))
NEWTON_SOURCES = ("csrc/newton_mfma.hpp", "csrc/kernels_newton.hip")
CALIB_BYTES = 1 << 30      # the --calib-copy copy
TRAFFIC_TAG = "k_newton_traffic"


def newton_source_hash():
    """sha256 over the sources of the hex Newton kernels."""
    h = hashlib.sha256()
    for rel in NEWTON_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    name = name.replace("(anonymous namespace)::", "")
    name = name.split("(")[0]
    for pre in ("void ", "fpts::newton::", "fpts::"):
        name = name.replace(pre, "")
    return name.strip()


def stats_table(path, top=24):
    rows = list(csv.DictReader(open(path)))
    out = ["| Kernel | Calls | Avg ms | Total ms | % of GPU time |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %.4f | %.3f | %.2f |" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e6,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return "\n".join(out)


def _per_kernel(path, counter):
    """kernel -> (dispatches, summed counter, summed duration ms); also the
    counter value of the largest copy-kernel dispatch."""
    agg = OrderedDict()
    seen = set()
    copy_val, copy_grid = None, -1
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = short_name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        n, s, t = agg.get(k, (0, 0.0, 0.0))
        key = r["Dispatch_Id"]
        if key not in seen:
            seen.add(key)
            agg[k] = (n + 1, s + v, t + d)
        if "copyBuffer" in k and int(r["Grid_Size"]) > copy_grid:
            copy_grid, copy_val = int(r["Grid_Size"]), v
    return agg, copy_val


def traffic(fetch_csv, write_csv):
    """kernel -> dict(dispatches, ms, read_bytes, write_bytes) per dispatch,
    calibrated; plus the two calibration factors."""
    fa, fcopy = _per_kernel(fetch_csv, "FETCH_SIZE")
    wa, wcopy = _per_kernel(write_csv, "WRITE_SIZE")
    if not fcopy or not wcopy:
        raise SystemExit("no copy-kernel dispatch in the counter runs (use --calib-copy)")
    fr = CALIB_BYTES / (fcopy * 1024.0)
    fw = CALIB_BYTES / (wcopy * 1024.0)
    out = OrderedDict()
    for k, (n, s, t) in fa.items():
        if k not in wa:
            continue
        wn, ws, wt = wa[k]
        out[k] = dict(dispatches=n, ms=t / n, read=s * 1024.0 * fr / n,
                      write=ws * 1024.0 * fw / wn)
    return out, fr, fw


def sq_counters(paths, match=("k_newton", "k_nearest", "k_locate", "k_bin_", "k_eval")):
    """kernel -> {counter: value per dispatch} over the --pmc runs."""
    agg = OrderedDict()
    for path in paths:
        disp = {}
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            if not any(k.startswith(m) for m in match):
                continue
            d = agg.setdefault(k, OrderedDict())
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            disp.setdefault(k, {}).setdefault(r["Counter_Name"], set()).add(r["Dispatch_Id"])
        for k, cs in disp.items():
            for c, ids in cs.items():
                agg[k][c] /= len(ids)
    return agg


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        cmd = argv[2] if len(argv) > 2 else ""
        title = argv[3] if len(argv) > 3 else "rocprofv3 kernel statistics"
        print("# %s\n\nCommand (run from /tmp with TMPDIR=/tmp on the GPU host; REPO = the "
              "repository root):\n\n    %s\n\nSummary of `run_kernel_stats.csv` (python -m "
              "paper_2501_12349_amd.prof stats).\n" % (title, cmd))
        print(stats_table(argv[1]))
        return 0
    if len(argv) >= 3 and argv[0] == "traffic":
        fetch_dir, write_dir = argv[1], argv[2]
        cmd = argv[3] if len(argv) > 3 else ""
        title = argv[4] if len(argv) > 4 else "HBM traffic per dispatch"
        t, fr, fw = traffic(os.path.join(fetch_dir, "run_counter_collection.csv"),
                            os.path.join(write_dir, "run_counter_collection.csv"))
        print("# %s\n\nCommands (run from /tmp with TMPDIR=/tmp on the GPU host; REPO = the "
              "repository root), one counter per run:\n\n    %s\n"
              % (title, cmd.replace(" ;; ", "\n    ")))
        print("Calibration: a 1 GiB device copy in the same program reads FETCH_SIZE = %.0f KiB "
              "and WRITE_SIZE = %.0f KiB, so bytes = FETCH_SIZE x 1024 x %.4f and "
              "WRITE_SIZE x 1024 x %.4f.  Durations are those of the counter runs (kernels "
              "serialised by the profiler).\n" % (CALIB_BYTES / 1024 / fr, CALIB_BYTES / 1024 / fw,
                                                  fr, fw))
        print("| Kernel | Dispatches | ms | GB read | GB written | GB/s |")
        print("|---|---:|---:|---:|---:|---:|")
        for k, v in sorted(t.items(), key=lambda kv: -kv[1]["ms"]):
            if v["ms"] < 0.05:
                continue
            print("| `%s` | %d | %.3f | %.3f | %.3f | %.0f |" % (
                k, v["dispatches"], v["ms"], v["read"] / 1e9, v["write"] / 1e9,
                (v["read"] + v["write"]) / (v["ms"] * 1e-3) / 1e9))
        kn = [k for k in t if k.startswith("k_newton<")]
        if kn:
            v = t[kn[0]]
            print("\n%s: %s bytes=%d read=%d write=%d source=%s" % (
                TRAFFIC_TAG, kn[0], int(v["read"] + v["write"]), int(v["read"]),
                int(v["write"]), newton_source_hash()))
        return 0
    if len(argv) >= 3 and argv[0] == "sq":
        cmd = argv[3] if len(argv) > 3 else ""
        title = argv[4] if len(argv) > 4 else "SQ counters per dispatch"
        agg = sq_counters([os.path.join(argv[1], "run_counter_collection.csv"),
                           os.path.join(argv[2], "run_counter_collection.csv")])
        print("# %s\n\nCommands (run from /tmp with TMPDIR=/tmp on the GPU host; REPO = the "
              "repository root), eight SQ counters per run:\n\n    %s\n"
              % (title, cmd.replace(" ;; ", "\n    ")))
        print("Per dispatch.  SQ_WAVE_CYCLES and SQ_WAIT_INST_ANY count 4-cycle units summed "
              "over waves; SQ_VALU_MFMA_BUSY_CYCLES and SQ_LDS_BANK_CONFLICT are cycles summed "
              "over SIMDs / CUs.\n")
        names = []
        for d in agg.values():
            for c in d:
                if c not in names:
                    names.append(c)
        print("| Counter | " + " | ".join("`%s`" % k for k in agg) + " |")
        print("|---|" + "---:|" * len(agg))
        for c in names:
            print("| %s | %s |" % (c, " | ".join("%.4g" % agg[k].get(c, float("nan"))
                                                 for k in agg)))
        return 0
    print(__doc__)
    return 2


def read_newton_traffic(path):
    """Bytes per k_newton dispatch from a traffic summary, or None when the
    file is missing or the Newton sources changed since it was made."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith(TRAFFIC_TAG + ":"):
            fields = dict(f.split("=", 1) for f in ln.split()[2:] if "=" in f)
            if fields.get("source") != newton_source_hash():
                return None
            return int(fields["bytes"])
    return None


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
