#!/usr/bin/env python3
"""Benchmark: zone-updates/s of the patch MHD update on one MI355X.

Headline workload: 3D periodic 256^3 box as 512 patches of 32^3 (ghost width
4, the stencil minimum), rho = 1, P = 1, B = (0.1, 0, 0), seeded Gaussian
random velocity with a k^-5/3 spectrum at rms Mach 1, gamma = 5/3, CFL 0.4.
One step = ghost exchange + FP64 CFL reduction + the full CTU+CT MHDTVD
update (Steps 1-11) of all patches, replayed from a captured HIP graph, with
the state resident in HBM.  The headline value is the FP32 batch (FP32 sweeps
and CT, FP64 dt and floors); the FP64 batch of the same workload is reported
beside it, and so are the uneven 400-patch batch, the 512^3 Orszag-Tang batch
(patches of 64^3, 50 steps) and the 768^3 high-contrast batch (patches of
48^3).

Roofline: the algorithmic bytes of one step are those of the patch design
(16 + 24 ((1 + 2g/n)^3 - 1) words per interior zone-update for cubic patches
of edge n: the step reads and writes the 8 conserved words of every interior
zone, the ghost exchange reads and writes those of every ghost zone, and the
step reads the ghosts), over the step time measured with HIP events on the
library's stream around the timed graph replays.

Prints ONE JSON line.  --gpus > 1 is not supported (one GPU per process; the
multi-GPU design is documented, not built).
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec on 1 MI355X (FP32 batched vs FP64 plain) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
PROFILE_JSON = os.path.join(ROOT, "profiles", "turb256_512x32_fp32_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1701_07452_amd", "csrc", "wmb_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic bytes of one step, and their attribution to the kernel classes
# ---------------------------------------------------------------------------

def alg_words(descs, g):
    """Algorithmic words of one step over a batch of patches (8 conserved
    words per zone; the zone-centred field is carried, the face field is not
    counted separately), attributed to the kernel class that must move them:
      - the ghost exchange reads and writes 8 words of every ghost zone: the
        x-ghosts of interior rows are written by the update kernel (its push
        to the x-neighbours), the other ghosts by the y/z exchange passes;
      - the step reads q^n over the whole stored box (interior and ghosts):
        charged to the three Step-1 sweeps, a third each;
      - the step writes q^{n+1} over the interior: charged to the update.
    The total is 16 V_int + 24 (V_stored - V_int) per patch."""
    w = {"fill": 0, "sweep1_x": 0, "sweep1_y": 0, "sweep1_z": 0, "update": 0}
    for n, _ in descs:
        vi = n[0] * n[1] * n[2]
        vs = (n[0] + 2 * g) * (n[1] + 2 * g) * (n[2] + 2 * g)
        gx = 2 * g * n[1] * n[2]
        w["update"] += 16 * gx + 8 * vi
        w["fill"] += 16 * (vs - vi - gx)
        for k in ("sweep1_x", "sweep1_y", "sweep1_z"):
            w[k] += 8 * vs / 3.0
    return w


def profile_record():
    """The committed rocprofv3 counter summary (copy-calibrated FETCH_SIZE /
    WRITE_SIZE bytes and VALU utilisation per kernel class of one step), or
    None when the kernel source has changed since it was taken."""
    try:
        rec = json.load(open(PROFILE_JSON))
        cur = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernels_source_sha256") == cur else None


def roofline(descs, g, es, zones, ms_step, kern_ms, prof=None):
    """Step-level HBM roofline at the algorithmic bytes, with per-kernel
    shares (each kernel's algorithmic bytes over the step time; the shares sum
    to the step fraction) and the measured traffic and VALU utilisation from
    the committed counter summary when it is current."""
    words = alg_words(descs, g)
    step_bytes = sum(words.values()) * es
    t = ms_step * 1e-3
    achieved = step_bytes / t / 1e9
    per = {}
    for k, ms in (kern_ms or {}).items():
        ab = words.get(k, 0) * es
        per[k] = {"alg_bytes": ab, "frac_share": round(ab / t / 1e9 / HBM_PEAK_GBS, 5), "eager_ms": round(ms, 4),
                  "frac_own_time": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None}
        if prof and k in prof.get("per_class", {}):
            pc = prof["per_class"][k]
            per[k]["design_bytes"] = pc.get("fetch_bytes", 0) + pc.get("write_bytes", 0)
            per[k]["valu_busy"] = pc.get("valu_busy")
    traffic = None
    if prof and es == 4:
        traffic = sum(v.get("fetch_bytes", 0) + v.get("write_bytes", 0) for v in prof["per_class"].values())
    dom = max(kern_ms, key=kern_ms.get) if kern_ms else None
    return {
        "kernel": "step (one graph replay: exchange, dt, Steps 1-11 of every patch)",
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": traffic,
        "alg_bytes_per_step": step_bytes,
        "alg_bytes_per_zone_update": round(step_bytes / zones, 3),
        "ms_per_step": ms_step,
        "measured_traffic_GBs": round(traffic / t / 1e9, 1) if traffic else None,
        "dominant_kernel": dom,
        "per_kernel": per,
    }


# ---------------------------------------------------------------------------
# rocprofv3 counter summary (written into profiles/, read back by roofline())
# ---------------------------------------------------------------------------

TUNING32_PROF = "1x32=12,1y32=16,1z32=16,2x32=2,2y32=16,2z32=-256,6x0=9"
TUNING64_PROF = "1x32=6,1y32=-256,1z32=-256,2x32=3,2y32=-64,2z32=-64,6x0=0"
COUNTER_ARGS = ("--steps 2 --warmup 1 --prof-steps 0 --no-fp64 --no-cpu-baseline --schedule 1 --calib-copy "
                "--tuning32 " + TUNING32_PROF)
SQ_COUNTERS = "SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE"
TRACE_ARGS = ("--steps 5 --warmup 1 --prof-steps 3 --no-cpu-baseline --no-uneven --no-c4 --no-c5 --no-divb "
              "--no-scratch-groups --schedule 1 "
              "--tuning32 " + TUNING32_PROF + " --tuning64 " + TUNING64_PROF)


def kernel_class(name):
    """Kernel class of a dispatch name (as in kernels_ms), or None outside the step."""
    import re

    m = re.search(r"(?:sweep|march)_kernel<(?:float|double), (\d), (\d)", name)
    if m:
        # stage 3: the z corrector from the records the fused corrector stored
        return "sweep%s_%s" % ("2" if m.group(2) == "3" else m.group(2), "xyz"[int(m.group(1))])
    if "corr_xy_kernel" in name:  # the fused x/y corrector: counted in the x class
        return "sweep2_x"
    for key, cls in (("fill_pass_kernel", "fill"), ("ct_half_kernel", "ct_half"), ("update_kernel", "update"),
                     ("dt_finalize_kernel", "dt")):
        if key in name:
            return cls
    return None


def short_name(name):
    name = name.replace("void ", "").replace("wmb::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def read_counter_csv(path):
    """Dispatches of a rocprofv3 counter_collection.csv, in dispatch order:
    [{"name", "ns", counter: value, ...}]."""
    import csv

    disp = {}
    for r in csv.DictReader(open(path)):
        d = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"],
                                                    "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                                                    "vgpr": r.get("VGPR_Count")})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


def last_step(disp):
    """The dispatches of the last step before the trailing diagnostics: back
    from the last update launch to the previous step's update."""
    cls = [kernel_class(d["name"]) for d in disp]
    last = max(i for i, c in enumerate(cls) if c == "update")
    j = last
    while j > 0 and cls[j - 1] == "update":
        j -= 1
    k = j - 1
    while k >= 0 and cls[k] != "update":
        k -= 1
    return disp[k + 1:last + 1]


def find_one(root, pattern):
    import glob

    hits = sorted(glob.glob(os.path.join(root, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit("no %s under %s" % (pattern, root))
    return hits[-1]


def summarize_counters(root):
    """Turn the rocprofv3 runs under `root` (fetch/, write/, sq/: one counter
    pass each of COUNTER_ARGS; trace/: --kernel-trace --stats of TRACE_ARGS,
    with its bench line in trace/bench.json; kernels.sha256: the kernel
    source the runs were built from) into the committed summaries."""
    sha = open(os.path.join(root, "kernels.sha256")).read().split()[0]
    cur = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if sha != cur:
        log("summarize: the runs were made from another kernel source (%s, now %s)" % (sha[:12], cur[:12]))
    fetch = read_counter_csv(find_one(os.path.join(root, "fetch"), "*counter_collection.csv"))
    write = read_counter_csv(find_one(os.path.join(root, "write"), "*counter_collection.csv"))
    sq = read_counter_csv(find_one(os.path.join(root, "sq"), "*counter_collection.csv"))
    copy_bytes = 1 << 30

    def calib(disp, counter):
        copies = [d for d in disp if "copyBuffer" in d["name"]]
        return max(d.get(counter, 0.0) for d in copies)

    fetch_kib, write_kib = calib(fetch, "FETCH_SIZE"), calib(write, "WRITE_SIZE")
    fs, ws = copy_bytes / 1024 / fetch_kib, copy_bytes / 1024 / write_kib
    steps = {"fetch": last_step(fetch), "write": last_step(write), "sq": last_step(sq)}
    names = [d["name"] for d in steps["fetch"]]
    for k in ("write", "sq"):
        if [d["name"] for d in steps[k]] != names:
            raise SystemExit("the three passes launched different kernels in their last step")
    rows, per_class = [], {}
    for i, nm in enumerate(names):
        f = steps["fetch"][i].get("FETCH_SIZE", 0.0) * 1024 * fs
        w = steps["write"][i].get("WRITE_SIZE", 0.0) * 1024 * ws
        s = steps["sq"][i]
        cyc = s.get("GRBM_GUI_ACTIVE", 0.0) / 8
        rows.append({"kernel": short_name(nm), "class": kernel_class(nm), "fetch": f, "write": w,
                     "ms": steps["fetch"][i]["ns"] / 1e6, "waves": s.get("SQ_WAVES", 0.0),
                     "valu": s.get("SQ_INSTS_VALU", 0.0), "active_valu": s.get("SQ_ACTIVE_INST_VALU", 0.0),
                     "cyc": cyc, "vgpr": s.get("vgpr")})
    for r in rows:
        pc = per_class.setdefault(r["class"], {"launches": 0, "fetch_bytes": 0.0, "write_bytes": 0.0, "ms": 0.0,
                                               "waves": 0.0, "valu": 0.0, "active_valu": 0.0, "cyc": 0.0})
        pc["launches"] += 1
        for a, b in (("fetch_bytes", "fetch"), ("write_bytes", "write"), ("ms", "ms"), ("waves", "waves"),
                     ("valu", "valu"), ("active_valu", "active_valu"), ("cyc", "cyc")):
            pc[a] += r[b]
    for pc in per_class.values():
        pc["valu_busy"] = round(pc["active_valu"] * 4 / (1024 * pc["cyc"]), 4) if pc["cyc"] else None
        pc["valu_insts_per_wave"] = round(pc["valu"] / pc["waves"], 1) if pc["waves"] else None
        pc["fetch_bytes"], pc["write_bytes"] = round(pc["fetch_bytes"]), round(pc["write_bytes"])
        pc["ms"] = round(pc["ms"], 4)
        for k in ("waves", "valu", "active_valu", "cyc"):
            del pc[k]
    tot_f = sum(r["fetch"] for r in rows)
    tot_w = sum(r["write"] for r in rows)
    tot_ms = sum(r["ms"] for r in rows)
    rec = {
        "workload": "turbulence 256^3 as 512 x 32^3, ghost 4, FP32, one step (the last of the run)",
        "kernels_source_sha256": sha,
        "commands": {"fetch": "rocprofv3 --pmc FETCH_SIZE -- python3 bench.py " + COUNTER_ARGS,
                     "write": "rocprofv3 --pmc WRITE_SIZE -- python3 bench.py " + COUNTER_ARGS,
                     "sq": "rocprofv3 --pmc " + SQ_COUNTERS + " -- python3 bench.py " + COUNTER_ARGS},
        "calibration": {"copy_bytes": copy_bytes, "fetch_kib": fetch_kib, "write_kib": write_kib,
                        "fetch_scale": fs, "write_scale": ws},
        "per_class": per_class,
        "whole_step": {"fetch_bytes": round(tot_f), "write_bytes": round(tot_w), "kernel_ms": round(tot_ms, 4)},
    }
    with open(PROFILE_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    md = ["# HBM traffic and VALU issue per kernel: 256^3 turbulence as 512 x 32^3, FP32 batch", "",
          "Commands (TMPDIR=/tmp, run from /tmp, `<repo>` the repository root, one pass each, "
          "`--output-format csv -d <out>/{fetch,write,sq} -o run`):", "```"]
    for k in ("fetch", "write", "sq"):
        md.append(rec["commands"][k].replace("python3 bench.py", "python3 <repo>/bench.py"))
    md += ["```", "Summarised by `python bench.py --summarize-counters <out>`, which writes this file and "
           "`%s` (read by `bench.py`'s roofline while the kernel source's sha256 matches)." %
           os.path.basename(PROFILE_JSON), "",
           "Calibration: each run first copies 1 GiB device to device (`--calib-copy`). For that copy "
           "`FETCH_SIZE` reads %.0f KiB and `WRITE_SIZE` %.0f KiB against 1048576 KiB moved each way, so fetch "
           "values are scaled by %.3f and write values by %.3f." % (fetch_kib, write_kib, fs, ws), "",
           "Values are those of the dispatches of the run's last step (the profiler serialises the "
           "kernels; durations are those of the FETCH_SIZE pass). VALU busy = SQ_ACTIVE_INST_VALU x 4 / "
           "(1024 SIMDs x GRBM_GUI_ACTIVE / 8): GRBM_GUI_ACTIVE reads the busy cycles of the 8 XCDs summed, "
           "and a wave64 FP32 VALU instruction holds a 16-lane SIMD for 4 cycles.", "",
           "| Kernel | Fetch (GB) | Write (GB) | Duration (ms) | Measured TB/s | VALU instr. per wave | VALU busy |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        busy = r["active_valu"] * 4 / (1024 * r["cyc"]) if r["cyc"] else 0.0
        md.append("| `%s` | %.3f | %.3f | %.3f | %.2f | %.0f | %.0f%% |" % (
            r["kernel"], r["fetch"] / 1e9, r["write"] / 1e9, r["ms"], (r["fetch"] + r["write"]) / (r["ms"] * 1e9),
            r["valu"] / r["waves"] if r["waves"] else 0, 100 * busy))
    md.append("| **whole step** | %.3f | %.3f | %.3f | %.2f | | |" % (tot_f / 1e9, tot_w / 1e9, tot_ms,
                                                                       (tot_f + tot_w) / (tot_ms * 1e9)))
    md += ["", "The step moves %.2f GB of measured traffic in %.3f ms of serialised kernel time (%.2f TB/s); "
           "its algorithmic bytes are 2.609 GB (155.5 B per zone-update)." % ((tot_f + tot_w) / 1e9, tot_ms,
                                                                             (tot_f + tot_w) / (tot_ms * 1e9))]
    base = PROFILE_JSON[:-len(".json")]
    with open(base + ".md", "w") as fh:
        fh.write("\n".join(md) + "\n")
    summarize_trace(os.path.join(root, "trace"), sha)
    log("summarize: wrote %s(.json, .md)" % base)


def summarize_trace(root, sha):
    """profiles/turb256_512x32_kernel_stats.md from a --kernel-trace --stats run of TRACE_ARGS."""
    import csv

    stats = list(csv.DictReader(open(find_one(root, "*kernel_stats.csv"))))
    trace = list(csv.DictReader(open(find_one(root, "*kernel_trace.csv"))))
    bench = json.loads(open(os.path.join(root, "bench.json")).read().strip().splitlines()[-1])
    durs = {}
    for r in sorted(trace, key=lambda r: int(r["Start_Timestamp"])):
        durs.setdefault(short_name(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    md = ["# rocprofv3 kernel statistics: 256^3 turbulence as 512 patches of 32^3 (FP32 and FP64 batches)", "",
          "Command (TMPDIR=/tmp, run from /tmp; `<repo>` is the repository root):", "```",
          "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o run -- \\",
          "  python3 <repo>/bench.py " + TRACE_ARGS, "```",
          "Kernel source sha256 %s. Per precision the run does 1 warm-up step, 5 graph-replayed timed steps "
          "and 3 eager profiled steps (`wmb_profile_step`: the same launches, one kernel at a time), plus "
          "set-up and diagnostics kernels. `Avg` is rocprofv3's `AverageNs` over all calls: in the replayed "
          "steps the three sweeps of a stage run concurrently and share the GPU, so their average lies above "
          "the one-at-a-time time. `Eager` is the mean of each kernel's last 3 dispatches (the profiled "
          "steps). The last column is `bench.py`'s own HIP-event time for the kernel class in the same run "
          "(`kernels_ms`; FP32 `%s` ms/step, FP64 `%s` ms/step in the graph)." % (
              sha[:16], "%.3f" % bench["ms_per_step"], "%.3f" % bench["fp64"]["ms_per_step"]), "",
          "| Kernel | Calls | Avg (ms) | Min (ms) | Max (ms) | Eager (ms) | bench.py HIP-event (ms) |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    km = {"float": bench.get("kernels_ms") or {}, "double": (bench.get("fp64") or {}).get("kernels_ms") or {}}
    seen = set()
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        nm = short_name(r["Name"])
        cls = kernel_class(nm)
        prec = "double" if "<double" in nm else "float"
        eager = durs.get(nm, [])[-3:]
        hip = ""
        if cls and (prec, cls) not in seen and cls in km[prec]:
            hip = "%.3f" % km[prec][cls]
            seen.add((prec, cls))
        md.append("| `%s` | %s | %.4f | %.4f | %.4f | %s | %s |" % (
            nm, r["Calls"], float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            "%.4f" % (sum(eager) / len(eager)) if eager else "", hip))
    md += ["", "`bench.py`'s class times sum the launches of a class in a step (the fill's y and z passes; the "
           "Step-1 x sweep's launches); its column sits on the class's first row."]
    with open(os.path.join(ROOT, "profiles", "turb256_512x32_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")


# ---------------------------------------------------------------------------
# CPU baseline (the oracle as it stands)
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(q, b, dx, ghost, budget_s=12.0):
    """The FP64 oracle as it stands, timed on this host's cores on a bounded
    sample: a 2x2xk block of the workload's 32^3 patches (periodic sample box),
    one warm-up step then timed steps until about budget_s seconds.  Also the
    one-patch linear-wave case (32^3, 10 steps) in CPU seconds."""
    import numpy as np

    from oracle import OracleSim, default_params
    from paper_1701_07452_amd import inputs as I

    nblk = int(os.environ.get("WMB_CPU_SAMPLE_PATCHES", "16"))
    kz = max(1, nblk // 4)
    sub = I.uniform_grid((64, 64, 32 * kz), 32)
    qs = np.ascontiguousarray(q[:, :32 * kz, :64, :64])
    bs = np.ascontiguousarray(b[:, :32 * kz, :64, :64])
    orc = OracleSim(default_params(dx=dx, ghost=ghost), sub.descs)
    for ip, (qp, bp) in enumerate(I.split(sub, qs, bs)):
        orc.set_state(ip, qp, bp)
    orc.run_steps(1)
    steps, t0 = 0, time.perf_counter()
    while True:
        orc.run_steps(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 50:
            break
    zones = sub.zones()
    threads = orc.num_threads()
    orc.close()
    # one periodic 32^3 patch, linear fast wave, FP64, 10 steps (the oracle
    # runs patches in parallel, so one patch runs on one core)
    qw, bw, _ = I.fast_wave_diagonal(32)
    Gw = I.uniform_grid(32, 32)
    ow = OracleSim(default_params(dx=(1 / 32,) * 3), Gw.descs)
    ow.set_state(0, qw, bw)
    c0 = time.process_time()
    w0 = time.perf_counter()
    ow.run_steps(10)
    c1_wall = time.perf_counter() - w0
    c1_cpu = time.process_time() - c0
    ow.close()
    # the same 32^3 box as 8 patches of 16^3 on all the oracle's threads
    G8 = I.uniform_grid(32, 16)
    o8 = OracleSim(default_params(dx=(1 / 32,) * 3), G8.descs)
    for ip, (qp, bp) in enumerate(I.split(G8, qw, bw)):
        o8.set_state(ip, qp, bp)
    c0 = time.process_time()
    w0 = time.perf_counter()
    o8.run_steps(10)
    c8_wall = time.perf_counter() - w0
    c8_cpu = time.process_time() - c0
    c8_threads = min(o8.num_threads(), G8.npatch)
    o8.close()
    return {
        "value": zones * steps / el,
        "unit": "zone-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d patches of 32^3 (%d zones) cut from the workload, periodic sample box, FP64, %d steps in %.1f s"
                  % (sub.npatch, zones, steps, el),
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "linear_wave_32cubed_10_steps": {"wall_s": round(c1_wall, 3), "cpu_s": round(c1_cpu, 3), "cores_used": 1,
                                         "note": "one patch: the oracle parallelises over patches only"},
        "linear_wave_32cubed_10_steps_8x16cubed": {"wall_s": round(c8_wall, 3), "cpu_s": round(c8_cpu, 3),
                                                   "cores_used": c8_threads,
                                                   "note": "the same box as 8 patches of 16^3, one a thread"},
    }


# ---------------------------------------------------------------------------
# one batch on the GPU
# ---------------------------------------------------------------------------

def free_device_memory():
    import gc

    import torch

    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def make_sim(W, G, q, b, dx, prec, ghost, stream, **params):
    from paper_1701_07452_amd import inputs as I

    sim = W.Sim(W.make_params(dx=dx, precision=prec, ghost=ghost, **params), G.descs, origins=G.origin, stream=stream)
    for ip, (qp, bp) in enumerate(I.iter_split(G, q, b)):
        sim.set_state(ip, qp, bp)
    return sim


SCHEDULE = 0  # captured-step schedule: 0 picks 1, 2 or 3 patch groups by timing during the warm-up


def pick_schedule(sim, stream, reps=3):
    """Time `reps` graph replays under 1, 2 and 3 patch groups (warm-up steps:
    the state advances) and keep the fastest; returns {groups: ms per step}."""
    import torch

    times = {}
    for groups in (1, 2, 3):
        sim.set_schedule(groups)
        sim.run_steps(1)  # captures the graphs of this schedule
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.run_steps(reps)
        e1.record(stream)
        stream.synchronize()
        times[groups] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    sim.set_schedule(best)
    return best, times


def run_batch(W, G, q, b, dx, prec, ghost, steps, warmup, prof_steps, tuning=None, freeze=(), divb_at=(), **params):
    """Time `steps` graph replays after `warmup` ones; per-kernel eager
    durations from prof_steps profiled steps; optionally the normalised div b
    of a fresh run after each step count in divb_at."""
    import torch

    stream = torch.cuda.Stream()
    sim = make_sim(W, G, q, b, dx, prec, ghost, stream, **params)
    if tuning:
        sim.set_tuning(tuning)
    else:
        tuning = sim.autotune(reps=3)
    log("bench: pencils per block %s" % W.tuning_to_str(tuning))
    if params.get("scratch_groups", 0) > 1:  # the schedule is the scratch groups, one after another
        groups, sched_ms = params["scratch_groups"], None
    elif SCHEDULE:
        groups, sched_ms = SCHEDULE, None
        sim.set_schedule(groups)
    else:
        groups, sched_ms = pick_schedule(sim, stream)
    log("bench: schedule %d patch group(s) %s" % (groups, "" if sched_ms is None else
                                                   {g: round(t, 3) for g, t in sched_ms.items()}))
    sim.run_steps(max(warmup, 1))  # captures the graphs
    stream.synchronize()
    freeze_ms = None
    if freeze:
        # freeze patches between graph replays: the same graphs run on
        t0 = time.perf_counter()
        for ip in freeze:
            sim.set_active(ip, False)
        freeze_ms = (time.perf_counter() - t0) * 1e3 / len(freeze)
        sim.run_steps(1)
        stream.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.run_steps(steps)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    # per-kernel durations: the same launches, HIP events after every kernel class
    kern = None
    for _ in range(prof_steps):
        k = sim.profile_step()
        kern = {c: kern[c] + k[c] for c in k} if kern else k
    if kern:
        kern = {c: v / prof_steps for c, v in kern.items()}
    tot, dn, dr, nfl = sim.diagnostics()
    nprot = sim.protected_faces()
    sim.close()
    diag = {"max_divb_norm": dn, "max_divb_raw": dr, "floors": nfl, "protected_faces": nprot,
            "tuning": W.tuning_to_str(tuning), "schedule_groups": groups, "schedule_ms": sched_ms}
    if freeze:
        diag["freeze_ms_per_patch"] = freeze_ms
    if divb_at:
        # normalised div b against the step count, from the initial state
        sim = make_sim(W, G, q, b, dx, prec, ghost, stream, **params)
        sim.set_tuning(tuning)
        if params.get("scratch_groups", 0) <= 1:
            sim.set_schedule(groups)
        done, curve = 0, {}
        for n in sorted(divb_at):
            sim.run_steps(n - done)
            done = n
            _, dnn, _, _ = sim.diagnostics()
            curve[str(n)] = dnn
        sim.close()
        diag["divb_norm_vs_steps"] = curve
    del sim
    free_device_memory()
    return ms, wall, kern, diag


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ghost", type=int, default=4)
    ap.add_argument("--prof-steps", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning32", default="", help="sweep shapes for FP32 (e.g. 1x32=16,...); default: autotune")
    ap.add_argument("--tuning64", default="", help="sweep shapes for FP64; default: autotune")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven 400-patch batch (reported beside)")
    ap.add_argument("--no-c4", action="store_true", help="skip the 512^3 Orszag-Tang batch of 64^3 patches")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the 768^3 high-contrast batch of 48^3 patches (210 GB pool, about a minute of set-up)")
    ap.add_argument("--protection", action="store_true",
                    help="also time the Mach-5 lognormal-density batch (384^3 as 512 x 48^3, FP32) with the protection "
                         "floors off and on (reported beside)")
    ap.add_argument("--outflow", action="store_true",
                    help="also time the FP32 batch with outflow boundaries on every side of the domain")
    ap.add_argument("--frozen", action="store_true",
                    help="also time the FP32 batch with every other patch frozen (checkerboard), graphs reused")
    ap.add_argument("--no-divb", action="store_true", help="skip the div b against step count runs")
    ap.add_argument("--no-scratch-groups", action="store_true",
                    help="skip the FP32 batch with the step intermediates shared by 4 patch groups (reported beside)")
    ap.add_argument("--planar", action="store_true",
                    help="also time the planar Orszag-Tang vortex (192^2 and 2048^2) run as one-patch-thin 3D boxes")
    ap.add_argument("--patch-sweep", action="store_true",
                    help="also time the FP32 turbulence box cut into patches of 16, 24, 32, 48 and 64 zones an edge")
    ap.add_argument("--schedule", type=int, default=0,
                    help="captured-step schedule: 1 (concurrent sweep branches), 2 or 3 patch groups; 0 picks by timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--summarize-counters", metavar="DIR", default="",
                    help="no run: summarise the rocprofv3 passes under DIR into profiles/")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU sharding is a documented design, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    W.load_library()
    global SCHEDULE
    SCHEDULE = args.schedule
    t_start = time.perf_counter()

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prof = profile_record()
    N, n, g = 256, 32, args.ghost
    dx = (1.0 / N,) * 3
    log("bench: building the 256^3 turbulence state")
    q, b = I.turbulence(N)
    G = I.uniform_grid(N, n)
    zones = G.zones()
    divb_at = (10, 20, 50) if args.prof_steps > 0 and not args.no_divb else ()

    log("bench: FP32 batch, %d warm-up + %d timed steps" % (args.warmup, args.steps))
    ms32, wall32, kern32, diag32 = run_batch(W, G, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, args.prof_steps,
                                             W.tuning_from_str(args.tuning32), divb_at=divb_at)
    value = zones * args.steps / (ms32 / 1e3)
    log("bench: FP32 %.3f ms/step, %.3e zone-updates/s" % (ms32 / args.steps, value))
    fp64 = None
    if not args.no_fp64:
        log("bench: FP64 batch")
        ms64, wall64, kern64, diag64 = run_batch(W, G, q, b, dx, W.WMB_FP64, g, args.steps, args.warmup,
                                                 args.prof_steps, W.tuning_from_str(args.tuning64))
        fp64 = {"value": zones * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps, "dtype": "f64",
                "kernels_ms": kern64, **diag64}
        if kern64:
            fp64["roofline"] = roofline(G.descs, g, 8, zones, ms64 / args.steps, kern64)
        log("bench: FP64 %.3f ms/step" % (ms64 / args.steps))

    uneven = None
    if not args.no_uneven and args.prof_steps > 0:
        # the uneven batch (patch edges from {16, 24, 32, 48, 64} per slab, 8 x 10 x 5
        # patches, turbulence seed 170107454, dx = 1/256): FP32, reported beside
        Gu = I.uneven_grid()
        Nz, Ny, Nx = Gu.shape
        log("bench: uneven batch, %d patches, %d zones" % (Gu.npatch, Gu.zones()))
        qu, bu = I.turbulence(None, seed=170107454, shape=Gu.shape, box=(Nx / 256, Ny / 256, Nz / 256))
        msu, wallu, kernu, diagu = run_batch(W, Gu, qu, bu, (1.0 / 256,) * 3, W.WMB_FP32, g, args.steps,
                                             args.warmup, 1)
        del qu, bu
        uneven = {"workload": "uneven batch: 400 patches, 8 x 10 x 5 slabs with edges from {16,24,32,48,64}, "
                              "turbulence, ghost %d, FP32" % g,
                  "zones": Gu.zones(), "patches": Gu.npatch, "ms_per_step": msu / args.steps,
                  "value": Gu.zones() * args.steps / (msu / 1e3), "kernels_ms": kernu, **diagu,
                  "roofline": roofline(Gu.descs, g, 4, Gu.zones(), msu / args.steps, kernu)}
        log("bench: uneven FP32 %.3f ms/step, %.3e zone-updates/s" % (msu / args.steps, uneven["value"]))

    shared = None
    if not args.no_scratch_groups and args.prof_steps > 0:
        # the same batch with the step intermediates shared by 4 patch groups
        # whose steps run one after another: a smaller pool for a slower step
        log("bench: FP32 batch with 4 scratch groups")
        mss, _, kerns, diags = run_batch(W, G, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, 1,
                                         W.tuning_from_str(args.tuning32), scratch_groups=4)
        p1 = W.pool_bytes(W.make_params(dx=dx, precision=W.WMB_FP32, ghost=g), G.descs)
        p4 = W.pool_bytes(W.make_params(dx=dx, precision=W.WMB_FP32, ghost=g, scratch_groups=4), G.descs)
        shared = {"workload": "the FP32 batch with scratch_groups = 4 (22 + 51/4 words a ghosted zone)",
                  "pool_bytes": p4, "pool_bytes_default": p1, "ms_per_step": mss / args.steps,
                  "value": zones * args.steps / (mss / 1e3), "kernels_ms": kerns, **diags}
        log("bench: scratch groups 4: %.3f ms/step, pool %.2f GB against %.2f GB" % (mss / args.steps, p4 / 1e9,
                                                                                    p1 / 1e9))

    c4 = None
    if not args.no_c4 and args.prof_steps > 0:
        N4, n4, s4 = 512, 64, 50
        G4 = I.uniform_grid(N4, n4)
        log("bench: 512^3 Orszag-Tang batch, %d patches of 64^3" % G4.npatch)
        q4, b4 = I.orszag_tang_3d(N4)
        ms4, _, kern4, diag4 = run_batch(W, G4, q4, b4, (1.0 / N4,) * 3, W.WMB_FP32, g, s4, args.warmup, 1,
                                         divb_at=(10, 20, 50))
        del q4, b4
        c4 = {"workload": "3D Orszag-Tang extension, 512^3 as 512 patches of 64^3, ghost %d, FP32, %d graph-replayed "
                          "steps" % (g, s4),
              "zones": G4.zones(), "patches": G4.npatch, "steps": s4, "ms_per_step": ms4 / s4,
              "value": G4.zones() * s4 / (ms4 / 1e3), "kernels_ms": kern4, **diag4,
              "roofline": roofline(G4.descs, g, 4, G4.zones(), ms4 / s4, kern4)}
        log("bench: C4 FP32 %.3f ms/step, %.3e zone-updates/s" % (ms4 / s4, c4["value"]))

    c5 = None
    if not args.no_c5 and args.prof_steps > 0:
        N5, n5 = 768, 48
        G5 = I.uniform_grid(N5, n5)
        log("bench: 768^3 high-contrast batch, %d patches of 48^3" % G5.npatch)
        q5, b5 = I.high_contrast_turbulence(N5, workers=-1)
        ms5, _, kern5, diag5 = run_batch(W, G5, q5, b5, (1.0 / N5,) * 3, W.WMB_FP32, g, args.steps, args.warmup, 1,
                                         rho_floor=1e-8, p_floor=1e-8)
        del q5, b5
        c5 = {"workload": "high-contrast turbulence (lognormal rho, sigma 1.5, Mach 5, beta 1), 768^3 as 4096 patches "
                          "of 48^3, ghost %d, FP32, FP64 floors 1e-8" % g,
              "zones": G5.zones(), "patches": G5.npatch, "ms_per_step": ms5 / args.steps,
              "value": G5.zones() * args.steps / (ms5 / 1e3), "kernels_ms": kern5, **diag5,
              "roofline": roofline(G5.descs, g, 4, G5.zones(), ms5 / args.steps, kern5)}
        log("bench: C5 FP32 %.3f ms/step, %.3e zone-updates/s" % (ms5 / args.steps, c5["value"]))

    protection = None
    if args.protection:
        Nh = 384
        Gh = I.uniform_grid(Nh, 48)
        log("bench: Mach-5 lognormal batch %d^3 as %d x 48^3" % (Nh, Gh.npatch))
        qh, bh = I.high_contrast_turbulence(Nh)
        protection = {"workload": "Mach-5 solenoidal turbulence, lognormal rho (sigma 1.5), beta 1, %d^3 as %d "
                                  "patches of 48^3, ghost %d, FP32, floors 1e-8" % (Nh, Gh.npatch, g)}
        for tag, pf in (("off", 0.0), ("on", 1e-4)):
            msh, _, kernh, diagh = run_batch(W, Gh, qh, bh, (1.0 / Nh,) * 3, W.WMB_FP32, g, 10, args.warmup, 1,
                                             rho_floor=1e-8, p_floor=1e-8, rho_protect=pf, p_protect=pf)
            protection[tag] = {"protect_floor": pf, "ms_per_step": msh / 10, "value": Gh.zones() * 10 / (msh / 1e3),
                               "kernels_ms": kernh, **diagh}
            log("bench: protection %s: %.3f ms/step, %d protected faces, %d floors" %
                (tag, msh / 10, diagh["protected_faces"], diagh["floors"]))
        del qh, bh

    outflow = None
    if args.outflow:
        Go = I.uniform_grid(N, n, periodic=(False, False, False))
        log("bench: FP32 batch with outflow on every side")
        mso, _, kerno, diago = run_batch(W, Go, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, 1,
                                         W.tuning_from_str(args.tuning32) or None)
        outflow = {"workload": "the FP32 batch with outflow (zero-gradient) boundaries on all six sides",
                   "ms_per_step": mso / args.steps, "value": zones * args.steps / (mso / 1e3), "kernels_ms": kerno,
                   **diago}
        log("bench: outflow: %.3f ms/step, %.3e zone-updates/s" % (mso / args.steps, outflow["value"]))

    frozen = None
    if args.frozen:
        px, py, pz = G.nblocks
        half = [(k * py + j) * px + i for k in range(pz) for j in range(py) for i in range(px) if (i + j + k) % 2]
        log("bench: FP32 batch with %d of %d patches frozen" % (len(half), G.npatch))
        msf, _, kernf, diagf = run_batch(W, G, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, 1,
                                         W.tuning_from_str(args.tuning32) or None, freeze=half)
        active = zones - len(half) * n ** 3
        frozen = {"workload": "the FP32 batch with every other patch (checkerboard) frozen after graph capture",
                  "frozen_patches": len(half), "active_zones": active, "ms_per_step": msf / args.steps,
                  "value": active * args.steps / (msf / 1e3), "kernels_ms": kernf, **diagf}
        log("bench: frozen half: %.3f ms/step, %.3e active zone-updates/s, %.2f ms per set_active" %
            (msf / args.steps, frozen["value"], diagf["freeze_ms_per_patch"]))

    planar = None
    if args.planar:
        # planar problems run as 3D boxes one patch thin (5 zones, periodic) across z
        planar = {"workload": "planar Orszag-Tang vortex as an N x N x 5 box of 32 x 32 x 5 patches, ghost %d, "
                              "FP32; per planar zone-update and per stored 3D zone-update" % g}
        for N2 in (192, 2048):
            G2 = I.patch_grid([32] * (N2 // 32), [32] * (N2 // 32), [5])
            q2, b2 = I.orszag_tang_2d(N2)
            log("bench: planar Orszag-Tang %d^2 as %d patches of 32 x 32 x 5" % (N2, G2.npatch))
            ms2, _, kern2, diag2 = run_batch(W, G2, q2, b2, (1.0 / N2,) * 3, W.WMB_FP32, g, args.steps, args.warmup,
                                             1)
            del q2, b2
            planar[str(N2)] = {"ms_per_step": ms2 / args.steps, "patches": G2.npatch,
                               "planar_zone_updates_per_s": N2 * N2 * args.steps / (ms2 / 1e3),
                               "zone_updates_per_s_3d": G2.zones() * args.steps / (ms2 / 1e3),
                               "kernels_ms": kern2, **diag2}
            log("bench: planar %d^2: %.3f ms/step, %.3e planar zone-updates/s" %
                (N2, ms2 / args.steps, planar[str(N2)]["planar_zone_updates_per_s"]))

    sweep = None
    if args.patch_sweep:
        # the same turbulence recipe cut into cubic patches of each edge: 256^3
        # where the edge divides it, else 240^3
        sweep = {"workload": "turbulence box (256^3, or 240^3 for edges 24 and 48) as periodic cubic patches, "
                             "ghost %d, FP32, autotuned" % g}
        for e in (16, 24, 32, 48, 64):
            Ne = 256 if 256 % e == 0 else 240
            Ge = I.uniform_grid(Ne, e)
            qe, be = I.turbulence(Ne)
            log("bench: patch sweep %d^3 as %d patches of %d^3" % (Ne, Ge.npatch, e))
            mse, _, kerne, diage = run_batch(W, Ge, qe, be, (1.0 / Ne,) * 3, W.WMB_FP32, g, args.steps, args.warmup, 1)
            del qe, be
            sweep[str(e)] = {"box": Ne, "patches": Ge.npatch, "ms_per_step": mse / args.steps,
                             "value": Ge.zones() * args.steps / (mse / 1e3), "kernels_ms": kerne,
                             "tuning": diage["tuning"], "schedule_groups": diage["schedule_groups"]}
            log("bench: patch sweep edge %d: %.3f ms/step, %.3e zone-updates/s" %
                (e, mse / args.steps, sweep[str(e)]["value"]))

    if not kern32:  # counter-collection runs skip the per-kernel pass
        print(json.dumps({"metric": METRIC, "value": value, "unit": "zone-updates/s", "partial": True}), flush=True)
        return
    roof = roofline(G.descs, g, 4, zones, ms32 / args.steps, kern32, prof)
    if prof:
        roof["valu_busy_sweeps"] = {k: v.get("valu_busy") for k, v in prof["per_class"].items() if k.startswith("sweep")}
        roof["profile"] = os.path.relpath(PROFILE_JSON, ROOT)
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU baseline (oracle)")
        cpu = cpu_baseline(q, b, dx, g)
        log("bench: CPU %.3e zone-updates/s on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "turbulence 256^3 as 512 patches of 32^3, ghost 4, FP32 sweeps+CT, FP64 dt/floors, 20-step run",
            "zones": zones, "patches": G.npatch, "patch_edge": n, "ghost": g, "gamma": 5.0 / 3.0, "cfl": 0.4,
            "rms_mach": 1.0, "B0": [0.1, 0.0, 0.0], "seed": 170107452,
        },
        "wall_s_timed": wall32,
        "kernels_ms": kern32,
        "fp32_diag": diag32,
        "fp64": fp64,
        "uneven_fp32": uneven,
        "scratch_groups_fp32": shared,
        "c4_fp32": c4,
        "c5_fp32": c5,
        "protection_fp32": protection,
        "frozen_half_fp32": frozen,
        "outflow_fp32": outflow,
        "planar_fp32": planar,
        "patch_sweep_fp32": sweep,
        "roofline": roof,
        "cpu_baseline": cpu,
        "bench_wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
