#!/usr/bin/env python3
"""Benchmark: zone-updates/s of the patch MHD update on one MI355X.

Workload: 3D periodic 256^3 box as 512 patches of 32^3 (ghost width 4, the
stencil minimum), rho = 1, P = 1, B = (0.1, 0, 0), seeded Gaussian random
velocity with a k^-5/3 spectrum at rms Mach 1, gamma = 5/3, CFL 0.4.
One step = ghost exchange + FP64 CFL reduction + the full CTU+CT MHDTVD
update (Steps 1-11) of all patches, replayed from a captured HIP graph, with
the state resident in HBM.  The headline value is the FP32 batch (FP32 sweeps
and CT, FP64 dt and floors); the FP64 batch is reported beside it.

Prints ONE JSON line.  --gpus > 1 is not supported (one GPU per process; the
multi-GPU design is documented, not built).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec on 1 MI355X (FP32 batched vs FP64 plain) + % HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic bytes per launch of each kernel class (unique words each launch
# must read or write at least once, times the word size)
# ---------------------------------------------------------------------------

def alg_bytes(kclass, n, g, es, npatch):
    """n: interior edge, g: ghost width, es: bytes per word (uniform patches)."""
    def box(lo, hi):
        return (n + hi - lo + 1) ** 3

    N = n + 2 * g
    if kclass == "fill":
        # y and z passes (the step before wrote the x-ghosts): 11 words read +
        # 11 written per ghost zone of whole y-ghost rows and z-ghost planes
        per = 22 * (2 * g * N * n + 2 * g * N * N)
    elif kclass == "dt":
        per = 0                                          # finalize only: the reduction is folded into "update"
    elif kclass.startswith("sweep1"):
        T, P = n + 6, n + 8
        per = 9 * P * T * T + 7 * (P - 3) * T * T        # q + b_par in; 7 flux rows out
        if kclass == "sweep1_x":
            per += 3 * box(-3, 2)                        # and the Step-2 reference EMF
    elif kclass.startswith("sweep2"):
        T, P = n + 2, n + 6
        per = (8 + 2 * 7 + 3 + 1) * P * T * T + 7 * (P - 3) * T * T  # q, 2 transverse fluxes, b, b^{n+1/2}; flux out
    elif kclass == "ct_half":
        # Steps 3-4 fused: Step-1 flux rows 0, 5, 6 (3 dirs), E^r and b^n in,
        # b^{n+1/2} out, over the box [-2, n+2]^3
        per = (9 + 3 + 3 + 3) * box(-2, 2)
    elif kclass == "update":
        # Steps 8-11 fused: q^n rho, m + flux rows 0-3 + b^{n+1/2} over the E^r
        # box [-1, n]; flux rows 5-6 over the edge box [0, n]; q^n E, flux row 4,
        # b^n in and q^{n+1}, b^{n+1} out over the interior
        per = (4 + 12 + 3) * box(-1, 0) + 6 * box(0, 0) + (1 + 3 + 3 + 11) * n ** 3
        per += 11 * 2 * g * n * n                        # the x-ghosts it writes into the neighbours
    else:
        raise KeyError(kclass)
    return per * es * npatch


def measured_traffic(kclass):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when the kernel
    source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "turb256_512x32_fp32_hbm_traffic.json")
    src = os.path.join(ROOT, "paper_1701_07452_amd", "csrc", "wmb_kernels.hip")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_source_sha256") != cur or kclass not in rec.get("per_launch_bytes", {}):
        return None
    return rec["per_launch_bytes"][kclass]["total"]


def cpu_baseline(q, b, G, dx, ghost, budget_s=12.0):
    """The FP64 oracle as it stands, timed on this host's cores on a bounded
    sample: a 2x2xk block of the workload's 32^3 patches (periodic sample box),
    one warm-up step then timed steps until about budget_s seconds."""
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
    return {
        "value": zones * steps / el,
        "unit": "zone-updates/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": "%d patches of 32^3 (%d zones) cut from the workload, periodic sample box, FP64, %d steps in %.1f s"
                  % (sub.npatch, zones, steps, el),
    }


def run_precision(W, G, q, b, dx, prec, ghost, steps, warmup, prof_steps, tuning=None, freeze=(), **params):
    import torch

    from paper_1701_07452_amd import inputs as I

    stream = torch.cuda.Stream()
    sim = W.Sim(W.make_params(dx=dx, precision=prec, ghost=ghost, **params), G.descs, origins=G.origin, stream=stream)
    for ip, (qp, bp) in enumerate(I.split(G, q, b)):
        sim.set_state(ip, qp, bp)
    if tuning:
        sim.set_tuning(tuning)
    else:
        tuning = sim.autotune(reps=3)
    log("bench: pencils per block %s" % W.tuning_to_str(tuning))
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
    extra = {"freeze_ms_per_patch": freeze_ms} if freeze else {}
    return ms, wall, kern, {"max_divb_norm": dn, "max_divb_raw": dr, "floors": nfl, "protected_faces": nprot,
                            "tuning": W.tuning_to_str(tuning), **extra}


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
    ap.add_argument("--protection", action="store_true",
                    help="also time the Mach-5 lognormal-density batch (384^3 as 512 x 48^3, FP32) with the protection "
                         "floors off and on (reported beside)")
    ap.add_argument("--outflow", action="store_true",
                    help="also time the FP32 batch with outflow boundaries on every side of the domain")
    ap.add_argument("--frozen", action="store_true",
                    help="also time the FP32 batch with every other patch frozen (checkerboard), graphs reused")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU sharding is a documented design, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1701_07452_amd import inputs as I
    from paper_1701_07452_amd import wmb as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    W.load_library()

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    N, n, g = 256, 32, args.ghost
    dx = (1.0 / N,) * 3
    log("bench: building the 256^3 turbulence state")
    q, b = I.turbulence(N)
    G = I.uniform_grid(N, n)
    zones = G.zones()

    log("bench: FP32 batch, %d warm-up + %d timed steps" % (args.warmup, args.steps))
    ms32, wall32, kern32, diag32 = run_precision(W, G, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, args.prof_steps,
                                                 W.tuning_from_str(args.tuning32))
    value = zones * args.steps / (ms32 / 1e3)
    log("bench: FP32 %.3f ms/step, %.3e zone-updates/s" % (ms32 / args.steps, value))
    fp64 = None
    if not args.no_fp64:
        log("bench: FP64 batch")
        ms64, wall64, kern64, diag64 = run_precision(W, G, q, b, dx, W.WMB_FP64, g, args.steps, args.warmup,
                                                     args.prof_steps, W.tuning_from_str(args.tuning64))
        fp64 = {"value": zones * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps,
                "kernels_ms": kern64, **diag64}
        log("bench: FP64 %.3f ms/step" % (ms64 / args.steps))

    uneven = None
    if not args.no_uneven and args.prof_steps > 0:
        # the uneven batch (patch edges from {16, 24, 32, 48, 64} per slab, 8 x 10 x 5
        # patches, turbulence seed 170107454, dx = 1/256): FP32, reported beside
        Gu = I.uneven_grid()
        Nz, Ny, Nx = Gu.shape
        log("bench: uneven batch, %d patches, %d zones" % (Gu.npatch, Gu.zones()))
        qu, bu = I.turbulence(None, seed=170107454, shape=Gu.shape, box=(Nx / 256, Ny / 256, Nz / 256))
        msu, wallu, kernu, diagu = run_precision(W, Gu, qu, bu, (1.0 / 256,) * 3, W.WMB_FP32, g, args.steps,
                                                 args.warmup, 1)
        del qu, bu
        uneven = {"workload": "uneven batch: 400 patches, 8 x 10 x 5 slabs with edges from {16,24,32,48,64}, "
                              "turbulence, ghost %d, FP32" % g,
                  "zones": Gu.zones(), "patches": Gu.npatch, "ms_per_step": msu / args.steps,
                  "value": Gu.zones() * args.steps / (msu / 1e3), "kernels_ms": kernu, **diagu}
        log("bench: uneven FP32 %.3f ms/step, %.3e zone-updates/s" % (msu / args.steps, uneven["value"]))

    protection = None
    if args.protection:
        Nh = 384
        Gh = I.uniform_grid(Nh, 48)
        log("bench: Mach-5 lognormal batch %d^3 as %d x 48^3" % (Nh, Gh.npatch))
        qh, bh = I.high_contrast_turbulence(Nh)
        protection = {"workload": "Mach-5 solenoidal turbulence, lognormal rho (sigma 1.5), beta 1, %d^3 as %d "
                                  "patches of 48^3, ghost %d, FP32, floors 1e-8" % (Nh, Gh.npatch, g)}
        for tag, pf in (("off", 0.0), ("on", 1e-4)):
            msh, _, kernh, diagh = run_precision(W, Gh, qh, bh, (1.0 / Nh,) * 3, W.WMB_FP32, g, 10, args.warmup, 1,
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
        mso, _, kerno, diago = run_precision(W, Go, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, 1,
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
        msf, _, kernf, diagf = run_precision(W, G, q, b, dx, W.WMB_FP32, g, args.steps, args.warmup, 1,
                                             W.tuning_from_str(args.tuning32) or None, freeze=half)
        active = zones - len(half) * n ** 3
        frozen = {"workload": "the FP32 batch with every other patch (checkerboard) frozen after graph capture",
                  "frozen_patches": len(half), "active_zones": active, "ms_per_step": msf / args.steps,
                  "value": active * args.steps / (msf / 1e3), "kernels_ms": kernf, **diagf}
        log("bench: frozen half: %.3f ms/step, %.3e active zone-updates/s, %.2f ms per set_active" %
            (msf / args.steps, frozen["value"], diagf["freeze_ms_per_patch"]))

    if not kern32:  # counter-collection runs skip the per-kernel pass
        print(json.dumps({"metric": METRIC, "value": value, "unit": "zone-updates/s", "partial": True}), flush=True)
        return
    # roofline of the dominant kernel class (FP32 batch)
    dom = max(kern32, key=kern32.get)
    per_launch = alg_bytes(dom, n, g, 4, G.npatch)
    achieved = per_launch / (kern32[dom] * 1e-3) / 1e9
    step_bytes = sum(alg_bytes(k, n, g, 4, G.npatch) for k in kern32)
    traffic = measured_traffic(dom)
    roof = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_GBs": round(traffic / (kern32[dom] * 1e-3) / 1e9, 1) if traffic else None,
        "alg_bytes_per_launch": per_launch,
        "avg_launch_ms": kern32[dom],
        "step_alg_bytes": step_bytes,
        "step_alg_frac": round(step_bytes / (ms32 / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU baseline (oracle)")
        cpu = cpu_baseline(q, b, G, dx, g)
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
        "protection_fp32": protection,
        "frozen_half_fp32": frozen,
        "outflow_fp32": outflow,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
