"""Benchmark: zone-updates/s of the FP64 SSP-RK3 step on the 256^3 turbulent
SRMHD box (one MI355X), with the dominant kernel's roofline and the FP64
oracle timed on the host as a CPU baseline.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--precision fp64|fp32]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 128 FP64 flop/clk
FP32_VECTOR_PEAK_TFLOPS = 157.3


def algorithmic_units():
    """Per-unit algorithmic figures of each kernel class (opcounts.json):
    FP64 flops per face/edge/zone counted from the kernel arithmetic, and the
    compulsory HBM bytes per element."""
    path = os.path.join(ROOT, "paper_1810_04597_amd", "opcounts.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def measured_traffic(kernel):
    """HBM bytes per launch from the counter passes, or None when the kernel
    sources changed since they were taken."""
    t = _traffic_table()
    if t is None:
        return None
    k = t["kernels"].get(kernel)
    return None if k is None else k["bytes"]


def _traffic_table():
    path = os.path.join(ROOT, "paper_1810_04597_amd", "traffic.json")
    if not os.path.exists(path):
        return None
    from paper_1810_04597_amd.traffic import source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None
    return t


# Compulsory HBM bytes per interior zone of one SSP-RK3 stage when a stage
# reads and writes the state once: stage 1 reads P^n and U^n and writes U^(1)
# and P^(1) (4 x 8 FP64 fields); stages 2 and 3 also read U^n beside the
# current stage state (5 x 8 fields).  896 bytes per zone per step.
STAGE_BYTES = (256.0, 320.0, 320.0)
STEP_BYTES = sum(STAGE_BYTES)


def launch_units(kernel, n):
    """Number of units (faces, edges or zones) one launch of `kernel` processes."""
    g = 5
    ng = n + 2 * g
    if kernel.startswith("sweep"):
        return (n + 5) * ng * ng
    if kernel.startswith("edge"):
        return (n + 5) * (n + 5) * n
    return n ** 3


def rooflines(prof, n, steps, ms_step, precision):
    """(roofline of the dominant kernel, roofline of the whole step, per-kernel
    figures) from the HIP-event profile {class: (total ms, launches)} of
    `steps` steps.

    Dominant kernel (largest total time): when it is the stage update, its
    algorithmic bytes are the stage's compulsory bytes (the mean of
    STAGE_BYTES per zone, n^3 zones per launch), which credits it with the
    state traffic of the whole stage; another dominant kernel is priced at its
    own compulsory bytes per face, edge or zone (opcounts.json).  `traffic` is
    the counter-measured HBM bytes per launch of that kernel (None when the
    kernel sources changed since the counters were taken) and
    traffic_over_algorithmic their ratio.
    Step: STEP_BYTES per zone over the step time, and the counter-measured
    bytes of every launch of a step (sum over classes of bytes per launch x
    launches per step) over the same time."""
    if not prof:
        return None, None, {}
    units = algorithmic_units()
    tot_ms = sum(v[0] for v in prof.values())
    kernels = {}
    for k, (tot, cnt) in prof.items():
        kernels[k] = {"avg_ms": tot / cnt, "launches": cnt, "share": tot / tot_ms}
        u = units.get(k, {})
        if "bytes" in u and k != "update":
            kb = u["bytes"] * launch_units(k, n)
            kernels[k]["own_bytes_per_launch"] = kb
            kernels[k]["own_GBs"] = kb / (tot / cnt / 1e3) / 1e9
    zones = n ** 3
    dom = max(prof, key=lambda k: prof[k][0])
    avg_s = prof[dom][0] / prof[dom][1] / 1e3
    traffic = measured_traffic(dom) if n == 256 and precision == "fp64" else None
    if dom == "update":
        alg = sum(STAGE_BYTES) / len(STAGE_BYTES) * zones
        basis = "stage compulsory bytes, mean of %s B/zone x %d zones" % (list(STAGE_BYTES), zones)
    else:
        alg = units.get(dom, {}).get("bytes", float("nan")) * launch_units(dom, n)
        basis = "kernel's own compulsory bytes per unit x units per launch"
    achieved = alg / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "avg_ms": avg_s * 1e3, "algorithmic_bytes_per_launch": alg, "basis": basis,
                "traffic_over_algorithmic": (traffic / alg) if traffic else None}
    step_alg = STEP_BYTES * zones
    step = {"algorithmic_bytes": step_alg, "ms": ms_step,
            "achieved": step_alg / (ms_step / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    step["frac"] = step["achieved"] / HBM_PEAK_GBS
    t = _traffic_table() if n == 256 and precision == "fp64" else None
    if t is not None and all(k in t["kernels"] for k in prof if k != "advance"):
        meas = sum(t["kernels"][k]["bytes"] * prof[k][1] / steps for k in prof if k != "advance")
        step.update(measured_bytes=meas, measured_achieved=meas / (ms_step / 1e3) / 1e9,
                    measured_frac=meas / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                    traffic_over_algorithmic=meas / step_alg)
    else:
        step.update(measured_bytes=None, measured_achieved=None, measured_frac=None,
                    traffic_over_algorithmic=None)
    return roofline, step, kernels


def cpu_baseline(seconds_target=12.0):
    """FP64 oracle on the host: 32^3 turbulent box (the same generator),
    RK3 steps until about `seconds_target` of work."""
    import numpy as np  # noqa: F401
    from workloads import box
    from oracle.scheme import Solver
    n = 32
    g, d = box.turbulent_box(n)
    s = Solver(g)
    s.curl_potential(d)
    s.set_primitives(d)
    steps = 0
    w0, c0 = time.perf_counter(), time.process_time()
    while True:
        s.rk_step()
        steps += 1
        if time.perf_counter() - w0 > seconds_target or steps >= 20:
            break
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    cores = max(1, int(round(cpu / wall)))
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n ** 3 * steps / wall, "unit": "zone-updates/s",
            "cores": cores, "kind": "oracle",
            "sample": "FP64 NumPy oracle, 32^3 turbulent SRMHD box (same seeded generator), "
                      "%d SSP-RK3 steps, %.1f s wall; %d core used of %d on %s" % (
                          steps, wall, cores, os.cpu_count() or 0, model)}


def precision_report(args):
    """Both forms on the same seeded grid with the same fixed dt (the FP64
    CFL step of the initial state), timed separately; per-field maximum error
    of the FP32-flux form relative to the FP64 form after the steps."""
    import numpy as np
    import torch
    from workloads import box
    from paper_1810_04597_amd.grid import Grid, PRIM
    from paper_1810_04597_amd import _lib as L
    n = args.n
    g, d = box.turbulent_box(n)
    grids = {}
    for name, prec in (("fp64", L.FP64), ("fp32", L.FP32_FLUX)):
        G = Grid(g, precision=prec)
        G.curl_potential(d)
        G.set_primitives(d)
        grids[name] = G
    del d
    dt = grids["fp64"].compute_dt()
    res = {}
    for name, G in grids.items():
        G.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        for _ in range(args.steps):
            G.rk_step(dt)
        e1.record(G.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[name] = {"ms_per_step": ms / args.steps, "zone_updates_per_s": n ** 3 * args.steps / (ms / 1e3)}
        print("bench: %s form done" % name, file=sys.stderr, flush=True)
    errs = {}
    A, B = grids["fp32"], grids["fp64"]
    gg = g.ng
    for f, k in enumerate(PRIM):
        a = A.field_view(A.prim, f)[gg:-gg, gg:-gg, gg:-gg]
        b = B.field_view(B.prim, f)[gg:-gg, gg:-gg, gg:-gg]
        if k in ("rho", "p"):
            errs[k] = float(((a - b).abs() / b.abs()).max())
        else:
            errs[k] = float((a - b).abs().max() / b.abs().max())
    out = {"metric": "zone-updates/s per RK3 step, FP32-flux form vs FP64 (%d^3)" % n,
           "value": res["fp32"]["zone_updates_per_s"], "unit": "zone-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": res["fp32"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32-flux/f64", "data": "synthetic",
           "config": {"workload": "turbulent SRMHD box %d^3, fixed dt %.3e, seed 1810" % (n, dt)},
           "fp64": res["fp64"], "rel_error_vs_fp64": errs,
           "speedup_vs_fp64": res["fp32"]["zone_updates_per_s"] / res["fp64"]["zone_updates_per_s"]}
    for G in grids.values():
        G.close()
    print(json.dumps(out))


def recon_report(args):
    """The reconstructions on the turbulent box: each grid starts from the
    same seeded data (MP7 on a grid with six ghost layers, the others on
    five), runs args.warmup steps, then args.steps timed RK3 steps with the
    device CFL step; per-kernel HIP-event averages."""
    import torch
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    n = args.n
    res = {}
    for name in ("mp5", "weno5", "plm", "mp7"):
        g, d = box.turbulent_box(n, ng=6 if name == "mp7" else 5)
        G = Grid(g, recon=name)
        G.curl_potential(d)
        G.set_primitives(d)
        for _ in range(args.warmup):
            G.rk_step()
        G.synchronize()
        G.set_profiling(True)
        G.profile(reset=True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(G.stream)
        for _ in range(args.steps):
            G.rk_step()
        e1.record(G.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prof = G.profile(reset=True)
        dg = G.diagnostics()
        res[name] = {"ms_per_step": ms / args.steps,
                     "zone_updates_per_s": n ** 3 * args.steps / (ms / 1e3),
                     "kernels_avg_ms": {k: t / c for k, (t, c) in prof.items()},
                     "max_divb": dg["max_divb"], "n_c2p_fail": dg["n_c2p_fail"], "t": dg["t"]}
        G.close()
        del G
        print("bench: %s done" % name, file=sys.stderr, flush=True)
    out = {"metric": "zone-updates/s per RK3 step by reconstruction (%d^3)" % n,
           "value": res["mp5"]["zone_updates_per_s"], "unit": "zone-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["mp5"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "turbulent SRMHD box %d^3, device CFL 0.4, seed 1810" % n},
           "recon": res}
    print(json.dumps(out))


def split_report(args):
    """Split inversion (Newton load balance).  (a) Inversions with a large
    spread of Newton iterations: the Kerr-Schild torus (args.torus) whose
    stored primitives are replaced by a uniform state (a poor warm start),
    and the same with the cold start Gamma U, each timed for first-pass
    limits K = 0 (one pass), 2, 3, 4, 6 (the inversion's and the second
    pass's HIP-event times, median of 5 calls, the same conserved state each
    call).  (b) The regular FP64 box step with K = 0 and K = 3."""
    import torch
    from workloads.torus import torus
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    n1, n2, n3 = (int(x) for x in args.torus.split(","))
    g, d, tab = torus(n1, n2, n3)
    inv = {}
    for label, guess in (("poor_warm", L.GUESS_WARM), ("cold", L.GUESS_COLD)):
        G = Grid(g, tables=tab, guess=guess)
        G.curl_potential(d)
        G.set_primitives(d)
        cons0 = G.cons.clone()
        res = {}
        for k in (0, 2, 3, 4, 6):
            G.set_newton_split(k)
            times = []
            for rep in range(5):
                G.cons.copy_(cons0)
                for f, val in ((0, 1.0), (1, 0.0), (2, 0.0), (3, 0.0), (4, 1.0)):
                    G._interior(G.field_view(G.prim, f)).fill_(val)
                G.synchronize()
                G.set_profiling(True)
                G.profile(reset=True)
                nf = G.cons2prim()
                prof = G.profile(reset=True)
                G.set_profiling(False)
                times.append((prof["cons2prim"][0], prof.get("newton_split", (0.0, 0))[0]))
            times.sort(key=lambda x: x[0] + x[1])
            dg = G.diagnostics()
            first, second = times[len(times) // 2]
            res["K=%d" % k] = {"first_pass_ms": first, "second_pass_ms": second,
                               "total_ms": first + second, "n_fail": nf,
                               "iters_per_zone": dg["newton_iters_sum"] / g.zones,
                               "iters_max_per_pass": dg["newton_iters_max"]}
        G.close()
        del G
        inv[label] = res
        print("bench: split %s done" % label, file=sys.stderr, flush=True)
    del d
    gb, db = box.turbulent_box(args.n)
    step = {}
    for k in (0, 3):
        G = Grid(gb)
        G.set_newton_split(k)
        G.curl_potential(db)
        G.set_primitives(db)
        for _ in range(args.warmup):
            G.rk_step()
        G.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(G.stream)
        for _ in range(args.steps):
            G.rk_step()
        e1.record(G.stream)
        torch.cuda.synchronize()
        step["K=%d" % k] = e0.elapsed_time(e1) / args.steps
        G.close()
        del G
    base = inv["poor_warm"]["K=0"]["total_ms"]
    best = min(inv["poor_warm"].items(), key=lambda kv: kv[1]["total_ms"])
    out = {"metric": "inversion time, split vs one pass, KS torus %dx%dx%d, poor warm start" % (n1, n2, n3),
           "value": best[1]["total_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": step["K=3"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Kerr-Schild a=0.9 torus %dx%dx%d, stored primitives uniform "
                                  "(rho = p = 1, u = 0) before the inversion; box %d^3 step" % (n1, n2, n3, args.n)},
           "best_K": best[0], "speedup_vs_one_pass": base / best[1]["total_ms"],
           "inversion": inv, "box_step_ms": step}
    print(json.dumps(out))


def torus_report(args):
    """Plain FP64 GRMHD torus (Kerr-Schild a = 0.9, tabulated metric, floors,
    device CFL step): zone-updates/s and per-kernel times (--recon and
    --fallback as for torus-long)."""
    import torch
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    n1, n2, n3 = (int(x) for x in args.torus.split(","))
    g, d, tab = torus(n1, n2, n3)
    G = Grid(g, tables=tab, recon=args.recon, fallback=args.fallback)
    G.curl_potential(d)
    G.set_primitives(d)
    for _ in range(args.warmup):
        G.rk_step()
    G.set_profiling(True)
    G.profile(reset=True)
    G.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(G.stream)
    for _ in range(args.steps):
        G.rk_step()
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = G.profile(reset=True)
    dg = G.diagnostics()
    # fluxes through the spheres (accretion rate -F_D, magnetic flux) at the
    # first shell outside the horizon r+ = 1 + sqrt(1 - a^2), and their cost
    import math
    import numpy as np
    sh = G.shell_fluxes()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(G.stream)
    for _ in range(10):
        G.shell_fluxes()
    ev1.record(G.stream)
    torch.cuda.synchronize()
    r = np.exp(g.x0[0] + (np.arange(n1) + 0.5) * g.dx[0])
    ih = int(np.argmax(r > 1.0 + math.sqrt(1.0 - 0.9 ** 2)))
    out = {"metric": "zone-updates/s per RK3 step, KS torus %dx%dx%d (FP64)" % (n1, n2, n3),
           "value": g.zones * args.steps / (ms / 1e3), "unit": "zone-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "Kerr-Schild a=0.9 torus %dx%dx%d, r 1.2-50, 2%% noise, beta 100, floors, device CFL, %s%s"
                                  % (n1, n2, n3, args.recon.upper(),
                                     " with the lower-order fallback" if args.fallback else "")},
           "kernels": {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in prof.items()},
           "diag": {k: dg[k] for k in ("t", "max_divb", "rho_min", "rho_max", "w_max", "n_floor_rho",
                                       "n_floor_p", "n_wcap", "n_c2p_fail", "newton_iters_sum",
                                       "newton_iters_max", "n_nonfinite")},
           "shell_fluxes": {"r_horizon_shell": float(r[ih]), "mdot": float(-sh["F_D"][ih]),
                            "energy_flux": float(sh["F_tau"][ih]), "phi_abs": float(sh["Phi"][ih]),
                            "phi_signed": float(sh["Phi_s"][ih]),
                            "call_ms_incl_copy": ev0.elapsed_time(ev1) / 10}}
    G.close()
    print(json.dumps(out))


def fallback_report(args):
    """The lower-order fallback (grmhd_grid_desc.fallback).  (a) The
    Kerr-Schild torus (args.torus) with MP5 and WENO5, with and without the
    fallback: args.warmup steps, then args.steps timed steps at the device
    CFL step; failed inversions and troubled zones over the timed steps, the
    step time and the per-class kernel times (the fix kernel is its own
    class; with the option on, 'update' counts two launches per stage, the
    hydro and the induction parts).  (b) The turbulent box (args.n^3) with
    and without it, where no zone is troubled: the cost of the split update
    and of the fix kernel's early exit."""
    import torch
    from workloads.torus import torus
    from workloads import box
    from paper_1810_04597_amd.grid import Grid

    def timed_run(G, steps):
        for _ in range(args.warmup):
            G.rk_step()
        G.synchronize()
        G.reset_run_counters()
        G.set_profiling(True)
        G.profile(reset=True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        for _ in range(steps):
            G.rk_step()
        e1.record(G.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prof = G.profile(reset=True)
        dg = G.diagnostics()
        return {"ms_per_step": ms / steps,
                "zone_updates_per_s": G.spec.zones * steps / (ms / 1e3),
                "c2p_fail": dg["run_c2p_fail"], "troubled": dg["run_troubled"],
                "floor_rho": dg["run_floor_rho"], "floor_p": dg["run_floor_p"], "t": dg["t"],
                "kernels_avg_ms": {k: t / c for k, (t, c) in prof.items()},
                "kernels_launches": {k: c for k, (t, c) in prof.items()}}

    n1, n2, n3 = (int(x) for x in args.torus.split(","))
    g, d, tab = torus(n1, n2, n3)
    tor = {}
    for recon in ("mp5", "weno5"):
        for fb in (False, True):
            G = Grid(g, tables=tab, recon=recon, fallback=fb)
            G.curl_potential(d)
            G.set_primitives(d)
            tor["%s_%s" % (recon, "fallback" if fb else "plain")] = timed_run(G, args.steps)
            G.close()
            del G
            print("bench: torus %s fallback=%s done" % (recon, fb), file=sys.stderr, flush=True)
    gb, db = box.turbulent_box(args.n)
    bx = {}
    for fb in (False, True):
        G = Grid(gb, fallback=fb)
        G.curl_potential(db)
        G.set_primitives(db)
        bx["fallback" if fb else "plain"] = timed_run(G, args.steps)
        G.close()
        del G
        print("bench: box fallback=%s done" % fb, file=sys.stderr, flush=True)
    w = tor["weno5_fallback"]
    out = {"metric": "zone-updates/s per RK3 step with the lower-order fallback, KS torus %dx%dx%d, WENO5"
                     % (n1, n2, n3),
           "value": w["zone_updates_per_s"], "unit": "zone-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": w["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "Kerr-Schild a=0.9 torus %dx%dx%d (floors, device CFL), MP5 and WENO5, "
                                  "fallback off/on; turbulent box %d^3" % (n1, n2, n3, args.n)},
           "torus": tor, "box": bx}
    print(json.dumps(out))


def torus_long_report(args):
    """Long Kerr-Schild torus run (device CFL step): every --every steps the
    diagnostics, the fluxes through the first sphere outside the horizon
    (accretion rate -F_D, magnetic flux) and the MRI resolution of the torus
    body (rho > --mri-rho-cut: mass-weighted mean Q along theta and phi, the
    fraction of body zones with Q >= 8); wall time per step over the run.
    --recon and --fallback select the reconstruction and the lower-order
    fallback; failed inversions and troubled zones are counted over the run."""
    import math
    import numpy as np
    import torch
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    n1, n2, n3 = (int(x) for x in args.torus.split(","))
    g, d, tab = torus(n1, n2, n3)
    G = Grid(g, tables=tab, recon=args.recon, fallback=args.fallback)
    G.curl_potential(d)
    G.set_primitives(d)
    r = np.exp(g.x0[0] + (np.arange(n1) + 0.5) * g.dx[0])
    ih = int(np.argmax(r > 1.0 + math.sqrt(1.0 - 0.9 ** 2)))
    series = []
    w0 = time.perf_counter()
    for s in range(1, args.steps + 1):
        G.rk_step()
        if s % args.every == 0 or s == args.steps:
            dg = G.diagnostics()
            sh = G.shell_fluxes()
            mq = G.mri_quality(args.mri_rho_cut)
            rec = {"step": s, "t": dg["t"], "dt": dg["dt"], "mdot_horizon": float(-sh["F_D"][ih]),
                   "phi_horizon": float(sh["Phi"][ih]), "max_divb": dg["max_divb"],
                   "max_divb_norm": dg["max_divb_norm"],
                   "mri_Q2": mq["Q2_mean"], "mri_Q3": mq["Q3_mean"],
                   "mri_frac_Q2_ok": mq["frac_Q2_ok"], "mri_frac_Q3_ok": mq["frac_Q3_ok"],
                   "sum_D": dg["sum_cons"][0], "w_max": dg["w_max"], "n_c2p_fail": dg["n_c2p_fail"],
                   "n_nonfinite": dg["n_nonfinite"], "newton_iters_max": dg["newton_iters_max"],
                   "run_c2p_fail": dg["run_c2p_fail"], "run_troubled": dg["run_troubled"]}
            series.append(rec)
            print("bench: step %d t %.3f mdot %.3e divb %.2e failed %d troubled %d"
                  % (s, rec["t"], rec["mdot_horizon"], rec["max_divb"], rec["run_c2p_fail"], rec["run_troubled"]),
                  file=sys.stderr, flush=True)
            if dg["n_nonfinite"]:
                break
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    out = {"metric": "long torus run, KS %dx%dx%d (FP64)" % (n1, n2, n3), "value": series[-1]["t"],
           "unit": "t (M)", "n_gpus": 1, "steps": series[-1]["step"], "warmup": 0,
           "ms_per_step": 1e3 * wall / series[-1]["step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Kerr-Schild a=0.9 torus %dx%dx%d, device CFL, diagnostics every %d steps, "
                                  "%s%s" % (n1, n2, n3, args.every, args.recon.upper(),
                                            " with the lower-order fallback" if args.fallback else ""),
                      "r_shell": float(r[ih])},
           "series": series}
    G.close()
    print(json.dumps(out))


def learned_report(args):
    """Train the learned Newton guess on the GPU (seeded samples, own kernels),
    then run the Kerr-Schild torus with three forms on the same GPU: plain
    FP64 (warm guess), FP32 flux + learned guess, FP32 flux + warm guess;
    fixed dt; density error of the FP32 forms against FP64."""
    import numpy as np
    import torch
    from workloads.mlp_data import sample_prims, init_weights
    from workloads.torus import torus
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L
    n1, n2, n3 = (int(x) for x in args.torus.split(","))
    g, d, tab = torus(n1, n2, n3)
    # --- training on 2^k seeded samples
    T = Grid(g, tables=tab)
    prims = sample_prims(args.train_samples)
    T.mlp_set_weights(L.mlp_pack(init_weights()), np.ones(32, np.float32))
    feat, targ = T.mlp_datagen(prims, set_norm=True)
    del prims
    batch = 4096
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for epoch in range(args.epochs):
        lr = 1e-3 if epoch < (2 * args.epochs) // 3 else 3e-4
        for s0 in range(0, feat.shape[0], batch):
            l = T.mlp_train_step(feat[s0:s0 + batch], targ[s0:s0 + batch], lr, want_loss=(s0 == 0))
            if s0 == 0:
                losses.append(l)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    flat, norm = T.mlp_get_weights()
    print("bench: trained %d epochs in %.1f s, loss %s" % (args.epochs, train_s, losses[-1]),
          file=sys.stderr, flush=True)
    # unseen samples: Newton iterations from the cold start and from the network
    test = sample_prims(1 << 18, seed=99)
    ft, tt, cons = T.mlp_datagen(test, want_cons=True)
    out = T.mlp_forward(ft)
    y0 = ((cons[:, 4] + cons[:, 0]) * torch.pow(10.0, out[:, 0].double() * float(norm[24]) + float(norm[16]))).contiguous()
    _, ic = T.cons2prim_points(cons)
    _, im = T.cons2prim_points(cons, y0)
    ic, im = ic.cpu().numpy(), im.cpu().numpy()
    ok = (ic > 0) & (im > 0)
    T.close()
    del feat, targ
    # the network's own gain on this workload: the torus' conserved state
    # inverted from the cold start, from the network's guess alone (every
    # zone deferred to the learned pass) and from the warm start (the exact
    # previous primitives); Newton iterations and inversion time
    starts = {}
    for name, guess in (("cold", L.GUESS_COLD), ("network_only", L.GUESS_MLP), ("warm", L.GUESS_WARM)):
        G = Grid(g, tables=tab, guess=guess)
        if guess == L.GUESS_MLP:
            G.mlp_set_weights(flat, norm)
            G.set_learned_guess(0.0, L.LEARNED_ONLY)
        G.curl_potential(d)
        G.set_primitives(d)
        G.cons2prim()
        G.set_profiling(True)
        G.profile(reset=True)
        G.reset_run_counters()
        G.cons2prim()
        prof = G.profile(reset=True)
        G.set_profiling(False)
        dg = G.diagnostics()
        starts[name] = {"newton_iters_per_zone": dg["newton_iters_sum"] / g.zones,
                        "newton_iters_max": dg["newton_iters_max"],
                        "inversion_ms": sum(v[0] for k, v in prof.items() if k in ("cons2prim", "learned_guess")),
                        "network_chosen": dg["run_mlp_chosen"], "network_fallbacks": dg["run_mlp_fallback"]}
        G.close()
    print("bench: start comparison %s" % json.dumps(starts), file=sys.stderr, flush=True)
    forms = {"fp64_warm": (L.FP64, L.GUESS_WARM), "fp32_learned": (L.FP32_FLUX, L.GUESS_MLP),
             "fp32_warm": (L.FP32_FLUX, L.GUESS_WARM)}
    res, grids = {}, {}
    dt = None
    for name, (prec, guess) in forms.items():
        G = Grid(g, tables=tab, precision=prec, guess=guess)
        if guess == L.GUESS_MLP:
            G.mlp_set_weights(flat, norm)
        G.curl_potential(d)
        G.set_primitives(d)
        if dt is None:
            dt = G.compute_dt()
        G.synchronize()
        G.set_profiling(True)
        G.profile(reset=True)
        G.reset_run_counters()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        for _ in range(args.steps):
            G.rk_step(dt)
        e1.record(G.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prof = G.profile(reset=True)
        G.set_profiling(False)
        dg = G.diagnostics()
        res[name] = {"ms_per_step": ms / args.steps, "zone_updates_per_s": g.zones * args.steps / (ms / 1e3),
                     "newton_iters_per_zone_last": dg["newton_iters_sum"] / g.zones,
                     "learned_fallbacks_last": dg["n_mlp_fallback"],
                     "learned_chosen_last": dg["n_mlp_chosen"], "c2p_fail_last": dg["n_c2p_fail"],
                     "run": {"stages": 3 * args.steps, "deferred_to_network": dg["run_mlp_deferred"],
                             "network_chosen": dg["run_mlp_chosen"],
                             "network_fallbacks": dg["run_mlp_fallback"], "c2p_fail": dg["run_c2p_fail"],
                             "floor_rho": dg["run_floor_rho"], "floor_p": dg["run_floor_p"],
                             "wcap": dg["run_wcap"]},
                     "kernels_avg_ms": {k: v[0] / v[1] for k, v in prof.items()}}
        grids[name] = G
        print("bench: %s done" % name, file=sys.stderr, flush=True)
    ref = grids["fp64_warm"]
    gg = g.ng
    b = ref.field_view(ref.prim, 0)[gg:-gg, gg:-gg, gg:-gg]
    for name in ("fp32_learned", "fp32_warm"):
        a = grids[name].field_view(grids[name].prim, 0)[gg:-gg, gg:-gg, gg:-gg]
        rel = ((a - b).abs() / b.abs())
        res[name]["rho_rel_err_max"] = float(rel.max())
        res[name]["rho_rel_err_median"] = float(rel.median())
        body = b > 0.05
        res[name]["rho_rel_err_max_body"] = float(rel[body].max())
    for G in grids.values():
        G.close()
    out = {"metric": "zone-updates/s, FP32 flux + learned Newton guess vs FP64, KS torus %dx%dx%d" % (n1, n2, n3),
           "value": res["fp32_learned"]["zone_updates_per_s"], "unit": "zone-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 0, "ms_per_step": res["fp32_learned"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32-flux/f64 + bf16 mlp", "data": "synthetic",
           "config": {"workload": "Kerr-Schild a=0.9 torus %dx%dx%d, fixed dt %.3e, 2%% noise, beta 100" % (n1, n2, n3, dt),
                      "train_samples": args.train_samples, "epochs": args.epochs},
           "training": {"seconds": train_s, "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1]},
           "inversion_of_torus_state_by_start": starts,
           "unseen_samples_newton_iters": {"cold": float(ic[ok].mean()), "learned": float(im[ok].mean()),
                                           "n": int(ok.sum())},
           "forms": res}
    print(json.dumps(out))


CALIB_COPY_BYTES = 1 << 30


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, one plain device copy of CALIB_COPY_BYTES "
                         "(reference for scaling the HBM traffic counters)")
    ap.add_argument("--profile-kernels", action="store_true", default=True)
    ap.add_argument("--eager", action="store_true",
                    help="time steps launched one by one instead of graph replays")
    ap.add_argument("--mode", default="step",
                    choices=["step", "precision", "learned", "torus", "torus-long", "recon", "split",
                             "fallback"],
                    help="step: the FP64 RK3 step (default); precision: FP32-flux form "
                         "against FP64 on the same grid, fixed dt, per-field error; learned: "
                         "train the Newton-guess network on the GPU, then the Kerr-Schild "
                         "torus in plain FP64 vs FP32 flux + learned guess; recon: the step "
                         "with MP5, WENO5 and PLM-MC reconstruction; split: the split "
                         "(load-balanced) Newton inversion against one pass; fallback: the "
                         "lower-order fallback on the torus and the box, off and on")
    ap.add_argument("--train-samples", type=int, default=1 << 22)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--torus", default="384,192,192")
    ap.add_argument("--every", type=int, default=250, help="torus-long: steps between diagnostics")
    ap.add_argument("--recon", default="mp5", choices=["mp5", "weno5", "plm"],
                    help="torus, torus-long: reconstruction")
    ap.add_argument("--fallback", action="store_true",
                    help="torus, torus-long: the lower-order fallback at troubled zones")
    ap.add_argument("--mri-rho-cut", type=float, default=1e-2,
                    help="torus-long: density above which a zone counts as torus body")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs one grid block on one GPU (no domain decomposition across GPUs); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.mode == "precision":
        return precision_report(args)
    if args.mode == "learned":
        return learned_report(args)
    if args.mode == "torus":
        return torus_report(args)
    if args.mode == "torus-long":
        return torus_long_report(args)
    if args.mode == "recon":
        return recon_report(args)
    if args.mode == "split":
        return split_report(args)
    if args.mode == "fallback":
        return fallback_report(args)

    import torch
    from workloads import box
    from paper_1810_04597_amd.grid import Grid
    from paper_1810_04597_amd import _lib as L

    n = args.n
    t0 = time.perf_counter()
    g, d = box.turbulent_box(n)
    print("bench: generated %d^3 initial data in %.1f s" % (n, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    prec = L.FP64 if args.precision == "fp64" else L.FP32_FLUX
    # the grid's own stream (default priority), so a step can be captured
    G = Grid(g, precision=prec, stream=torch.cuda.Stream())
    G.curl_potential(d)
    G.set_primitives(d)
    del d
    for _ in range(args.warmup):
        G.rk_step()
    if not args.eager:
        G.rk_steps_graph(1)         # captures the step's graph
    G.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)
    # the timed steps run without the library's per-launch timing events
    # (the per-kernel breakdown comes from a later pass of the same length);
    # by default each step is one replay of the captured graph of the step
    stream = G.stream

    def timed_steps(graph):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        t0 = time.perf_counter()
        if graph:
            G.rk_steps_graph(args.steps)
        else:
            for _ in range(args.steps):
                G.rk_step()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - t0

    ms, wall = timed_steps(not args.eager)
    ms_eager = ms if args.eager else timed_steps(False)[0]
    prof = {}
    if args.profile_kernels:
        G.set_profiling(True)
        G.profile(reset=True)
        for _ in range(args.steps):
            G.rk_step()
        prof = G.profile(reset=True)
        G.set_profiling(False)
    diag = G.diagnostics()
    if args.calib_copy:
        src = torch.ones(CALIB_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    zones = n ** 3
    value = zones * args.steps / (ms / 1e3)
    roofline, step_roofline, kernels = rooflines(prof, n, args.steps, ms / args.steps, args.precision)
    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    out = {
        "metric": "zone-updates/s per RK3 step (256^3)",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-flux/f64",
        "data": "synthetic",
        "config": {"workload": "turbulent SRMHD box %d^3, Minkowski, MP5+HLL+UCT, SSP-RK3, "
                               "device CFL 0.4, seed 1810" % n,
                   "zones": zones, "precision": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_roofline": step_roofline,
        "kernels": kernels,
        "algorithmic_hbm_GBs": STEP_BYTES * value / 1e9,
        "wall_s": wall,
        "launch": "eager" if args.eager else "graph",
        "ms_per_step_eager": ms_eager / args.steps,
        "diag": {"max_divb": diag["max_divb"], "n_c2p_fail": diag["n_c2p_fail"],
                 "rho_min": diag["rho_min"], "t": diag["t"]},
    }
    G.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
