"""Summary of a profiled FP64 RK3 step (markdown) from rocprofv3 outputs.

    rocprofv3 --kernel-trace --stats --output-format csv -d <dir_t> -o run -- \
        python -u bench.py --steps 5 --warmup 1 --no-cpu-baseline --eager --calib-copy
    rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 \
        SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU --output-format csv -d <dir_v> -o run -- \
        python -u bench.py --steps 1 --warmup 1 --no-cpu-baseline --eager
    rocprofv3 --pmc SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY \
        SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM SQ_LDS_BANK_CONFLICT \
        --output-format csv -d <dir_s> -o run -- python -u bench.py --steps 1 --warmup 1 \
        --no-cpu-baseline --eager
    python -m paper_1810_04597_amd.profsum --ktrace <dir_t> --valu <dir_v> --stall <dir_s> \
        --bench <bench log> --out <file.md> [--n 256]

Per kernel class: calls and average duration (kernel trace), HBM bytes per
launch (traffic.json, written by paper_1810_04597_amd.traffic from the
FETCH_SIZE / WRITE_SIZE passes), algorithmic bytes and FLOP per launch
(opcounts.json), FP64 FLOP counted by the SQ instruction counters (64 lanes
per wavefront instruction, FMA = 2; masked lanes are counted too, so this is
an upper bound) and the VALU issue fraction (4 cycles per wavefront
instruction on a 16-lane SIMD, 1024 SIMDs at 2.4 GHz).

Per step (the stage kernels run three times per step): measured HBM bytes
over the step time against the 8 TB/s peak and against the plain device
copy's rate in the same trace; the algorithmic rate 896 B per zone-update;
the FP64 VALU utilisation (counted FP64 FLOP over 78.6 TFLOP/s).
"""
import argparse
import csv
import glob
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK = 8.0e12
FP64_PEAK = 78.6e12
SIMDS, CLOCK = 1024, 2.4e9
STAGE_CLASSES = ("sweep_x1", "sweep_x2", "sweep_x3", "edge_x1", "edge_x2", "edge_x3", "update",
                 "cons2prim")

CLASS_OF = [(r"k_sweep(_lds)?<0", "sweep_x1"), (r"k_sweep(_lds)?<1", "sweep_x2"),
            (r"k_sweep(_lds)?<2", "sweep_x3"), (r"k_edge(_lds)?<0", "edge_x1"),
            (r"k_edge(_lds)?<1", "edge_x2"), (r"k_edge(_lds)?<2", "edge_x3"),
            (r"k_update", "update"), (r"k_c2p<", "cons2prim"), (r"k_bc_centred", "bc_centred"),
            (r"k_bc_faces", "bc_faces"), (r"k_cfl", "cfl"), (r"k_dt_final", "dt_final"),
            (r"k_advance", "advance"), (r"__amd_rocclr_copyBuffer", "copy_calib")]
# rows of the update split by RK stage (template argument after the metric)
# (k_update_zm<metric, stage, derivative order, flux storage, parts>)
STAGE_ROW = [(r"k_update_zm<.*>, 1, [0-9], ", "update (stage 1: U^n in, U^(1) out)"),
             (r"k_update_zm<.*>, 2, [0-9], ", "update (stage 2, in place)"),
             (r"k_update_zm<.*>, 3, [0-9], ", "update (stage 3: U^(3) over U^n)")]


def class_of(name):
    cls = None
    for pat, c in CLASS_OF:
        if re.search(pat, name):
            cls = c
    return cls


def row_of(name):
    for pat, r in STAGE_ROW:
        if re.search(pat, name):
            return r
    return class_of(name)


def units(cls, n):
    ng = n + 10
    if cls.startswith("sweep"):
        return (n + 5) * ng * ng
    if cls.startswith("edge"):
        return (n + 5) * (n + 5) * n
    return n ** 3


def read_counters(d):
    """{class: {counter: mean value over the class's largest-grid dispatches}}"""
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    raw = {}
    for r in csv.DictReader(open(f)):
        cls = class_of(r["Kernel_Name"])
        if cls is None:
            continue
        raw.setdefault(cls, {}).setdefault(r["Counter_Name"], []).append(
            (int(r["Grid_Size"]), float(r["Counter_Value"])))
    out = {}
    for cls, cs in raw.items():
        out[cls] = {}
        for c, lst in cs.items():
            g = max(x for x, _ in lst)
            v = [val for x, val in lst if x == g]
            out[cls][c] = sum(v) / len(v)
    return out


def copy_rate(dir_t):
    """Bytes/s of the largest plain device copy in the trace (read + write)."""
    f = glob.glob(os.path.join(dir_t, "**", "*kernel_trace.csv"), recursive=True)
    if not f:
        return None
    best = None
    for r in csv.DictReader(open(f[0])):
        if "copyBuffer" not in r["Kernel_Name"]:
            continue
        g = int(r["Grid_Size_X"])
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        if best is None or g > best[0] or (g == best[0] and dt < best[1]):
            best = (g, dt)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ktrace", required=True)
    ap.add_argument("--valu")
    ap.add_argument("--stall", help="counter pass with SQ_WAVE_CYCLES, SQ_WAIT_ANY, SQ_WAIT_INST_ANY, "
                    "SQ_ACTIVE_INST_ANY, SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS, SQ_LDS_BANK_CONFLICT")
    ap.add_argument("--bench", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--traffic", default=os.path.join(HERE, "traffic.json"),
                    help="per-launch HBM bytes written by paper_1810_04597_amd.traffic")
    ap.add_argument("--title", default="FP64 SSP-RK3 step, turbulent SRMHD box 256^3 (MI355X)")
    ap.add_argument("--commands", default="", help="text block: the commands that made the inputs")
    a = ap.parse_args(argv)
    traffic = json.load(open(a.traffic))
    ops = json.load(open(os.path.join(HERE, "opcounts.json")))
    bench = [json.loads(l) for l in open(a.bench) if l.startswith("{")][-1]
    valu = read_counters(a.valu) if a.valu else {}
    stats = glob.glob(os.path.join(a.ktrace, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = []
    for r in csv.DictReader(open(stats)):
        cls = class_of(r["Name"])
        if cls is None or cls == "copy_calib":
            continue
        us = float(r["AverageNs"]) / 1e3
        calls = int(r["Calls"])
        t = traffic["kernels"].get(cls)
        meas = t["bytes"] if t else None
        u = units(cls, a.n)
        alg_b = ops.get(cls, {}).get("bytes")
        fl = ops.get(cls, {}).get("flops")
        v = valu.get(cls, {})
        f64 = None
        if "SQ_INSTS_VALU_FMA_F64" in v:
            f64 = 64.0 * (v["SQ_INSTS_VALU_ADD_F64"] + v["SQ_INSTS_VALU_MUL_F64"] +
                          2.0 * v["SQ_INSTS_VALU_FMA_F64"])
        busy = v["SQ_INSTS_VALU"] * 4.0 / (SIMDS * CLOCK * us * 1e-6) if "SQ_INSTS_VALU" in v else None
        rows.append((row_of(r["Name"]), calls, us, meas, alg_b * u if alg_b else None,
                     fl * u / (us * 1e-6) if fl else None, f64 / (us * 1e-6) if f64 else None, busy))
    rows.sort(key=lambda x: -x[2])
    fmt = lambda val, s: "-" if val is None else s % val
    out = ["# Kernel trace, HBM traffic and FP64 VALU counters: %s\n" % a.title]
    if a.commands:
        out.append("Commands (from the repository root, library built in-tree):\n")
        out += ["    " + l for l in a.commands.strip().split("\n")]
        out.append("")
    out.append("HBM traffic: FETCH_SIZE and WRITE_SIZE per dispatch scaled by what they read for a "
               "plain 1 GiB device copy (FETCH x %.4f, WRITE x %.4f of the copied bytes); kernel "
               "source hash %s. Counter values are averages over a class's launches (the update's "
               "over its three stages: stage 1 reads no U^n, stages 2 and 3 do).\n" % (
                   1 / traffic["fetch_scale"], 1 / traffic["write_scale"], traffic["source_hash"]))
    out.append("| kernel | calls | avg us | HBM GB/launch (measured) | measured TB/s | algorithmic "
               "GB/launch | FP64 TFLOP/s (algorithmic) | FP64 TFLOP/s (SQ counters) | VALU busy |")
    out.append("|---|---|---|---|---|---|---|---|---|")
    for name, calls, us, meas, alg, tf, tfc, busy in rows:
        out.append("| %s | %d | %.1f | %s | %s | %s | %s | %s | %s |" % (
            name, calls, us, fmt(meas and meas / 1e9, "%.2f"),
            fmt(meas and meas / (us * 1e-6) / 1e12, "%.2f"), fmt(alg and alg / 1e9, "%.2f"),
            fmt(tf and tf / 1e12, "%.1f"), fmt(tfc and tfc / 1e12, "%.1f"), fmt(busy, "%.2f")))
    # whole step
    ms = bench["ms_per_step"]
    zps = bench["value"]
    step_bytes = sum(3 * traffic["kernels"][c]["bytes"] for c in STAGE_CLASSES
                     if c in traffic["kernels"])
    out.append("\nWhole step (bench.py in the same GPU call: %.2f ms per step, %.3g zone-updates/s, "
               "%s launch):\n" % (ms, zps, bench.get("launch", "eager")))
    hbm = step_bytes / (ms * 1e-3)
    cp = copy_rate(a.ktrace)
    line = "1. measured HBM: %.1f GB per step (stage kernels, three launches each) = %.2f TB/s, " \
           "%.2f of the 8 TB/s peak" % (step_bytes / 1e9, hbm / 1e12, hbm / HBM_PEAK)
    rate = 2.0 * a.copy_bytes / cp[1] if cp and cp[1] > 0 else None
    if rate and rate <= HBM_PEAK:   # the 1 GiB calibration copy is in the trace
        line += ", %.2f of the %.2f TB/s a plain 1 GiB device copy reaches in the same trace" % (
            hbm / rate, rate / 1e12)
    out.append(line)
    alg = 896.0 * zps
    out.append("2. algorithmic: 896 B per zone-update (state in and out, three stages) x %.3g/s = "
               "%.3f TB/s (%.3f of peak)" % (zps, alg / 1e12, alg / HBM_PEAK))
    if valu:
        f64_step = 0.0
        for c in STAGE_CLASSES:
            v = valu.get(c, {})
            if "SQ_INSTS_VALU_FMA_F64" in v:
                f64_step += 3 * 64.0 * (v["SQ_INSTS_VALU_ADD_F64"] + v["SQ_INSTS_VALU_MUL_F64"] +
                                        2.0 * v["SQ_INSTS_VALU_FMA_F64"])
        vt = sum(3 * valu.get(c, {}).get("SQ_INSTS_VALU", 0.0) for c in STAGE_CLASSES)
        out.append("3. FP64 VALU: %.2f TFLOP per step counted (upper bound: masked lanes count) = "
                   "%.1f TFLOP/s, %.3f of the 78.6 TFLOP/s FP64 vector peak; all VALU instructions "
                   "keep the SIMDs %.2f busy over the step" % (
                       f64_step / 1e12, f64_step / (ms * 1e-3) / 1e12,
                       f64_step / (ms * 1e-3) / FP64_PEAK, vt * 4.0 / (SIMDS * CLOCK * ms * 1e-3)))
    if a.stall:
        sc = read_counters(a.stall)
        out.append("\nWave states (SQ counters, fractions of the wave-cycles of each class: "
                   "SQ_WAIT_ANY, waiting on a dependency or counter; SQ_WAIT_INST_ANY, waiting for "
                   "an instruction to be issued (arbitration with the other wavefronts of the SIMD, "
                   "instruction fetch); SQ_ACTIVE_INST_ANY, _VALU, _LDS, issuing; LDS bank "
                   "conflict cycles):\n")
        out.append("| kernel | wait (dependency) | wait (issue) | issuing | issuing VALU | issuing LDS "
                   "| LDS bank conflicts |")
        out.append("|---|---|---|---|---|---|---|")
        for c in STAGE_CLASSES:
            v = sc.get(c, {})
            w = v.get("SQ_WAVE_CYCLES")
            if not w:
                continue
            out.append("| %s | %.2f | %.2f | %.2f | %.2f | %.3f | %d |" % (
                c, v["SQ_WAIT_ANY"] / w, v["SQ_WAIT_INST_ANY"] / w, v["SQ_ACTIVE_INST_ANY"] / w,
                v["SQ_ACTIVE_INST_VALU"] / w, v["SQ_ACTIVE_INST_LDS"] / w,
                int(v.get("SQ_LDS_BANK_CONFLICT", 0))))
    text = "\n".join(out) + "\n"
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
