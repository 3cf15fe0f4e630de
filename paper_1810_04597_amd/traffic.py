"""Measured HBM traffic per kernel launch from two rocprofv3 counter passes.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir_f> -o run -- python bench.py --calib-copy ...
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir_w> -o run -- python bench.py --calib-copy ...
    python -m paper_1810_04597_amd.traffic <dir_f> <dir_w>

The counters (KiB per dispatch) are scaled by what they read for the plain
device copy of 1 GiB that bench.py --calib-copy runs after its steps:
factor = known bytes / counter bytes, separately for FETCH and WRITE.
Writes traffic.json with the hash of the kernel sources, so the benchmark
reports the traffic only while the kernels are unchanged.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                    glob.glob(os.path.join(HERE, "csrc", "*.hpp"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


CLASS_OF = [(r"k_sweep(_lds)?<0", "sweep_x1"), (r"k_sweep(_lds)?<1", "sweep_x2"),
            (r"k_sweep(_lds)?<2", "sweep_x3"), (r"k_edge(_lds)?<0", "edge_x1"),
            (r"k_edge(_lds)?<1", "edge_x2"), (r"k_edge(_lds)?<2", "edge_x3"),
            (r"k_update", "update"), (r"k_c2p", "cons2prim"), (r"k_bc_centred", "bc_centred"),
            (r"k_bc_faces", "bc_faces"), (r"k_cfl", "cfl"), (r"__amd_rocclr_copyBuffer", "copy_calib")]


def _read(d, counter):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    out = {}
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        cls = None
        for pat, c in CLASS_OF:
            if re.search(pat, name):
                cls = c
        if cls is None:
            continue
        out.setdefault(cls, []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def compute(dir_f, dir_w, copy_bytes=1 << 30):
    """Per-class HBM bytes per launch (the largest-grid launches of each
    class), scaled by the calibration copy's counter readings."""
    fetch = _read(dir_f, "FETCH_SIZE")
    write = _read(dir_w, "WRITE_SIZE")
    known_kib = copy_bytes / 1024.0
    big = lambda lst: [v for g, v in lst if g == max(x for x, _ in lst)]
    cf = known_kib / (sum(big(fetch["copy_calib"])) / len(big(fetch["copy_calib"])))
    cw = known_kib / (sum(big(write["copy_calib"])) / len(big(write["copy_calib"])))
    res = {"source_hash": source_hash(), "fetch_scale": cf, "write_scale": cw, "kernels": {}}
    for cls in fetch:
        if cls == "copy_calib":
            continue
        fv = big(fetch[cls])
        wv = big(write.get(cls, [(0, 0.0)]))
        fb = sum(fv) / len(fv) * cf * 1024
        wb = sum(wv) / len(wv) * cw * 1024
        res["kernels"][cls] = {"fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    return res


def main(dir_f, dir_w, copy_bytes=1 << 30, out=None):
    res = compute(dir_f, dir_w, copy_bytes)
    with open(out or os.path.join(HERE, "traffic.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 1 << 30)
