"""Algorithmic operation counts of the kernels (host only, no GPU).

Builds the harness csrc/opcount.cpp, which runs the kernels' own per-face,
per-edge and per-zone bodies with an operation-counting number type on the
seeded turbulent box, and writes the per-unit means to opcounts.json (used by
bench.py for the roofline line).

python -m paper_1810_04597_amd.opcount [--n 24]
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def build_harness():
    out = os.path.join(HERE, "_build", "opcount")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-x", "c++", "-I", "/opt/rocm/include",
           "-I", os.path.join(HERE, "csrc"), "-I", os.path.join(ROOT, "include"),
           "-D__HIP_PLATFORM_AMD__", os.path.join(HERE, "csrc", "opcount.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=24)
    args = ap.parse_args()
    from workloads import box
    g, d = box.turbulent_box(args.n)
    exe = build_harness()
    with tempfile.NamedTemporaryFile(suffix=".bin", delete=False) as f:
        np.array([float(args.n)]).tofile(f)
        for k in ("rho", "u1", "u2", "u3", "p"):
            np.ascontiguousarray(d[k], dtype=np.float64).tofile(f)
        for k in ("A1", "A2", "A3"):
            np.ascontiguousarray(d[k], dtype=np.float64).tofile(f)
        path = f.name
    try:
        r = subprocess.run([exe, path], check=True, capture_output=True, text=True)
    finally:
        os.unlink(path)
    counts = json.loads(r.stdout)
    with open(os.path.join(HERE, "opcounts.json"), "w") as fo:
        json.dump(counts, fo, indent=1)
    print(json.dumps(counts, indent=1))


if __name__ == "__main__":
    main()
