#!/usr/bin/env python3
"""Online-solve throughput of SubApSnap on one MI355X.

Default workload: 3-D diffusion -div(a grad u) = 1 on the unit cube, 7-point
finite differences on a 215^3 grid (n = 9,938,375),
a = exp(sum_k p_k phi_k) with four sin/cos product modes, r = 40 snapshots
(GPU conjugate-gradient solves, Householder QR), s = 160 rows by rounds of
pivoted QR, and a batch of 65,536 parameters p* uniform in [-1, 1]^4, all
resident in HBM.  All inputs are synthetic and seeded (subap_inputs).

A step is one subap_solve_batch call on the whole batch: the face
coefficients of the selected rows, S A(p) Q from the FP64 face-difference
table, the FP64 Householder least squares, y, the sketched residual and the
status of every parameter, fused in one kernel.
A solve counts toward the metric when its status is OK and it is within
delta_res = |A(p) Q (y - y_ref)| / |b| <= 1e-6 over all n rows of the
reference: the FP64 form is the reference itself and is checked against the
FP64 CPU oracle on sampled parameters of the same launch; reduced-precision
forms are measured against the FP64 form by subap_delta_residual on the GPU.

--workload selects the other lines (bench_configs.py): krr (kernel ridge
regression, n = 16384, 4096 parameters), uneven, surrogate, lift, leverage,
delay.  Prints one JSON line.  --gpus N with N > 1 exits: this benchmark uses
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TOL = 1e-6
PEAKS = {  # MI355X published dense peaks
    "bf16_mfma_tflops": 2500.0,
    "fp32_mfma_tflops": 157.3,
    "fp64_tflops": 78.6,
    "hbm_gbs": 8000.0,
}
WORKLOADS = ["diffusion3d", "krr", "uneven", "surrogate", "lift", "leverage", "delay"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-sample", type=int, default=256, help="parameters solved one per call")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle timing budget")
    ap.add_argument("--oracle-sample", type=int, default=4,
                    help="parameters of the timed launch the FP64 CPU oracle recomputes")
    ap.add_argument("--workload", default="diffusion3d", choices=WORKLOADS,
                    help="diffusion3d (default, the headline line) or one of the other configurations "
                         "(lift: the FP32 lift alone on an N^3 grid, --grid N)")
    ap.add_argument("--grid", type=int, default=215, help="diffusion3d/surrogate/lift/leverage: nodes per axis")
    ap.add_argument("--delay-n", type=int, default=10 ** 7, help="delay: system size n")
    ap.add_argument("--table-sample", type=int, default=64,
                    help="delay: parameters for the full-residual / transfer-function error columns")
    ap.add_argument("--apsnap-sample", type=int, default=8, help="delay: parameters solved by ApSnap")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a device-to-device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--given-basis", action="store_true",
                    help="diffusion3d, krr: seeded orthonormal basis instead of snapshot solves (profiling "
                         "runs; the online kernels do the same work for any basis)")
    ap.add_argument("--profile-only", action="store_true",
                    help="diffusion3d, krr: time the headline form only (no validity check, other forms or "
                         "CPU baseline)")
    return ap.parse_args()


def timed(fn, steps, stream):
    """Average milliseconds of fn over steps calls, HIP events on the launch stream."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the single-GPU online solve; multi-GPU runs are not part of this "
              "benchmark (the batch shards over parameters with no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch

    import bench_configs
    import subap_inputs as si
    from paper_2510_04825_amd import binding as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    out = getattr(bench_configs, args.workload)(args, B, si, torch, dev, stream, timed, PEAKS, TOL)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
