"""Long oracle runs that are too slow for the test suite, for the full-size
validation of the GPU path.  Cases (`--case`):

  large_dt_512   the large-dT cavity (Sec. IV-C): 512 x 512, walls at
                 T0 (1 +/- 0.6), Ra = 1e5, Pr = 0.71, Sutherland viscosity,
                 mu_r = 0.06, s_e = s_zeta = 1.5, pure-conduction start,
                 200,000 steps;
  periodic_1024  the bandwidth sweep's periodic 1024 x 1024 grid with
                 Gaussian perturbations (sigma 1e-3), 1000 steps;
  periodic_4096  the same on 4096 x 4096, 10 steps;
  channel        the acoustic channel 2048 x 256 (source at x = 0, amplitude
                 0.01, period 200 steps, Eq. 53-54), its first 5000 steps;
  large_dt_sweep_1e3 / _1e4 / _1e5
                 the paper's large-dT runs (Sec. IV-C): walls at T0 (1 +/- 0.6),
                 Sutherland viscosity, tau_e = tau_zeta = tau_f, Ra = 1e3, 1e4,
                 1e5 on 100, 150, 200 cells (101, 151, 201 nodes) with
                 mu_r = 0.1, 0.1, 0.06, conduction start; 100,000, 200,000 and
                 300,000 steps.

Runs only the FP64 oracle and writes its macroscopic fields (rho, ux, uy, T)
with the step count to an .npz file; checkpoints every `--every` steps so
that an interrupted run resumes (cases without a time-dependent boundary).
`--golden` also writes the fields on every `--stride`-th node in x and
`--stride-y`-th in y (default: the same), the fixtures under tests/golden/
that tests/test_gpu_validation.py compares the GPU runs with, plus the
temperature of the three columns next to each x-side (T_left3, T_right3)
for the wall heat fluxes.  Usage:

    python -m tests.reference_runs --case large_dt_512 --out ref.npz [--steps N] [--every 10000] \
        [--golden tests/golden/large_dt_512_sample.npz --stride 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1109_6672_amd import workloads as W  # noqa: E402


def large_dt_512():
    """The energy-mode rates are untied (s_e = s_zeta = 1.5): with
    tau_e = tau_zeta = tau_f at every node this grid diverges near the cold
    bottom corner after about 15,000 steps.  Sec. III allows tau_e != tau_f
    for low-Mach flows, where the bulk viscosity hardly enters the energy
    equation."""
    p = W.cavity(512, 1e5, 1.2, 0.06, sutherland=True)
    p.update(s_e=1.5, s_zeta=1.5)
    return p, W.conduction_fields(p)


def periodic_1024():
    p = W.periodic(1024)
    return p, W.gaussian_fields(p, sigma=1e-3)


def periodic_4096():
    p = W.periodic(4096)
    return p, W.gaussian_fields(p, sigma=1e-3)


def channel():
    p = W.channel()
    return p, W.rest_fields(p)


def large_dt_sweep(n, Ra, mu_r):
    p = W.cavity(n, Ra, 1.2, mu_r, sutherland=True)
    return p, W.conduction_fields(p)


CASES = {"large_dt_512": (large_dt_512, 200_000), "periodic_1024": (periodic_1024, 1000),
         "periodic_4096": (periodic_4096, 10), "channel": (channel, 5000),
         "large_dt_sweep_1e3": (lambda: large_dt_sweep(101, 1e3, 0.1), 100_000),
         "large_dt_sweep_1e4": (lambda: large_dt_sweep(151, 1e4, 0.1), 200_000),
         "large_dt_sweep_1e5": (lambda: large_dt_sweep(201, 1e5, 0.06), 300_000)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="large_dt_512", choices=sorted(CASES))
    ap.add_argument("--out", required=True)
    ap.add_argument("--steps", type=int, default=0, help="default: the case's length")
    ap.add_argument("--every", type=int, default=10_000)
    ap.add_argument("--golden", default="")
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--stride-y", type=int, default=0)
    args = ap.parse_args()
    make, steps = CASES[args.case]
    args.steps = args.steps or steps
    sy = args.stride_y or args.stride
    if args.golden and os.path.exists(args.out):
        write_golden(args.out, args.golden, args.stride, sy)
        return
    p, f = make()
    o = O.Oracle(p).init(*f)
    ck = args.out + ".ckpt.npz"
    n = 0  # the cavity has no time-dependent boundary, so a resumed state needs only its step count
    if os.path.exists(ck) and args.case != "channel":
        z = np.load(ck)
        o.set_pops(z["pops"])
        n = int(z["time"])
        print(f"resumed at step {n}", flush=True)
    t0 = time.time()
    while n < args.steps:
        k = min(args.every, args.steps - n)
        o.step(k)
        n += k
        if args.case != "channel":
            np.savez(ck, pops=o.pops(), time=n)
        d = o.diag()
        print(f"step {n}: mass {d['mass']:.10f} bad {d['bad']} ({time.time() - t0:.0f} s)", flush=True)
    rho, ux, uy, T = o.macros()
    np.savez(args.out, rho=rho, ux=ux, uy=uy, T=T, time=n)
    print(f"wrote {args.out}", flush=True)
    if args.golden:
        write_golden(args.out, args.golden, args.stride, sy)


def write_golden(full: str, golden: str, stride: int, stride_y: int):
    z = np.load(full)
    off, offy = stride // 2, stride_y // 2
    sl = (slice(offy, None, stride_y), slice(off, None, stride))
    np.savez_compressed(golden, rho=z["rho"][sl], ux=z["ux"][sl], uy=z["uy"][sl], T=z["T"][sl],
                        time=z["time"], stride=stride, offset=off, stride_y=stride_y, offset_y=offy,
                        T_left3=z["T"][:, :3], T_right3=z["T"][:, -3:])
    print(f"wrote {golden} ({z['rho'][sl].shape} nodes every {stride} from {off} in x, every {stride_y} "
          f"from {offy} in y)", flush=True)


if __name__ == "__main__":
    main()
