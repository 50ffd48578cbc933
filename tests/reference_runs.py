"""Long oracle runs that are too slow for the test suite, for the full-size
validation of the large-dT cavity (Sec. IV-C): 512 x 512, walls at
T0 (1 +/- 0.6), Ra = 1e5, Pr = 0.71, Sutherland viscosity, mu_r = 0.06,
s_e = s_zeta = 1.5, pure-conduction start, 200,000 steps.

Runs only the FP64 oracle and writes its macroscopic fields (rho, ux, uy, T)
with the step count to an .npz file; checkpoints every `--every` steps so
that an interrupted run resumes.  `--golden` also writes the fields on every
`--stride`-th node in x and y (the fixture tests/golden/large_dt_512_sample.npz
that tests/test_gpu_validation.py compares the GPU run with).  Usage:

    python -m tests.reference_runs --out ref.npz [--steps 200000] [--every 10000] \
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--every", type=int, default=10_000)
    ap.add_argument("--golden", default="")
    ap.add_argument("--stride", type=int, default=8)
    args = ap.parse_args()
    if args.golden and os.path.exists(args.out):
        write_golden(args.out, args.golden, args.stride)
        return
    p, f = large_dt_512()
    o = O.Oracle(p).init(*f)
    ck = args.out + ".ckpt.npz"
    n = 0  # the cavity has no time-dependent boundary, so a resumed state needs only its step count
    if os.path.exists(ck):
        z = np.load(ck)
        o.set_pops(z["pops"])
        n = int(z["time"])
        print(f"resumed at step {n}", flush=True)
    t0 = time.time()
    while n < args.steps:
        k = min(args.every, args.steps - n)
        o.step(k)
        n += k
        np.savez(ck, pops=o.pops(), time=n)
        d = o.diag()
        print(f"step {n}: mass {d['mass']:.10f} bad {d['bad']} ({time.time() - t0:.0f} s)", flush=True)
    rho, ux, uy, T = o.macros()
    np.savez(args.out, rho=rho, ux=ux, uy=uy, T=T, time=n)
    print(f"wrote {args.out}", flush=True)
    if args.golden:
        write_golden(args.out, args.golden, args.stride)


def write_golden(full: str, golden: str, stride: int):
    z = np.load(full)
    off = stride // 2
    sl = (slice(off, None, stride), slice(off, None, stride))
    np.savez_compressed(golden, rho=z["rho"][sl], ux=z["ux"][sl], uy=z["uy"][sl], T=z["T"][sl],
                        time=z["time"], stride=stride, offset=off)
    print(f"wrote {golden} ({z['rho'][sl].shape} nodes every {stride} from {off})", flush=True)


if __name__ == "__main__":
    main()
