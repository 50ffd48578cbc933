"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same seeded inputs and compare the macroscopic fields."""
import numpy as np

from oracle import oracle as O
from paper_1109_6672_amd import lbddf, workloads as W

TOL = {"f32": 1e-5, "f16": 2e-3, "bf16": 2e-3}


def rel_errors(g, r):
    """Max relative errors of rho, u, T: pointwise for rho and T, and
    max |u - u_ref| / max |u_ref| for the velocity."""
    err_rho = float(np.max(np.abs(g[0] - r[0]) / np.abs(r[0])))
    err_T = float(np.max(np.abs(g[3] - r[3]) / np.abs(r[3])))
    umax = float(np.max(np.hypot(r[1], r[2])))
    err_u = float(np.max(np.hypot(g[1] - r[1], g[2] - r[2])) / umax) if umax > 0 else float(
        np.max(np.hypot(g[1], g[2])))
    return err_rho, err_u, err_T


def run_pair(p, fields, steps, label=""):
    print(f"[case] {label} nx={p['nx']} ny={p['ny']} storage={p.get('storage')} steps={steps}", flush=True)
    s = lbddf.Solver(p).init(*fields).step(steps)
    o = O.Oracle(p).init(*fields).step(steps)
    g, r = s.macros(), o.macros()
    e = rel_errors(g, r)
    print(f"       rel err rho {e[0]:.3e}  u {e[1]:.3e}  T {e[2]:.3e}", flush=True)
    return s, o, g, r, e
