"""Validation of the HIP path at the full sizes of the paper's test problems,
against what the paper and the mathematics fix there:

* the bench workload (periodic 8192 x 8192) element by element against the
  FP64 oracle after 5 steps;
* the periodic 1024^2 (1000 steps) and 4096^2 (10 steps) grids and the
  first 5000 steps of the 2048 x 256 channel against sampled oracle fields;
* the small-dT cavity (128 x 128, Ra = 1e4) run to convergence against the
  'Present' row of Table II and against the oracle, and the other Table II
  rows (Ra = 1e3, 1e5; Ra = 1e4 at the paper's temperatures on 151^2);
* the acoustic channel (2048 x 256, sinusoidal source at x = 0) against the
  attenuation law Eq. 55-56 before the outlet reflection returns, then on to
  100,000 steps;
* the large-dT cavity (Sutherland viscosity) on its 64 x 64 form and at
  512 x 512 against the FP64 oracle after 200,000 steps in FP32, FP16 and
  BF16 storage, the heat-flux balance of its two walls, and the paper's Ra
  sweep on 101^2, 151^2 and 201^2.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1109_6672_amd import lbddf, postproc as P, workloads as W
from paper_1109_6672_amd.serving import Plateau
from tests.gpu_common import TOL, rel_errors

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _converge(s, check=1000, tol=1e-8, cap=600_000):
    """Runs until the FP64 residual ||T^n - T^(n-check)|| / ||T^n|| falls below
    tol, stalls at its floor (the server's plateau test) or the step cap is
    reached."""
    s.residual(update=True)
    pl, r = Plateau(), math.inf
    while s.time < cap:
        s.step(check)
        r = s.residual(update=True)
        if r < tol:
            return "converged", r
        if pl.update(r):
            return "plateau", r
    return "step_cap", r


@pytest.fixture(scope="module")
def bench_reference():
    """The FP64 oracle on the workload bench.py times (periodic 8192 x 8192,
    Gaussian sigma = 1e-3), 5 steps: about 20 GB of host memory, a few
    seconds per step on the host cores."""
    from oracle import oracle as O

    p = W.periodic(8192)
    f = W.gaussian_fields(p, sigma=1e-3)
    print("[case] oracle on the bench workload, periodic 8192x8192, 5 steps", flush=True)
    o = O.Oracle(p).init(*f).step(5)
    ref = o.macros()
    del o
    return p, f, ref


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_bench_workload_at_full_size_against_the_oracle(bench_reference, storage):
    """Full-size parity in the launch configuration bench.py times (8192^2,
    lockstep blocks, 8-row strips), element by element after 5 steps."""
    p, f, ref = bench_reference
    s = lbddf.Solver(dict(p, storage=storage)).init(*f).step(5)
    e = rel_errors(s.macros(), ref)
    print(f"[case] bench workload 8192x8192 {storage}, 5 steps (strip rows {s.strip_rows}): rel err rho {e[0]:.3e} "
          f"u {e[1]:.3e} T {e[2]:.3e}", flush=True)
    s.close()
    assert max(e) < TOL[storage], e


def test_small_dT_cavity_reproduces_table_ii():
    with open(os.path.join(HERE, "golden", "table2_cavity.json")) as fh:
        tab = json.load(fh)
    row = dict(zip(tab["columns"], next(r for r in tab["rows"] if r[0] == 1e4)))
    p = W.cavity(128, 1e4, 0.02, 0.02)
    print(f"[case] Table II Ra=1e4 cavity 128x128 tau_f={3 * 0.02 + 0.5:.2f} g={p['g']:.4e}", flush=True)
    s = lbddf.Solver(p).init(*W.noisy_temperature_fields(p))
    state, r = _converge(s)
    rho, ux, uy, T = s.macros()
    m = P.cavity_metrics(p, ux, uy, T)
    print(f"       {state} after {s.time} steps (r = {r:.2e}): " + ", ".join(f"{k} {v:.4f}" for k, v in m.items()),
          flush=True)
    print("       paper: " + ", ".join(f"{k} {row[k]:.4f}" for k in ("Nu", "u_max", "y_max", "v_max", "x_max")),
          flush=True)
    assert state != "step_cap"
    # grid 128 against the paper's 150, and a slightly compressible model
    for k in ("Nu", "u_max", "v_max"):
        assert abs(m[k] / row[k] - 1) < 0.02, (k, m[k], row[k])
    for k in ("y_max", "x_max"):
        assert abs(m[k] - row[k]) < 0.02, (k, m[k], row[k])


@pytest.mark.parametrize("Ra,n,mu_r,cap", [(1e3, 101, 0.05, 1_000_000), (1e5, 201, 0.02, 4_000_000)])
def test_small_dT_cavity_table_ii_other_rows(Ra, n, mu_r, cap):
    """The Ra = 1e3 and 1e5 rows of Table II on the paper's grids (100 and 200
    cells, H = n - 1), run to convergence (Ra = 1e5 stops on the plateau test
    near r = 3e-8 after about 3.3 million steps).  The paper's table is the
    Boussinesq limit, which a compressible model approaches as the
    stratification g H / (R T0) shrinks: 0.053 at Ra = 1e3 (mu_r = 0.05),
    0.21 at Ra = 1e5 (mu_r = 0.02; smaller mu_r, tau_f = 0.53 or 0.545,
    diverges within 10,000 steps here, with or without untied bulk rates or a
    conduction start).  At Ra = 1e5, u_max is held to 4 %: the paper's value
    and its two references already spread by 3 % for that quantity."""
    with open(os.path.join(HERE, "golden", "table2_cavity.json")) as fh:
        tab = json.load(fh)
    row = dict(zip(tab["columns"], next(r for r in tab["rows"] if r[0] == Ra)))
    p = W.cavity(n, Ra, 0.02, mu_r)
    print(f"[case] Table II Ra={Ra:g} cavity {n}x{n} tau_f={3 * mu_r + 0.5:.2f} g={p['g']:.4e}", flush=True)
    s = lbddf.Solver(p).init(*W.noisy_temperature_fields(p))
    state, r = _converge(s, check=2000, cap=cap)
    rho, ux, uy, T = s.macros()
    m = P.cavity_metrics(p, ux, uy, T)
    print(f"       {state} after {s.time} steps (r = {r:.2e}): " + ", ".join(f"{k} {v:.4f}" for k, v in m.items()),
          flush=True)
    print("       paper: " + ", ".join(f"{k} {row[k]:.4f}" for k in ("Nu", "u_max", "y_max", "v_max", "x_max")),
          flush=True)
    assert state != "step_cap" and s.diag()["bad"] == 0
    for k in ("Nu", "u_max", "v_max"):
        bar = 0.04 if (Ra >= 1e5 and k == "u_max") else 0.02
        assert abs(m[k] / row[k] - 1) < bar, (k, m[k], row[k])
    for k in ("y_max", "x_max"):
        assert abs(m[k] - row[k]) < 2.0 / (n - 1) + 1e-9, (k, m[k], row[k])


def test_table_ii_ra1e4_at_the_papers_temperatures_and_grid():
    """Table II's Ra = 1e4 row at the paper's own conditions: walls at 315 K
    and 285 K (dT / T0 = 0.1 about T_r = 300 K) on 150 cells (151 x 151
    nodes), mu_r = 0.05 (tau_f = 0.65, g H / R T0 = 0.047), run to
    convergence.  Nu, u_max and v_max within 2 % of the 'Present' row, the
    positions within two lattice spacings."""
    with open(os.path.join(HERE, "golden", "table2_cavity.json")) as fh:
        tab = json.load(fh)
    row = dict(zip(tab["columns"], next(r for r in tab["rows"] if r[0] == 1e4)))
    p = W.cavity(151, 1e4, 0.1, 0.05)
    print(f"[case] Table II Ra=1e4, dT/T0=0.1, 151x151, g={p['g']:.4e}", flush=True)
    s = lbddf.Solver(p).init(*W.noisy_temperature_fields(p))
    state, r = _converge(s, check=1000, cap=2_000_000)
    rho, ux, uy, T = s.macros()
    m = P.cavity_metrics(p, ux, uy, T)
    print(f"       {state} after {s.time} steps (r = {r:.2e}): " + ", ".join(f"{k} {v:.4f}" for k, v in m.items()),
          flush=True)
    assert state != "step_cap" and s.diag()["bad"] == 0
    for k in ("Nu", "u_max", "v_max"):
        assert abs(m[k] / row[k] - 1) < 0.02, (k, m[k], row[k])
    for k in ("y_max", "x_max"):
        assert abs(m[k] - row[k]) < 2.0 / 150 + 1e-9, (k, m[k], row[k])


def test_small_dT_cavity_converged_state_against_the_oracle():
    """Config 2 run 268,000 steps (its convergence above) on the GPU and in the
    FP64 oracle: FP32 storage within 1e-5 in rho, u and T (measured 9.0e-8 /
    1.2e-6 / 2.1e-8 with the walled step's FP64 sums), and the Table II
    quantities agree to 1e-4.  This flow's velocity (about 3.5e-3) is driven by a buoyancy
    fifty times smaller than the hydrostatic forces (dT/T0 = 0.02), so a
    steady per-step bias of the energy balance shows up in u: before the
    zeroth moment of h_eq was closed on the node's energy, the rounding of the
    lattice weights added such a bias and u was off by 5e-4.  The FP64-
    arithmetic library meets the bar as well."""
    from oracle import oracle as O

    p = W.cavity(128, 1e4, 0.02, 0.02)
    f = W.noisy_temperature_fields(p)
    print("[case] Table II Ra=1e4 cavity 128x128, 268000 steps, GPU (FP32 and FP64 arithmetic) and oracle",
          flush=True)
    g = lbddf.Solver(p).init(*f).step(268_000).macros()
    g64 = lbddf.Solver(p, arith="f64").init(*f).step(268_000).macros()
    r = O.Oracle(p).init(*f).step(268_000).macros()
    e64 = rel_errors(g64, r)
    print(f"       FP64 arithmetic: rel err rho {e64[0]:.3e} u {e64[1]:.3e} T {e64[2]:.3e}", flush=True)
    assert max(e64) < TOL["f32"], e64
    e = rel_errors(g, r)
    mg, mr = P.cavity_metrics(p, *g[1:]), P.cavity_metrics(p, *r[1:])
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e}; Nu {mg['Nu']:.5f} / {mr['Nu']:.5f}, "
          f"u_max {mg['u_max']:.4f} / {mr['u_max']:.4f}, v_max {mg['v_max']:.4f} / {mr['v_max']:.4f}", flush=True)
    assert max(e) < TOL["f32"], e
    for k in ("Nu", "u_max", "v_max"):
        assert abs(mg[k] / mr[k] - 1) < 1e-4, (k, mg[k], mr[k])
    assert mg["y_max"] == mr["y_max"] and mg["x_max"] == mr["x_max"]


def _beta_eq56(mu, Pr, b, period):
    """Spatial attenuation rate of Eq. 56 for a source of frequency 1/period
    (lattice units, rho0 = 1, R T0 = 1/3)."""
    gamma = (b + 2) / b
    cs = math.sqrt(gamma / 3)
    cv, cp = b / 2 / 3, (b + 2) / 2 / 3
    fp = 1.0 / period
    return 2 * math.pi ** 2 * fp ** 2 / cs ** 3 * (
        (4 / 3) * mu + 2 * (1 / 3 - 1 / b) * mu + (1 / cv - 1 / cp) * mu * cp / Pr)


def test_acoustic_channel_follows_eq56_at_full_size():
    import torch

    period, U0 = 200.0, 0.01
    p = W.channel(2048, 256, U0=U0, period=period)
    mu = (p["tau_f"] - 0.5) * p["R"] * p["T0"]
    cs = math.sqrt((p["b"] + 2) / p["b"] / 3)
    beta = _beta_eq56(mu, p["Pr"], p["b"], period)
    print(f"[case] acoustic channel 2048x256 U0={U0} period={period} beta(Eq. 56)={beta:.4e}", flush=True)
    s = lbddf.Solver(p).init(*W.rest_fields(p))
    t_m = 2600  # the front (x = c_s t = 1937) has not reached the outlet
    s.step(t_m - int(period))
    env = None
    for _ in range(int(period)):
        s.step(1)
        ux = s.macros_device()[1].abs()
        env = ux if env is None else torch.maximum(env, ux)
    env = env.cpu().numpy().astype(np.float64)
    spread = float(np.max(np.abs(env - env[0:1])))
    lam = cs * period
    x = np.arange(20, int(cs * t_m - 3 * lam))
    e = env[0, x]
    fit, amp = P.envelope_fit(x, e)
    dev = float(np.max(np.abs(e / (U0 * np.exp(-beta * x)) - 1)))
    print(f"       fitted beta {fit:.4e} ({fit / beta - 1:+.3%}), amplitude {amp:.5f}, max deviation from "
          f"U0 exp(-beta x) {dev:.3%}, spread over rows {spread:.1e}", flush=True)
    assert spread == 0.0  # a plane wave: every row computes the same values
    assert abs(fit / beta - 1) < 0.05
    assert dev < 0.05
    s.step(100_000 - s.time)
    d = s.diag()
    rho, ux, uy, T = s.macros()
    print(f"       after {s.time} steps: bad nodes {d['bad']}, max |u| {np.max(np.hypot(ux, uy)):.4f}, "
          f"rho in [{rho.min():.5f}, {rho.max():.5f}]", flush=True)
    assert d["bad"] == 0 and np.max(np.abs(ux)) < 3 * U0


@pytest.fixture(scope="module")
def large_dT_reference():
    from oracle import oracle as O

    p = W.cavity(64, 1e5, 1.2, 0.06, sutherland=True)
    f = W.conduction_fields(p)
    print(f"[case] large-dT cavity 64x64 oracle, 200000 steps", flush=True)
    o = O.Oracle(p).init(*f).step(200_000)
    return p, f, o.macros()


def test_large_dT_cavity_downscale_against_the_oracle(large_dT_reference):
    """The 64 x 64 form (g = 1.7e-3, g H / R T0 = 0.32) after 200,000 steps,
    FP32 storage: within 1e-5 of the oracle (measured 4.1e-7 / 3.3e-7 /
    3.2e-7).  The deviations from the rest state are O(1) here (rho from 0.6
    to 2.5); the bounded-grid step forms the moments, m - m_eq, h - h_eq and
    the wall rebuild in FP64 and rounds its FP32 sums without bias (FP32
    throughout: 3.5e-5 / 1.5e-5 / 1.3e-5)."""
    p, f, ref = large_dT_reference
    s = lbddf.Solver(p).init(*f).step(200_000)
    e = rel_errors(s.macros(), ref)
    print(f"[case] large-dT cavity 64x64 f32 after 200000 steps: rel err rho {e[0]:.3e} u {e[1]:.3e} "
          f"T {e[2]:.3e}", flush=True)
    assert s.diag()["bad"] == 0
    assert max(e) < TOL["f32"], e


def _finite_or_raise(e, s):
    """A non-finite error or an unstable node is a failure of its own (not the
    expected miss of a storage bar): RuntimeError, which xfail does not take."""
    if not all(np.isfinite(e)) or s.diag()["bad"] != 0:
        raise RuntimeError(f"non-finite or unstable result: errors {e}")


@pytest.mark.xfail(raises=AssertionError, strict=True,
                   reason="16-bit storage of O(1) deviations from rest: FP16 measured 1.9e-3 / 2.6e-3 / 1.3e-3, "
                          "BF16 1.2e-2 / 2.5e-2 / 1.2e-2 against 2e-3")
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_large_dT_cavity_downscale_16bit_against_the_oracle(large_dT_reference, storage):
    p, f, ref = large_dT_reference
    s = lbddf.Solver(dict(p, storage=storage)).init(*f).step(200_000)
    e = rel_errors(s.macros(), ref)
    print(f"[case] large-dT cavity 64x64 {storage} after 200000 steps: rel err rho {e[0]:.3e} u {e[1]:.3e} "
          f"T {e[2]:.3e}", flush=True)
    _finite_or_raise(e, s)
    assert max(e) < TOL[storage], e


def test_large_dT_cavity_downscale_fp64_arithmetic(large_dT_reference):
    """The 64 x 64 large-dT form with the step's arithmetic in FP64
    (liblbddf_fp64.so) and FP32 storage: within 1e-5 of the oracle after
    200,000 steps (FP32 arithmetic: 3.4e-5)."""
    p, f, ref = large_dT_reference
    s = lbddf.Solver(p, arith="f64").init(*f).step(200_000)
    e = rel_errors(s.macros(), ref)
    print(f"[case] large-dT cavity 64x64, FP64 arithmetic, 200000 steps: rel err rho {e[0]:.3e} u {e[1]:.3e} "
          f"T {e[2]:.3e}", flush=True)
    assert max(e) < TOL["f32"], e


def _large_dt_512(storage, arith):
    path = os.path.join(HERE, "golden", "large_dt_512_sample.npz")
    z = np.load(path)
    stride, off, steps = int(z["stride"]), int(z["offset"]), int(z["time"])
    p = W.cavity(512, 1e5, 1.2, 0.06, sutherland=True, storage=storage)
    p.update(s_e=1.5, s_zeta=1.5)
    print(f"[case] large-dT cavity 512x512 {storage} storage, {arith} arithmetic, {steps} steps, every {stride}th "
          "node", flush=True)
    s = lbddf.Solver(p, arith=arith).init(*W.conduction_fields(p)).step(steps)
    g = tuple(a[off::stride, off::stride] for a in s.macros())
    e = rel_errors(g, (z["rho"], z["ux"], z["uy"], z["T"]))
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e}", flush=True)
    return s, e


@pytest.mark.parametrize("arith", ["f32", "f64"])
def test_large_dT_cavity_512_against_the_oracle(arith):
    """Config 3 at full size: 512 x 512, 200,000 steps, FP32 storage, against
    the FP64 oracle's fields on every 8th node
    (tests/golden/large_dt_512_sample.npz, written by tests/reference_runs.py
    from an oracle-only run).  Measured: the FP32 library 2.8e-7 / 2.9e-6 /
    2.9e-7 (with the moments, the non-equilibrium parts and the wall rebuild
    in FP32 and plain rounding: 8e-5 / 7.5e-5 / 1.3e-4); the FP64-arithmetic
    library 2.8e-7 / 3.4e-6 / 3.1e-7."""
    s, e = _large_dt_512("f32", arith)
    assert s.diag()["bad"] == 0
    assert max(e) < TOL["f32"], e


@pytest.mark.xfail(raises=AssertionError, strict=True,
                   reason="16-bit storage of O(1) deviations from rest: FP16 measured 2.4e-3 / 2.7e-2 / 2.4e-3, "
                          "BF16 1.8e-2 / 1.9e-1 / 1.8e-2 against 2e-3")
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_large_dT_cavity_512_16bit_against_the_oracle(storage):
    s, e = _large_dt_512(storage, "f32")
    _finite_or_raise(e, s)
    assert max(e) < TOL[storage], e


def test_large_dT_cavity_512_heat_balance():
    """512 x 512, 200,000 steps: in FP32 and FP16 storage the cold wall carries
    the steeper temperature gradient (the conductivity falls with T under
    Sutherland's law, and the wall fluxes balance)."""
    p = W.cavity(512, 1e5, 1.2, 0.06, sutherland=True)
    p.update(s_e=1.5, s_zeta=1.5)  # tied to tau_f this grid diverges at the cold bottom corner
    f = W.conduction_fields(p)
    for storage in ("f32", "f16"):
        s = lbddf.Solver(dict(p, storage=storage)).init(*f).step(200_000)
        d = s.diag()
        rho, ux, uy, T = s.macros()
        hot = np.abs(-3 * T[:, 0] + 4 * T[:, 1] - T[:, 2]) / 2
        cold = np.abs(3 * T[:, -1] - 4 * T[:, -2] + T[:, -3]) / 2
        print(f"[case] large-dT cavity 512x512 {storage}: bad {d['bad']}, mean |dT/dx| hot {hot.mean():.4e} "
              f"cold {cold.mean():.4e}, max |u| {np.max(np.hypot(ux, uy)):.4f}", flush=True)
        assert d["bad"] == 0
        assert cold.mean() > hot.mean()
        s.close()


def _sampled(name):
    z = np.load(os.path.join(HERE, "golden", name))
    sx, ox = int(z["stride"]), int(z["offset"])
    sy, oy = int(z["stride_y"]), int(z["offset_y"])
    return z, (slice(oy, None, sy), slice(ox, None, sx)), int(z["time"])


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("n,name", [(1024, "periodic_1024_sample.npz"), (4096, "periodic_4096_sample.npz")])
def test_bandwidth_sweep_grids_against_the_oracle(n, name, storage):
    """Config 4a at its sizes: periodic 1024 x 1024 for its full 1000 steps
    and 4096 x 4096 for 10 steps (Gaussian sigma = 1e-3 on rho, u, T),
    against the FP64 oracle on every 16th (1024^2) or 64th (4096^2) node
    (fixtures written by tests/reference_runs.py from oracle-only runs), in
    the launch configuration bench.py times."""
    z, sl, steps = _sampled(name)
    p = W.periodic(n, storage=storage)
    print(f"[case] periodic {n}x{n} {storage}, {steps} steps, sampled oracle", flush=True)
    s = lbddf.Solver(p).init(*W.gaussian_fields(p, sigma=1e-3)).step(steps)
    g = tuple(a[sl] for a in s.macros())
    e = rel_errors(g, (z["rho"], z["ux"], z["uy"], z["T"]))
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e} (strip rows {s.strip_rows})", flush=True)
    assert s.diag()["bad"] == 0
    assert max(e) < TOL[storage], e


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_channel_first_5000_steps_against_the_oracle(storage):
    """Config 4b at full size: the 2048 x 256 acoustic channel (source at
    x = 0, amplitude 0.01, period 200 steps, Eq. 53-54; outlet at x = nx - 1)
    after its first 5000 steps, against the FP64 oracle on every 8th node in
    x and 64th in y (the wave is plane: all rows agree)."""
    z, sl, steps = _sampled("channel_5000_sample.npz")
    p = W.channel(storage=storage)
    print(f"[case] channel 2048x256 {storage}, {steps} steps, sampled oracle", flush=True)
    s = lbddf.Solver(p).init(*W.rest_fields(p)).step(steps)
    g = tuple(a[sl] for a in s.macros())
    e = rel_errors(g, (z["rho"], z["ux"], z["uy"], z["T"]))
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e}", flush=True)
    assert s.diag()["bad"] == 0
    assert max(e) < TOL[storage], e


def _vortex_centre(rho, ux):
    """Centre of the primary vortex: the extremum of the stream function
    psi(x, y) = sum over rows below y of rho u_x (one row per lattice
    spacing), as fractions of the cavity width from the hot wall (x) and the
    bottom (y)."""
    psi = np.cumsum(rho * ux, axis=0)
    j, i = np.unravel_index(np.argmax(np.abs(psi)), psi.shape)
    return i / (rho.shape[1] - 1), j / (rho.shape[0] - 1)


@pytest.mark.parametrize("Ra,n,mu_r", [(1e3, 101, 0.1), (1e4, 151, 0.1), (1e5, 201, 0.06)])
def test_large_dT_cavity_paper_sweep_against_the_oracle(Ra, n, mu_r):
    """The paper's large-dT runs (Sec. IV-C, Eq. 57-59): walls at 960 K and
    240 K (T0 (1 +/- 0.6)), Sutherland viscosity, tau_e = tau_zeta = tau_f at
    every node, Ra = 1e3, 1e4, 1e5 on 100, 150, 200 cells with
    mu_r = 0.1, 0.1, 0.06, from the conduction profile; 100,000, 200,000 and
    300,000 steps in FP32 storage against the FP64 oracle on every 5th node
    (tests/golden/large_dt_sweep_*.npz, written by tests/reference_runs.py
    from oracle-only runs).  On the GPU's full fields the wall heat fluxes
    balance (cold-wall over hot-wall mean gradient within 7 % of
    mu(T_h) / mu(T_l) = 2.619) and, at Ra = 1e3 and 1e4, the centre of the
    primary vortex lies right of and below the cavity centre (the asymmetry
    of Figs. 7-8)."""
    name = f"large_dt_sweep_{'1e%d' % round(math.log10(Ra))}.npz"
    z, sl, steps = _sampled(name)
    p = W.cavity(n, Ra, 1.2, mu_r, sutherland=True)
    print(f"[case] large-dT cavity {n}x{n} Ra {Ra:g} f32, {steps} steps, sampled oracle", flush=True)
    s = lbddf.Solver(p).init(*W.conduction_fields(p)).step(steps)
    rho, ux, uy, T = s.macros()
    e = rel_errors((rho[sl], ux[sl], uy[sl], T[sl]), (z["rho"], z["ux"], z["uy"], z["T"]))
    xc, yc = _vortex_centre(rho, ux)
    hot = np.abs(-3 * T[:, 0] + 4 * T[:, 1] - T[:, 2]).mean() / 2
    cold = np.abs(3 * T[:, -1] - 4 * T[:, -2] + T[:, -3]).mean() / 2
    mu_ratio = 1.6 ** 1.5 / 0.4 ** 1.5 * (0.4 + 110.5 / 600) / (1.6 + 110.5 / 600)  # Eq. 59
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e}; vortex centre ({xc:.3f}, {yc:.3f}); "
          f"cold/hot wall gradient {cold / hot:.3f} (mu ratio {mu_ratio:.3f})", flush=True)
    assert s.diag()["bad"] == 0
    assert max(e) < TOL["f32"], e
    assert abs(cold / hot / mu_ratio - 1) < 0.07
    if Ra < 1e5:
        assert xc > 0.55 and yc < 0.45


@pytest.mark.xfail(raises=AssertionError, strict=True,
                   reason="FP16 storage of O(1) deviations from rest: u measured 2.2e-2, 9.2e-3 and 8.5e-3 against 2e-3 "
                          "at Ra = 1e3, 1e4, 1e5 (rho and T 1.1e-3 to 2.1e-3)")
@pytest.mark.parametrize("Ra,n,mu_r", [(1e3, 101, 0.1), (1e4, 151, 0.1), (1e5, 201, 0.06)])
def test_large_dT_cavity_paper_sweep_16bit(Ra, n, mu_r):
    """The paper's large-dT sweep in FP16 storage against the same oracle
    fields as the FP32 runs above."""
    name = f"large_dt_sweep_{'1e%d' % round(math.log10(Ra))}.npz"
    z, sl, steps = _sampled(name)
    p = W.cavity(n, Ra, 1.2, mu_r, sutherland=True, storage="f16")
    print(f"[case] large-dT cavity {n}x{n} Ra {Ra:g} f16, {steps} steps, sampled oracle", flush=True)
    s = lbddf.Solver(p).init(*W.conduction_fields(p)).step(steps)
    rho, ux, uy, T = s.macros()
    e = rel_errors((rho[sl], ux[sl], uy[sl], T[sl]), (z["rho"], z["ux"], z["uy"], z["T"]))
    print(f"       rel err rho {e[0]:.3e} u {e[1]:.3e} T {e[2]:.3e}", flush=True)
    _finite_or_raise(e, s)
    assert max(e) < TOL["f16"], e
