"""GPU parity: the HIP path against the FP64 oracle, element by element, on
seeded inputs of every configuration at sizes the oracle finishes in seconds
(several wavefront tiles and strips, ragged tails).

Tolerance (max relative error of rho, u, T): 1e-5 with FP32 storage, 2e-3
with 16-bit weight-shifted storage."""
import numpy as np
import pytest

from paper_1109_6672_amd import lbddf, workloads as W
from tests.gpu_common import TOL, rel_errors, run_pair

pytestmark = pytest.mark.gpu


def _check(e, storage):
    tol = TOL[storage]
    assert e[0] < tol and e[1] < tol and e[2] < tol, (storage, e)


_BF16_MISS = pytest.mark.xfail(raises=AssertionError, strict=True,
                               reason="BF16 (8-bit mantissa) misses 2e-3 in u: measured 7.8e-3 on periodic noise, "
                                      "5.9e-3 on the Couette flow")


def _finite(e):
    if not all(np.isfinite(e)):
        raise RuntimeError(f"non-finite result: errors {e}")


@pytest.mark.parametrize("storage", ["f32", "f16", pytest.param("bf16", marks=_BF16_MISS)])
def test_periodic_noise(gpu, storage):
    p = W.periodic(150, 77, storage=storage)
    f = W.gaussian_fields(p, sigma=1e-3)
    _, _, _, _, e = run_pair(p, f, 200, "periodic noise")
    _finite(e)
    _check(e, storage)


@pytest.mark.parametrize("collision", ["mrt", "bgk"])
def test_periodic_mean_flow(gpu, collision):
    """Noise advected by a mean flow (u ~ 0.06): exercises the O(u^2) terms
    and exact momentum conservation over many steps."""
    p = W.periodic(150, 77)
    p["collision"] = collision
    rho, ux, uy, T = W.gaussian_fields(p, sigma=1e-3)
    _, _, _, _, e = run_pair(p, (rho, ux + 0.05, uy + 0.03, T), 600, f"periodic mean flow {collision}")
    _check(e, "f32")


@pytest.mark.parametrize("variant", ["bgk", "decoupled", "internal", "noheat", "strip4"])
def test_periodic_variants(gpu, variant):
    p = W.periodic(130, 66)
    if variant == "bgk":
        p["collision"] = "bgk"
    elif variant == "decoupled":
        p["coupled"] = False
    elif variant == "internal":
        p.update(energy="internal", heating=False, g=1e-5)
    elif variant == "noheat":
        p.update(heating=False, s_e=1.2, s_zeta=1.1)
    f = W.gaussian_fields(p, sigma=2e-3)
    s = lbddf.Solver(p).init(*f)
    if variant == "strip4":
        s.set_strip_rows(4)
    s.step(150)
    from oracle import oracle as O
    o = O.Oracle(p).init(*f).step(150)
    e = rel_errors(s.macros(), o.macros())
    print(f"[case] periodic {variant}: rel err {e}", flush=True)
    _check(e, "f32")


@pytest.mark.parametrize("storage", ["f32", "f16", pytest.param("bf16", marks=_BF16_MISS)])
def test_couette(gpu, storage):
    p = W.couette(storage=storage)
    _, _, _, _, e = run_pair(p, W.rest_fields(p), 3000, "couette")
    _finite(e)
    _check(e, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_couette_full_length(gpu, storage):
    """The Couette workload at its full length (20,000 steps)."""
    p = W.couette(storage=storage)
    _, _, _, _, e = run_pair(p, W.rest_fields(p), 20000, "couette 20k")
    _check(e, storage)


def test_paper_couette_power_law_adiabatic(gpu):
    p = W.couette_paper(1.0, 0.35)
    _, _, _, _, e = run_pair(p, W.rest_fields(p), 2000, "couette mu~T adiabatic")
    _check(e, "f32")


_F16_GRAVITY_MISS = pytest.mark.xfail(
    raises=AssertionError, strict=True,
    reason="FP16 storage of the gravity-stratified deviations from rest: u measured 7.8e-3 against 2e-3 after "
           "12,000 steps (7.4e-3 after 4000; rho and T 2.4e-4 and 2.0e-4)")


@pytest.mark.parametrize("storage,steps", [("f32", 12000), ("f16", 1000),
                                           pytest.param("f16", 12000, marks=_F16_GRAVITY_MISS)])
def test_cavity_small_dT(gpu, storage, steps):
    """Gravity-driven small-dT cavity, tau_f = 0.56 as in the 128^2 case
    (0.536 is unstable in the oracle itself).  FP32 storage over 12,000 steps
    (measured 4.8e-8 / 1.2e-6 / 5.1e-8; the full convergence run is in the
    validation tests).  FP16 storage meets the 16-bit bar over the first 1000
    steps only: the flow's velocity is a small residue of stratified
    populations whose FP16 rounding noise accumulates in u."""
    p = W.cavity(70, 1e4, 0.02, 0.02, storage=storage)
    _, _, _, _, e = run_pair(p, W.noisy_temperature_fields(p), steps, "cavity small dT")
    _finite(e)
    _check(e, storage)


@pytest.mark.parametrize("Ra", [1e3, 1e4, 1e5])
def test_cavity_large_dT_sutherland(gpu, Ra):
    """The large-dT cavity (T0 (1 +/- 0.6), Sutherland viscosity) at the
    Rayleigh numbers of the paper's large-dT figures, from the conduction
    state.  At Ra = 1e3 the flow is ten times slower while rho and T still
    deviate by O(1) from rest, so u relative to its small maximum is the
    hardest of the three."""
    p = W.cavity(66, Ra, 1.2, 0.06, sutherland=True)
    _, _, _, _, e = run_pair(p, W.conduction_fields(p), 1500, f"cavity large dT sutherland Ra={Ra:g}")
    _check(e, "f32")


def test_channel_inlet_outlet(gpu):
    p = W.channel(nx=190, ny=9, U0=0.01, period=40.0)
    _, _, g, r, e = run_pair(p, W.rest_fields(p), 600, "acoustic channel")
    _check(e, "f32")


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 5), (7, 1), (2, 3), (65, 1), (64, 2), (3, 130)])
def test_degenerate_periodic_grids(gpu, nx, ny):
    """Grids narrower than a tile, one row or one node: the periodic wrap folds
    every neighbour back onto the grid, one strip covers it all."""
    p = W.periodic(nx, ny)
    _, _, _, _, e = run_pair(p, W.gaussian_fields(p, sigma=1e-3), 50, "degenerate periodic")
    _check(e, "f32")


@pytest.mark.parametrize("case", ["couette 1x3", "couette 4x3", "adiabatic couette 2x4", "cavity 4x4",
                                  "cavity 5x5", "channel 3x1", "channel 5x2"])
def test_smallest_bounded_grids(gpu, case):
    """The smallest grids the library accepts with walls (3 nodes across a
    Dirichlet pair, 4 with an adiabatic side) or an inlet and an outlet (3
    columns): almost every node is a boundary node.  The cavities have hot and
    cold side walls, an adiabatic floor and an adiabatic lid moving at 0.05,
    and no gravity: a buoyant flow in a 5 x 5 box moves at ~3e-4, where the
    FP32 floor of stratified deviations (~5e-9 in u) would be what is
    measured, not the boundary code."""
    kind, shape = case.rsplit(" ", 1)
    nx, ny = (int(v) for v in shape.split("x"))
    if kind == "couette":
        p, f = W.couette(nx=nx, ny=ny), None
    elif kind == "adiabatic couette":
        p, f = W.couette_paper(1.0, 0.35, nx=nx, ny=ny), None
    elif kind == "cavity":
        p = W.cavity(nx, 100.0, 0.02, 0.01)
        p["g"] = 0.0
        p["sides"][3] = W.side("adiabatic", 0.05, 0.0, 1.0)
        f = W.noisy_temperature_fields(p)
    else:
        p, f = W.channel(nx=nx, ny=ny, period=20.0), None
    _, _, _, _, e = run_pair(p, f if f is not None else W.rest_fields(p), 100, f"smallest {case}")
    _check(e, "f32")


def test_zero_steps_change_nothing(gpu):
    p = W.periodic(70, 33)
    s = lbddf.Solver(p).init(*W.gaussian_fields(p, sigma=1e-3))
    before = s.populations()
    s.step(0)
    assert s.time == 0
    np.testing.assert_array_equal(s.populations(), before)


def test_deterministic_and_strip_invariant(gpu):
    """Bitwise identical results for repeated runs and for any strip height."""
    p = W.cavity(70, 1e4, 0.2, 0.05)
    f = W.noisy_temperature_fields(p)
    outs = []
    for rows in (0, 4, 16, 64):
        s = lbddf.Solver(p).init(*f)
        if rows:
            s.set_strip_rows(rows)
        s.step(300)
        outs.append(s.populations())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_populations_match_the_oracle(gpu):
    p = W.cavity(40, 1e4, 0.2, 0.05)
    f = W.noisy_temperature_fields(p)
    s, o, _, _, _ = run_pair(p, f, 200, "cavity populations")
    gp, rp = s.populations(), o.pops()
    scale = np.abs(rp).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(gp - rp) / scale) < 1e-5


@pytest.mark.parametrize("storage,mant", [("f16", 10), ("bf16", 7)])
def test_16bit_codec_rounding_bound(gpu, storage, mant):
    """Stored values are the deviations from the rest equilibria, rounded
    stochastically to the 16-bit format (after a power-of-two plane scale for
    FP16): each decoded population lies within one unit in the last place of
    its deviation, 2^-mant |dev| (or the format's smallest step), of the FP64
    equilibrium of the initial fields."""
    from oracle import oracle as O

    p = W.periodic(130, 70, storage=storage)
    f = W.gaussian_fields(p, sigma=1e-2)
    gp = lbddf.Solver(p).init(*f).populations()
    rp = O.Oracle(p).init(*f).pops()
    rest = O.Oracle(p).init(*W.rest_fields(p)).pops()[:, :1, :1]
    dev = np.abs(rp - rest)
    tiny = 2.0 ** -24 if storage == "f16" else 2.0 ** -133
    bound = np.maximum(dev * 2.0 ** -mant, tiny) + 1e-7 * np.abs(rp)
    err = np.abs(gp - rp)
    print(f"[case] {storage} codec: max err / bound {np.max(err / bound):.3f}", flush=True)
    assert np.all(err <= bound)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_stochastic_rounding_is_unbiased(gpu, storage):
    """A uniform state stores the same deviation x at every node. Stochastic
    rounding puts each stored value on one of the two format neighbours of x
    (FP16 after its power-of-two plane scale, BF16 directly), taking the upper
    one with probability (x - lo) / (hi - lo): over 65,536 nodes the mean of
    the stored values sits on x within a few standard errors, where rounding to
    nearest would sit up to half a step away. The neighbours and the exact x
    come from the format's definition and the FP64 oracle, not from the
    kernel."""
    from oracle import oracle as O

    p = W.periodic(256, 256, storage=storage)
    shape = (p["ny"], p["nx"])
    # the values the library receives (it takes the fields in FP32)
    vals = [float(np.float32(v)) for v in (1.02, 0.05, -0.03, 1.05)]
    f = tuple(np.full(shape, v) for v in vals)
    gp = lbddf.Solver(p).init(*f).populations()
    rp = O.Oracle(p).init(*f).pops()
    rest = O.Oracle(p).init(*W.rest_fields(p)).pops()[:, 0, 0]
    mant = 10 if storage == "f16" else 7
    n = gp[0].size
    straddled = 0
    for q in range(18):
        a = q % 9
        s = 1.0 if storage == "bf16" else (512.0 if a == 0 else (2048.0 if a < 5 else 8192.0))
        x = (rp[q, 0, 0] - rest[q]) * s
        obs = (gp[q].ravel() - rest[q]) * s
        gap = 2.0 ** (np.floor(np.log2(abs(x))) - mant)
        lo = np.floor(x / gap) * gap
        p_up = (x - lo) / gap
        assert np.all(np.abs(obs - x) < gap * (1 + 1e-3)), (q, x, np.unique(obs))
        assert len(np.unique(np.round(obs / gap * 8) / 8)) <= 2, (q, np.unique(obs))
        bias = (obs.mean() - x) / gap
        print(f"[case] {storage} plane {q}: p_up {p_up:.3f} observed {np.mean(obs > x):.3f} bias {bias:+.4f} step",
              flush=True)
        assert abs(bias) < 5 * 0.5 / np.sqrt(n) + 0.02
        if 0.1 < p_up < 0.9:
            straddled += 1
            assert abs(np.mean(obs > x) - p_up) < 5 * np.sqrt(p_up * (1 - p_up) / n) + 0.02
    assert straddled >= 6

    p = W.periodic(256, 192)
    f = W.gaussian_fields(p, sigma=1e-3)
    s = lbddf.Solver(p).init(*f)
    d0 = s.diag()
    s.step(1000)
    d1 = s.diag()
    from oracle import oracle as O
    o = O.Oracle(p).init(*f)
    r0 = o.diag()
    assert abs(d0["mass"] - r0["mass"]) < 1e-6 * r0["mass"]
    assert abs(d0["energy"] - r0["energy"]) < 1e-6 * r0["energy"]
    print(f"[case] conservation drift mass {d1['mass'] - d0['mass']:.3e} energy {d1['energy'] - d0['energy']:.3e}")
    assert abs(d1["mass"] - d0["mass"]) < 1e-6 * d0["mass"]
    assert abs(d1["energy"] - d0["energy"]) < 1e-6 * d0["energy"]
    assert d1["bad"] == 0 and d1["time"] == 1000


def test_checkpoint_resume_is_bitwise(gpu):
    p = W.channel(nx=130, ny=8, period=30.0)
    f = W.rest_fields(p)
    a = lbddf.Solver(p).init(*f).step(200)
    blob = a.save()
    a.step(150)
    b = lbddf.Solver(p).load(blob)
    assert b.time == 200
    b.step(150)
    np.testing.assert_array_equal(a.populations(), b.populations())


def test_residual_matches_the_oracle(gpu):
    p = W.cavity(40, 1e4, 0.2, 0.05)
    f = W.noisy_temperature_fields(p)
    from oracle import oracle as O
    s, o = lbddf.Solver(p).init(*f), O.Oracle(p).init(*f)
    assert s.residual() == float("inf") and o.residual() == float("inf")
    s.step(100)
    o.step(100)
    rs, ro = s.residual(), o.residual()
    print(f"[case] residual gpu {rs:.6e} oracle {ro:.6e}")
    assert abs(rs - ro) < 1e-3 * ro


@pytest.mark.parametrize("case", ["periodic", "cavity", "channel"])
def test_graph_replays_match_host_launches_bitwise(gpu, case):
    """lb_step replays a captured graph of 32 launches whose arguments are
    fixed (the step index comes from a device clock, the inlet phase is
    computed on the device from it).  Every replay, with eager work (macros,
    diagnostics) and synchronisation between replays, gives the populations
    that launches one by one from the host give after the same steps, bit
    for bit; so do the 4 single launches after the last replay."""
    if case == "periodic":
        p = W.periodic(130, 66)
        f = W.gaussian_fields(p, sigma=1e-3)
    elif case == "cavity":
        p = W.cavity(70, 1e5, 1.2, 0.06, sutherland=True)
        f = W.conduction_fields(p)
    else:
        p = W.channel(nx=190, ny=9, U0=0.01, period=37.5)
        f = W.rest_fields(p)
    a = lbddf.Solver(p).init(*f)
    a.set_graph_steps(0)
    b = lbddf.Solver(p).init(*f)
    print(f"[case] graph vs host launches, {case} {p['nx']}x{p['ny']}, 4 replays of 32 steps + 4", flush=True)
    for i in range(4):
        a.step(32)
        b.step(32)
        b.macros()
        b.diag(check=False)
        assert a.time == b.time == 32 * (i + 1)
        assert np.array_equal(a.populations(), b.populations()), f"replay {i}"
    a.step(4)
    b.step(4)
    assert a.time == b.time == 132
    assert np.array_equal(a.populations(), b.populations())
