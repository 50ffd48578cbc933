"""Seeded synthetic workloads: problem set-ups and initial fields.

This module is the one place that both the FP64 oracle and the GPU path take
their inputs from.  It holds no lattice Boltzmann arithmetic: it only

* draws seeded random numbers (SplitMix64, Box-Muller), and
* writes the physical set-ups of the paper's test problems down as plain
  parameter dictionaries in lattice units (delta_x = delta_t = c = 1, so
  R*T0 = 1/3, Sec. II / Sec. IV-A).

Every solver (oracle or GPU) turns such a dictionary into its own relaxation
rates, equilibria and boundary rules by itself.

Parameter dictionary keys (all optional except nx, ny):

  nx, ny           node counts, boundary nodes included (walls sit on nodes)
  rho0, T0, R, b   reference density / temperature, gas constant, degrees of
                   freedom (gamma = (b+2)/b, Sec. III-C-1)
  Pr               Prandtl number, Pr = (tau_f - 1/2)/tau_h (Sec. III-C-2)
  tau_f            shear relaxation time of the MRT scheme (viscosity
                   mu = (tau_f - 1/2) p) for visc == "const_tau"
  s_e, s_zeta, s_q relaxation rates of the non-hydrodynamic moments (Eq. 40);
                   s_e / s_zeta <= 0 means "tied to 1/tau_f"
  tau_rho, tau_j   relaxation times of the conserved moments (Eq. 40)
  visc             "const_tau" | "const_mu" | "power" | "sutherland"
  mu_ref, T_ref    viscosity at the reference temperature
  visc_n           exponent of the power law mu ~ T^n (Sec. IV-A)
  suth_S           Sutherland constant S in lattice temperature units (Eq. 59)
  g                gravity; the force density is a = (0, -rho g) (Sec. IV-C)
  energy           "total" (Eq. 18b / 47) | "internal" (internal-energy form,
                   Eq. 38)
  heating          viscous-heating coupling term of Eq. 47 on/off
  correction       D2Q9 correction term of Eq. 48-50 on/off
  coupled          True: theta-coupled equilibria (Eq. 18); False: the
                   decoupled theta = 1, p = rho R T0 model (Eq. 8)
  collision        "mrt" (Eq. 44) | "bgk" (Eq. 34)
  rho_extrap       "pressure" | "density": how a Dirichlet-temperature wall
                   takes its density from the fluid neighbour
  sides            four dicts for x-, x+, y-, y+ with keys kind ("periodic",
                   "wall", "adiabatic", "inlet", "outlet"), ux, uy, T,
                   amp (inlet velocity amplitude), period (inlet period, steps)
  storage          "f32" | "f16" | "bf16" (GPU population storage only)
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1109667200

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of Steele, Lea & Flood's SplitMix64.

    The k-th output (0-based) is the mix function applied to
    seed + (k+1) * 0x9E3779B97F4A7C15 (mod 2**64), so the stream can be
    evaluated for any index range without generating its prefix.
    """
    z = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    t = np.empty_like(z)
    with np.errstate(over="ignore"):
        # in place: the same arithmetic without a temporary per operation
        np.multiply(z, _GAMMA, out=z)
        np.add(z, np.uint64(seed & 0xFFFFFFFFFFFFFFFF), out=z)
        for sh, m in ((30, _M1), (27, _M2)):
            np.right_shift(z, np.uint64(sh), out=t)
            np.bitwise_xor(z, t, out=z)
            np.multiply(z, m, out=z)
        np.right_shift(z, np.uint64(31), out=t)
        np.bitwise_xor(z, t, out=z)
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, count, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(seed: int, count: int) -> np.ndarray:
    """Standard normal deviates by the Box-Muller transform of SplitMix64.

    Outputs 2k and 2k+1 of the generator give u1 in (0, 1] and u2 in [0, 1);
    they yield r cos(2 pi u2) and r sin(2 pi u2) with r = sqrt(-2 ln u1).
    """
    npairs = (count + 1) // 2
    out = np.empty(2 * npairs, dtype=np.float64)
    chunk = 1 << 22  # pairs per chunk, bounds the temporaries
    for p0 in range(0, npairs, chunk):
        n = min(chunk, npairs - p0)
        z = splitmix64(seed, 2 * n, start=2 * p0)
        u1 = ((z[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)
        u2 = (z[1::2] >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        r = np.sqrt(-2.0 * np.log(u1))
        ang = (2.0 * math.pi) * u2
        out[2 * p0:2 * (p0 + n):2] = r * np.cos(ang)
        out[2 * p0 + 1:2 * (p0 + n):2] = r * np.sin(ang)
    return out[:count]


# --------------------------------------------------------------------------
# parameter dictionaries
# --------------------------------------------------------------------------
def side(kind="periodic", ux=0.0, uy=0.0, T=1.0, amp=0.0, period=1.0) -> dict:
    return dict(kind=kind, ux=float(ux), uy=float(uy), T=float(T), amp=float(amp), period=float(period))


def base_params(nx: int, ny: int, **kw) -> dict:
    """Lattice-unit defaults: rho0 = T0 = 1, R = 1/3 so that c = sqrt(3 R T0) = 1."""
    p = dict(
        nx=int(nx), ny=int(ny), rho0=1.0, T0=1.0, R=1.0 / 3.0, b=3.0, Pr=0.71,
        tau_f=0.8, s_e=0.0, s_zeta=0.0, s_q=1.5, tau_rho=1.0, tau_j=1.0,
        visc="const_tau", mu_ref=0.1, T_ref=1.0, visc_n=1.0, suth_S=110.5 / 600.0,
        g=0.0, energy="total", heating=True, correction=True, coupled=True,
        collision="mrt", rho_extrap="pressure",
        sides=[side(), side(), side(), side()], storage="f32",
    )
    p.update(kw)
    return p


def cavity_gravity(Ra: float, Pr: float, mu_r: float, dT: float, H: float, T_r: float = 1.0,
                   rho0: float = 1.0) -> float:
    """Gravity from the Rayleigh number of Eq. 57 with beta = 1/T_r (Eq. 58).

    Ra = g beta dT H^3 Pr / nu_r^2 with nu_r = mu_r / rho0.
    """
    nu = mu_r / rho0
    return Ra * nu * nu * T_r / (dT * H ** 3 * Pr)


# --------------------------------------------------------------------------
# the test problems (Sec. IV) as synthetic set-ups
# --------------------------------------------------------------------------
def couette(nx=4, ny=64, U=0.1, Pr=0.71, tau_f=1.25, storage="f32") -> dict:
    """Thermal Couette flow with both walls at T0 (viscous heating only).

    Lower wall at rest, upper wall moving at U, x periodic, total-energy
    form with the heating term, no correction term (Sec. IV-A).
    Relaxation rates as in Sec. IV-A: s_e = s_zeta = s_q = 1.5.
    """
    return base_params(
        nx, ny, Pr=Pr, tau_f=tau_f, s_e=1.5, s_zeta=1.5, s_q=1.5,
        energy="total", heating=True, correction=False,
        sides=[side(), side(), side("wall", 0.0, 0.0, 1.0), side("wall", U, 0.0, 1.0)],
        storage=storage,
    )


def couette_paper(Pr: float, Ma: float, nx=10, ny=62, b=3.0, mu0=0.25, storage="f32") -> dict:
    """The paper's Couette case: adiabatic lower wall, mu = mu0 (T/T0)^n, n = 1.

    Upper wall at T0 moving at U = Ma sqrt(gamma R T0) (Sec. IV-A, Eq. 52).
    """
    gamma = (b + 2.0) / b
    U = Ma * math.sqrt(gamma / 3.0)
    return base_params(
        nx, ny, b=b, Pr=Pr, s_e=1.5, s_zeta=1.5, s_q=1.5, visc="power", mu_ref=mu0, T_ref=1.0,
        visc_n=1.0, energy="total", heating=True, correction=False,
        sides=[side(), side(), side("adiabatic", 0.0, 0.0, 1.0), side("wall", U, 0.0, 1.0)],
        storage=storage,
    )


def cavity(n: int, Ra: float, dT_over_T0: float, mu_r: float, Pr=0.71, sutherland=False,
           storage="f32") -> dict:
    """Differentially heated square cavity (Sec. IV-C).

    Hot wall at x = 0, cold wall at x = H, adiabatic top and bottom, walls on
    the outermost nodes (H = n - 1).  Internal-energy form (Eq. 38) with the
    correction term and gravity a = (0, -rho g).  T0 = T_r = 1.
    """
    H = n - 1
    g = cavity_gravity(Ra, Pr, mu_r, dT_over_T0, H)
    return base_params(
        n, n, Pr=Pr, s_e=0.0, s_zeta=0.0, s_q=1.5,
        visc="sutherland" if sutherland else "const_mu", mu_ref=mu_r, T_ref=1.0,
        g=g, energy="internal", heating=False, correction=True,
        sides=[side("wall", 0.0, 0.0, 1.0 + dT_over_T0 / 2), side("wall", 0.0, 0.0, 1.0 - dT_over_T0 / 2),
               side("adiabatic"), side("adiabatic")],
        storage=storage,
    )


def periodic(n: int, ny: int | None = None, storage="f32", tau_f=0.8) -> dict:
    """Fully periodic box, total energy with heating and the correction term."""
    return base_params(n, ny if ny is not None else n, tau_f=tau_f, s_q=1.5, energy="total",
                       heating=True, correction=True, storage=storage)


def channel(nx=2048, ny=256, U0=0.01, period=200.0, tau_f=0.8, Pr=0.71, b=3.0, storage="f32",
            correction=True, coupled=True) -> dict:
    """Acoustic channel: velocity/density/temperature source at x = 0 (Eq. 53-54),
    zero-gradient outlet at x = nx-1, periodic in y (Sec. IV-B)."""
    return base_params(
        nx, ny, tau_f=tau_f, Pr=Pr, b=b, s_q=1.5, energy="total", heating=True,
        correction=correction, coupled=coupled,
        sides=[side("inlet", amp=U0, period=period), side("outlet"), side(), side()],
        storage=storage,
    )


# --------------------------------------------------------------------------
# initial fields (row-major [y][x] float64 arrays)
# --------------------------------------------------------------------------
def rest_fields(p: dict):
    shape = (p["ny"], p["nx"])
    return (np.full(shape, p["rho0"]), np.zeros(shape), np.zeros(shape), np.full(shape, p["T0"]))


def gaussian_fields(p: dict, sigma: float = 1e-3, k: int = 4):
    """Independent N(0, sigma^2) perturbations of rho (about rho0), u_x, u_y and
    T/T0 (about 1), drawn from one stream in the order rho, u_x, u_y, T."""
    ny, nx = p["ny"], p["nx"]
    n = nx * ny
    z = gaussian(SEED_BASE + k, 4 * n) * sigma
    rho = p["rho0"] + z[0:n]
    ux = z[n:2 * n]
    uy = z[2 * n:3 * n]
    T = p["T0"] * (1.0 + z[3 * n:4 * n])
    return tuple(a.reshape(ny, nx) for a in (rho, ux, uy, T))


def noisy_temperature_fields(p: dict, amp: float = 1e-6, k: int = 2):
    """Rest state with T = T0 (1 + U(-1, 1) * amp)."""
    ny, nx = p["ny"], p["nx"]
    u = uniform01(SEED_BASE + k, nx * ny).reshape(ny, nx)
    rho, ux, uy, _ = rest_fields(p)
    T = p["T0"] * (1.0 + amp * (2.0 * u - 1.0))
    return rho, ux, uy, T


def conduction_fields(p: dict, amp: float = 1e-6, k: int = 3):
    """Pure-conduction start of the cavity: T linear between the x walls,
    uniform pressure (rho = rho0 T0 / T), fluid at rest, plus seeded uniform
    noise T0 U(-1, 1) amp on T (the paper states no initial condition)."""
    ny, nx = p["ny"], p["nx"]
    Th, Tc = p["sides"][0]["T"], p["sides"][1]["T"]
    x = np.arange(nx) / (nx - 1)
    T = np.broadcast_to(Th + (Tc - Th) * x, (ny, nx)).copy()
    u = uniform01(SEED_BASE + k, nx * ny).reshape(ny, nx)
    T[:, 1:-1] += p["T0"] * amp * (2.0 * u[:, 1:-1] - 1.0)
    rho = p["rho0"] * p["T0"] / T
    return rho, np.zeros((ny, nx)), np.zeros((ny, nx)), T


def serving_mix(n_requests: int, sizes=(64, 128, 256, 512, 1024), Ra_range=(1e3, 1e6), dT_range=(0.02, 1.2),
                rate: float = 50.0, Pr: float = 0.71, storage: str = "f32", k: int = 5, u_target: float = 0.05,
                tau_min: float = 0.56, nu_max: float = 0.1):
    """Seeded stream of cavity requests with Poisson arrivals.

    Per request, from one SplitMix64 stream (seed SEED_BASE + k): the
    exponential arrival gap (rate per second), the grid edge (uniform over
    `sizes`), Ra (log-uniform) and dT/T0 (uniform).  The viscosity is chosen
    so that the buoyancy velocity nu sqrt(Ra / Pr) / H equals `u_target`,
    with tau_f(T_r) = 3 nu + 1/2 kept >= tau_min (requests at that bound are
    flagged "under_resolved") and nu <= nu_max (flagged "viscosity_capped");
    large dT (> 0.2) uses the Sutherland law and energy-mode rates
    s_e = s_zeta = 1.5.  Returns a
    list of dicts with keys t (arrival, s), params, n, Ra, dT, flags.
    """
    u = uniform01(SEED_BASE + k, 4 * n_requests).reshape(n_requests, 4)
    out, t = [], 0.0
    for i in range(n_requests):
        t += -math.log(1.0 - u[i, 0]) / rate
        n = int(sizes[min(int(u[i, 1] * len(sizes)), len(sizes) - 1)])
        Ra = 10.0 ** (math.log10(Ra_range[0]) + u[i, 2] * (math.log10(Ra_range[1]) - math.log10(Ra_range[0])))
        dT = dT_range[0] + u[i, 3] * (dT_range[1] - dT_range[0])
        H = n - 1
        nu = u_target * H * math.sqrt(Pr / Ra)
        flags = []
        if 3 * nu + 0.5 < tau_min:
            nu = (tau_min - 0.5) / 3
            flags.append("under_resolved")
        elif nu > nu_max:
            # the paper's viscosities stay at or below 0.1 (Sec. IV-C); larger
            # ones (tau_f near 2 at a hot wall) diverge at large dT
            nu = nu_max
            flags.append("viscosity_capped")
        p = cavity(n, Ra, dT, nu, Pr=Pr, sutherland=dT > 0.2, storage=storage)
        if dT > 0.2:
            # large dT: energy-mode rates untied from tau_f (allowed for
            # low-Mach flows, Sec. III), as the tied form diverges at the
            # cold bottom corner on fine grids
            p.update(s_e=1.5, s_zeta=1.5)
        out.append(dict(t=t, params=p, n=n, Ra=Ra, dT=dT, flags=flags))
    return out
