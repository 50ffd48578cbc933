"""The paper's acoustic set-up (Sec. IV-B): a 600 x 4 channel (periodic in y)
driven at x = 0 by a sound source of density amplitude 0.01 and wavelength
50 (Eq. 53-54), sampled over the last period before t = 800, for the
Prandtl numbers of Fig. 3 (0.2, 0.5, 5 at gamma = 5/3) and the ratios of
specific heats of Fig. 4 (5/3, 7/5, 9/7 at Pr = 2), coupled and decoupled
(theta = 1, Fig. 5).  On the GPU path the coupled model's amplitude envelope
follows Eq. 55-56 (fitted decay rate within 3 %, envelope within 7 %: Eq. 56
is the small-attenuation limit, and Pr = 0.2 attenuates most), the
decoupled model's misses it by more than 25 % (the claim of Fig. 5), and
both runs match the FP64 oracle's to the FP32 bar at t = 800.

Coupled at Pr = 5 the scheme (omega_h = 1.79, coupling coefficient
(Pr - 1)/tau_f = 5) carries a growing mode: the FP64 oracle itself
diverges by t = 1600 from rest, and by t = 100 once seeded with 1e-10 of
transverse noise.  The GPU fields are compared with the oracle's at
t = 400, before that mode has grown out of the FP32 rounding; the envelope
is still taken at t = 800."""
import math

import numpy as np
import pytest

from paper_1109_6672_amd import lbddf, workloads as W
from tests.gpu_common import TOL, rel_errors

pytestmark = pytest.mark.gpu

NX, NY, T_M, LAM, MU = 600, 4, 800, 50.0, 0.1


def _setup(Pr, gamma, coupled):
    b = 2.0 / (gamma - 1.0)
    cs = math.sqrt(gamma / 3.0)
    period = LAM / cs
    U = cs * 0.01  # Eq. 54: u = c_s drho / rho0 with drho = 0.01 rho0
    p = W.channel(nx=NX, ny=NY, U0=U, period=period, tau_f=3 * MU + 0.5, Pr=Pr, b=b, correction=False,
                  coupled=coupled)
    cv, cp = b / 6.0, (b + 2.0) / 6.0
    fp = cs / LAM
    beta = 2 * math.pi ** 2 * fp ** 2 / cs ** 3 * ((4 / 3) * MU + 2 * (1 / 3 - 1 / b) * MU
                                                    + (1 / cv - 1 / cp) * MU * cp / Pr)
    return p, cs, period, U, beta


def _envelope(stepper, macros, period):
    """Max |u_x| over the last period before t = T_M."""
    stepper(T_M - int(period) - 1)
    env = np.zeros(NX)
    for _ in range(int(period) + 1):
        stepper(1)
        env = np.maximum(env, np.abs(macros()[1][0]))
    return env


@pytest.mark.parametrize("Pr,gamma", [(0.2, 5 / 3), (0.5, 5 / 3), (5.0, 5 / 3), (2.0, 5 / 3), (2.0, 7 / 5),
                                      (2.0, 9 / 7)])
@pytest.mark.parametrize("coupled", [True, False])
def test_paper_acoustic_setup(gpu, Pr, gamma, coupled):
    from oracle import oracle as O

    p, cs, period, U, beta = _setup(Pr, gamma, coupled)
    s = lbddf.Solver(p).init(*W.rest_fields(p))
    o = O.Oracle(p).init(*W.rest_fields(p))
    t_cmp = 400 if (coupled and Pr >= 5) else T_M  # before the growing mode (see the module docstring)
    if t_cmp < T_M:
        s.step(t_cmp)
        e = rel_errors(s.macros(), o.step(t_cmp).macros())
        s.init(*W.rest_fields(p))
    env = _envelope(lambda n: s.step(n), s.macros, period)
    if t_cmp == T_M:
        e = rel_errors(s.macros(), o.step(T_M).macros())
    x = np.arange(NX)
    sel = (x >= 20) & (x <= min(500, int(cs * (T_M - period)) - 20))
    want = U * np.exp(-beta * x[sel])
    dev = np.abs(env[sel] / want - 1).max()
    fit = -np.polyfit(x[sel], np.log(env[sel]), 1)[0]
    print(f"[case] acoustic Pr={Pr} gamma={gamma:.4f} coupled={coupled}: GPU vs oracle at t={t_cmp} {e}, "
          f"beta fit/Eq.56 {fit / beta:.4f}, envelope max dev {dev:.3f}", flush=True)
    assert max(e) < TOL["f32"], e
    if coupled:
        assert abs(fit / beta - 1) < 0.03 and dev < 0.07
    else:
        assert dev > 0.25
