"""Host-side post-processing of macroscopic fields into the quantities the
paper reports for its test problems (no part of the time step).

cavity_metrics - Table II quantities of the differentially heated cavity
                 (Sec. IV-C): average Nusselt number on the cold wall, peak
                 velocities on the mid-lines and where they occur.
envelope_fit   - decay rate of an amplitude profile U(x) = U0 exp(-beta x)
                 (Sec. IV-B, Eq. 55).
"""
from __future__ import annotations

import numpy as np


def _midline(a: np.ndarray, axis: int) -> np.ndarray:
    """Values on the mid-line of a field of shape [ny][nx] (axis 1: the
    vertical line x = H/2; axis 0: the horizontal line y = H/2).  With an
    even node count the line falls between two columns (rows) and their mean
    is taken."""
    n = a.shape[axis]
    i = (n - 1) // 2
    take = (lambda k: a[:, k]) if axis == 1 else (lambda k: a[k, :])
    return take(i) if n % 2 == 1 else 0.5 * (take(i) + take(i + 1))


def cavity_metrics(p: dict, ux: np.ndarray, uy: np.ndarray, T: np.ndarray) -> dict:
    """Table II quantities for a square cavity whose walls lie on the
    outermost nodes (H = n - 1 lattice spacings), hot wall at x = 0, cold
    wall at x = H.

    Nu: (1/dT) times the integral over the cold wall of |dT/dx| (second-order
        one-sided difference, trapezoidal rule).
    u_max, y_max: peak horizontal velocity on the vertical mid-line and its
        height; v_max, x_max: peak vertical velocity on the horizontal
        mid-line and its abscissa.  Velocities in units of chi / H with the
        thermal diffusivity chi = nu / Pr at the reference state, positions
        in units of H (the nodes themselves, no interpolation).
    """
    ny, nx = T.shape
    H = nx - 1
    T_hot, T_cold = p["sides"][0]["T"], p["sides"][1]["T"]
    dT = T_hot - T_cold
    if p["visc"] == "const_tau":
        nu = (p["tau_f"] - 0.5) * p["R"] * p["T0"]
    else:
        nu = p["mu_ref"] / p["rho0"]
    chi = nu / p["Pr"]
    dTdx = (3.0 * T[:, -1] - 4.0 * T[:, -2] + T[:, -3]) / 2.0
    g = np.abs(dTdx)
    Nu = float(np.sum(0.5 * (g[1:] + g[:-1]))) / dT
    u_line = _midline(ux, 1)
    v_line = _midline(uy, 0)
    iu, iv = int(np.argmax(u_line)), int(np.argmax(v_line))
    return dict(Nu=Nu, u_max=float(u_line[iu]) * H / chi, y_max=iu / H, v_max=float(v_line[iv]) * H / chi,
                x_max=iv / H)


def envelope_fit(x: np.ndarray, env: np.ndarray) -> tuple[float, float]:
    """Least-squares fit of log(env) = log(U0) - beta x; returns (beta, U0)."""
    slope, icpt = np.polyfit(np.asarray(x, dtype=np.float64), np.log(np.asarray(env, dtype=np.float64)), 1)
    return float(-slope), float(np.exp(icpt))
