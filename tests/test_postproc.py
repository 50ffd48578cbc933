"""Post-processing of the validation quantities on fields with known answers."""
import math

import numpy as np
import pytest

from paper_1109_6672_amd import postproc as P, workloads as W


@pytest.mark.parametrize("n", [33, 40])
def test_pure_conduction_has_unit_nusselt_number(n):
    p = W.cavity(n, 1e4, 0.02, 0.02)
    H = n - 1
    x = np.arange(n) / H
    T = np.tile(1.01 - 0.02 * x, (n, 1))
    m = P.cavity_metrics(p, np.zeros_like(T), np.zeros_like(T), T)
    assert abs(m["Nu"] - 1.0) < 1e-12


def test_nusselt_integrates_a_varying_wall_gradient_exactly():
    """T quadratic in x near the wall (the one-sided difference is exact) with
    a wall gradient linear in y (the trapezoidal rule is exact)."""
    n = 41
    H = n - 1
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    a, c = 1e-6, -5e-4
    # dT/dx at x = H: 2 a H (1 + y/H) + c (1 + y/H) = (2 a H + c)(1 + y/H)
    T = 1.0 + (a * X ** 2 + c * X) * (1 + Y / H)
    p = W.cavity(n, 1e4, 0.02, 0.02)
    m = P.cavity_metrics(p, np.zeros_like(T), np.zeros_like(T), T)
    g = abs(2 * a * H + c)
    want = g * 1.5 * H / 0.02
    assert abs(m["Nu"] / want - 1) < 1e-12


@pytest.mark.parametrize("n", [41, 42])
def test_midline_peaks_and_their_positions(n):
    H = n - 1
    p = W.cavity(n, 1e4, 0.02, 0.02)
    chi = 0.02 / 0.71
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    ux = 1e-3 * np.exp(-((Y - 30) / 4.0) ** 2) * np.ones_like(X)       # peak at y = 30 on every column
    uy = 2e-3 * np.exp(-((X - 7) / 3.0) ** 2) * np.ones_like(Y)        # peak at x = 7 on every row
    m = P.cavity_metrics(p, ux, uy, np.ones_like(X))
    assert m["y_max"] == 30 / H and m["x_max"] == 7 / H
    assert abs(m["u_max"] - 1e-3 * H / chi) < 1e-12 * H / chi
    assert abs(m["v_max"] - 2e-3 * H / chi) < 1e-12 * H / chi


def test_even_grid_midline_averages_the_two_central_lines():
    n = 42
    ux = np.zeros((n, n))
    ux[10, 20] = 1.0
    ux[10, 21] = 3.0
    p = W.cavity(n, 1e4, 0.02, 0.02)
    m = P.cavity_metrics(p, ux, np.zeros_like(ux), np.ones_like(ux))
    assert abs(m["u_max"] - 2.0 * (n - 1) / (0.02 / 0.71)) < 1e-9


def test_envelope_fit_recovers_the_decay_rate():
    x = np.arange(20, 1500, dtype=float)
    beta, U0 = P.envelope_fit(x, 0.01 * np.exp(-2.7e-4 * x))
    assert abs(beta / 2.7e-4 - 1) < 1e-9 and abs(U0 / 0.01 - 1) < 1e-9
    assert math.isfinite(beta)
