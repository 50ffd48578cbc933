"""Pins of the oracle's local algebra against what the paper and the mathematics fix.

Every check compares the oracle's output with an independent statement:
quadrature identities of the lattice, the moment-basis polynomials that the
rows of M stand for, exact rational inverses, the velocity moments that
Eq. 19-21 and Eq. 26/28 prescribe, the textbook decoupled equilibria (Eq. 8),
and conservation properties that hold for any input.
"""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle import oracle as O
from paper_1109_6672_amd import workloads as W

RNG = np.random.default_rng(11096672)


def _ora(**kw):
    return O.Oracle(W.base_params(1, 1, **kw))


def _random_states(n=20, T0=1.0, big=False):
    for _ in range(n):
        rho = RNG.uniform(0.5, 2.0)
        ux, uy = RNG.uniform(-0.2, 0.2, 2)
        T = T0 * RNG.uniform(0.4, 1.6) if big else T0 * RNG.uniform(0.9, 1.1)
        yield rho, ux, uy, T


# ---------------------------------------------------------------- lattice
def test_lattice_is_a_fifth_degree_quadrature():
    """Eq. 6 + weights: sum w e^(2k) moments of the Gauss-Hermite rule with RT0 = 1/3."""
    ex, ey, w = O.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    assert abs(w.sum() - 1) < 1e-15
    for i in range(2):
        assert abs((w * e[:, i]).sum()) < 1e-15
    cs2 = 1.0 / 3.0
    for i, j in product(range(2), repeat=2):
        assert abs((w * e[:, i] * e[:, j]).sum() - cs2 * (i == j)) < 1e-15
    for i, j, k in product(range(2), repeat=3):
        assert abs((w * e[:, i] * e[:, j] * e[:, k]).sum()) < 1e-15
    d = np.eye(2)
    for i, j, k, l in product(range(2), repeat=4):
        want = cs2 * cs2 * (d[i, j] * d[k, l] + d[i, k] * d[j, l] + d[i, l] * d[j, k])
        assert abs((w * e[:, i] * e[:, j] * e[:, k] * e[:, l]).sum() - want) < 1e-15
    # nine distinct velocities, rest + 4 axis + 4 diagonal, ordered as in Eq. 6
    assert len({(a, b) for a, b in zip(ex, ey)}) == 9
    assert list(ex[1:5] ** 2 + ey[1:5] ** 2) == [1, 1, 1, 1]
    assert list(ex[5:] ** 2 + ey[5:] ** 2) == [2, 2, 2, 2]
    ang = np.degrees(np.arctan2(ey[1:], ex[1:])) % 360
    assert list(ang) == [0, 90, 180, 270, 45, 135, 225, 315]


# ---------------------------------------------------------------- matrices
def _frac(M):
    return [[Fraction(float(x)).limit_denominator(1000) for x in row] for row in M]


def test_transform_matrices_are_exact_inverses():
    """Eq. B1 times Eq. B2 is the identity in exact rational arithmetic."""
    M, Mi = O.matrices()
    A, B = _frac(M), _frac(Mi)
    for r in range(9):
        for c in range(9):
            s = sum(A[r][k] * B[k][c] for k in range(9))
            assert s == (1 if r == c else 0), (r, c, s)


def test_transform_rows_are_the_named_moments():
    """Rows of M are the moments (rho, e, zeta, j_x, q_x, j_y, q_y, p_xx, p_xy)
    of the D2Q9 MRT basis, written as polynomials of the velocity."""
    M, _ = O.matrices()
    ex, ey, _ = O.lattice()
    e2 = ex ** 2 + ey ** 2
    rows = [
        np.ones(9), 3 * e2 - 4, (9 * e2 ** 2 - 21 * e2 + 8) / 2, ex, (3 * e2 - 5) * ex, ey,
        (3 * e2 - 5) * ey, ex ** 2 - ey ** 2, ex * ey,
    ]
    for k, row in enumerate(rows):
        np.testing.assert_array_equal(M[k], row)
    # orthogonal rows (M M^T diagonal)
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=0)


# ---------------------------------------------------------------- equilibria
@pytest.mark.parametrize("T0,R", [(1.0, 1.0 / 3.0), (2.0, 1.0 / 6.0)])
def test_feq_moments_eq19a_and_eq20(T0, R):
    o = _ora(T0=T0, R=R)
    ex, ey, _ = O.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    d = np.eye(2)
    RT0 = R * T0
    for rho, ux, uy, T in _random_states(T0=T0, big=True):
        f = o.feq(rho, ux, uy, T)
        u = np.array([ux, uy])
        RT = R * T
        th = T / T0
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(e.T @ f, rho * u, atol=1e-14)
        P = np.einsum("a,ai,aj->ij", f, e, e)
        np.testing.assert_allclose(P, rho * np.outer(u, u) + rho * RT * d, atol=1e-14)
        # Eq. 20: third moment, with the diagonal deviation 3 rho RT0 u (1 - theta)
        for i, j, k in product(range(2), repeat=3):
            got = (f * e[:, i] * e[:, j] * e[:, k]).sum()
            want = rho * RT * (u[k] * d[i, j] + u[j] * d[i, k] + u[i] * d[j, k])
            if i == j == k:
                want += 3 * rho * RT0 * u[i] * (1 - th)
            assert abs(got - want) < 1e-14, (i, j, k)


@pytest.mark.parametrize("T0,R", [(1.0, 1.0 / 3.0), (2.0, 1.0 / 6.0)])
def test_heq_moments_eq19b(T0, R):
    o = _ora(T0=T0, R=R, b=3.0)
    ex, ey, _ = O.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    d = np.eye(2)
    for rho, ux, uy, T in _random_states(T0=T0, big=True):
        h = o.heq(rho, ux, uy, T)
        u = np.array([ux, uy])
        p = rho * R * T
        E = 0.5 * (3.0 * R * T + u @ u)
        assert abs(h.sum() - rho * E) < 1e-14
        np.testing.assert_allclose(e.T @ h, (rho * E + p) * u, atol=1e-14)
        P = np.einsum("a,ai,aj->ij", h, e, e)
        np.testing.assert_allclose(P, (rho * E + 2 * p) * np.outer(u, u) + p * (E + R * T) * d, atol=1e-14)


def test_internal_energy_equilibrium():
    """Internal-energy form: h_eq = b R T f_eq / 2, so sum h_eq = rho c_v T."""
    o = _ora(energy="internal", heating=False, b=5.0)
    for rho, ux, uy, T in _random_states():
        h, f = o.heq(rho, ux, uy, T), o.feq(rho, ux, uy, T)
        np.testing.assert_allclose(h, 2.5 * T / 3.0 * f, rtol=1e-15)
        assert abs(h.sum() - rho * 2.5 * T / 3.0) < 1e-14


def test_decoupled_and_theta1_reduce_to_eq8():
    """theta = 1, p = p0 gives the decoupled equilibria of Eq. 8 (the textbook
    second-order D2Q9 f_eq, and the total-energy h_eq of Eq. 8b)."""
    ex, ey, w = O.lattice()
    oc = _ora()
    od = _ora(coupled=False)
    for rho, ux, uy, T in _random_states(big=True):
        eu = ex * ux + ey * uy
        u2 = ux * ux + uy * uy
        f8 = rho * w * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * u2)
        E = 0.5 * (3.0 * T / 3.0 + u2)
        p0 = rho / 3.0
        h8 = E * f8 + w * p0 * (3 * eu + 9 * eu ** 2 - 3 * u2 + 0.5 * (3 * (ex ** 2 + ey ** 2) - 2))
        np.testing.assert_allclose(od.feq(rho, ux, uy, T), f8, atol=1e-15)
        np.testing.assert_allclose(od.heq(rho, ux, uy, T), h8, atol=1e-15)
        # the coupled model at T = T0 is the same model
        np.testing.assert_allclose(oc.feq(rho, ux, uy, 1.0), f8, atol=1e-15)
        E1 = 0.5 * (1.0 + u2)
        h81 = E1 * f8 + w * p0 * (3 * eu + 9 * eu ** 2 - 3 * u2 + 0.5 * (3 * (ex ** 2 + ey ** 2) - 2))
        np.testing.assert_allclose(oc.heq(rho, ux, uy, 1.0), h81, atol=1e-15)


def test_moment_equilibria_eq41_is_M_feq():
    o = _ora()
    M, _ = O.matrices()
    for rho, ux, uy, T in _random_states(big=True):
        np.testing.assert_allclose(o.meq(rho, ux, uy, T), M @ o.feq(rho, ux, uy, T), atol=1e-14)


# ---------------------------------------------------------------- sources
def test_correction_eq49_is_Minv_Chat_and_meets_eq26_eq28():
    M, Mi = O.matrices()
    ex, ey, _ = O.lattice()
    for _ in range(10):
        dQx, dQy = RNG.normal(size=2)
        phix, phiy = 3 * (dQx + dQy), dQx - dQy  # Eq. 48
        C = O.correction(phix, phiy)
        Chat = np.zeros(9)
        Chat[1], Chat[7] = phix, phiy
        np.testing.assert_allclose(C, Mi @ Chat, atol=1e-15)
        np.testing.assert_allclose(M @ C, Chat, atol=1e-14)
        assert abs(C.sum()) < 1e-15                                   # Eq. 26
        assert abs((ex * C).sum()) < 1e-15 and abs((ey * C).sum()) < 1e-15
        assert abs((ex * ey * C).sum()) < 1e-15                       # Eq. 28
        assert abs((ex * ex * C).sum() - dQx) < 1e-14
        assert abs((ey * ey * C).sum() - dQy) < 1e-14


def test_forcing_moments_and_eq51():
    """F_alpha has moments (0, a, u a + a u); M F is Eq. 51 with p_xx = 2(u_x a_x - u_y a_y)."""
    o = _ora()
    M, _ = O.matrices()
    ex, ey, _ = O.lattice()
    e = np.stack([ex, ey], 1).astype(float)
    for _ in range(10):
        ux, uy, ax, ay = RNG.normal(size=4) * 0.1
        Fv, Fh = o.forcing(ux, uy, ax, ay)
        u, a = np.array([ux, uy]), np.array([ax, ay])
        assert abs(Fv.sum()) < 1e-15
        np.testing.assert_allclose(e.T @ Fv, a, atol=1e-15)
        np.testing.assert_allclose(np.einsum("a,ai,aj->ij", Fv, e, e), np.outer(u, a) + np.outer(a, u), atol=1e-15)
        np.testing.assert_allclose(M @ Fv, Fh, atol=1e-15)
        assert abs(Fh[7] - 2 * (ux * ax - uy * ay)) < 1e-15


# ---------------------------------------------------------------- transport
def test_transport_relations():
    """mu = (tau_f - 1/2) p; Pr = (tau_f - 1/2)/tau_h; tau_hf = tau_f/(Pr - 1);
    tau_f = mu/p + 1/2 for the viscosity laws; Sutherland ratio (Eq. 59)."""
    o = _ora(Pr=0.71, tau_f=0.8, s_e=0.0, s_zeta=0.0, s_q=1.5)
    t = o.transport(1.0, 1.0)
    tau_h = 2.0 / t["omega_h"] / 2 - 0.5
    assert abs((0.8 - 0.5) / tau_h - 0.71) < 1e-14
    assert abs(t["inv_tau_hf"] - (0.71 - 1) / 0.8) < 1e-15
    np.testing.assert_allclose(t["s"], [1, 1 / 0.8, 1 / 0.8, 1, 1.5, 1, 1.5, 1 / 0.8, 1 / 0.8], rtol=1e-15)
    # tau_hf consistency: mu_energy = (tau_f tau_h / tau_hf + tau_h) p equals (tau_f - 1/2) p
    assert abs((0.8 * tau_h * t["inv_tau_hf"] + tau_h) - 0.3) < 1e-14
    S = 110.5 / 600
    os_ = _ora(visc="sutherland", mu_ref=0.06, T_ref=1.0, suth_S=S)
    for T in (0.4, 1.0, 1.6):
        rho = 1.3
        mu = (os_.transport(rho, T)["tau_f"] - 0.5) * rho * T / 3.0
        Tstar = 273.0 / 600.0  # mu/mu* with mu* = mu(T_ref)/((1/T*)^1.5 (T*+S)/(1+S))
        mustar = 0.06 / ((1 / Tstar) ** 1.5 * (Tstar + S) / (1 + S))
        assert abs(mu - mustar * (T / Tstar) ** 1.5 * (Tstar + S) / (T + S)) < 1e-14
    op = _ora(visc="power", mu_ref=0.25, visc_n=1.0)
    for T in (0.8, 1.2):
        assert abs((op.transport(1.1, T)["tau_f"] - 0.5) * 1.1 * T / 3.0 - 0.25 * T) < 1e-14


# ---------------------------------------------------------------- collision
def _random_pops(o, rho=1.0, T=1.0, scale=0.02):
    f = o.feq(rho, 0.05, -0.03, T) * (1 + scale * RNG.normal(size=9))
    h = o.heq(rho, 0.05, -0.03, T) * (1 + scale * RNG.normal(size=9))
    return np.concatenate([f, h])


@pytest.mark.parametrize("energy,g", [("total", 0.0), ("total", 1e-3), ("internal", 1e-3)])
def test_collision_conserves_mass_momentum_energy(energy, g):
    """Per node: sum f* = sum f, sum e f* = sum e f + a, sum h* = sum h,
    including the coupling term (Z = e.u) and the correction term."""
    o = _ora(energy=energy, heating=(energy == "total"), g=g, Pr=0.71, tau_f=0.7, s_q=1.2, s_e=1.1, s_zeta=1.3)
    ex, ey, _ = O.lattice()
    for _ in range(10):
        pin = _random_pops(o, rho=RNG.uniform(0.8, 1.2), T=RNG.uniform(0.7, 1.3))
        phix, phiy = RNG.normal(size=2) * 1e-2
        out = o.node_collide(pin, phix, phiy)
        rho = pin[:9].sum()
        assert abs(out[:9].sum() - rho) < 1e-14
        assert abs((ex * out[:9]).sum() - (ex * pin[:9]).sum()) < 1e-14
        assert abs((ey * out[:9]).sum() - ((ey * pin[:9]).sum() - rho * g)) < 1e-14
        assert abs(out[9:].sum() - pin[9:].sum()) < 1e-14


def test_mrt_with_single_rate_is_bgk():
    """S = (1/tau_f) I turns Eq. 44 into the BGK scheme Eq. 34 (with its source
    sign as Eq. 32-33 give it) - also with correction, forcing and heating."""
    kw = dict(tau_f=0.7, Pr=0.71, g=2e-3, tau_rho=0.7, tau_j=0.7, s_e=1 / 0.7, s_zeta=1 / 0.7, s_q=1 / 0.7)
    om, ob = _ora(collision="mrt", **kw), _ora(collision="bgk", **kw)
    for _ in range(10):
        pin = _random_pops(om, T=RNG.uniform(0.8, 1.2))
        phix, phiy = RNG.normal(size=2) * 1e-2
        np.testing.assert_allclose(om.node_collide(pin, phix, phiy), ob.node_collide(pin, phix, phiy), atol=2e-16 * 8)


def test_equilibrium_is_a_fixed_point_of_the_collision():
    o = _ora(tau_f=0.9, Pr=2.0)
    for rho, ux, uy, T in _random_states(big=True):
        pin = np.concatenate([o.feq(rho, ux, uy, T), o.heq(rho, ux, uy, T)])
        np.testing.assert_allclose(o.node_collide(pin), pin, atol=1e-15)


def test_moments_recover_the_state():
    """Eq. 46 and Eq. 37 invert the equilibria (T from the total energy)."""
    o = _ora()
    for rho, ux, uy, T in _random_states(big=True):
        pin = np.concatenate([o.feq(rho, ux, uy, T), o.heq(rho, ux, uy, T)])
        np.testing.assert_allclose(o.node_moments(pin), [rho, ux, uy, T], atol=1e-14)
    og = _ora(g=1e-3)
    for rho, ux, uy, T in _random_states(big=True):
        pin = np.concatenate([og.feq(rho, ux, uy, T), og.heq(rho, ux, uy, T)])
        r, vx, vy, _ = og.node_moments(pin)
        # rho u = sum e f + a/2 with a = (0, -rho g)
        assert abs(vx - ux) < 1e-15 and abs(vy - (uy - 0.5e-3)) < 1e-15
