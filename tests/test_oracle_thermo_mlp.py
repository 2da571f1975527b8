"""Pins of the oracle's van der Waals thermodynamics and of its FP64 network.

Thermodynamics: the equal-area densities must have equal pressure and equal
chemical potential (checked with formulas independent of the solver), obey
the law of corresponding states, and approach the mean-field critical law
(rho_l - rho_v)/rho_c = 4 sqrt(1 - T/Tc) near T_c; the surface tension of the
square-gradient model scales as sqrt(kappa) and vanishes as (1 - T/Tc)^{3/2}.

Network: back-propagated gradients against central finite differences, and
Adam against its textbook form on a quadratic.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle.mlp as M
import oracle.thermo as TH
import synth


@pytest.mark.parametrize("Tr", [0.65, 0.8, 0.9, 0.97])
def test_maxwell_equal_pressure_chemical_potential_and_area(Tr):
    a, b = synth.A_ATTR, synth.B_EXCL
    T = Tr * synth.T_CRIT
    rl, rv, Pc = TH.coexistence(T, a=a, b=b)
    assert rl > 1.0 > rv > 0
    assert TH.pressure(rl, T, a, b) == pytest.approx(Pc, rel=1e-10)
    assert TH.pressure(rv, T, a, b) == pytest.approx(Pc, rel=1e-10)
    # chemical potential from the Gibbs-Duhem integral of dP/rho along the
    # isotherm (numerical quadrature over the whole loop)
    dmu, _ = quad(lambda r: (T / (1 - b * r) ** 2 - 2 * a * r) / r, rv, rl, limit=200, epsrel=1e-12)
    assert abs(dmu) < 1e-9 * T
    # equal area in the P-v plane, by quadrature
    area, _ = quad(lambda v: T / (v - b) - a / v ** 2 - Pc, 1 / rl, 1 / rv, limit=400, epsrel=1e-12)
    assert abs(area) < 1e-9 * Pc / rv


def test_corresponding_states_and_critical_law():
    base = [TH.coexistence(0.9 * 0.02, a=27 * (1 / 3) * 0.02 / 8, b=1 / 3)]
    other = TH.coexistence(0.9 * 0.5, a=27 * 0.1 * 0.5 / 8, b=0.1)  # rho_c = 10/3
    assert other[0] * 0.3 == pytest.approx(base[0][0], rel=1e-9)
    assert other[1] * 0.3 == pytest.approx(base[0][1], rel=1e-9)
    for eps in (1e-4, 1e-5):
        rl, rv, _ = TH.coexistence((1 - eps) * 0.02)
        assert (rl - rv) / (4 * math.sqrt(eps)) == pytest.approx(1.0, abs=4 * math.sqrt(eps) + 1e-6)


def test_surface_tension_scaling():
    s1 = TH.surface_tension(0.9 * 0.02, 0.1)
    s2 = TH.surface_tension(0.9 * 0.02, 0.4)
    assert s2 / s1 == pytest.approx(2.0, rel=1e-9)
    a = TH.surface_tension((1 - 1e-3) * 0.02, 0.1)
    b = TH.surface_tension((1 - 4e-3) * 0.02, 0.1)
    assert b / a == pytest.approx(8.0, rel=0.02)  # (1 - T/Tc)^{3/2}
    assert TH.surface_tension(0.65 * 0.02, 0.1) > TH.surface_tension(0.9 * 0.02, 0.1) > 0


def test_cs_critical_point_and_virial_series():
    """Carnahan-Starling contact factor with mean-field attraction,
    P = rho RT Z(eta) - a rho^2, eta = b rho/4: the critical point has
    eta_c = 0.1304 and Z_c = P_c/(rho_c R T_c) = 0.3590 whatever a and b
    (R T_c = 0.3773 a/b); the hard-sphere factor reproduces the virial series
    Z = 1 + 4 eta + 10 eta^2 + 18 eta^3 + ... that the Carnahan-Starling form
    is built on (its coefficients are n^2 + n - 2)."""
    for a, b in ((synth.A_CS, synth.B_CS), (0.1, 0.25)):
        rc, Tc, Pc = TH.critical_point(1.0, a, b, "cs")
        assert b * rc / 4 == pytest.approx(0.1304, abs=1e-4)
        assert Pc / (rc * Tc) == pytest.approx(0.3590, abs=1e-4)
        assert Tc * b / a == pytest.approx(0.3773, abs=1e-4)
        # the critical point is where dP/drho and d2P/drho2 vanish (central differences)
        h = 1e-4 * rc
        P = lambda r: TH.pressure(r, Tc, a, b, "cs")
        assert abs(P(rc + h) - P(rc - h)) / (2 * h) < 1e-6 * Pc / rc
        assert abs(P(rc + h) - 2 * P(rc) + P(rc - h)) / h ** 2 < 1e-4 * Pc / rc ** 2
    b = 0.4
    for eta in (1e-3, 2e-3):
        Z = TH.compressibility(4 * eta / b, b, "cs")
        assert (Z - 1 - 4 * eta - 10 * eta ** 2) / eta ** 3 == pytest.approx(18.0 + 28.0 * eta, rel=1e-3)


@pytest.mark.parametrize("Tr", [0.6, 0.75, 0.9, 0.97])
def test_cs_maxwell_equal_pressure_chemical_potential_and_area(Tr):
    """The equal-area densities of the Carnahan-Starling fluid have equal
    pressure and equal chemical potential: the chemical potential by the
    Gibbs-Duhem integral of (1/rho) dP/drho along the isotherm with dP/drho
    from finite differences (independent of the closed-form mu), and the
    closed-form mu agrees; the free energy satisfies rho mu - psi = P."""
    a, b = synth.A_CS, synth.B_CS
    _, Tc, _ = TH.critical_point(1.0, a, b, "cs")
    T = Tr * Tc
    rl, rv, Pc = TH.coexistence(T, 1.0, a, b, "cs")
    assert rl > 1.0 > rv > 0
    assert TH.pressure(rl, T, a, b, "cs") == pytest.approx(Pc, rel=1e-9)
    assert TH.pressure(rv, T, a, b, "cs") == pytest.approx(Pc, rel=1e-9)
    dPdr = lambda r: (TH.pressure(r * (1 + 1e-7), T, a, b, "cs") - TH.pressure(r * (1 - 1e-7), T, a, b, "cs")) / (2e-7 * r)
    dmu, _ = quad(lambda r: dPdr(r) / r, rv, rl, limit=200, epsrel=1e-11)
    assert abs(dmu) < 1e-7 * T
    assert TH.chemical_potential(rl, T, a, b, "cs") - TH.chemical_potential(rv, T, a, b, "cs") == \
        pytest.approx(0.0, abs=1e-9 * T)
    for r in (rv, 0.5 * (rl + rv), rl):
        mu = TH.chemical_potential(r, T, a, b, "cs")
        assert r * mu - TH.free_energy_density(r, T, a, b, "cs") == pytest.approx(TH.pressure(r, T, a, b, "cs"),
                                                                                  rel=1e-10, abs=1e-15)


def test_vdw_free_energy_and_quadrature_construction_agree():
    """The quadrature form of the equal-area rule (used for any closure)
    reproduces the closed-form van der Waals construction."""
    for Tr in (0.65, 0.9):
        T = Tr * synth.T_CRIT
        ref = TH.coexistence(T)
        got = TH._coexistence_quadrature(T, 1.0, synth.A_ATTR, synth.B_EXCL, "vdw")
        np.testing.assert_allclose(got, ref, rtol=1e-10)


def _batch(n=37, seed=3):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0.65, 0.95, n), rng.uniform(15, 80, n), rng.uniform(0, 3, n)], 1)
    Y = rng.uniform(0.05, 2.2, n)
    return X, Y


def test_mlp_shapes_and_gradient_matches_finite_differences():
    """Backprop against central differences (h = 1e-6)."""
    theta = synth.xavier_params()
    assert theta.size == M.NPARAM == 8641
    theta = theta + 0.05 * np.random.default_rng(1).standard_normal(theta.size)  # non-zero biases
    X, Y = _batch()
    g = M.grad(theta, X, Y)
    idx = np.random.default_rng(2).choice(theta.size, 120, replace=False)
    idx = np.concatenate([idx, [8640, 8639, 8576, 0, 191, 192]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (M.loss(theta + e, X, Y) - M.loss(theta - e, X, Y)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_matches_textbook_on_quadratic():
    """Adam on L = |p|^2/2 from p0: the first step moves every coordinate by
    -lr sign(p0) (bias-corrected m/sqrt(v) = g/|g|)."""
    p0 = np.array([1.0, -2.0, 0.5])
    p1, m, v = M.adam_step(p0, np.zeros(3), np.zeros(3), p0.copy(), 1, lr=1e-2)
    assert np.allclose(p1, p0 - 1e-2 * np.sign(p0) * (np.abs(p0) / (np.abs(p0) + 1e-8)), rtol=1e-14)
    # many steps converge to the minimum
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = M.adam_step(p, m, v, p.copy(), t, lr=1e-2)
    assert np.abs(p).max() < 1e-2


def test_mlp_training_reduces_loss():
    X, _ = _batch(200, 4)
    Y = 1.0 + 0.5 * np.tanh((X[:, 2] - 1.0) * 3.0)
    theta, hist = M.train(synth.xavier_params(), X, Y, 300, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
