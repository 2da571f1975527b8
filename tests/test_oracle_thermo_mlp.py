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
