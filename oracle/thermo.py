"""Van der Waals thermodynamics for the oracle (test infrastructure only).

The paper's closure (eq. EVforce1 and the text after it) gives the Enskog
pressure P_E = rho R T/(1 - b rho) and the mean-field pressure P_V = -a rho^2,
so the bulk pressure is the van der Waals equation P = P_E + P_V.  Figure 1
of the paper compares simulated coexistence densities with Maxwell's
equal-area construction; this module computes that construction and the
flat-interface surface tension of the square-gradient (capillarity kappa)
model, by plain numerical quadrature and bracketing root finding.
"""
from __future__ import annotations

import math

from scipy.integrate import quad
from scipy.optimize import brentq


def pressure(rho, RT, a, b):
    """van der Waals pressure P = rho RT/(1 - b rho) - a rho^2."""
    return rho * RT / (1.0 - b * rho) - a * rho * rho


def critical_point(R, a, b):
    """(rho_c, T_c, P_c) of the van der Waals equation."""
    return 1.0 / (3.0 * b), 8.0 * a / (27.0 * b * R), a / (27.0 * b * b)


def _spinodal_volumes(RT, a, b):
    """Specific volumes where dP/dv = 0 (v = 1/rho), bracketing the unstable branch."""
    # P(v) = RT/(v - b) - a/v^2; dP/dv = -RT/(v-b)^2 + 2a/v^3
    dP = lambda v: -RT / (v - b) ** 2 + 2.0 * a / v ** 3
    vc = 3.0 * b
    lo = brentq(dP, b * (1 + 1e-12), vc)
    hi = brentq(dP, vc, 1e6 * b)
    return lo, hi


def coexistence(T, R=1.0, a=0.0225, b=1.0 / 3.0):
    """Liquid and vapour densities from Maxwell's equal-area rule in the P-v plane.

    For a trial pressure Pc between the spinodal pressures, v_l and v_v are the
    outer roots of P(v) = Pc; the rule demands that the integral of P(v) - Pc
    from v_l to v_v vanishes.  Returns (rho_l, rho_v, P_coex).
    """
    RT = R * T
    _, Tc, _ = critical_point(R, a, b)
    if not (0 < T < Tc):
        raise ValueError("T must lie below T_c")
    P = lambda v: RT / (v - b) - a / (v * v)
    v1, v2 = _spinodal_volumes(RT, a, b)
    Pmin, Pmax = P(v1), P(v2)

    def outer_roots(Pc):
        vl = brentq(lambda v: P(v) - Pc, b * (1 + 1e-14), v1, xtol=1e-300, rtol=1e-15)
        # P(v) < RT/(v - b), so P < Pc/2 at v = b + 2 RT/Pc: a bracket for the vapour root
        vv = brentq(lambda v: P(v) - Pc, v2, b + 2.0 * RT / Pc, xtol=1e-300, rtol=1e-15)
        return vl, vv

    def area(Pc):
        # int (P(v) - Pc) dv with the antiderivative RT ln(v - b) + a/v of P
        vl, vv = outer_roots(Pc)
        return RT * math.log((vv - b) / (vl - b)) + a / vv - a / vl - Pc * (vv - vl)

    lo = max(Pmin, 0.0) + 1e-12 * Pmax
    hi = Pmax * (1 - 1e-12)
    Pc = brentq(area, lo, hi, xtol=1e-300, rtol=1e-15)
    vl, vv = outer_roots(Pc)
    return 1.0 / vl, 1.0 / vv, Pc


def chemical_potential(rho, RT, a, b):
    """mu = RT ln(rho/(1 - b rho)) + RT/(1 - b rho) - 2 a rho (up to a T-only constant)."""
    return RT * math.log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho) - 2.0 * a * rho


def surface_tension(T, kappa, R=1.0, a=0.0225, b=1.0 / 3.0):
    """Flat-interface tension of the square-gradient model with capillarity kappa.

    The force kappa rho grad(lap rho) of the text after eq. EVforce1 is the
    square-gradient term of a free energy with gradient coefficient kappa; the
    first integral of the planar profile gives (kappa/2) rho'^2 = dOmega(rho),
    dOmega = psi(rho) - mu_coex rho + P_coex, psi the Helmholtz free-energy
    density, hence sigma = int_{rho_v}^{rho_l} sqrt(2 kappa dOmega) d rho.
    """
    RT = R * T
    rl, rv, Pc = coexistence(T, R, a, b)
    mu_c = chemical_potential(rl, RT, a, b)

    def psi(r):
        # Helmholtz free-energy density up to a term linear in rho, chosen so
        # that d psi/d rho = chemical_potential and rho mu - psi = P.
        return r * RT * math.log(r / (1.0 - b * r)) - a * r * r

    def dOmega(r):
        return max(psi(r) - mu_c * r + Pc, 0.0)

    val, _ = quad(lambda r: math.sqrt(2.0 * kappa * dOmega(r)), rv, rl, limit=400, epsrel=1e-12)
    return val
