"""Thermodynamics of the model's equation of state for the oracle (test
infrastructure only).

The paper's closure (eq. EVforce1 and the text after it) gives the Enskog
pressure P_E = rho R T/(1 - b rho) and the mean-field pressure P_V = -a rho^2,
so the bulk pressure is the van der Waals equation P = P_E + P_V.  Enskog's
pressure is rho R T (1 + b rho chi) with chi the contact value of the pair
distribution; eos = "cs" takes Carnahan & Starling's hard-sphere value
chi = (1 - eta/2)/(1 - eta)^3, eta = b rho/4, with the same mean field.
Figure 1 of the paper compares simulated coexistence densities with Maxwell's
equal-area construction; this module computes that construction and the
flat-interface surface tension of the square-gradient (capillarity kappa)
model, by plain numerical quadrature and bracketing root finding.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq


def compressibility(rho, b, eos="vdw"):
    """Z = P_E/(rho R T): 1/(1 - b rho) (van der Waals) or
    (1 + eta + eta^2 - eta^3)/(1 - eta)^3 with eta = b rho/4 (Carnahan-Starling)."""
    if eos == "cs":
        eta = 0.25 * b * rho
        return (1.0 + eta + eta * eta - eta ** 3) / (1.0 - eta) ** 3
    return 1.0 / (1.0 - b * rho)


def pressure(rho, RT, a, b, eos="vdw"):
    """Bulk pressure P = P_E + P_V = rho RT Z(rho) - a rho^2 (van der Waals:
    rho RT/(1 - b rho) - a rho^2)."""
    return rho * RT * compressibility(rho, b, eos) - a * rho * rho


def free_energy_density(rho, RT, a, b, eos="vdw"):
    """Helmholtz free-energy density up to a term linear in rho:
    rho RT [ln rho - 1 + f_ex/RT] - a rho^2 with the hard-core excess free
    energy per particle f_ex/RT = -ln(1 - b rho) (van der Waals) or
    (4 eta - 3 eta^2)/(1 - eta)^2 (Carnahan-Starling).  Its derivative is
    the chemical potential and rho mu - psi the pressure."""
    if eos == "cs":
        eta = 0.25 * b * rho
        fex = (4.0 * eta - 3.0 * eta * eta) / (1.0 - eta) ** 2
    else:
        fex = -math.log(1.0 - b * rho)
    return rho * RT * (math.log(rho) - 1.0 + fex) - a * rho * rho


def critical_point(R, a, b, eos="vdw"):
    """(rho_c, T_c, P_c): closed form for van der Waals; for Carnahan-Starling
    plus mean field, the density where dP/drho = d^2P/drho^2 = 0, i.e. where
    q(rho) = rho Z(rho) has q' = rho q'' (then RT_c = 2 a/q''), found by
    bracketing with q', q'' from central differences of the closed form."""
    if eos != "cs":
        return 1.0 / (3.0 * b), 8.0 * a / (27.0 * b * R), a / (27.0 * b * b)
    q = lambda r: r * compressibility(r, b, "cs")

    def d1(r, h):
        return (q(r + h) - q(r - h)) / (2 * h)

    def d2(r, h):
        return (q(r + h) - 2 * q(r) + q(r - h)) / (h * h)

    def cond(r):
        h = 1e-4 * r
        return d1(r, h) - r * d2(r, h)

    rc = brentq(cond, 0.2 / b, 1.0 / b, xtol=1e-15, rtol=1e-14)
    h = 1e-4 * rc
    RTc = 2.0 * a / d2(rc, h)
    return rc, RTc / R, pressure(rc, RTc, a, b, "cs")


def _spinodal_volumes(RT, a, b):
    """Specific volumes where dP/dv = 0 (v = 1/rho), bracketing the unstable branch."""
    # P(v) = RT/(v - b) - a/v^2; dP/dv = -RT/(v-b)^2 + 2a/v^3
    dP = lambda v: -RT / (v - b) ** 2 + 2.0 * a / v ** 3
    vc = 3.0 * b
    lo = brentq(dP, b * (1 + 1e-12), vc)
    hi = brentq(dP, vc, 1e6 * b)
    return lo, hi


def _coexistence_quadrature(T, R, a, b, eos):
    """Maxwell's equal-area rule in the P-v plane for any pressure closure:
    spinodals by bracketing dP/dv = 0 around the critical volume, the outer
    roots of P(v) = Pc by bracketing, and int_{v_l}^{v_v} (P(v) - Pc) dv = 0
    by adaptive quadrature.  Returns (rho_l, rho_v, P_coex)."""
    RT = R * T
    rc, Tc, _ = critical_point(R, a, b, eos)
    if not (0 < T < Tc):
        raise ValueError("T must lie below T_c")
    P = lambda v: pressure(1.0 / v, RT, a, b, eos)
    hdv = 1e-7
    dP = lambda v: (P(v * (1 + hdv)) - P(v * (1 - hdv))) / (2 * hdv * v)
    vc = 1.0 / rc
    vmin = (b / 4.0 if eos == "cs" else b) * (1 + 1e-9)
    grid = np.geomspace(vmin * 1.0001, vc, 400)
    k = np.argmax([dP(v) > 0 for v in grid])  # first volume past the liquid spinodal
    v1 = brentq(dP, grid[k - 1], grid[k])
    grid = np.geomspace(vc, 1e4 * vc, 800)
    k = np.argmax([dP(v) < 0 for v in grid])
    v2 = brentq(dP, grid[k - 1], grid[k])
    Pmin, Pmax = P(v1), P(v2)

    def outer_roots(Pc):
        vl = brentq(lambda v: P(v) - Pc, vmin, v1, xtol=1e-300, rtol=1e-15)
        hi = v2
        while P(hi) > Pc:
            hi *= 2.0
        vv = brentq(lambda v: P(v) - Pc, v2, hi, xtol=1e-300, rtol=1e-15)
        return vl, vv

    def area(Pc):
        vl, vv = outer_roots(Pc)
        val, _ = quad(lambda v: P(v) - Pc, vl, vv, limit=400, epsabs=0.0, epsrel=1e-13)
        return val

    lo = max(Pmin, 0.0) + 1e-12 * Pmax
    Pc = brentq(area, lo, Pmax * (1 - 1e-12), xtol=1e-300, rtol=1e-14)
    vl, vv = outer_roots(Pc)
    return 1.0 / vl, 1.0 / vv, Pc


def coexistence(T, R=1.0, a=0.0225, b=1.0 / 3.0, eos="vdw"):
    """Liquid and vapour densities from Maxwell's equal-area rule in the P-v plane.
    eos = "cs": the same rule by quadrature (_coexistence_quadrature).

    For a trial pressure Pc between the spinodal pressures, v_l and v_v are the
    outer roots of P(v) = Pc; the rule demands that the integral of P(v) - Pc
    from v_l to v_v vanishes.  Returns (rho_l, rho_v, P_coex).
    """
    if eos != "vdw":
        return _coexistence_quadrature(T, R, a, b, eos)
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


def chemical_potential(rho, RT, a, b, eos="vdw"):
    """mu = d psi/d rho (up to a T-only constant): van der Waals
    RT ln(rho/(1 - b rho)) + RT/(1 - b rho) - 2 a rho; Carnahan-Starling
    RT [ln rho + (8 eta - 9 eta^2 + 3 eta^3)/(1 - eta)^3] - 2 a rho."""
    if eos == "cs":
        eta = 0.25 * b * rho
        return RT * (math.log(rho) + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1.0 - eta) ** 3) - 2.0 * a * rho
    return RT * math.log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho) - 2.0 * a * rho


def surface_tension(T, kappa, R=1.0, a=0.0225, b=1.0 / 3.0, eos="vdw"):
    """Flat-interface tension of the square-gradient model with capillarity kappa.

    The force kappa rho grad(lap rho) of the text after eq. EVforce1 is the
    square-gradient term of a free energy with gradient coefficient kappa; the
    first integral of the planar profile gives (kappa/2) rho'^2 = dOmega(rho),
    dOmega = psi(rho) - mu_coex rho + P_coex, psi the Helmholtz free-energy
    density, hence sigma = int_{rho_v}^{rho_l} sqrt(2 kappa dOmega) d rho.
    """
    RT = R * T
    rl, rv, Pc = coexistence(T, R, a, b, eos)
    mu_c = chemical_potential(rl, RT, a, b, eos)

    def psi(r):
        # Helmholtz free-energy density up to a term linear in rho, chosen so
        # that d psi/d rho = chemical_potential and rho mu - psi = P.
        if eos == "cs":
            return free_energy_density(r, RT, a, b, eos)
        return r * RT * math.log(r / (1.0 - b * r)) - a * r * r

    def dOmega(r):
        return max(psi(r) - mu_c * r + Pc, 0.0)

    val, _ = quad(lambda r: math.sqrt(2.0 * kappa * dOmega(r)), rv, rl, limit=400, epsrel=1e-12)
    return val
