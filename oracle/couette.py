"""Steady planar thermal Couette flow of the model's continuum limit (test
infrastructure only): the analytic profile the paper's second validation
(the Couette paragraph after eq. P0E, Fig. 2) compares with.

Fluid between a wall at rest (x = 0) and a wall moving with U_w along y
(x = L), both at T_w, no flow across (u_x = 0), uniform in y.  From the
momentum balance eq. momentum_balance with T_NS = -mu S and the kinetic
energy balance eq. LB_energy_balance with k = (5/2) R mu:
  - x-momentum: the pressure P = P_E - a rho^2 is uniform (kappa = 0);
  - y-momentum: mu du/dx = tau_w, a constant;
  - energy: k dT/dx + mu u du/dx = const, so with mu du/dx = tau_w and
    k = c_p mu/Pr (c_p = 5R/2; Pr = 1 in the paper), (c_p/Pr) dT/du = c - u,
    and T(0) = T(U_w) = T_w gives T(u) = T_w + Pr u (U_w - u)/(5 R),
    whatever mu(rho, T);
  - rho(u) solves P_E(rho, T(u)) - a rho^2 = P;
  - x(u) = (1/tau_w) int_0^u mu du' with mu = tau P_E (eq. viscosity under
    eq. P0E, dt = 1), tau_w = int_0^U_w mu du / L;
  - P follows from the mass per unit length, int_0^L rho dx = rho_mean L.
The Mach number is u/c with c^2 = (dP/drho)_T + (dP/dT)_rho P_E/(rho^2 c_v),
c_v = 3R/2 (the adiabatic sound speed of the fluid).
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq

from . import thermo as TH


def _rho_at(P, RT, a, b, eos):
    """Density of pressure P on the isotherm RT (the single root of a
    supercritical isotherm; the largest density range the closure allows)."""
    top = (1.0 / b if eos == "vdw" else 4.0 / b) * (1 - 1e-12)
    f = lambda r: TH.pressure(r, RT, a, b, eos) - P
    return brentq(f, 1e-12, top, xtol=1e-15, rtol=1e-14)


def sound_speed(rho, RT, a, b, eos="vdw", R=1.0):
    h = 1e-7 * rho
    Prho = (TH.pressure(rho + h, RT, a, b, eos) - TH.pressure(rho - h, RT, a, b, eos)) / (2 * h)
    Z = TH.compressibility(rho, b, eos)
    PE = rho * RT * Z
    PT = rho * R * Z
    return np.sqrt(Prho + PT * PE / (rho * rho * 1.5 * R))


def profile(L, rho_mean, Tw, Uw, a, b, tau, eos="vdw", R=1.0, n=4001, Pr=1.0):
    """Steady profile on a fine grid of u in [0, U_w]: dict of arrays x, u, T,
    rho, Mach and the pressure P and wall stress tau_w."""
    us = np.linspace(0.0, Uw, n)
    T = Tw + Pr * us * (Uw - us) / (5.0 * R)

    def fields(P):
        rho = np.array([_rho_at(P, R * t, a, b, eos) for t in T])
        mu = tau * rho * R * T * TH.compressibility(rho, b, eos)
        # x(u) by the trapezoidal rule on the fine u grid
        xi = np.concatenate([[0.0], np.cumsum(0.5 * (mu[1:] + mu[:-1]) * np.diff(us))])
        tauw = xi[-1] / L
        return rho, mu, xi / tauw, tauw

    def mass_defect(P):
        rho, mu, x, _ = fields(P)
        return np.trapezoid(rho, x) / L - rho_mean

    P0 = TH.pressure(rho_mean, R * Tw, a, b, eos)
    lo, hi = 0.5 * P0, 2.0 * P0
    while mass_defect(lo) > 0:
        lo *= 0.5
    while mass_defect(hi) < 0:
        hi *= 2.0
    P = brentq(mass_defect, lo, hi, xtol=1e-16, rtol=1e-13)
    rho, mu, x, tauw = fields(P)
    c = np.array([sound_speed(r, R * t, a, b, eos, R) for r, t in zip(rho, T)])
    return dict(x=x, u=us, T=T, rho=rho, Mach=us / c, P=P, tau_w=tauw)


def at(prof, xs):
    """Profile values (u, T, rho, Mach) interpolated at positions xs."""
    return {k: np.interp(xs, prof["x"], prof[k]) for k in ("u", "T", "rho", "Mach")}


def wall_speed_for_mach(L, rho_mean, Tw, Ma, a, b, tau, eos="vdw", R=1.0, Pr=1.0):
    """U_w that puts the Mach number at the moving wall at Ma (fixed point:
    the wall's density depends on U_w through the heating)."""
    rho = rho_mean
    U = Ma * sound_speed(rho, R * Tw, a, b, eos, R)
    for _ in range(50):
        pr = profile(L, rho_mean, Tw, U, a, b, tau, eos, R, n=801, Pr=Pr)
        Un = Ma * sound_speed(pr["rho"][-1], R * Tw, a, b, eos, R)
        if abs(Un - U) < 1e-13 * U:
            break
        U = Un
    return U
