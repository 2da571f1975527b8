"""Pins of the oracle's walls and of the supersonic thermal Couette flow (the
paper's second validation: the Couette paragraph after eq. P0E, Fig. 2).

The paper gives the wall values (u = 0 and T = T_w at x = 0; u_y = U_w and
T = T_w at x = L) but no wall scheme.  The oracle's reading: diffuse
reflection at walls half a cell outside the first and last cells, and linear
extrapolation of every stencil's field beyond a wall.  Pinned here by exact
properties (a resting equilibrium between walls at its own temperature is a
fixed point; the walls conserve mass) and by the steady profile of the
continuum limit the paper derives (oracle.couette: uniform pressure,
mu du/dx = const, T(u) = T_w + u (U_w - u)/(5R) from k = (5/2) R mu).
"""
import numpy as np
import pytest

import oracle as O
import oracle.couette as C
import synth

A, B = synth.A_ATTR, synth.B_EXCL


def _channel(nx, Tw, Uw, tau=1.0, D=2, nz=1, ny=1):
    L = O.Lattice(D, nx, ny, nz)
    L.set_params(R=1.0, a=A, b=B, kappa=0.0, tau=tau, lam=tau)
    L.set_walls(Tw, Uw)
    return L


@pytest.mark.parametrize("D", [2, 3])
def test_rest_state_between_walls_is_a_fixed_point(D):
    """A uniform fluid at rest at the walls' temperature: each wall re-emits
    exactly the equilibrium populations that left, so nothing changes."""
    nx, Tw = 9, 1.3 * synth.T_CRIT
    shape = (3 if D == 3 else 1, 4, nx)
    L = _channel(nx, Tw, 0.0, D=D, nz=shape[0], ny=4)
    L.init(np.full(shape, 0.9), np.full(shape, Tw))
    f0, g0 = L.get_pops()
    L.step(20)
    f1, g1 = L.get_pops()
    assert np.abs(f1 - f0).max() < 1e-14 and np.abs(g1 - g0).max() < 1e-14


def test_walls_conserve_mass():
    nx, Tw = 24, 1.5 * synth.T_CRIT
    L = _channel(nx, Tw, 0.3, ny=3)
    rho = 1.0 + 0.05 * np.sin(2 * np.pi * np.arange(nx) / nx)
    L.init(np.broadcast_to(rho, (1, 3, nx)).copy(), np.full((1, 3, nx), 1.2 * Tw))
    m0 = L.global_sums()[0]
    L.step(3000)
    assert abs(L.global_sums()[0] / m0 - 1) < 1e-13


def test_supersonic_couette_converges_to_the_continuum_profile():
    """A 32-cell channel of the dense van der Waals gas (mean density rho_c,
    T_w = 1.5 T_c, kappa = 0), started at rest at T_w, driven by the wall
    speed that makes the Mach number 1.2 at the moving wall, after 6e4 steps
    (about 2.5 momentum-diffusion times): density, temperature and velocity
    against the continuum profile.  Measured: e_rho 1.8e-2, e_T 8.4e-3 (of
    T), e_u 2.4e-2 (of U_w), Mach at the moving wall's cell 1.168 against
    1.191; the residual is the velocity slip and temperature jump of diffuse
    walls (64 cells: e_rho 9.2e-3, e_T 4.2e-3, e_u 1.25e-2)."""
    nx, Tw, tau = 32, 1.5 * synth.T_CRIT, 1.0
    U = C.wall_speed_for_mach(float(nx), 1.0, Tw, 1.2, A, B, tau)
    pr = C.profile(float(nx), 1.0, Tw, U, A, B, tau)
    an = C.at(pr, np.arange(nx) + 0.5)
    L = _channel(nx, Tw, U, tau)
    L.init(np.ones((1, 1, nx)), np.full((1, 1, nx), Tw))
    L.step(60000)
    r, u, T, _ = L.moments()
    e_rho = np.abs(r[0, 0] - an["rho"]).max() / an["rho"].max()
    e_T = np.abs(T[0, 0] - an["T"]).max() / an["T"].max()
    e_u = np.abs(u[1, 0, 0] - an["u"]).max() / U
    Ma = u[1, 0, 0, -1] / C.sound_speed(r[0, 0, -1], T[0, 0, -1], A, B)
    print(f"Couette 32: e_rho {e_rho:.2e} e_T {e_T:.2e} e_u {e_u:.2e} Mach {Ma:.3f} vs {an['Mach'][-1]:.3f}")
    assert e_rho < 2.5e-2 and e_T < 1e-2 and e_u < 3e-2
    assert Ma == pytest.approx(an["Mach"][-1], abs=0.03)
    assert np.abs(u[0]).max() < 1e-4
