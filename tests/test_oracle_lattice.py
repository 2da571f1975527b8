"""Lattice-level pins of the FP64 oracle stepper.

Expected values come from exact invariants of the scheme (fixed points,
conservation), the exact z-reduction of D3Q27 to D2Q9, and the hydrodynamic
limit the paper states: viscosity mu = (1/(2 beta) - 1/2) dt P0 with zero bulk
viscosity (eq. viscosity), Prandtl number 1 (k = (5/2) R mu after
eq. LB_energy_balance), independence of lambda (comment (ii) after
eq. viscosity), the van der Waals adiabatic sound speed, and Maxwell's
equal-area coexistence (Fig. 1).
"""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

import oracle as O
import oracle.thermo as TH
import synth

P = synth.params()


def _lattice(D, shape, **kw):
    nz, ny, nx = shape
    L = O.Lattice(D, nx, ny, nz)
    q = dict(P)
    q.update(kw)
    L.set_params(**q)
    return L


@pytest.mark.parametrize("D,shape", [(2, (1, 6, 7)), (3, (5, 4, 6))])
def test_uniform_states_are_fixed_points(D, shape):
    """A uniform state at rest or in uniform motion is unchanged by the
    step: streaming a uniform field is the identity, all stencils vanish, so
    F = Phi = q' = 0 and f* = f^eq = fh."""
    L = _lattice(D, shape)
    rho = np.full(shape, 1.3)
    T = np.full(shape, 0.017)
    for u in (None, np.stack([np.full(shape, v) for v in (0.07, -0.04, 0.02)[:D]])):
        L.init(rho, T, u)
        f0, g0 = L.get_pops()
        L.step(7)
        f1, g1 = L.get_pops()
        assert np.abs(f1 - f0).max() < 1e-14 * np.abs(f0).max()
        assert np.abs(g1 - g0).max() < 1e-14 * np.abs(g0).max()
        r, uu, TT, F = L.moments()
        assert np.allclose(r, 1.3, rtol=1e-15)
        assert np.allclose(TT, 0.017, rtol=1e-13)
        if u is not None:
            assert np.allclose(uu, u, atol=1e-15)


def _slab_state(D, shape, Tr=0.9, noise=1e-3):
    T0 = Tr * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    rho = synth.slab(shape, rl, rv, noise=noise)
    return rho, np.full(shape, T0)


@pytest.mark.parametrize("D,shape", [(2, (1, 12, 40)), (3, (6, 8, 40))])
def test_collision_conserves_locally(D, shape):
    """Per cell, sum f is unchanged, sum c f gains F dt, sum g gains
    (u.F + Qtilde) dt with Qtilde = 0 (eq. pre_LBM with eq. u_shift, T_shift)."""
    L = _lattice(D, shape)
    rho, T = _slab_state(D, shape)
    L.init(rho, T)
    L.step(20)
    d = L.step(1, diag=True)
    k = 0
    rho_h = d[k]; k += 1
    sum_f = d[k]; k += 1
    j = d[k:k + D]; k += D
    sum_cf = d[k:k + D]; k += D
    F = d[k:k + D]; k += D
    e = d[k]; k += 1
    sum_g = d[k]; k += 1
    uF = d[k]
    assert np.abs(sum_f - rho_h).max() < 1e-14 * rho_h.max()
    assert np.abs(sum_cf - (j + F)).max() < 1e-14 * rho_h.max()
    assert np.abs(F).max() > 1e-5  # the force really acts
    assert np.abs(sum_g - (e + uF)).max() < 1e-14 * np.abs(e).max()


@pytest.mark.parametrize("D,shape,steps", [(2, (1, 16, 48), 300), (3, (8, 8, 24), 40)])
def test_global_mass_conserved(D, shape, steps):
    """Total mass is invariant on a periodic lattice."""
    L = _lattice(D, shape)
    rho, T = _slab_state(D, shape)
    L.init(rho, T)
    m0 = L.global_sums()[0]
    L.step(steps)
    m1 = L.global_sums()[0]
    assert abs(m1 - m0) < 1e-13 * m0


def test_d3q27_with_one_plane_equals_d2q9():
    """A D3Q27 lattice one cell thick in z reproduces D2Q9 field by field."""
    shape2 = (1, 10, 36)
    rho, T = _slab_state(2, shape2)
    L2 = _lattice(2, shape2)
    L2.init(rho, T)
    L3 = _lattice(3, shape2)
    L3.init(rho, T)
    L2.step(60)
    L3.step(60)
    r2, u2, T2, _ = L2.moments()
    r3, u3, T3, _ = L3.moments()
    assert np.abs(r3 - r2).max() < 1e-12
    assert np.abs(u3[:2] - u2).max() < 1e-13
    assert np.abs(u3[2]).max() < 1e-15
    assert np.abs(T3 - T2).max() < 1e-13
    f2, g2 = L2.get_pops()
    f3, g3 = L3.get_pops()
    c3, _ = O.lattice(3)
    c2, _ = O.lattice(2)
    for i in range(9):
        sel = np.all(c3[:, :2] == c2[i, :2], axis=1)
        assert np.abs(f3[sel].sum(0) - f2[i]).max() < 1e-13
        assert np.abs(g3[sel].sum(0) - g2[i]).max() < 1e-13


def _decay(mode, sphi=-1.0, RT=0.02, lam=1.0, nx=128, steps=3000, A=1e-4, kind="ideal"):
    if kind == "ideal":
        L = _lattice(2, (1, 1, nx), a=0.0, b=0.0, kappa=0.0, lam=lam, sphi=sphi)
        rho0 = 1.0
    else:
        L = _lattice(2, (1, 1, nx), kappa=0.0, lam=lam, sphi=sphi)
        rho0 = kind
    x = np.arange(nx)
    cs = np.cos(2 * np.pi * x / nx)
    u = None
    if mode == "sound":      # isentropic: dT/T = (gamma - 1) d rho/rho (ideal gas)
        rho = rho0 * (1 + A * cs)
        T = RT * (1 + (2.0 / 3.0) * A * cs)
    elif mode == "shear":
        rho = np.full(nx, rho0)
        T = np.full(nx, RT)
        u = np.zeros((2, 1, 1, nx))
        u[1, 0, 0] = A * cs
    else:                    # isobaric temperature mode
        rho = rho0 * (1 - A * cs)
        T = RT * (1 + A * cs)
    L.init(rho.reshape(1, 1, nx), T.reshape(1, 1, nx), u)
    amp = []
    for _ in range(steps):
        r, uu, TT, _ = L.moments()
        q = {"sound": r[0, 0] - rho0, "shear": uu[1, 0, 0], "thermal": TT[0, 0] - RT}[mode]
        amp.append(2.0 * (q * cs).sum() / nx)
        L.step(1)
    return np.arange(steps), np.array(amp)


@pytest.mark.parametrize("RT", [0.05, 0.15])
def test_ideal_gas_sound_attenuation_decides_phi_sign(RT):
    """With a = b = kappa = 0 the model is a compressible Navier-Stokes
    fluid with nu = tau P0/rho, zero bulk viscosity and Pr = 1, so a standing
    sound wave decays at (k^2/2)[(4/3) nu + (gamma - 1) chi] = nu k^2 and
    oscillates at sqrt(5/3 RT) k.  The lattice third moment c^3 = c misses the
    Maxwellian's by M_a = rho u_a (u_a^2 + 3 theta - 1), which eq. correction_u
    removes.  A Chapman-Enskog expansion of eq. pre_LBM puts the defect into the
    normal stress with the sign that makes -d_a M_a the needed correction; with
    the printed + the defect is doubled instead, an extra longitudinal viscosity
    2 tau rho (1 - 3 theta) that raises the decay rate to
    nu k^2 [1 + (1 - 3 theta)/theta].  Both predictions are checked."""
    k = 2 * np.pi / 128
    nu = P["tau"] * RT
    w0 = np.sqrt(5.0 / 3.0 * RT) * k
    fit = {}
    for s in (-1.0, 1.0):
        t, a = _decay("sound", sphi=s, RT=RT)
        p, _ = curve_fit(lambda t, A, w, ph, G: A * np.cos(w * t + ph) * np.exp(-G * t), t, a,
                         p0=[a[0], w0, 0.0, nu * k * k])
        fit[s] = p
    assert fit[-1.0][3] / (nu * k * k) == pytest.approx(1.0, abs=0.015)
    assert fit[-1.0][1] / w0 == pytest.approx(1.0, abs=0.01)
    assert fit[1.0][3] / (nu * k * k) == pytest.approx(1.0 + (1.0 - 3.0 * RT) / RT, rel=0.03)


@pytest.mark.parametrize("lam", [1.0, 2.0])
def test_ideal_gas_shear_and_thermal_decay(lam):
    """Shear and isobaric temperature modes decay at nu k^2
    (Pr = 1: chi = k/(rho c_p) = nu), independently of lambda."""
    k = 2 * np.pi / 128
    RT = 0.05
    nu = P["tau"] * RT
    for mode in ("shear", "thermal"):
        t, a = _decay(mode, RT=RT, lam=lam, steps=2000)
        p, _ = curve_fit(lambda t, A, G: A * np.exp(-G * t), t[50:], a[50:], p0=[a[0], nu * k * k])
        assert p[1] / (nu * k * k) == pytest.approx(1.0, abs=0.02), mode


def test_vdw_sound_speed():
    """In a stable van der Waals state the adiabatic sound speed is
    c^2 = (5/3) RT/(1 - b rho)^2 - 2 a rho (c_v = 3R/2, P = P_E - a rho^2)."""
    rho0, Tr = 0.6, 1.3
    RT = Tr * synth.T_CRIT
    k = 2 * np.pi / 128
    c2 = 5.0 / 3.0 * RT / (1 - P["b"] * rho0) ** 2 - 2 * P["a"] * rho0
    L = _lattice(2, (1, 1, 128), kappa=0.0)
    x = np.arange(128)
    cs = np.cos(k * x)
    A = 1e-4
    # isentropic perturbation of the van der Waals gas: dT = (2/3) T/(1 - b rho) d rho/rho
    rho = rho0 * (1 + A * cs)
    T = RT * (1 + (2.0 / 3.0) * A * cs / (1 - P["b"] * rho0))
    L.init(rho.reshape(1, 1, 128), T.reshape(1, 1, 128))
    amp = []
    for _ in range(2500):
        r, _, _, _ = L.moments()
        amp.append(2 * ((r[0, 0] - rho0) * cs).sum() / 128)
        L.step(1)
    t = np.arange(len(amp))
    p, _ = curve_fit(lambda t, A, w, ph, G: A * np.cos(w * t + ph) * np.exp(-G * t), t, amp,
                     p0=[amp[0], np.sqrt(c2) * k, 0.0, 1e-4])
    assert p[1] / (np.sqrt(c2) * k) == pytest.approx(1.0, abs=0.01)


def _nsf_modes(rho0, RT, q, a, b, tau, R=1.0):
    """Roots s of the linearised Navier-Stokes-Fourier system for a plane wave
    exp(i q x + s t) of the fluid the paper's hydrodynamic limit describes:
    continuity (eq. macro_mass), momentum (eq. momentum_balance) with the
    pressure P = P_E - a rho^2 (kappa = 0), shear viscosity mu = tau P_E
    (eq. viscosity with P0 = P_E, dt = 1) and zero bulk viscosity, and the
    energy balance eq. LB_energy_balance, which at linear order reads
    rho c_v dT/dt + P_E div u = k lap T with c_v = 3R/2 and k = (5/2) R mu.
    Unknowns (d rho, u, d T):
        s d rho + i q rho0 u = 0
        rho0 s u + i q P_rho d rho + i q P_T d T + (4/3) mu q^2 u = 0
        rho0 c_v s d T + i q P_E u + k q^2 d T = 0
    with P_rho = RT/(1 - b rho)^2 - 2 a rho and P_T = rho R/(1 - b rho); the
    determinant is a cubic in s.  Returns (sound root, thermal root, P_rho, P_T)."""
    PE = rho0 * RT / (1 - b * rho0)
    Prho = RT / (1 - b * rho0) ** 2 - 2 * a * rho0
    PT = rho0 * R / (1 - b * rho0)
    mu = tau * PE
    kT = 2.5 * R * mu
    cv = 1.5 * R
    a1, a2 = 4.0 / 3.0 * mu * q * q, kT * q * q
    roots = np.roots([rho0 * rho0 * cv, rho0 * a2 + a1 * rho0 * cv,
                      a1 * a2 + q * q * PT * PE + q * q * rho0 * rho0 * cv * Prho, q * q * rho0 * Prho * a2])
    sound = roots[np.argmax(np.abs(roots.imag))]
    thermal = roots[np.argmin(np.abs(roots.imag))].real
    return sound, thermal, Prho, PT


def _vdw_mode(mode, rho0, Tr, steps, nx=128, A=1e-4):
    """Amplitude of the cos(q x) component of d rho (sound), d T (thermal)
    or u_y (shear) over `steps` steps on a 128 x 1 D2Q9 lattice in a stable
    single-phase van der Waals state (kappa = 0, so the flat state is a
    fluid with P = P_E - a rho^2)."""
    q = 2 * np.pi / nx
    RT = Tr * synth.T_CRIT
    L = _lattice(2, (1, 1, nx), kappa=0.0)
    cs = np.cos(q * np.arange(nx))
    _, _, Prho, PT = _nsf_modes(rho0, RT, q, P["a"], P["b"], P["tau"])
    u = None
    if mode == "sound":      # adiabatic: dT/T = (2/3) (d rho/rho)/(1 - b rho)
        rho = rho0 * (1 + A * cs)
        T = RT * (1 + (2.0 / 3.0) * A * cs / (1 - P["b"] * rho0))
    elif mode == "thermal":  # isobaric: P_rho d rho + P_T d T = 0
        dT = A * RT * cs
        rho = rho0 - PT * dT / Prho
        T = RT + dT
    else:
        rho, T = np.full(nx, rho0), np.full(nx, RT)
        u = np.zeros((2, 1, 1, nx))
        u[1, 0, 0] = A * cs
    L.init(rho.reshape(1, 1, nx), T.reshape(1, 1, nx), u)
    amp = []
    for _ in range(steps):
        r, uu, TT, _ = L.moments()
        v = {"sound": r[0, 0] - rho0, "thermal": TT[0, 0] - RT, "shear": uu[1, 0, 0]}[mode]
        amp.append(2.0 * (v * cs).sum() / nx)
        L.step(1)
    return np.arange(steps), np.array(amp), q, RT


def _two_mode(t, A, w, ph, G, B, GT):
    return A * np.cos(w * t + ph) * np.exp(-G * t) + B * np.exp(-GT * t)


@pytest.mark.parametrize("rho0", [0.6, 1.2])
def test_vdw_transport_pins_gamma0_and_heat_flux_correction(rho0):
    """Dense (b rho = 0.2 and 0.4), supercritical (T/Tc = 1.3) van der Waals
    gas with kappa = 0: the sound, thermal and shear modes of the oracle decay
    at the rates of the linearised Navier-Stokes-Fourier system the paper
    derives (eq. momentum_balance with mu = tau P_E from eq. viscosity under
    eq. P0E and zero bulk viscosity; eq. LB_energy_balance with
    k = (5/2) R mu), computed from the exact dispersion cubic (_nsf_modes).

    This pins the parts of the step that vanish for an ideal gas:
      - gamma_0 (eq. gamma) and Phi' (eq. correction_gamma), which keep the
        bulk viscosity zero: sound attenuation;
      - the first term of q' (eq. correction_q), which turns the lattice's
        heat flux in grad(P0/rho) into the Fourier flux in grad T: the
        isobaric thermal mode (and sound attenuation);
      - mu = tau P_E: the shear mode.
    Measured ratios (fit / prediction) at rho0 = 0.6 / 1.2: sound 1.009 /
    1.007, thermal 0.996 / 1.006, shear 0.998 / 0.998.  With a copy of the
    oracle whose gamma_0 drops the (2/3)(P_E/(rho R T)) term the sound ratio
    is 0.668 / 0.570; with the sign of the first term of q' flipped the
    thermal ratio is 0.606 / -0.577 (growing) and the sound ratio 1.236 /
    1.640.  The tolerances (2 % sound and thermal, 1 % shear) reject both."""
    b, a, tau = P["b"], P["a"], P["tau"]
    t, amp, q, RT = _vdw_mode("sound", rho0, 1.3, 3000)
    sound, thermal, _, _ = _nsf_modes(rho0, RT, q, a, b, tau)
    p, _ = curve_fit(_two_mode, t, amp, p0=[amp[0], abs(sound.imag), 0.0, -sound.real, 0.0, -thermal],
                     maxfev=20000)
    assert p[3] / -sound.real == pytest.approx(1.0, abs=0.02)
    assert p[1] / abs(sound.imag) == pytest.approx(1.0, abs=0.005)
    t, amp, q, RT = _vdw_mode("thermal", rho0, 1.3, 3000)
    p, _ = curve_fit(_two_mode, t, amp, p0=[0.0, abs(sound.imag), 0.0, -sound.real, amp[0], -thermal],
                     maxfev=20000)
    assert p[5] / -thermal == pytest.approx(1.0, abs=0.02)
    t, amp, q, RT = _vdw_mode("shear", rho0, 1.3, 2000)
    nu = tau * RT / (1 - b * rho0)   # mu/rho = tau P_E/rho
    p, _ = curve_fit(lambda t, A, G: A * np.exp(-G * t), t[50:], amp[50:], p0=[amp[0], nu * q * q])
    assert p[1] / (nu * q * q) == pytest.approx(1.0, abs=0.01)


def test_flat_interface_coexistence():
    """Fig. 1: the flat liquid-vapour interface of the 128 x 32, T/Tc = 0.9,
    FP64 workload after 2000 steps.  The liquid sits on Maxwell's equal-area
    density at the measured liquid temperature within 1 %.  The vapour, whose
    temperature lags (latent heat; thermal equilibration across the slab takes
    ~1e5 steps), is within 5 % -- a looser check that is reported, not claimed."""
    shape = (1, 32, 128)
    rho, T = _slab_state(2, shape)
    L = _lattice(2, shape)
    L.init(rho, T)
    L.step(2000)
    r, u, TT, _ = L.moments()
    Tl = TT[0, :, 56:72].mean()
    rl_m = r[0, :, 56:72].mean()
    rv_m = np.concatenate([r[0, :, 0:8], r[0, :, 120:128]], 1).mean()
    rl, rv, _ = TH.coexistence(Tl)
    assert rl_m == pytest.approx(rl, rel=0.01)
    assert rv_m == pytest.approx(rv, rel=0.05)
    assert np.abs(u).max() < 5e-3


@pytest.mark.parametrize("D,shape", [(2, (1, 14, 17)), (3, (11, 12, 13))])
def test_windowed_step_equals_full_step(D, shape):
    """The sampled evaluation behind full-size parity: a cell's new
    populations depend only on stored populations within Chebyshev distance 4
    (pull 1 + force chain 3), so stepping a 9-wide periodic window reproduces
    the full lattice's step at the window's centre."""
    nz, ny, nx = shape
    L = _lattice(D, shape)
    rho = synth.droplet(shape, 4.0, 1.9, 0.25, noise=1e-3, seed=synth.SEED + 11)
    L.init(rho, np.full(shape, 0.8 * synth.T_CRIT))
    L.step(3)
    f, g = L.get_pops()
    L.step(1)
    f1, g1 = L.get_pops()
    cells = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny // 2, nz // 2), (3, ny - 2, 1)]
    cells = [(x, y, z if D == 3 else 0) for (x, y, z) in cells]
    sf, sg = O.step_sampled(D, f, g, cells, P)
    for k, (x, y, z) in enumerate(cells):
        np.testing.assert_allclose(sf[k], f1[:, z, y, x], rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(sg[k], g1[:, z, y, x], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("D,u0", [(2, (0.0, 0.0, 0.0)), (2, (0.02, -0.015, 0.0)), (3, (0.0, 0.0, 0.0)),
                                   (3, (0.02, -0.015, 0.01))])
def test_positivity_and_speed_diagnostics_on_uniform_states(D, u0):
    """The last two global sums, max |u| and the smallest streamed population
    (the positivity diagnostic), on uniform states where both have closed
    forms.  The equilibrium of eq. feq is rho prod_a psi(c_a; u_a, theta +
    u_a^2) with psi(0) = 1 - theta - u_a^2 and psi(+-1) = (theta + u_a^2 +-
    u_a)/2 (eq. phi).  With |u_a| < theta + u_a^2 < 2/3 on every axis all
    factors are positive and the factor against the flow, (theta + u_a^2 -
    |u_a|)/2, is the smallest of the three, so the smallest member is the
    direction against the flow on every axis:
    rho prod_a (theta + u_a^2 - |u_a|)/2 over the D axes; max |u| is |u0|.
    (theta = RT/(1 - b rho) for the van der Waals closure: 0.0318 here.)"""
    shape = (1, 6, 7) if D == 2 else (5, 4, 6)
    rho0, RT0 = 1.3, 0.9 * synth.T_CRIT
    L = _lattice(D, shape)
    u = np.zeros((D,) + shape)
    for a in range(D):
        u[a] = u0[a]
    L.init(np.full(shape, rho0), np.full(shape, RT0), u)
    s = L.global_sums()
    theta = RT0 / (1.0 - P["b"] * rho0)
    fmin = rho0
    for a in range(D):
        fmin *= 0.5 * (theta + u0[a] ** 2 - abs(u0[a]))
    assert s[7] == pytest.approx(fmin, rel=1e-13)
    assert s[6] == pytest.approx(math.sqrt(sum(v * v for v in u0[:D])), rel=1e-13, abs=1e-15)
