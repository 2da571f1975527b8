"""Physics of the GPU path: the FP64 region measurement against a host
recomputation from the read-out fields, the flat-interface surface tension
against the square-gradient first integral and Laplace's law on
droplets."""
import math

import numpy as np
import pytest

import oracle.thermo as TH
import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")


def _bulk_pressure(rho, T, p):
    return rho * p["R"] * T / (1.0 - p["b"] * rho) - p["a"] * rho * rho


def _region_means(rho, T, mask, p):
    P = _bulk_pressure(rho, T, p)
    return rho[mask].mean(), T[mask].mean(), P[mask].mean(), int(mask.sum())


def test_measure_slab_matches_host_recompute():
    p = synth.params()
    T0 = 0.85 * synth.T_CRIT
    rl, rv, _ = ev.eos_coexistence(T0, p["R"], p["a"], p["b"])
    shape = (1, 32, 128)
    L = ev.Lattice(2, 128, 32, 1, storage="f64")
    L.set_params(**p)
    L.init_fields(synth.slab(shape, rl, rv), np.full(shape, T0))
    L.step(300)
    out = L.measure_slab((56, 72), (0, 8), (120, 128))
    rho, _, T = L.moments()
    x = np.arange(128)[None, None, :] * np.ones(shape)
    liq = (x >= 56) & (x < 72)
    vap = (x < 8) | ((x >= 120) & (x < 128))
    ri, Ti, Pi, ni = _region_means(rho, T, liq, p)
    ro, To, Po, no = _region_means(rho, T, vap, p)
    assert out[7] == ni
    np.testing.assert_allclose(out[[0, 2, 4]], [ri, Ti, Pi], rtol=1e-12)
    np.testing.assert_allclose(out[[1, 3, 5]], [ro, To, Po], rtol=1e-12)


@pytest.mark.parametrize("D,shape,R", [(2, (1, 80, 96), 20.0), (3, (40, 36, 32), 9.0)])
def test_measure_droplet_matches_host_recompute(D, shape, R):
    p = synth.params()
    T0 = 0.8 * synth.T_CRIT
    rl, rv, _ = ev.eos_coexistence(T0, p["R"], p["a"], p["b"])
    nz, ny, nx = shape
    L = ev.Lattice(D, nx, ny, nz, storage="f64")
    L.set_params(**p)
    L.init_fields(synth.droplet(shape, R, rl, rv), np.full(shape, T0))
    L.step(200)
    c = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2 if D == 3 else 0.0)
    r_in, r_out = R / 2, R + 6
    out = L.measure_droplet(c[:D] if D == 2 else c, r_in, r_out)
    rho, _, T = L.moments()
    r = synth.radius_field(shape)
    ri, Ti, Pi, ni = _region_means(rho, T, r < r_in, p)
    ro, To, Po, _ = _region_means(rho, T, r > r_out, p)
    assert out[7] == ni
    np.testing.assert_allclose(out[:6], [ri, ro, Ti, To, Pi, Po], rtol=1e-12)
    excess = (rho.sum() - ro * rho.size) / (ri - ro)   # equimolar area (2D) or volume (3D)
    Re = math.sqrt(excess / math.pi) if D == 2 else (3.0 * excess / (4.0 * math.pi)) ** (1.0 / 3.0)
    assert out[6] == pytest.approx(Re, rel=1e-10)


@pytest.mark.parametrize("Tr", [0.7, 0.8, 0.9])
def test_flat_interface_surface_tension(Tr):
    """sigma = kappa sum_x (d rho/dx)^2 across one interface of a
    relaxed flat slab matches sigma = int sqrt(2 kappa dOmega) d rho of the vdW
    free energy at the measured liquid temperature.  Measured ratio after
    6e4 steps: 0.984, 0.974, 0.985 at T/Tc = 0.7, 0.8, 0.9; the bound allows
    for the O(h^2) stencils on 7-15 cell interfaces and the residual
    temperature difference between the phases."""
    p = synth.params()
    T0 = Tr * synth.T_CRIT
    rl, rv, _ = ev.eos_coexistence(T0, p["R"], p["a"], p["b"])
    nx = 256
    shape = (1, 4, nx)
    L = ev.Lattice(2, nx, 4, 1, storage="f64")
    L.set_params(**p)
    L.init_fields(synth.slab(shape, rl, rv, noise=0), np.full(shape, T0))
    L.step(60000)
    rho, _, T = L.moments()
    prof = rho[0].mean(0)
    d = (np.roll(prof, -1) - np.roll(prof, 1)) / 2.0   # the isotropic gradient of a y-uniform field
    sigma = p["kappa"] * np.sum(d[: nx // 2] ** 2)
    Tl = T[0].mean(0)[nx // 2 - 8: nx // 2 + 8].mean()
    sigma_th = TH.surface_tension(Tl, p["kappa"], p["R"], p["a"], p["b"])
    print(f"T/Tc {Tr}: sigma {sigma:.6f}, theory {sigma_th:.6f} at T_l/Tc {Tl / synth.T_CRIT:.4f}", flush=True)
    assert sigma == pytest.approx(sigma_th, rel=0.05)


def test_laplace_law_2d():
    """Droplets R = 30, 40, 60 on a 512^2 periodic D2Q9 lattice at
    T/Tc = 0.8 (FP32, 6e4 steps): the pressure jump between the bulk phases
    falls as 1/R_e with slope sigma.  The fitted slope through the origin
    (measured 0.0209) is within 5 % of the flat-interface tension of the
    square-gradient theory at the measured liquid temperature (0.0216); the
    liquid is still ~0.7 % warmer than the vapour at this horizon, and
    dP/dT ~ 5.6 in the liquid makes that the dominant residual."""
    p = synth.params()
    T0 = 0.8 * synth.T_CRIT
    rl, rv, _ = ev.eos_coexistence(T0, p["R"], p["a"], p["b"])
    n = 512
    Re, dp, Tl = [], [], []
    for R in (30.0, 40.0, 60.0):
        L = ev.Lattice(2, n, n, 1, storage="f32")
        L.set_params(**p)
        L.init_fields(synth.droplet((1, n, n), R, rl, rv, noise=1e-4), np.full((1, n, n), T0))
        L.step(60000)
        out = L.measure_droplet(((n - 1) / 2, (n - 1) / 2), R / 2, R + 20)
        print(f"R {R}: dp {out[4] - out[5]:.4e}, R_e {out[6]:.3f}, dp R_e {(out[4] - out[5]) * out[6]:.5f}", flush=True)
        Re.append(out[6])
        dp.append(out[4] - out[5])
        Tl.append(out[2])
    Re, dp = np.array(Re), np.array(dp)
    assert np.all(np.diff(dp) < 0)
    slope = np.sum(dp / Re) / np.sum(1.0 / Re ** 2)
    sigma_th = TH.surface_tension(float(np.mean(Tl)), p["kappa"], p["R"], p["a"], p["b"])
    print(f"slope {slope:.5f}, sigma {sigma_th:.5f}", flush=True)
    assert slope == pytest.approx(sigma_th, rel=0.05)


def test_flat_interface_converges_to_maxwell_with_resolution():
    """Fig. 1 at the scheme's steady state, at two interface resolutions:
    FP64 256 x 4 slabs at T/Tc = 0.8 of the workload fluid (RT_c = 0.02) and
    of the same fluid with a halved (RT_c = 0.01, interfaces sqrt(2) wider at
    equal kappa), 2e6 steps each on its own stream.  The steady state keeps
    the liquid warmer than the vapour and the vapour below Maxwell's
    equal-area density; both deviations are discretisation errors of second
    order in the interface resolution, so halving a must shrink each by well
    over 1.5 (measured: vapour -6.05 % -> -3.50 %, temperature difference
    0.0050 -> 0.0028 T_c, liquid -0.52 % -> -0.29 %)."""
    p = synth.params()
    n, q = 256, 16
    out = []
    Ls = []
    for s_ in (1.0, 0.5):
        pp = dict(p)
        pp["a"] *= s_
        L = ev.Lattice(2, n, 4, 1, storage="f64")
        L.set_params(**pp)
        L.init_slab(0.8, seed=synth.SEED + 1, noise=1e-3)
        Ls.append((L, pp))
    for _ in range(20):
        for L, _ in Ls:
            L.step(100000)
    for L, pp in Ls:
        # a flat interface carries no spurious current at the steady state
        # (measured max |u| 7e-7 at 2e6 steps)
        assert L.global_sums()[6] < 1e-5
        m = L.measure_slab((n / 2 - q, n / 2 + q), (0, q), (n - q, n))
        _, Tc, _ = TH.critical_point(pp["R"], pp["a"], pp["b"])
        rl, rv, _ = TH.coexistence(0.5 * (m[2] + m[3]), pp["R"], pp["a"], pp["b"])
        out.append((m[0] / rl - 1, m[1] / rv - 1, (m[2] - m[3]) / Tc))
        print(f"RT_c {pp['R'] * Tc:.3f}: rho_l {out[-1][0]:+.4%} rho_v {out[-1][1]:+.4%} "
              f"(T_l - T_v)/T_c {out[-1][2]:+.5f}", flush=True)
    (l1, v1, t1), (l2, v2, t2) = out
    assert -0.08 < v1 < -0.04 and abs(l1) < 0.01 and t1 > 0
    assert v1 / v2 > 1.5 and l1 / l2 > 1.5 and t1 / t2 > 1.5
