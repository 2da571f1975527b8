"""The Prandtl-number option (EVLBM_OPT_PRANDTL) through the C ABI against the
oracle's reading of the quasi-equilibrium relaxation of g: the D2Q9 step,
the D3Q27 one-pass step (the two-pass step is checked against it in
test_gpu_push.py) and the walls, then the
subsonic Couette temperature rise Pr U_w^2/(20 R)."""
import numpy as np
import pytest

import oracle
import oracle.couette as C
import oracle.thermo as TH
import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")
P = synth.params()
SQ3 = np.sqrt(3.0)


def _errs(g, o):
    rg, ug, Tg = g.moments()
    ro, uo, To, _ = o.moments()
    return np.abs(rg - ro).max() / ro.max(), np.abs(ug - uo).max() * SQ3, np.abs(Tg - To).max() / To.max()


@pytest.mark.parametrize("D,shape,steps", [(2, (1, 37, 70), 300), (3, (13, 11, 37), 100)])
@pytest.mark.parametrize("Pr", [0.5, 2.0])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_prandtl_matches_oracle(D, shape, steps, Pr, storage, tol):
    nz, ny, nx = shape
    T0 = 0.8 * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    rho = synth.droplet(shape, 0.3 * min(s for s in shape if s > 1), rl, rv, noise=1e-3)
    T = np.full(shape, T0)
    g = ev.Lattice(D, nx, ny, nz, storage=storage)
    g.set_params(**P, Pr=Pr)
    g.init_fields(rho, T)
    o = oracle.Lattice(D, nx, ny, nz)
    o.set_params(**P, Pr=Pr)
    o.init(rho, T)
    g.step(steps)
    o.step(steps)
    e = _errs(g, o)
    print(f"Pr {Pr} D={D} {storage}: e_rho={e[0]:.3e} e_u={e[1]:.3e} e_T={e[2]:.3e}", flush=True)
    assert max(e) < tol


@pytest.mark.parametrize("Pr", [0.5, 2.0])
def test_prandtl_walls_match_oracle_and_couette_rise(Pr):
    """Walls with Pr != 1: 1000 steps against the oracle (FP64), then the
    subsonic Couette flow (32 cells, U_w = 0.2) to its steady state: the
    central temperature rise against the continuum Pr U_w^2/(20 R) within 3 %
    (the oracle measured 1.002 and 1.019)."""
    nx, Tw, U = 32, 1.5 * synth.T_CRIT, 0.2
    p = dict(R=1.0, a=P["a"], b=P["b"], kappa=0.0, tau=1.0, lam=1.0)
    g = ev.Lattice(2, nx, 1, 1, storage="f64")
    g.set_params(**p, Pr=Pr)
    g.set_walls(Tw, U)
    g.init_fields(np.ones((1, 1, nx)), np.full((1, 1, nx), Tw))
    o = oracle.Lattice(2, nx, 1, 1)
    o.set_params(**p, Pr=Pr)
    o.set_walls(Tw, U)
    o.init(np.ones((1, 1, nx)), np.full((1, 1, nx), Tw))
    g.step(1000)
    o.step(1000)
    e = _errs(g, o)
    print(f"walls Pr {Pr}: e_rho={e[0]:.3e} e_u={e[1]:.3e} e_T={e[2]:.3e}", flush=True)
    assert max(e) < 1e-10
    g.step(39000)
    _, _, T = g.moments()
    an = C.at(C.profile(float(nx), 1.0, Tw, U, P["a"], P["b"], 1.0, Pr=Pr), np.arange(nx) + 0.5)
    ratio = (T.max() / Tw - 1) / (an["T"].max() / Tw - 1)
    print(f"Couette Pr {Pr}: temperature rise ratio {ratio:.4f}", flush=True)
    assert ratio == pytest.approx(1.0, abs=0.03)
