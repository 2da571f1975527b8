"""GPU parity with the FP64 oracle for Carnahan-Starling's contact factor in
Enskog's pressure (EVLBM_OPT_EOS = EVLBM_EOS_CS), through the C ABI: the
flat-interface workload of 128 x 32 cells at T/Tc = 0.9 (FP64, 1000 steps),
a ragged D3Q27 droplet through the one-pass step (FP64 and FP32), a batched
domain, and the library's bulk pressure measurement.  Tolerances as for the
van der Waals closure: 1e-10 (FP64), 1e-5 (FP32) on moments."""
import numpy as np
import pytest

import oracle
import oracle.thermo as TH
import synth

pytestmark = pytest.mark.gpu

ev = pytest.importorskip("paper_2508_00577_amd")
P = synth.params_cs()
_, TC, _ = TH.critical_point(1.0, P["a"], P["b"], "cs")
SQ3 = np.sqrt(3.0)


def _errs(a, b):
    (r1, u1, T1), (r2, u2, T2) = a, b
    return (np.abs(r1 - r2).max() / np.abs(r2).max(), np.abs(u1 - u2).max() * SQ3,
            np.abs(T1 - T2).max() / np.abs(T2).max())


def _fields(kind, shape, Tr, noise=1e-3):
    T0 = Tr * TC
    rl, rv, _ = TH.coexistence(T0, 1.0, P["a"], P["b"], "cs")
    if kind == "slab":
        rho = synth.slab(shape, rl, rv, noise=noise)
    else:
        rho = synth.droplet(shape, 0.3 * min(s for s in shape if s > 1), rl, rv, noise=noise)
    return rho, np.full(shape, T0)


def _pair(D, shape, storage, rho, T):
    nz, ny, nx = shape
    g = ev.Lattice(D, nx, ny, nz, storage=storage)
    g.set_params(**P)
    g.init_fields(rho, T)
    o = oracle.Lattice(D, nx, ny, nz)
    o.set_params(**P)
    o.init(rho, T)
    return g, o


def test_cs_library_coexistence_matches_oracle():
    for Tr in (0.7, 0.9):
        got = ev.eos_coexistence(Tr * TC, 1.0, P["a"], P["b"], eos="cs")
        ref = TH.coexistence(Tr * TC, 1.0, P["a"], P["b"], "cs")
        np.testing.assert_allclose(got, ref, rtol=1e-8)
    rc, Tc, Pc = ev.eos_critical(1.0, P["a"], P["b"], eos="cs")
    assert Tc == pytest.approx(TC, rel=1e-7)


def test_cs_flat_interface_f64_1000_steps():
    shape = (1, 32, 128)
    rho, T = _fields("slab", shape, 0.9)
    g, o = _pair(2, shape, "f64", rho, T)
    for n, tol in ((1, 1e-12), (99, 1e-11), (900, 1e-10)):
        g.step(n)
        o.step(n)
        rg, ug, Tg = g.moments()
        ro, uo, To, _ = o.moments()
        e = _errs((rg, ug, Tg), (ro, uo, To))
        print(f"CS slab f64 step {g.step_count}: e_rho={e[0]:.3e} e_u={e[1]:.3e} e_T={e[2]:.3e}", flush=True)
        assert max(e) < tol


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_cs_3d_droplet_ragged_one_pass(storage, tol):
    shape = (13, 11, 37)
    rho, T = _fields("droplet", shape, 0.8, 1e-4)
    g, o = _pair(3, shape, storage, rho, T)
    g.step(100)
    o.step(100)
    rg, ug, Tg = g.moments()
    ro, uo, To, _ = o.moments()
    e = _errs((rg, ug, Tg), (ro, uo, To))
    print(f"CS 3d droplet {storage} step 100: e_rho={e[0]:.3e} e_u={e[1]:.3e} e_T={e[2]:.3e}", flush=True)
    assert max(e) < tol


def test_cs_batch_domain_matches_oracle_f64():
    sizes = [(70, 21), (33, 40)]
    B = ev.Batch(sizes, storage="f64")
    B.set_params(**P)
    o = []
    for k, (nx, ny) in enumerate(sizes):
        rho, T = _fields("droplet", (1, ny, nx), 0.85)
        B.init_domain(k, rho, T)
        L = oracle.Lattice(2, nx, ny, 1)
        L.set_params(**P)
        L.init(rho, T)
        o.append(L)
    B.step(200)
    for k, L in enumerate(o):
        L.step(200)
        e = _errs(B.moments(k), L.moments()[:3])
        print(f"CS batch domain {k}: e_rho={e[0]:.3e} e_u={e[1]:.3e} e_T={e[2]:.3e}", flush=True)
        assert max(e) < 1e-11


def test_cs_measured_pressure_uses_the_closure():
    """evlbm_measure's bulk pressure is rho RT Z - a rho^2 of the closure."""
    shape = (1, 16, 64)
    rho, T = _fields("slab", shape, 0.9)
    g, _ = _pair(2, shape, "f64", rho, T)
    g.step(10)
    r, u, TT = g.moments()
    out = g.measure_slab((24, 40), (0, 8), (56, 64))
    sel = np.zeros(64, bool)
    sel[24:40] = True
    Pf = TH.pressure(r[0], TT[0], P["a"], P["b"], "cs")
    assert out[4] == pytest.approx(Pf[:, sel].mean(), rel=1e-12)
