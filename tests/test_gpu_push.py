"""The one-pass D3Q27 step (moments of the next step pushed by the collision,
completed by the fix-up of the tile-chunk shells) against the two-pass step
(moments pulled again before every collision), through the C ABI.

Both compute the same sums of the same stored values, in a different order,
so FP64 runs agree to rounding and the FP32 moment fields agree to a few
ulps.  The shapes cover several tiles with ragged tails in x, y and z, a
lattice one tile wide (its own neighbour), single planes, rows and columns,
and lattices smaller than the stencil halo."""
import numpy as np
import pytest

import oracle.thermo as TH
import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")
P = synth.params()
SQ3 = np.sqrt(3.0)

SHAPES = [(13, 11, 37), (70, 12, 20), (33, 8, 130), (1, 9, 17), (2, 5, 6), (40, 1, 3), (3, 4, 1), (1, 1, 1)]


def _state(shape, noise=1e-3, seed=synth.SEED + 11):
    T0 = 0.85 * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    R = max(0.3 * min(shape), 0.5)
    return synth.droplet(shape, R, rl, rv, noise=noise, seed=seed), np.full(shape, T0)


def _lattice(shape, storage, push, rho, T, graph=True, Pr=1.0):
    nz, ny, nx = shape
    L = ev.Lattice(3, nx, ny, nz, storage=storage)
    L.set_params(**P, Pr=Pr)
    L.set_option(ev.OPT_PUSH_MOMENTS, 1 if push else 0)
    L.set_option(ev.OPT_USE_GRAPH, 1 if graph else 0)
    L.init_fields(rho, T)
    return L


def _errs(a, b):
    (r1, u1, T1), (r2, u2, T2) = a, b
    return (np.abs(r1 - r2).max() / np.abs(r2).max(), np.abs(u1 - u2).max() * SQ3,
            np.abs(T1 - T2).max() / np.abs(T2).max())


@pytest.mark.parametrize("shape", SHAPES)
def test_one_pass_matches_two_pass_f64(shape):
    rho, T = _state(shape)
    print(f"one-pass vs two-pass f64 {shape}", flush=True)
    a = _lattice(shape, "f64", True, rho, T)
    b = _lattice(shape, "f64", False, rho, T)
    a.step(25)
    b.step(25)
    fa, ga = a.get_populations()
    fb, gb = b.get_populations()
    ef = np.abs(fa - fb).max() / np.abs(fb).max()
    eg = np.abs(ga - gb).max() / np.abs(gb).max()
    e = _errs(a.moments(), b.moments())
    print(f"  e_f={ef:.2e} e_g={eg:.2e} e_rho={e[0]:.2e} e_u={e[1]:.2e} e_T={e[2]:.2e}", flush=True)
    assert ef < 1e-12 and eg < 1e-12
    assert max(e) < 1e-12


@pytest.mark.parametrize("Pr", [0.5, 2.0])
@pytest.mark.parametrize("shape", [(13, 11, 37), (70, 12, 20), (2, 5, 6)])
def test_one_pass_matches_two_pass_prandtl_f64(shape, Pr):
    """The one-pass step with the quasi-equilibrium term (Pr != 1) against
    the two-pass step: populations within 1e-12 after 25 steps."""
    rho, T = _state(shape)
    a = _lattice(shape, "f64", True, rho, T, Pr=Pr)
    b = _lattice(shape, "f64", False, rho, T, Pr=Pr)
    a.step(25)
    b.step(25)
    fa, ga = a.get_populations()
    fb, gb = b.get_populations()
    ef = np.abs(fa - fb).max() / np.abs(fb).max()
    eg = np.abs(ga - gb).max() / np.abs(gb).max()
    print(f"one-pass vs two-pass Pr {Pr} f64 {shape}: e_f={ef:.2e} e_g={eg:.2e}", flush=True)
    assert ef < 1e-12 and eg < 1e-12


@pytest.mark.parametrize("Pr", [1.0, 2.0])
@pytest.mark.parametrize("shape", [(5, 6, 65), (3, 4, 1), (1, 1, 1), (4, 9, 129), (13, 11, 37), (41, 5, 70)])
def test_one_pass_matches_two_pass_f32(shape, Pr):
    """FP32 storage (the 64-wide tile, one row per wave), including lattices
    whose last tile is one column wide (nx = 1, 65, 129), where one lane is
    both end lanes of its row, and a one-plane last z-chunk (nz = 41): the
    collision arithmetic is the same in both steps and the moments differ in
    summation order only.  Pr = 2 runs the kernels with the quasi-equilibrium
    term."""
    rho, T = _state(shape)
    print(f"one-pass vs two-pass f32 {shape} Pr {Pr}", flush=True)
    a = _lattice(shape, "f32", True, rho, T, Pr=Pr)
    b = _lattice(shape, "f32", False, rho, T, Pr=Pr)
    a.step(25)
    b.step(25)
    fa, ga = a.get_populations()
    fb, gb = b.get_populations()
    ef = np.abs(fa - fb).max() / np.abs(fb).max()
    eg = np.abs(ga - gb).max() / np.abs(gb).max()
    e = _errs(a.moments(), b.moments())
    print(f"  e_f={ef:.2e} e_g={eg:.2e} e_rho={e[0]:.2e} e_u={e[1]:.2e} e_T={e[2]:.2e}", flush=True)
    assert np.isfinite(fa).all() and np.isfinite(ga).all()
    assert max(ef, eg) < 2e-6 and max(e) < 2e-6


@pytest.mark.parametrize("storage,tol", [("f64", 1e-14), ("f32", 2e-6)])
@pytest.mark.parametrize("shape", [(13, 11, 37), (70, 12, 20), (2, 5, 6)])
def test_pushed_moments_equal_pulled(shape, storage, tol):
    """The moment field the one-pass step carries equals the moments pulled
    from the stored populations (switching the option off pulls them again)."""
    rho, T = _state(shape)
    L = _lattice(shape, storage, True, rho, T)
    L.step(40)
    pushed = L.moments()
    L.set_option(ev.OPT_PUSH_MOMENTS, 0)
    pulled = L.moments()
    e = _errs(pushed, pulled)
    print(f"pushed vs pulled {storage} {shape}: e_rho={e[0]:.2e} e_u={e[1]:.2e} e_T={e[2]:.2e}", flush=True)
    assert max(e) < tol


def test_one_pass_graph_replay_matches_eager():
    """Captured chunks of one-pass steps give the same bits as eager launches,
    across chunk boundaries and remainders."""
    shape = (40, 12, 70)
    rho, T = _state(shape)
    a = _lattice(shape, "f32", True, rho, T, graph=True)
    b = _lattice(shape, "f32", True, rho, T, graph=False)
    for n in (70, 5, 64, 33, 64):
        a.step(n)
        b.step(n)
        fa, ga = a.get_populations()
        fb, gb = b.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), f"after a call of {n} steps"
        ma, mb = a.moments(), b.moments()
        assert all(np.array_equal(x, y) for x, y in zip(ma, mb)), f"moments after a call of {n} steps"


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_one_pass_checkpoint_resume_is_bitwise(storage, tmp_path):
    shape = (36, 10, 70)
    rho, T = _state(shape)
    a = _lattice(shape, storage, True, rho, T)
    a.step(50)
    path = tmp_path / "ck3.evlbm"
    a.checkpoint_save(path)
    a.step(30)
    nz, ny, nx = shape
    b = ev.Lattice(3, nx, ny, nz, storage=storage)
    b.checkpoint_load(path)
    assert b.step_count == 50
    b.step(30)
    fa, ga = a.get_populations()
    fb, gb = b.get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("shape", [(1, 40, 96), (1, 9, 70), (1, 3, 5)])
def test_d2q9_one_pass_equals_two_pass_bitwise(shape, storage):
    """The one-pass D2Q9 step sums each tile's halo moments from the pulled
    populations in the order of the moment kernel, so it is the two-pass step
    bit for bit (ragged tiles in x and y; a lattice smaller than the halo;
    16-bit storage across two re-references, at steps 100 and 200)."""
    nz, ny, nx = shape
    T0 = 0.85 * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    rho = synth.droplet(shape, max(0.3 * min(nx, ny), 0.5), rl, rv, noise=1e-3, seed=synth.SEED + 12)
    T = np.full(shape, T0)
    runs = []
    for push in (1, 0):
        L = ev.Lattice(2, nx, ny, 1, storage=storage)
        L.set_params(**P)
        L.set_option(ev.OPT_PUSH_MOMENTS, push)
        L.init_fields(rho, T)
        L.step(230 if storage in ("f16dev", "bf16dev") else 45)
        runs.append(L)
    print(f"d2q9 one-pass vs two-pass {storage} {shape}", flush=True)
    fa, ga = runs[0].get_populations()
    fb, gb = runs[1].get_populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
