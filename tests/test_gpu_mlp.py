"""Warm-start network on the GPU against the FP64 oracle network, and the
learned warm start against the plain tanh initialisation."""
import numpy as np
import pytest

import oracle.mlp as OM
import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")

TENSORS = [("W1", 0, 192), ("b1", 192, 256), ("W2", 256, 4352), ("b2", 4352, 4416), ("W3", 4416, 8512),
           ("b3", 8512, 8576), ("W4", 8576, 8640), ("b4", 8640, 8641)]


def _params(seed=1):
    p = synth.xavier_params()
    p = p + 0.05 * np.random.default_rng(seed).standard_normal(p.size)
    return p.astype(np.float32).astype(np.float64)  # exactly representable in FP32


def _batch(n, seed=2):
    rng = np.random.default_rng(seed)
    X = np.stack([rng.uniform(0.65, 0.95, n), rng.uniform(15, 80, n), rng.uniform(0, 3, n)], 1)
    Y = 1.0 + 0.8 * np.tanh(2.0 * (1.0 - X[:, 2])) + 0.05 * rng.standard_normal(n)
    return X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1, 16, 100, 1000])
def test_forward_matches_oracle(n):
    p = _params()
    X, _ = _batch(n)
    net = ev.MLP(p)
    y = net.forward(X)
    yo = OM.forward(p, X)
    assert np.abs(y - yo).max() < 2e-5 * max(1.0, np.abs(yo).max())


@pytest.mark.parametrize("shape,centre,R,Tr", [((1, 37, 53), (26.0, 18.0, 0.0), 12.5, 0.8),
                                               ((13, 11, 29), (14.3, 5.0, 6.7), 4.0, 0.7),
                                               ((1, 96, 128), (63.5, 47.5, 0.0), 9.0, 0.85)])
def test_density_field_matches_oracle(shape, centre, R, Tr):
    """evlbm_mlp_density_field (the network evaluated at every cell, MFMA
    layers) against the FP64 oracle network at the same inputs
    (T/Tc, R, min(r/R, 3)), r/R rounded to FP32 as the kernel takes it; the
    last two grids reach r/R = 4 and 8, where the field keeps its value at
    r/R = 3 (the radial range of the training profiles)."""
    p = _params(9)
    net = ev.MLP(p)
    rho_c = 1.25
    got = net.density_field(shape, centre, R, Tr, rho_c).cpu().numpy()
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + ((z - centre[2]) ** 2 if nz > 1 else 0.0)
    rr = np.minimum((np.sqrt(d2) / R).astype(np.float32), np.float32(3.0)).astype(np.float64)
    X = np.stack([np.full(rr.size, np.float32(Tr)), np.full(rr.size, np.float32(R)), rr.ravel()], 1)
    want = rho_c * OM.forward(p, X).reshape(shape)
    err = np.abs(got - want).max() / rho_c
    print(f"density field {shape}: max |d rho|/rho_c = {err:.2e}", flush=True)
    assert err < 2e-5


def test_gradient_matches_oracle():
    """Per-tensor relative L2 error of the FP32 gradient
    against the FP64 oracle below 1e-4."""
    p = _params(3)
    X, Y = _batch(777, 4)
    net = ev.MLP(p)
    g, loss = net.grad(X, Y)
    go = OM.grad(p, X, Y)
    assert loss == pytest.approx(OM.loss(p, X, Y), rel=1e-5)
    for name, a, b in TENSORS:
        err = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        print(f"{name}: rel L2 {err:.2e}", flush=True)
        assert err < 1e-4, name


def test_adam_steps_match_oracle():
    p = _params(5)
    X, Y = _batch(300, 6)
    net = ev.MLP(p)
    hist = net.train(X, Y, 10, lr=1e-3)
    po = p.copy()
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    lo = []
    for t in range(1, 11):
        lo.append(OM.loss(po, X, Y))
        po, m, v = OM.adam_step(po, m, v, OM.grad(po, X, Y), t, lr=1e-3)
    assert np.allclose(hist, lo, rtol=1e-4)
    moved = np.abs(po - p)
    diff = np.abs(net.params() - po)
    assert diff.max() < 1e-3 * moved.max() + 1e-6


def test_tanh_droplet_init_matches_formula():
    shape = (1, 48, 64)
    L = ev.Lattice(2, 64, 48, 1, storage="f64")
    L.set_params(**synth.params())
    used = L.init_droplet(12.0, 0.8)
    assert not used
    rl, rv, _ = ev.eos_coexistence(0.8 * synth.T_CRIT)
    ref = synth.droplet(shape, 12.0, rl, rv, noise=0)
    o = ev.Lattice(2, 64, 48, 1, storage="f64")
    o.set_params(**synth.params())
    o.init_fields(ref, np.full(shape, 0.8 * synth.T_CRIT))
    fa, _ = L.get_populations()
    fb, _ = o.get_populations()
    assert np.abs(fa - fb).max() < 1e-13


def test_learned_warm_start_reduces_steps():
    """Train on long-run droplets of a small sweep, then seed a held-out droplet
    with the plain run's mass and energy.  Against the plain (tanh-seeded)
    run's state after 20000 steps, the warm start starts at least 3x closer
    and gets within 2 % of it in fewer steps.  (The slow thermal mode of this
    parameter set keeps both runs drifting for ~1e5 steps, so a 1e-3 bar is
    not reached within test time.)"""
    from paper_2508_00577_amd import warmstart as W
    params = synth.params()
    shape = (1, 96, 96)
    cases = [(R, Tr) for R in (10.0, 14.0, 18.0, 22.0) for Tr in (0.72, 0.8, 0.88)]
    X, Y = W.training_samples(cases, shape, params, steps=40000, rho_c=1.0)
    net, hist = W.train_network(X, Y, synth.xavier_params(), iters=3000, lr=2e-3)
    print(f"training samples {len(Y)}, loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    assert hist[-1] < 0.05 * hist[0]
    res = W.warm_start_study(net, [(15.0, 0.84)], shape, params, horizon=20000, check=500, tol=2e-2)
    print(res, flush=True)
    r = res[0]
    assert r["mlp_used"]
    assert r["err0_mlp_matched"] < r["err0_tanh"] / 3
    assert r["steps_mlp_matched"] is not None and r["steps_mlp_matched"] < r["steps_tanh"]
    # the trained box's edge (T/Tc = 0.88, held as FP32) is inside it for the
    # same value given in FP64 (R = 14: a training radius whose profiles reach
    # r/R = 3)
    L = ev.Lattice(2, shape[2], shape[1], 1, storage="f32")
    L.set_params(**params)
    assert L.init_droplet(14.0, 0.88, profile="mlp", mlp=net)


def test_network_is_trusted_only_on_its_training_box():
    """A new network has an empty (T/Tc, R) box, so droplets fall back to the
    tanh profile; training grows the box to the inputs' bounds; droplets
    outside it fall back too."""
    net = ev.MLP(synth.xavier_params())
    assert net.hull()[0] > net.hull()[1]
    L = ev.Lattice(2, 64, 48, 1, storage="f32")
    L.set_params(**synth.params())
    assert not L.init_droplet(14.0, 0.8, profile="mlp", mlp=net)
    rng = np.random.default_rng(synth.SEED + 9)
    X = np.stack([rng.uniform(0.72, 0.88, 64), rng.uniform(10.0, 22.0, 64), rng.uniform(0.0, 3.0, 64)], 1)
    Y = rng.uniform(0.2, 1.9, 64)
    net.train(X, Y, iters=2, lr=1e-3)
    lo_t, hi_t, lo_r, hi_r = net.hull()
    assert np.isclose(lo_t, np.float32(X[:, 0].min())) and np.isclose(hi_t, np.float32(X[:, 0].max()))
    assert np.isclose(lo_r, np.float32(X[:, 1].min())) and np.isclose(hi_r, np.float32(X[:, 1].max()))
    for R, Tr in ((30.0, 0.8), (14.0, 0.6), (14.0, 0.95)):
        assert not L.init_droplet(R, Tr, profile="mlp", mlp=net)
    net.set_hull(0.65, 0.97, 12.0, 90.0)
    assert net.hull() == (0.65, 0.97, 12.0, 90.0)
    with pytest.raises(ev.EvlbmError):
        net.set_hull(0.9, 0.8, 12.0, 90.0)
