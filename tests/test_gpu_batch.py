"""Batched uneven D2Q9 domains (one persistent launch per kernel and step)."""
import numpy as np
import pytest

import oracle
import oracle.thermo as TH
import synth

pytestmark = pytest.mark.gpu
ev = pytest.importorskip("paper_2508_00577_amd")
P = synth.params()


def _fields(kind, nx, ny, Tr, seed):
    T0 = Tr * synth.T_CRIT
    rl, rv, _ = TH.coexistence(T0)
    shape = (1, ny, nx)
    if kind == "slab":
        rho = synth.slab(shape, rl, rv, noise=1e-3, seed=seed)
    else:
        rho = synth.droplet(shape, 0.25 * min(nx, ny), rl, rv, noise=1e-4, seed=seed)
    return rho, np.full(shape, T0)


DOMS = [("slab", 70, 40, 0.85), ("droplet", 96, 64, 0.75), ("droplet", 33, 17, 0.9), ("slab", 130, 9, 0.7)]


def _batch(storage, variant=0):
    b = ev.Batch([(nx, ny) for _, nx, ny, _ in DOMS], storage=storage)
    b.set_params(**P)
    b.set_tile(variant)
    fields = []
    for k, (kind, nx, ny, Tr) in enumerate(DOMS):
        rho, T = _fields(kind, nx, ny, Tr, synth.SEED * 1000 + k)
        b.init_domain(k, rho, T)
        fields.append((rho, T))
    return b, fields


@pytest.mark.parametrize("storage,steps", [("f32", 70), ("f64", 70), ("f16dev", 230)])
def test_batch_domain_equals_single_lattice_bitwise(storage, steps):
    """With the same tile shape (64 x 16, a single lattice's D2Q9 tile)
    a batched domain evolves bit for bit as the same domain stepped alone (16-bit storage: across two
    re-references, at steps 100 and 200)."""
    b, fields = _batch(storage, 1)
    b.step(steps)
    for k, (kind, nx, ny, Tr) in enumerate(DOMS):
        L = ev.Lattice(2, nx, ny, 1, storage=storage)
        L.set_params(**P)
        L.init_fields(*fields[k])
        L.step(steps)
        fa, ga = b.get_populations(k)
        fb, gb = L.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), f"domain {k}"


# 64 x 16 tiles: 4 x 80 + 4 x 76 = 624, more than the persistent grid holds
# (at most two workgroups of 1024 threads per compute unit)
BIG = [("droplet", 300, 250, 0.8), ("slab", 250, 300, 0.9)] * 4


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_with_more_tiles_than_the_grid(storage):
    """Full rounds of the persistent loop, in which each XCD takes a
    contiguous run of the tile list, then a partial last round: every domain
    still evolves bit for bit as the same domain stepped alone (whose own
    launch deals its 80 or 76 tiles in XCD order), and in FP64 the first
    domain matches the oracle."""
    b = ev.Batch([(nx, ny) for _, nx, ny, _ in BIG], storage=storage)
    b.set_params(**P)
    b.set_tile(1)
    assert b.info()["tiles"] == 624
    fields = []
    for k, (kind, nx, ny, Tr) in enumerate(BIG):
        fields.append(_fields(kind, nx, ny, Tr, synth.SEED * 1000 + 50 + k))
        b.init_domain(k, *fields[k])
    print(f"batch of {len(BIG)} domains, 624 tiles, {storage}", flush=True)
    b.step(20)
    for k, (kind, nx, ny, Tr) in enumerate(BIG):
        L = ev.Lattice(2, nx, ny, 1, storage=storage)
        L.set_params(**P)
        L.init_fields(*fields[k])
        L.step(20)
        fa, ga = b.get_populations(k)
        fb, gb = L.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), f"domain {k}"
    if storage == "f64":
        kind, nx, ny, Tr = BIG[0]
        o = oracle.Lattice(2, nx, ny, 1)
        o.set_params(**P)
        o.init(*fields[0])
        o.step(20)
        fa, ga = b.get_populations(0)
        fo, go = o.get_pops()
        ef = np.abs(fa - fo).max() / np.abs(fo).max()
        eg = np.abs(ga - go).max() / np.abs(go).max()
        print(f"  domain 0 against the oracle: e_f={ef:.2e} e_g={eg:.2e}", flush=True)
        assert ef < 1e-12 and eg < 1e-12


# domains smaller than the radius-3 stencil halo, one row or column of tiles
# thick, next to an ordinary one
TINY = [("droplet", 1, 1, 0.8), ("slab", 2, 3, 0.85), ("slab", 5, 70, 0.7), ("droplet", 70, 5, 0.9),
        ("droplet", 40, 33, 0.8)]


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_tiny_domains(storage):
    """Each tiny domain evolves bit for bit as the same domain stepped alone
    (same 64 x 16 tile), its periodic images wrapping inside the tile; in
    FP64 every domain also matches the oracle."""
    b = ev.Batch([(nx, ny) for _, nx, ny, _ in TINY], storage=storage)
    b.set_params(**P)
    b.set_tile(1)
    fields = []
    for k, (kind, nx, ny, Tr) in enumerate(TINY):
        fields.append(_fields(kind, nx, ny, Tr, synth.SEED * 1000 + 80 + k))
        b.init_domain(k, *fields[k])
    print(f"tiny domains {[(nx, ny) for _, nx, ny, _ in TINY]}, {storage}", flush=True)
    b.step(40)
    for k, (kind, nx, ny, Tr) in enumerate(TINY):
        L = ev.Lattice(2, nx, ny, 1, storage=storage)
        L.set_params(**P)
        L.init_fields(*fields[k])
        L.step(40)
        fa, ga = b.get_populations(k)
        fb, gb = L.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), f"domain {k} ({nx} x {ny})"
        if storage == "f64":
            o = oracle.Lattice(2, nx, ny, 1)
            o.set_params(**P)
            o.init(*fields[k])
            o.step(40)
            fo, go = o.get_pops()
            ef = np.abs(fa - fo).max() / np.abs(fo).max()
            eg = np.abs(ga - go).max() / np.abs(go).max()
            print(f"  {nx} x {ny} against the oracle: e_f={ef:.2e} e_g={eg:.2e}", flush=True)
            assert ef < 1e-12 and eg < 1e-12, f"domain {k} ({nx} x {ny})"


def test_batch_graph_replays_match_eager_steps():
    """Steps replayed from the captured 32-step graph (a call of 64 steps: two
    replays) give the same bits as the same steps launched eagerly (calls of
    16 steps, below the graph chunk); every block is compared after a
    read-back, i.e. with eager work and synchronisation between replays."""
    a, _ = _batch("f32", 0)
    e, _ = _batch("f32", 0)
    for r in range(3):
        a.step(64)
        for _ in range(4):
            e.step(16)
        for k in range(len(DOMS)):
            fa, ga = a.get_populations(k)
            fe, ge = e.get_populations(k)
            assert np.array_equal(fa, fe) and np.array_equal(ga, ge), f"block {r}, domain {k}"


def test_batch_tile_shapes_agree():
    res = []
    for v in range(4):
        b, _ = _batch("f32", v)
        b.step(40)
        res.append([b.get_populations(k)[0] for k in range(len(DOMS))])
    for v in range(1, 4):
        for k in range(len(DOMS)):
            d = np.abs(res[v][k] - res[0][k]).max()
            assert d <= 1e-6 * np.abs(res[0][k]).max(), (v, k, d)
    print("bitwise across tile shapes:", all(np.array_equal(res[v][k], res[0][k]) for v in range(4)
                                                for k in range(len(DOMS))), flush=True)


def test_batch_against_oracle_f64():
    b, fields = _batch("f64", 1)
    b.step(100)
    for k, (kind, nx, ny, Tr) in enumerate(DOMS):
        o = oracle.Lattice(2, nx, ny, 1)
        o.set_params(**P)
        o.init(*fields[k])
        o.step(100)
        ro, uo, To, _ = o.moments()
        rg, ug, Tg = b.moments(k)
        assert np.abs(rg - ro).max() < 1e-10 * ro.max()
        assert np.abs(Tg - To).max() < 1e-10 * To.max()
        assert np.abs(ug - uo).max() * np.sqrt(3) < 1e-10


def test_batch_autotune_restores_state(tmp_path):
    b, _ = _batch("f32", 0)
    b.step(10)
    f0, _ = b.get_populations(1)
    entry = b.autotune(steps=5, cache=str(tmp_path / "tune.json"))
    assert entry["variant"] in range(4) and len(entry["ms_per_step"]) == 4
    f1, _ = b.get_populations(1)
    assert np.array_equal(f0, f1)
    again = b.autotune(steps=5, cache=str(tmp_path / "tune.json"))
    assert again["variant"] == entry["variant"]
    b.step(33)  # graph + eager remainder after the tuned shape is set
    assert np.isfinite(b.moments(0)[0]).all()


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_prandtl_domain_equals_single_lattice_and_oracle(storage):
    """Prandtl number 2 in the batch (the collision with the quasi-equilibrium
    term): every domain bit for bit as the same domain stepped alone on a
    lattice with the same tile shape, and in FP64 the first two domains within
    1e-12 of the oracle after 60 steps."""
    b = ev.Batch([(nx, ny) for _, nx, ny, _ in DOMS], storage=storage)
    b.set_params(**P, Pr=2.0)
    b.set_tile(1)
    fields = []
    for k, (kind, nx, ny, Tr) in enumerate(DOMS):
        rho, T = _fields(kind, nx, ny, Tr, synth.SEED * 1000 + 70 + k)
        b.init_domain(k, rho, T)
        fields.append((rho, T))
    b.step(60)
    for k, (kind, nx, ny, Tr) in enumerate(DOMS):
        L = ev.Lattice(2, nx, ny, 1, storage=storage)
        L.set_params(**P, Pr=2.0)
        L.init_fields(*fields[k])
        L.step(60)
        fa, ga = b.get_populations(k)
        fb, gb = L.get_populations()
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), f"domain {k}"
        if storage == "f64" and k < 2:
            o = oracle.Lattice(2, nx, ny, 1)
            o.set_params(**P, Pr=2.0)
            o.init(*fields[k])
            o.step(60)
            fo, go = o.get_pops()
            e = max(np.abs(fa - fo).max() / np.abs(fo).max(), np.abs(ga - go).max() / np.abs(go).max())
            print(f"Pr 2 batch domain {k} vs oracle: {e:.2e}", flush=True)
            assert e < 1e-12
